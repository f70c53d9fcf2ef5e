// Sampling-kernel instantiations for integrand id 1 (gauss).
#include "vsample.hpp"

namespace mcubes {

hipError_t launch_sample_f1(int dim, int blocks, int threads, size_t lds_bytes,
                             hipStream_t stream, const SampleArgs &args) {
    switch (dim) {
    case 1: return launch_sample_fd<1, 1>(blocks, threads, lds_bytes, stream, args);
    case 2: return launch_sample_fd<1, 2>(blocks, threads, lds_bytes, stream, args);
    case 3: return launch_sample_fd<1, 3>(blocks, threads, lds_bytes, stream, args);
    case 4: return launch_sample_fd<1, 4>(blocks, threads, lds_bytes, stream, args);
    case 5: return launch_sample_fd<1, 5>(blocks, threads, lds_bytes, stream, args);
    case 6: return launch_sample_fd<1, 6>(blocks, threads, lds_bytes, stream, args);
    case 7: return launch_sample_fd<1, 7>(blocks, threads, lds_bytes, stream, args);
    case 8: return launch_sample_fd<1, 8>(blocks, threads, lds_bytes, stream, args);
    case 9: return launch_sample_fd<1, 9>(blocks, threads, lds_bytes, stream, args);
    case 10: return launch_sample_fd<1, 10>(blocks, threads, lds_bytes, stream, args);
    case 11: return launch_sample_fd<1, 11>(blocks, threads, lds_bytes, stream, args);
    case 12: return launch_sample_fd<1, 12>(blocks, threads, lds_bytes, stream, args);
    case 13: return launch_sample_fd<1, 13>(blocks, threads, lds_bytes, stream, args);
    case 14: return launch_sample_fd<1, 14>(blocks, threads, lds_bytes, stream, args);
    case 15: return launch_sample_fd<1, 15>(blocks, threads, lds_bytes, stream, args);
    case 16: return launch_sample_fd<1, 16>(blocks, threads, lds_bytes, stream, args);
    default: return hipErrorInvalidValue;
    }
}

const void *sample_kernel_f1(int dim) {
    switch (dim) {
    case 1: return reinterpret_cast<const void *>(&vsample_kernel<1, 1>);
    case 2: return reinterpret_cast<const void *>(&vsample_kernel<1, 2>);
    case 3: return reinterpret_cast<const void *>(&vsample_kernel<1, 3>);
    case 4: return reinterpret_cast<const void *>(&vsample_kernel<1, 4>);
    case 5: return reinterpret_cast<const void *>(&vsample_kernel<1, 5>);
    case 6: return reinterpret_cast<const void *>(&vsample_kernel<1, 6>);
    case 7: return reinterpret_cast<const void *>(&vsample_kernel<1, 7>);
    case 8: return reinterpret_cast<const void *>(&vsample_kernel<1, 8>);
    case 9: return reinterpret_cast<const void *>(&vsample_kernel<1, 9>);
    case 10: return reinterpret_cast<const void *>(&vsample_kernel<1, 10>);
    case 11: return reinterpret_cast<const void *>(&vsample_kernel<1, 11>);
    case 12: return reinterpret_cast<const void *>(&vsample_kernel<1, 12>);
    case 13: return reinterpret_cast<const void *>(&vsample_kernel<1, 13>);
    case 14: return reinterpret_cast<const void *>(&vsample_kernel<1, 14>);
    case 15: return reinterpret_cast<const void *>(&vsample_kernel<1, 15>);
    case 16: return reinterpret_cast<const void *>(&vsample_kernel<1, 16>);
    default: return nullptr;
    }
}

}  // namespace mcubes
