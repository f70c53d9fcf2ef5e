// Sampling-kernel instantiations for integrand id 2 (corner).
#include "vsample.hpp"

namespace mcubes {

hipError_t launch_sample_f2(int dim, int blocks, int threads, size_t lds_bytes,
                             hipStream_t stream, const SampleArgs &args) {
    switch (dim) {
    case 1: return launch_sample_fd<2, 1>(blocks, threads, lds_bytes, stream, args);
    case 2: return launch_sample_fd<2, 2>(blocks, threads, lds_bytes, stream, args);
    case 3: return launch_sample_fd<2, 3>(blocks, threads, lds_bytes, stream, args);
    case 4: return launch_sample_fd<2, 4>(blocks, threads, lds_bytes, stream, args);
    case 5: return launch_sample_fd<2, 5>(blocks, threads, lds_bytes, stream, args);
    case 6: return launch_sample_fd<2, 6>(blocks, threads, lds_bytes, stream, args);
    case 7: return launch_sample_fd<2, 7>(blocks, threads, lds_bytes, stream, args);
    case 8: return launch_sample_fd<2, 8>(blocks, threads, lds_bytes, stream, args);
    case 9: return launch_sample_fd<2, 9>(blocks, threads, lds_bytes, stream, args);
    case 10: return launch_sample_fd<2, 10>(blocks, threads, lds_bytes, stream, args);
    case 11: return launch_sample_fd<2, 11>(blocks, threads, lds_bytes, stream, args);
    case 12: return launch_sample_fd<2, 12>(blocks, threads, lds_bytes, stream, args);
    case 13: return launch_sample_fd<2, 13>(blocks, threads, lds_bytes, stream, args);
    case 14: return launch_sample_fd<2, 14>(blocks, threads, lds_bytes, stream, args);
    case 15: return launch_sample_fd<2, 15>(blocks, threads, lds_bytes, stream, args);
    case 16: return launch_sample_fd<2, 16>(blocks, threads, lds_bytes, stream, args);
    default: return hipErrorInvalidValue;
    }
}

const void *sample_kernel_f2(int dim) {
    switch (dim) {
    case 1: return reinterpret_cast<const void *>(&vsample_kernel<2, 1>);
    case 2: return reinterpret_cast<const void *>(&vsample_kernel<2, 2>);
    case 3: return reinterpret_cast<const void *>(&vsample_kernel<2, 3>);
    case 4: return reinterpret_cast<const void *>(&vsample_kernel<2, 4>);
    case 5: return reinterpret_cast<const void *>(&vsample_kernel<2, 5>);
    case 6: return reinterpret_cast<const void *>(&vsample_kernel<2, 6>);
    case 7: return reinterpret_cast<const void *>(&vsample_kernel<2, 7>);
    case 8: return reinterpret_cast<const void *>(&vsample_kernel<2, 8>);
    case 9: return reinterpret_cast<const void *>(&vsample_kernel<2, 9>);
    case 10: return reinterpret_cast<const void *>(&vsample_kernel<2, 10>);
    case 11: return reinterpret_cast<const void *>(&vsample_kernel<2, 11>);
    case 12: return reinterpret_cast<const void *>(&vsample_kernel<2, 12>);
    case 13: return reinterpret_cast<const void *>(&vsample_kernel<2, 13>);
    case 14: return reinterpret_cast<const void *>(&vsample_kernel<2, 14>);
    case 15: return reinterpret_cast<const void *>(&vsample_kernel<2, 15>);
    case 16: return reinterpret_cast<const void *>(&vsample_kernel<2, 16>);
    default: return nullptr;
    }
}

}  // namespace mcubes
