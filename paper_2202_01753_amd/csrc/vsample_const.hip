// Sampling-kernel instantiations for integrand id 0 (const).
#include "vsample.hpp"

namespace mcubes {

hipError_t launch_sample_f0(int dim, int blocks, int threads, size_t lds_bytes,
                             hipStream_t stream, const SampleArgs &args) {
    switch (dim) {
    case 1: return launch_sample_fd<0, 1>(blocks, threads, lds_bytes, stream, args);
    case 2: return launch_sample_fd<0, 2>(blocks, threads, lds_bytes, stream, args);
    case 3: return launch_sample_fd<0, 3>(blocks, threads, lds_bytes, stream, args);
    case 4: return launch_sample_fd<0, 4>(blocks, threads, lds_bytes, stream, args);
    case 5: return launch_sample_fd<0, 5>(blocks, threads, lds_bytes, stream, args);
    case 6: return launch_sample_fd<0, 6>(blocks, threads, lds_bytes, stream, args);
    case 7: return launch_sample_fd<0, 7>(blocks, threads, lds_bytes, stream, args);
    case 8: return launch_sample_fd<0, 8>(blocks, threads, lds_bytes, stream, args);
    case 9: return launch_sample_fd<0, 9>(blocks, threads, lds_bytes, stream, args);
    case 10: return launch_sample_fd<0, 10>(blocks, threads, lds_bytes, stream, args);
    case 11: return launch_sample_fd<0, 11>(blocks, threads, lds_bytes, stream, args);
    case 12: return launch_sample_fd<0, 12>(blocks, threads, lds_bytes, stream, args);
    case 13: return launch_sample_fd<0, 13>(blocks, threads, lds_bytes, stream, args);
    case 14: return launch_sample_fd<0, 14>(blocks, threads, lds_bytes, stream, args);
    case 15: return launch_sample_fd<0, 15>(blocks, threads, lds_bytes, stream, args);
    case 16: return launch_sample_fd<0, 16>(blocks, threads, lds_bytes, stream, args);
    default: return hipErrorInvalidValue;
    }
}

const void *sample_kernel_f0(int dim) {
    switch (dim) {
    case 1: return reinterpret_cast<const void *>(&vsample_kernel<0, 1>);
    case 2: return reinterpret_cast<const void *>(&vsample_kernel<0, 2>);
    case 3: return reinterpret_cast<const void *>(&vsample_kernel<0, 3>);
    case 4: return reinterpret_cast<const void *>(&vsample_kernel<0, 4>);
    case 5: return reinterpret_cast<const void *>(&vsample_kernel<0, 5>);
    case 6: return reinterpret_cast<const void *>(&vsample_kernel<0, 6>);
    case 7: return reinterpret_cast<const void *>(&vsample_kernel<0, 7>);
    case 8: return reinterpret_cast<const void *>(&vsample_kernel<0, 8>);
    case 9: return reinterpret_cast<const void *>(&vsample_kernel<0, 9>);
    case 10: return reinterpret_cast<const void *>(&vsample_kernel<0, 10>);
    case 11: return reinterpret_cast<const void *>(&vsample_kernel<0, 11>);
    case 12: return reinterpret_cast<const void *>(&vsample_kernel<0, 12>);
    case 13: return reinterpret_cast<const void *>(&vsample_kernel<0, 13>);
    case 14: return reinterpret_cast<const void *>(&vsample_kernel<0, 14>);
    case 15: return reinterpret_cast<const void *>(&vsample_kernel<0, 15>);
    case 16: return reinterpret_cast<const void *>(&vsample_kernel<0, 16>);
    default: return nullptr;
    }
}

}  // namespace mcubes
