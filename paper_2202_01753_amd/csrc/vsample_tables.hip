// Sampling-kernel instantiations for integrand id 3 (tables).
#include "vsample.hpp"

namespace mcubes {

hipError_t launch_sample_f3(int dim, int blocks, int threads, size_t lds_bytes,
                             hipStream_t stream, const SampleArgs &args) {
    switch (dim) {
    case 4: return launch_sample_fd<3, 4>(blocks, threads, lds_bytes, stream, args);
    case 5: return launch_sample_fd<3, 5>(blocks, threads, lds_bytes, stream, args);
    case 6: return launch_sample_fd<3, 6>(blocks, threads, lds_bytes, stream, args);
    case 7: return launch_sample_fd<3, 7>(blocks, threads, lds_bytes, stream, args);
    case 8: return launch_sample_fd<3, 8>(blocks, threads, lds_bytes, stream, args);
    case 9: return launch_sample_fd<3, 9>(blocks, threads, lds_bytes, stream, args);
    case 10: return launch_sample_fd<3, 10>(blocks, threads, lds_bytes, stream, args);
    case 11: return launch_sample_fd<3, 11>(blocks, threads, lds_bytes, stream, args);
    case 12: return launch_sample_fd<3, 12>(blocks, threads, lds_bytes, stream, args);
    case 13: return launch_sample_fd<3, 13>(blocks, threads, lds_bytes, stream, args);
    case 14: return launch_sample_fd<3, 14>(blocks, threads, lds_bytes, stream, args);
    case 15: return launch_sample_fd<3, 15>(blocks, threads, lds_bytes, stream, args);
    case 16: return launch_sample_fd<3, 16>(blocks, threads, lds_bytes, stream, args);
    default: return hipErrorInvalidValue;
    }
}

const void *sample_kernel_f3(int dim) {
    switch (dim) {
    case 4: return reinterpret_cast<const void *>(&vsample_kernel<3, 4>);
    case 5: return reinterpret_cast<const void *>(&vsample_kernel<3, 5>);
    case 6: return reinterpret_cast<const void *>(&vsample_kernel<3, 6>);
    case 7: return reinterpret_cast<const void *>(&vsample_kernel<3, 7>);
    case 8: return reinterpret_cast<const void *>(&vsample_kernel<3, 8>);
    case 9: return reinterpret_cast<const void *>(&vsample_kernel<3, 9>);
    case 10: return reinterpret_cast<const void *>(&vsample_kernel<3, 10>);
    case 11: return reinterpret_cast<const void *>(&vsample_kernel<3, 11>);
    case 12: return reinterpret_cast<const void *>(&vsample_kernel<3, 12>);
    case 13: return reinterpret_cast<const void *>(&vsample_kernel<3, 13>);
    case 14: return reinterpret_cast<const void *>(&vsample_kernel<3, 14>);
    case 15: return reinterpret_cast<const void *>(&vsample_kernel<3, 15>);
    case 16: return reinterpret_cast<const void *>(&vsample_kernel<3, 16>);
    default: return nullptr;
    }
}

}  // namespace mcubes
