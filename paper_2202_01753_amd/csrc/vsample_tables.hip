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

const void *sample_kernel_f3(int dim, bool trace) {
    switch (dim) {
    case 4: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 4, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 4, false>);
    case 5: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 5, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 5, false>);
    case 6: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 6, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 6, false>);
    case 7: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 7, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 7, false>);
    case 8: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 8, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 8, false>);
    case 9: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 9, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 9, false>);
    case 10: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 10, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 10, false>);
    case 11: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 11, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 11, false>);
    case 12: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 12, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 12, false>);
    case 13: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 13, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 13, false>);
    case 14: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 14, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 14, false>);
    case 15: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 15, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 15, false>);
    case 16: return trace ? reinterpret_cast<const void *>(&vsample_kernel<3, 16, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<3, 16, false>);
    default: return nullptr;
    }
}

}  // namespace mcubes
