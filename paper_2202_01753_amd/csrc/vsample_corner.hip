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

const void *sample_kernel_f2(int dim, bool trace) {
    switch (dim) {
    case 1: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 1, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 1, false>);
    case 2: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 2, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 2, false>);
    case 3: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 3, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 3, false>);
    case 4: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 4, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 4, false>);
    case 5: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 5, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 5, false>);
    case 6: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 6, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 6, false>);
    case 7: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 7, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 7, false>);
    case 8: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 8, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 8, false>);
    case 9: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 9, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 9, false>);
    case 10: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 10, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 10, false>);
    case 11: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 11, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 11, false>);
    case 12: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 12, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 12, false>);
    case 13: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 13, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 13, false>);
    case 14: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 14, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 14, false>);
    case 15: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 15, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 15, false>);
    case 16: return trace ? reinterpret_cast<const void *>(&vsample_kernel<2, 16, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<2, 16, false>);
    default: return nullptr;
    }
}

}  // namespace mcubes
