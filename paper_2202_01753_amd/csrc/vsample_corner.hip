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

template <int F, int D>
static const void *symbol(bool trace, bool fp32) {
    if (fp32)
        return trace ? reinterpret_cast<const void *>(&vsample_kernel<F, D, true, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<F, D, false, true>);
    return trace ? reinterpret_cast<const void *>(&vsample_kernel<F, D, true, false>)
                 : reinterpret_cast<const void *>(&vsample_kernel<F, D, false, false>);
}

const void *sample_kernel_f2(int dim, bool trace, bool fp32) {
    switch (dim) {
    case 1: return symbol<2, 1>(trace, fp32);
    case 2: return symbol<2, 2>(trace, fp32);
    case 3: return symbol<2, 3>(trace, fp32);
    case 4: return symbol<2, 4>(trace, fp32);
    case 5: return symbol<2, 5>(trace, fp32);
    case 6: return symbol<2, 6>(trace, fp32);
    case 7: return symbol<2, 7>(trace, fp32);
    case 8: return symbol<2, 8>(trace, fp32);
    case 9: return symbol<2, 9>(trace, fp32);
    case 10: return symbol<2, 10>(trace, fp32);
    case 11: return symbol<2, 11>(trace, fp32);
    case 12: return symbol<2, 12>(trace, fp32);
    case 13: return symbol<2, 13>(trace, fp32);
    case 14: return symbol<2, 14>(trace, fp32);
    case 15: return symbol<2, 15>(trace, fp32);
    case 16: return symbol<2, 16>(trace, fp32);
    default: return nullptr;
    }
}

}  // namespace mcubes
