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

template <int F, int D>
static const void *symbol(bool trace, bool fp32) {
    if (fp32)
        return trace ? reinterpret_cast<const void *>(&vsample_kernel<F, D, true, true>)
                     : reinterpret_cast<const void *>(&vsample_kernel<F, D, false, true>);
    return trace ? reinterpret_cast<const void *>(&vsample_kernel<F, D, true, false>)
                 : reinterpret_cast<const void *>(&vsample_kernel<F, D, false, false>);
}

const void *sample_kernel_f3(int dim, bool trace, bool fp32) {
    switch (dim) {
    case 4: return symbol<3, 4>(trace, fp32);
    case 5: return symbol<3, 5>(trace, fp32);
    case 6: return symbol<3, 6>(trace, fp32);
    case 7: return symbol<3, 7>(trace, fp32);
    case 8: return symbol<3, 8>(trace, fp32);
    case 9: return symbol<3, 9>(trace, fp32);
    case 10: return symbol<3, 10>(trace, fp32);
    case 11: return symbol<3, 11>(trace, fp32);
    case 12: return symbol<3, 12>(trace, fp32);
    case 13: return symbol<3, 13>(trace, fp32);
    case 14: return symbol<3, 14>(trace, fp32);
    case 15: return symbol<3, 15>(trace, fp32);
    case 16: return symbol<3, 16>(trace, fp32);
    default: return nullptr;
    }
}

}  // namespace mcubes
