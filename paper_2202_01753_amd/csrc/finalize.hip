// Fixed-order reduction of the per-workgroup totals and the histogram
// accumulators of one sampling pass when the steps of Alg. 2 run on the host,
// and the dispatch of the sampling kernels by (integrand, dimension).
#include <algorithm>

#include "internal.hpp"
#include "merge.hpp"

namespace mcubes {

hipError_t launch_sample_f0(int, int, int, size_t, hipStream_t, const SampleArgs &);
hipError_t launch_sample_f1(int, int, int, size_t, hipStream_t, const SampleArgs &);
hipError_t launch_sample_f2(int, int, int, size_t, hipStream_t, const SampleArgs &);
hipError_t launch_sample_f3(int, int, int, size_t, hipStream_t, const SampleArgs &);
const void *sample_kernel_f0(int, bool, bool);
const void *sample_kernel_f1(int, bool, bool);
const void *sample_kernel_f2(int, bool, bool);
const void *sample_kernel_f3(int, bool, bool);

const void *sample_kernel(int integrand, int dim, bool trace, bool fp32) {
    switch (integrand) {
    case 0: return sample_kernel_f0(dim, trace, fp32);
    case 1: return sample_kernel_f1(dim, trace, fp32);
    case 2: return sample_kernel_f2(dim, trace, fp32);
    case 3: return sample_kernel_f3(dim, trace, fp32);
    default: return nullptr;
    }
}

hipError_t launch_sample(int integrand, int dim, int blocks, int threads, size_t lds_bytes,
                         hipStream_t stream, const SampleArgs &args) {
    switch (integrand) {
    case 0: return launch_sample_f0(dim, blocks, threads, lds_bytes, stream, args);
    case 1: return launch_sample_f1(dim, blocks, threads, lds_bytes, stream, args);
    case 2: return launch_sample_f2(dim, blocks, threads, lds_bytes, stream, args);
    case 3: return launch_sample_f3(dim, blocks, threads, lds_bytes, stream, args);
    default: return hipErrorInvalidValue;
    }
}

namespace {

using merge::kThreads;

// Blocks [0, nhb): kThreads bins per block, each thread one bin's
// accumulators summed in order into out and cleared for the next pass.
// Block nhb: the totals (merge::pass_totals) and the non-finite flag.
__global__ void __launch_bounds__(kThreads)
finalize_kernel(const double *__restrict__ part, double *__restrict__ hacc, int blocks, int nhist,
                int hist_stride, int nhb, uint32_t *flag, double *out) {
    if ((int)blockIdx.x < nhb) {
        const int b = blockIdx.x * kThreads + threadIdx.x;
        if (b < nhist) out[4 + b] = merge::take_bin(hacc, b, hist_stride);
        return;
    }
    double I = 0.0, V = 0.0;
    merge::pass_totals(part, blocks, &I, &V);
    if (threadIdx.x == 0) {
        out[0] = I;
        out[1] = V;
        out[2] = *flag ? 1.0 : 0.0;
        out[3] = 0.0;
        *flag = 0u;
    }
}

__global__ void clear_flag_kernel(uint32_t *flag) { *flag = 0u; }

__global__ void zero_kernel(double *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

}  // namespace

hipError_t launch_finalize(const double *partials, double *hist_acc, int blocks, int nhist, int hist_stride,
                           int with_hist, uint32_t *flag, double *out, hipStream_t stream) {
    const int nhb = with_hist ? (nhist + kThreads - 1) / kThreads : 0;
    hipLaunchKernelGGL(finalize_kernel, dim3(nhb + 1), dim3(kThreads), 0, stream, partials,
                       hist_acc, blocks, nhist, hist_stride, nhb, flag, out);
    return hipGetLastError();
}

hipError_t launch_clear_flag(uint32_t *flag, hipStream_t stream) {
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, stream, flag);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, size_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    const size_t blocks = std::min<size_t>((n + 255) / 256, 1024);
    hipLaunchKernelGGL(zero_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, n);
    return hipGetLastError();
}

}  // namespace mcubes
