// Fixed-order reduction of the per-workgroup partials of one sampling pass,
// and the dispatch of the sampling kernels by (integrand, dimension).
#include "internal.hpp"

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

constexpr int kFinThreads = 256;

__device__ __forceinline__ void two_sum_merge(double &s, double &c, double s2, double c2) {
    const double t = s + s2;
    const double bp = t - s;
    const double e = (s - (t - bp)) + (s2 - bp);
    s = t;
    c = (c + c2) + e;
}

// 16 bins per block and 16 groups of workgroup rows per bin: at d = 6,
// nb = 500 that is 188 blocks, which spread the read of the partials over
// most of the CUs (32 bins per block left 94 blocks and took 1.6x as long).
constexpr int kFinBins = 16;                        // bins per histogram block
constexpr int kFinGroups = kFinThreads / kFinBins;  // workgroup-row groups per bin

// Blocks [0, nhb): kFinBins bins per block; for each bin, group q sums the
// workgroup rows q, q + kFinGroups, ... in order and the groups are merged in
// order, so the result depends only on the number of workgroups.  Block nhb:
// the totals, each thread summing a strided subset of workgroups in order,
// then a fixed pairwise tree.  All merges are TwoSum-compensated.
__global__ void __launch_bounds__(kFinThreads)
finalize_kernel(const double *__restrict__ part, int blocks, int nhist, int hist_stride, int nhb,
                uint32_t *flag, double *out) {
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < nhb) {
        __shared__ double gs[kFinGroups][kFinBins], gc[kFinGroups][kFinBins];
        const int lane = tid % kFinBins, grp = tid / kFinBins;
        const int b = blockIdx.x * kFinBins + lane;
        double s = 0.0, c = 0.0;
        if (b < nhist) {
            const double *col = part + 4 * (size_t)blocks + b;
#pragma unroll 4
            for (int w = grp; w < blocks; w += kFinGroups)
                two_sum_merge(s, c, col[(size_t)w * hist_stride], 0.0);
        }
        gs[grp][lane] = s;
        gc[grp][lane] = c;
        __syncthreads();
        if (grp == 0 && b < nhist) {
            for (int q = 1; q < kFinGroups; ++q) two_sum_merge(s, c, gs[q][lane], gc[q][lane]);
            out[4 + b] = s + c;
        }
        return;
    }
    __shared__ double red[kFinThreads][4];
    double sI = 0.0, cI = 0.0, sV = 0.0, cV = 0.0;
    for (int w = tid; w < blocks; w += kFinThreads) {
        const double *o = part + 4 * (size_t)w;
        two_sum_merge(sI, cI, o[0], o[1]);
        two_sum_merge(sV, cV, o[2], o[3]);
    }
    red[tid][0] = sI;
    red[tid][1] = cI;
    red[tid][2] = sV;
    red[tid][3] = cV;
    __syncthreads();
    for (int half = kFinThreads / 2; half >= 1; half >>= 1) {
        if (tid < half) {
            two_sum_merge(red[tid][0], red[tid][1], red[tid + half][0], red[tid + half][1]);
            two_sum_merge(red[tid][2], red[tid][3], red[tid + half][2], red[tid + half][3]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        out[0] = red[0][0] + red[0][1];
        out[1] = red[0][2] + red[0][3];
        out[2] = *flag ? 1.0 : 0.0;
        out[3] = 0.0;
        *flag = 0u;
    }
}

__global__ void clear_flag_kernel(uint32_t *flag) { *flag = 0u; }

}  // namespace

hipError_t launch_finalize(const double *partials, int blocks, int nhist, int hist_stride,
                           int with_hist, uint32_t *flag, double *out, hipStream_t stream) {
    const int nhb = with_hist ? (nhist + kFinBins - 1) / kFinBins : 0;
    hipLaunchKernelGGL(finalize_kernel, dim3(nhb + 1), dim3(kFinThreads), 0, stream, partials,
                       blocks, nhist, hist_stride, nhb, flag, out);
    return hipGetLastError();
}

hipError_t launch_clear_flag(uint32_t *flag, hipStream_t stream) {
    hipLaunchKernelGGL(clear_flag_kernel, dim3(1), dim3(1), 0, stream, flag);
    return hipGetLastError();
}

}  // namespace mcubes
