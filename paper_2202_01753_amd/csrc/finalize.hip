// Fixed-order reduction of the per-workgroup totals and the histogram
// accumulators of one sampling pass (with the decision that follows it when
// the steps of Alg. 2 run on the device), and the dispatch of the sampling
// kernels by (integrand, dimension).
#include <algorithm>

#include "estimate.hpp"
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

// After pass c.it of a device-steps run: records (I, var), runs
// Weighted-Estimates over the passes so far and Check-Convergence (the same
// code and roundings as the host driver), ends the run if it converged or
// the pass saw a non-finite value, and mirrors all of it to the host.
__device__ void decide(const RunCtl &c, double I, double V, bool bad) {
    RunState *st = c.state;
    const int it = c.it, k = it + 1;
    c.iters[it] = I;
    c.iters[c.itmax + it] = V;
    double est[3] = {st->est[0], st->est[1], st->est[2]};
    int32_t status = kRunGoing;
    if (bad) {
        status = kRunNonFinite;
    } else {
        weighted_estimate(k, c.iters, c.iters + c.itmax, est);
        if (converged_after(k, est, c.tau_rel, c.chi2_max)) status = kRunConverged;
    }
    st->k = k;
    st->status = status;
    for (int i = 0; i < 3; ++i) st->est[i] = est[i];
    if (status != kRunGoing) st->last = it;
    if (c.host) {
        // everything else first, k last: a host that sees k has the rest
        c.host_iters[it] = I;
        c.host_iters[c.itmax + it] = V;
        c.host->status = status;
        for (int i = 0; i < 3; ++i) c.host->est[i] = est[i];
        if (status != kRunGoing) c.host->last = it;
        __threadfence_system();
        *(volatile int32_t *)&c.host->k = k;
        __threadfence_system();
    }
}

// Blocks [0, nhb): kFinThreads bins per block; each thread sums its bin's
// kHistAcc accumulators in order (TwoSum) into out and clears them for the
// next pass.  Block nhb: the totals, each thread summing a strided subset of
// workgroups in order, then a fixed pairwise tree.  All merges are
// TwoSum-compensated.  In a device-steps run the pass's decision follows,
// and the whole launch does nothing once the run has ended.
__global__ void __launch_bounds__(kFinThreads)
finalize_kernel(const double *__restrict__ part, double *__restrict__ hacc, int blocks, int nhist,
                int hist_stride, int nhb, uint32_t *flag, double *out, const RunCtl ctl) {
    // (this launch's own decision can only set last to ctl.it, which keeps
    // every block of it running)
    if (ctl.state && ctl.it > ctl.state->last) return;
    const int tid = threadIdx.x;
    if ((int)blockIdx.x < nhb) {
        const int b = blockIdx.x * kFinThreads + tid;
        if (b < nhist) {
            double *acc = hacc + b;
            double s = 0.0, c = 0.0;
#pragma unroll
            for (int x = 0; x < kHistAcc; ++x) {
                two_sum_merge(s, c, acc[(size_t)x * hist_stride], 0.0);
                acc[(size_t)x * hist_stride] = 0.0;
            }
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
        const double I = red[0][0] + red[0][1], V = red[0][2] + red[0][3];
        const bool bad = *flag != 0u;
        out[0] = I;
        out[1] = V;
        out[2] = bad ? 1.0 : 0.0;
        out[3] = 0.0;
        *flag = 0u;
        if (ctl.state) decide(ctl, I, V, bad);
    }
}

__global__ void clear_flag_kernel(uint32_t *flag) { *flag = 0u; }

__global__ void zero_kernel(double *p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

}  // namespace

hipError_t launch_finalize(const double *partials, double *hist_acc, int blocks, int nhist, int hist_stride,
                           int with_hist, uint32_t *flag, double *out, const RunCtl &ctl,
                           hipStream_t stream) {
    const int nhb = with_hist ? (nhist + kFinThreads - 1) / kFinThreads : 0;
    hipLaunchKernelGGL(finalize_kernel, dim3(nhb + 1), dim3(kFinThreads), 0, stream, partials,
                       hist_acc, blocks, nhist, hist_stride, nhb, flag, out, ctl);
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
