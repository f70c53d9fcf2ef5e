// Fixed-order merges of one sampling pass's results, shared by the finalize
// kernel (steps between passes on the host) and the steps kernel (on the
// device): the per-workgroup totals, the histogram accumulators, and the
// decision that ends a device-steps run.
#pragma once

#include "estimate.hpp"
#include "internal.hpp"

namespace mcubes {
namespace merge {

constexpr int kThreads = 256;  // threads of the workgroups that merge

__device__ __forceinline__ void two_sum_merge(double &s, double &c, double s2, double c2) {
    const double t = s + s2;
    const double bp = t - s;
    const double e = (s - (t - bp)) + (s2 - bp);
    s = t;
    c = (c + c2) + e;
}

// The per-workgroup totals of a pass (per workgroup: I sum and compensation,
// var sum and compensation) merged by one workgroup of kThreads in a fixed
// order: each thread a strided subset in workgroup order, then a pairwise
// tree; all merges TwoSum-compensated.  Thread 0 gets I and var.
__device__ inline void pass_totals(const double *part, int blocks, double *I, double *V) {
    __shared__ double red[kThreads][4];
    const int tid = threadIdx.x;
    double sI = 0.0, cI = 0.0, sV = 0.0, cV = 0.0;
    for (int w = tid; w < blocks; w += kThreads) {
        const double *o = part + 4 * (size_t)w;
        two_sum_merge(sI, cI, o[0], o[1]);
        two_sum_merge(sV, cV, o[2], o[3]);
    }
    red[tid][0] = sI;
    red[tid][1] = cI;
    red[tid][2] = sV;
    red[tid][3] = cV;
    __syncthreads();
    for (int half = kThreads / 2; half >= 1; half >>= 1) {
        if (tid < half) {
            two_sum_merge(red[tid][0], red[tid][1], red[tid + half][0], red[tid + half][1]);
            two_sum_merge(red[tid][2], red[tid][3], red[tid + half][2], red[tid + half][3]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        *I = red[0][0] + red[0][1];
        *V = red[0][2] + red[0][3];
    }
}

// Bin b of the histogram: its kHistAcc accumulators summed in order
// (TwoSum) and cleared for the next pass.
__device__ __forceinline__ double take_bin(double *hacc, size_t b, int hist_stride) {
    double *acc = hacc + b;
    double s = 0.0, c = 0.0;
#pragma unroll
    for (int x = 0; x < kHistAcc; ++x) {
        two_sum_merge(s, c, acc[(size_t)x * hist_stride], 0.0);
        acc[(size_t)x * hist_stride] = 0.0;
    }
    return s + c;
}

// After pass c.it of a device-steps run: records (I, var), runs
// Weighted-Estimates over the passes so far and Check-Convergence (the same
// code and roundings as the host driver), ends the run if it converged or
// the pass saw a non-finite value, and mirrors all of it to the host.
__device__ inline void decide(const RunCtl &c, double I, double V, bool bad) {
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

}  // namespace merge
}  // namespace mcubes
