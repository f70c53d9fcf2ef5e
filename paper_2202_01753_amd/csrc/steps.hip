// The steps of Alg. 2 between two sampling passes, on the device, for runs
// that keep them there: the start of a run (Init-Bins and the run state), and
// after each pass one launch that merges the pass's results, runs
// Weighted-Estimates and Check-Convergence, and Adjust-Bin-Bounds.
//
// The bin adjustment takes the host's steps (three-point smoothing, Lepage's
// damped compression, equal shares of the compressed weight per new bin)
// with the same comparisons and the same interpolation, one workgroup per
// axis.  Its sums are formed in a fixed order of its own (each thread a
// contiguous run of bins, then across the threads) rather than the host's
// one bin after another, and pow and log are the device library's, so the
// boundaries agree with the host's to rounding, not bit for bit; the result
// does not depend on timing.  Each new boundary is found by its own thread,
// with a binary search over the running sums for the bin where the host's
// scan would stop.
#include <cmath>

#include "internal.hpp"
#include "merge.hpp"

namespace mcubes {

namespace {

constexpr int kRefineThreads = 256;
static_assert(kRefineThreads == merge::kThreads, "the steps kernel's last workgroup merges the totals");

// The workgroup's threads each take a contiguous run of [first, last): the
// run of thread t.
__device__ __forceinline__ void thread_run(int first, int last, int *a, int *b) {
    const int per = (last - first + (int)blockDim.x - 1) / (int)blockDim.x;
    *a = min(first + (int)threadIdx.x * per, last);
    *b = min(*a + per, last);
}

// x[0] + ... + x[n-1] in a fixed order: each thread its run in order, then a
// butterfly across the wave (every lane ends with the same value), then the
// waves in order.  Returned to every thread.
__device__ double block_sum(const double *x, int n, double *wave_tmp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    int a, b;
    thread_run(0, n, &a, &b);
    double s = 0.0;
    for (int i = a; i < b; ++i) s = s + x[i];
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) s = s + __shfl_xor(s, off, 64);
    if (lane == 0) wave_tmp[wave] = s;
    __syncthreads();
    double t = 0.0;
    for (int w = 0; w < nw; ++w) t = t + wave_tmp[w];
    __syncthreads();
    return t;
}

// In place over [first, last): E[k] = max(lo, E[first], ..., E[k]).  Each
// thread its run, the runs' maxima scanned across the wave and the waves.
// Max is exact, so the grouping does not change the result.
__device__ void running_max(double *E, int first, int last, double lo, double *wave_tmp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int a, b;
    thread_run(first, last, &a, &b);
    double m = lo;
    for (int k = a; k < b; ++k) m = fmax(E[k], m);
    double x = m;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(x, off, 64);
        if (lane >= off) x = fmax(x, y);
    }
    if (lane == 63) wave_tmp[wave] = x;
    __syncthreads();
    double before = lo;
    for (int w = 0; w < wave; ++w) before = fmax(before, wave_tmp[w]);
    const double left = __shfl_up(x, 1, 64);
    if (lane > 0) before = fmax(before, left);
    double run = before;
    for (int k = a; k < b; ++k) {
        run = fmax(E[k], run);
        E[k] = run;
    }
    __syncthreads();
}

// Running sums P[0] = 0, P[i + 1] = x[0] + ... + x[i]: each thread its run
// in order, after the total of everything before it (the runs' totals
// scanned across the wave, then the waves in order).  The rounding of the
// cross-run sums can leave a later P an ulp below an earlier one, so P is
// then made non-decreasing (a running maximum, exact).
__device__ void running_sums(const double *x, int n, double *P, double *wave_tmp) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int a, b;
    thread_run(0, n, &a, &b);
    double s = 0.0;
    for (int i = a; i < b; ++i) s = s + x[i];
    double incl = s;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const double y = __shfl_up(incl, off, 64);
        if (lane >= off) incl = incl + y;
    }
    if (lane == 63) wave_tmp[wave] = incl;
    __syncthreads();
    double before = 0.0;
    for (int w = 0; w < wave; ++w) before = before + wave_tmp[w];
    const double left = __shfl_up(incl, 1, 64);
    if (lane > 0) before = before + left;
    double run = before;
    for (int i = a; i < b; ++i) {
        run = run + x[i];
        P[i + 1] = run;
    }
    if (threadIdx.x == 0) P[0] = 0.0;
    __syncthreads();
    running_max(P, 1, n + 1, 0.0, wave_tmp);
}

__global__ void __launch_bounds__(256) run_init_kernel(RunState *st, double *grid, double *host_grid, int d,
                                                       int nb, int itmax) {
    const int row = nb + 1;
    for (int i = threadIdx.x; i < d * row; i += blockDim.x) {
        const double b = (double)(i % row) / (double)nb;
        grid[i] = b;
        if (host_grid) host_grid[i] = b;
    }
    if (threadIdx.x == 0) {
        st->last = itmax - 1;
        st->status = kRunGoing;
        st->k = 0;
        st->pad = 0;
        st->est[0] = 0.0;
        st->est[1] = INFINITY;
        st->est[2] = NAN;
        st->pad2 = 0.0;
    }
    if (host_grid) __threadfence_system();
}

// Adjust-Bin-Bounds of axis j by one workgroup of kRefineThreads.  On entry
// C (nb doubles, in LDS or device memory) holds the axis's contributions and
// the LDS arrays follow lds: the compressed weights r (nb), their running
// sums P (nb + 1), the old boundaries (nb + 1) and the new ones E (nb + 1).
// grid row j is rewritten in place (m-Cubes1D, j = 0: and copied to every
// axis); host_grid, if not null, receives every boundary written to grid.
// C may be E itself: it is read before E is written.
__device__ __forceinline__ void adjust_axis(double *lds, const double *C, double *grid, double *host_grid, int j, int d,
                            int nb, int one_d, double alpha) {
    double *r = lds, *P = r + nb, *prev = P + nb + 1, *E = prev + nb + 1;
    __shared__ double wave_tmp[kRefineThreads / 64];
    const int tid = threadIdx.x;
    double *B = grid + (size_t)j * (nb + 1);
    for (int i = tid; i <= nb; i += kRefineThreads) prev[i] = B[i];
    // three-point smoothing (two points at the ends)
    for (int i = tid; i < nb; i += kRefineThreads) {
        double s;
        if (i == 0) s = (C[0] + C[1]) / 2.0;
        else if (i == nb - 1) s = (C[nb - 2] + C[nb - 1]) / 2.0;
        else s = ((C[i - 1] + C[i]) + C[i + 1]) / 3.0;
        r[i] = s;
    }
    __syncthreads();
    const double S = block_sum(r, nb, wave_tmp);
    bool moved = S > 0.0 && isfinite(S);  // else the axis keeps its boundaries
    if (moved) {
        // Lepage's damped compression of each bin's share
        for (int i = tid; i < nb; i += kRefineThreads) {
            const double s = r[i];
            r[i] = s == 0.0 ? 0.0 : (s == S ? 1.0 : pow((1.0 - s / S) / log(S / s), alpha));
        }
        __syncthreads();
        running_sums(r, nb, P, wave_tmp);
        moved = P[nb] > 0.0;
    }
    if (moved) {
        // boundary k closes k equal shares of the compressed weight: the
        // host's scan stops at the first bin s with s = nb - 1 or
        // P[s + 1] >= goal (P is non-decreasing, so that test is monotone in
        // s) and interpolates inside it
        const double per_bin = P[nb] / (double)nb;
        for (int k = 1 + tid; k < nb; k += kRefineThreads) {
            const double goal = (double)k * per_bin;
            int lo = 0, hi = nb - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (P[mid + 1] < goal) lo = mid + 1;
                else hi = mid;
            }
            const int src = lo;
            double frac = r[src] > 0.0 ? (goal - P[src]) / r[src] : 0.0;
            frac = fmin(fmax(frac, 0.0), 1.0);
            E[k] = __fma_rn(frac, prev[src + 1] - prev[src], prev[src]);
        }
        __syncthreads();
        // boundaries never decrease: each is at least the one before (the
        // first at least the old lower end)
        running_max(E, 1, nb, prev[0], wave_tmp);
        if (tid == 0) {
            E[0] = 0.0;
            E[nb] = 1.0;
        }
        __syncthreads();
        for (int i = tid; i <= nb; i += kRefineThreads) B[i] = E[i];
        if (host_grid)
            for (int i = tid; i <= nb; i += kRefineThreads) host_grid[(size_t)j * (nb + 1) + i] = E[i];
    }
    // m-Cubes1D: axis 0's boundaries, adjusted or not, on every axis
    if (one_d) {
        const double *src = moved ? E : prev;
        for (int c = 1; c < d; ++c)
            for (int i = tid; i <= nb; i += kRefineThreads) {
                B[(size_t)c * (nb + 1) + i] = src[i];
                if (host_grid) host_grid[(size_t)c * (nb + 1) + i] = src[i];
            }
    }
    if (host_grid) __threadfence_system();
}

// mc_refine_grid_device: one workgroup per axis (m-Cubes1D: one), the
// contributions read from hist.
__global__ void __launch_bounds__(kRefineThreads)
refine_kernel(double *grid, const double *hist, int d, int nb, int one_d, double alpha) {
    extern __shared__ double lds[];
    adjust_axis(lds, hist + (size_t)blockIdx.x * nb, grid, nullptr, blockIdx.x, d, nb, one_d, alpha);
}

// Everything between pass it and the next of a device-steps run, in one
// launch (nothing once the run has ended before pass it).  Workgroups
// [0, nref) adjust one axis each (nref = 0 in a No-Adjust pass), taking the
// axis's contributions from the histogram accumulators (summed in order and
// cleared, as the finalize does); workgroup nref merges the totals and takes
// the pass's decision.  The adjustment of pass it does not depend on that
// decision (a run refines after its last adjusting pass too).
__global__ void __launch_bounds__(kRefineThreads) steps_kernel(const StepsArgs A) {
    if (A.ctl.it > A.ctl.state->last) return;  // (this launch sets last to it at most)
    extern __shared__ double lds[];
    if ((int)blockIdx.x < A.nref) {
        const int j = blockIdx.x, nb = A.nb;
        double *C = lds + 3 * (size_t)nb + 2;  // the E array, free until the search
        for (int i = threadIdx.x; i < nb; i += kRefineThreads)
            C[i] = merge::take_bin(A.hist_acc, (size_t)j * nb + i, A.hist_stride);
        __syncthreads();
        adjust_axis(lds, C, A.grid, A.host_grid, j, A.d, nb, A.one_d, A.alpha);
        return;
    }
    double I = 0.0, V = 0.0;
    merge::pass_totals(A.partials, A.blocks, &I, &V);
    if (threadIdx.x == 0) {
        const bool bad = *A.flag != 0u;
        *A.flag = 0u;
        merge::decide(A.ctl, I, V, bad);
    }
}

}  // namespace

size_t refine_lds_bytes(int nb) { return sizeof(double) * (4 * (size_t)nb + 3); }

hipError_t launch_run_init(RunState *state, double *grid, double *host_grid, int d, int nb, int itmax,
                           hipStream_t stream) {
    hipLaunchKernelGGL(run_init_kernel, dim3(1), dim3(256), 0, stream, state, grid, host_grid, d, nb,
                       itmax);
    return hipGetLastError();
}

hipError_t launch_refine(double *grid, const double *hist, int d, int nb, int one_d, double alpha,
                         hipStream_t stream) {
    const size_t lds = refine_lds_bytes(nb);
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&refine_kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(refine_kernel, dim3(one_d ? 1 : d), dim3(kRefineThreads), lds, stream, grid,
                       hist, d, nb, one_d, alpha);
    return hipGetLastError();
}

hipError_t launch_steps(const StepsArgs &args, hipStream_t stream) {
    const size_t lds = args.nref ? refine_lds_bytes(args.nb) : 0;
    if (lds > 64 * 1024) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&steps_kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(steps_kernel, dim3(args.nref + 1), dim3(kRefineThreads), lds, stream, args);
    return hipGetLastError();
}

}  // namespace mcubes
