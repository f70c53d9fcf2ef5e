// Batched V-Sample: the sampling passes of many independent integrals (any
// mix of integrand, dimension and bin count) in one persistent launch.  The
// host splits the active integrals' sub-cubes into contiguous segments of
// bounded work and orders them largest first; the workgroups take segments
// from a shared counter until none is left, so they finish together whatever
// the actual cost of each integrand.  For each segment the workgroup loads
// that integral's grid into LDS, samples the segment's cubes
// with the same per-cube code as the single-integral kernel, writes the
// segment's totals to its own slot and adds its LDS histogram into the
// integral's.  A second kernel merges every integral's segment totals in
// order (so the totals do not depend on which workgroup took which segment),
// and a third adjusts the grids of the integrals still in their adjusting
// iterations, on the device, so that grids and histograms never leave it.
#include "estimate.hpp"
#include "vsample.hpp"

namespace mcubes {

namespace {

// The step's tables (items, segments, queue order) are written by the host
// before the launch and only read during it, so they are read through the
// constant address space (Const).

template <int F, int D, bool F32>
__device__ __forceinline__ void run_segment(Const<SampleArgs> &a, const BatchSegment &sg, int si,
                                            double *lds, const BatchArgs &B) {
    const LdsView<F32> v(lds, D, a.nb);
    load_lds<D, F32>(a, v);
    __syncthreads();
    const uint32_t g = (uint32_t)a.g;
    int32_t step[D];  // blockDim in base g
    {
        uint32_t sd[D];
        digits_of<D>((uint64_t)blockDim.x, g, sd);
#pragma unroll
        for (int j = 0; j < D; ++j) step[j] = (int32_t)sd[j];
    }
    uint64_t t = (uint64_t)sg.t0 + threadIdx.x;
    uint32_t dig[D];
    digits_of<D>(t, g, dig);
    double sI = 0.0, cI = 0.0, sV = 0.0, cV = 0.0;
    bool bad = false;
    while (t < (uint64_t)sg.t1) {
        double It, vt;
        // (plain, not volatile, constant loads: measured faster here, where
        // the cases' shared register allocation is set by other values; one
        // phase, raised priority for the first part of each sample)
        cube_pass<F, D, false, F32, false, false, false, false, true>(a, v, (Const<real_t<F32>> *)a.consts, t, dig,
                                                                      It, vt, bad);
        two_sum_add(sI, cI, It);
        two_sum_add(sV, cV, vt);
        t += blockDim.x;
        odometer_add<D>(dig, step, g);
    }
    block_totals(sI, cI, sV, cV, bad, B.seg_tot + 4 * (size_t)si, B.flags + sg.item);
    if (a.hist) {
        // into the integral's histogram in device memory (ordinary device
        // allocations, so the hardware FP64 atomic add applies); bins this
        // segment never reached are skipped
        double *dst = B.items[sg.item].out + 4;
        for (int i = threadIdx.x; i < D * a.nb; i += blockDim.x) {
            const double h = v.hist[i];
            if (h != 0.0) unsafeAtomicAdd(dst + i, h);
        }
    }
    __syncthreads();  // LDS is reused by the next segment
}

#define MC_CASE(F, D) \
    case (F) * 32 + (D): run_segment<F, D, F32>(a, sg, si, lds, B); break;
#define MC_CASES_1_10(F)                                                                           \
    MC_CASE(F, 1) MC_CASE(F, 2) MC_CASE(F, 3) MC_CASE(F, 4) MC_CASE(F, 5) MC_CASE(F, 6)           \
    MC_CASE(F, 7) MC_CASE(F, 8) MC_CASE(F, 9) MC_CASE(F, 10)

// Register budget: every (integrand, dimension) case of a kernel shares its
// allocation, so the largest case sets it.  With the arguments read through
// the constant address space every kernel fits 128 VGPRs (4 waves per SIMD);
// the table integrand, the largest, still has a kernel of its own so that its
// cases do not set the budget of the others.  (Splitting the closed forms by
// dimension, d <= 5 at 5 or 8 waves per SIMD, measured no faster: the extra
// launch groups cost more per step than the occupancy gained.)
template <bool F32, bool TABLES>
__global__ void __launch_bounds__(kBatchMaxBlock) __attribute__((amdgpu_waves_per_eu(4)))
vsample_batch_kernel(const BatchArgs B) {
    extern __shared__ double lds[];
    __shared__ int32_t next;
    for (;;) {
        // every workgroup leaves once the counter has passed hi
        if (threadIdx.x == 0) next = B.lo + (int32_t)atomicAdd(B.queue, 1u);
        __syncthreads();
        // the same for every lane: keep it (and all that is loaded through
        // it) in scalar registers
        const int32_t q = __builtin_amdgcn_readfirstlane(next);
        __syncthreads();
        if (q >= B.hi) break;
        const int si = ((Const<int32_t> *)B.order)[q];
        Const<BatchSegment> &sgc = ((Const<BatchSegment> *)B.segs)[si];
        const BatchSegment sg{sgc.item, 0, sgc.t0, sgc.t1};
        Const<BatchItem> &item = ((Const<BatchItem> *)B.items)[sg.item];
        // an integral that stopped in an earlier step (the host had not yet
        // seen it when it planned this one): nothing to do
        const uint32_t state = *(const volatile uint32_t *)item.state;
        if (__builtin_amdgcn_readfirstlane(state) != kItemRunning) continue;
        Const<SampleArgs> &a = item.a;
        if constexpr (TABLES) {
            switch (a.kind) {
                MC_CASE(3, 4) MC_CASE(3, 5) MC_CASE(3, 6) MC_CASE(3, 7) MC_CASE(3, 8) MC_CASE(3, 9)
                MC_CASE(3, 10)
                default: break;
            }
        } else {
            switch (a.kind) {
                MC_CASES_1_10(0)
                MC_CASES_1_10(1)
                MC_CASES_1_10(2)
                default: break;
            }
        }
    }
}

#undef MC_CASES_1_10
#undef MC_CASE

constexpr int kFinThreads = 64;  // one wavefront per integral

// One wavefront per integral: its segment totals merged with TwoSum, each
// lane over a strided subset in segment order and then across the lanes in
// a fixed butterfly (so the totals do not depend on which workgroup took
// which segment; an integral of a served step can have thousands of
// segments, too many for one lane); then the host steps of Alg. 2 that
// decide whether it goes on (Weighted-Estimates over all its iterations,
// Check-Convergence, the iteration cap), in the same code and roundings as
// the host driver.
__global__ void __launch_bounds__(kFinThreads) batch_finalize_kernel(const BatchArgs B) {
    const int item = blockIdx.x, lane = threadIdx.x;
    const BatchItem &it = B.items[item];
    double *r = B.res + (size_t)kResStride * item;
    if (*it.state != kItemRunning) {  // stopped earlier; its segments did nothing
        if (lane == 0) {
            for (int i = 0; i < kResStride; ++i) r[i] = 0.0;
            r[6] = kResSkipped;
            B.flags[item] = 0u;
        }
        return;
    }
    const int s0 = B.item_first[item], s1 = B.item_first[item + 1];
    double sI = 0.0, cI = 0.0, sV = 0.0, cV = 0.0;
    for (int s = s0 + lane; s < s1; s += kFinThreads) {
        const double *q = B.seg_tot + 4 * (size_t)s;
        two_sum_merge(sI, cI, q[0], q[1]);
        two_sum_merge(sV, cV, q[2], q[3]);
    }
#pragma unroll
    for (int off = kFinThreads / 2; off >= 1; off >>= 1) {
        const double s2 = __shfl_xor(sI, off, 64), c2 = __shfl_xor(cI, off, 64);
        const double v2 = __shfl_xor(sV, off, 64), e2 = __shfl_xor(cV, off, 64);
        two_sum_merge(sI, cI, s2, c2);
        two_sum_merge(sV, cV, v2, e2);
    }
    if (lane != 0) return;
    double *o = it.out;
    const double I = sI + cI, V = sV + cV;
    const bool bad = B.flags[item] != 0u;
    o[0] = r[0] = I;
    o[1] = r[1] = V;
    o[2] = r[2] = bad ? 1.0 : 0.0;
    o[3] = 0.0;
    B.flags[item] = 0u;
    double est[3] = {0.0, 0.0, NAN};
    bool conv = false;
    uint32_t state = kItemRunning;
    if (bad) {
        state = kItemFailed;
    } else {
        const int k = (int)it.a.iter + 1;  // iterations including this one
        it.iters[k - 1] = I;
        it.iters[it.itmax + k - 1] = V;
        weighted_estimate(k, it.iters, it.iters + it.itmax, est);
        conv = converged_after(k, est, it.tau_rel, it.chi2_max);
        if (conv || k >= it.itmax) state = kItemDone;
    }
    if (state != kItemRunning) *it.state = state;
    r[3] = est[0];
    r[4] = est[1];
    r[5] = est[2];
    r[6] = (double)state;
    r[7] = conv ? 1.0 : 0.0;
}

// Adjust-Bin-Bounds on the device, one block per (integral, axis): three-
// point smoothing and Lepage's damped compression ((1 - s_i/S)/ln(S/s_i))^alpha
// across the block, the running sums and the equal-share rebinning in order
// by one lane (the same steps and summation order as the host version; pow
// and log are the device library's).  Reads the axis's histogram from out
// and its boundaries from a.grid, writes the new boundaries to next; for the
// m-Cubes1D variant (only axis 0 listed) to every axis.
constexpr int kRefThreads = 64;

__global__ void __launch_bounds__(kRefThreads)
batch_refine_kernel(const BatchItem *items, const int32_t *axis_item, double *const *next_grid) {
    extern __shared__ double r[];  // nb doubles
    const int ax = blockIdx.x;
    const int item = axis_item[2 * ax], j = axis_item[2 * ax + 1];
    const BatchItem &it = items[item];
    if (*it.state != kItemRunning) return;  // stopped: its grid is not used again
    const int nb = it.a.nb;
    double *C = it.out + 4 + (size_t)j * nb;
    const double *B = it.a.grid + (size_t)j * (nb + 1);
    double *Bn = next_grid[item] + (size_t)j * (nb + 1);
    const double alpha = it.alpha;
    for (int i = threadIdx.x; i < nb; i += kRefThreads) {
        double s;
        if (i == 0) s = (C[0] + C[1]) / 2.0;
        else if (i == nb - 1) s = (C[nb - 2] + C[nb - 1]) / 2.0;
        else s = ((C[i - 1] + C[i]) + C[i + 1]) / 3.0;
        r[i] = s;
    }
    __syncthreads();
    // the row is read: clear it for the next collecting pass
    for (int i = threadIdx.x; i < nb; i += kRefThreads) C[i] = 0.0;
    __shared__ double total_s;
    __shared__ int usable;
    if (threadIdx.x == 0) {
        double S = 0.0;
        for (int i = 0; i < nb; ++i) S = S + r[i];
        total_s = S;
        usable = (S > 0.0) && isfinite(S);
    }
    __syncthreads();
    const int copies = it.a.one_d ? (it.a.kind & 31) : 1;
    if (!usable) {  // no usable weight: the axis keeps its boundaries
        for (int c = 0; c < copies; ++c)
            for (int i = threadIdx.x; i <= nb; i += kRefThreads) Bn[(size_t)c * (nb + 1) + i] = B[i];
        return;
    }
    const double S = total_s;
    for (int i = threadIdx.x; i < nb; i += kRefThreads) {
        const double s = r[i];
        r[i] = s == 0.0 ? 0.0 : (s == S ? 1.0 : pow((1.0 - s / S) / log(S / s), alpha));
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double R = 0.0;
    for (int i = 0; i < nb; ++i) R = R + r[i];
    if (!(R > 0.0)) {
        for (int c = 0; c < copies; ++c)
            for (int i = 0; i <= nb; ++i) Bn[(size_t)c * (nb + 1) + i] = B[i];
        return;
    }
    const double per_bin = R / (double)nb;
    int src = 0;
    double acc = 0.0, prev_edge = 0.0;
    Bn[0] = 0.0;
    for (int k = 1; k < nb; ++k) {
        const double goal = (double)k * per_bin;
        while (src < nb - 1 && acc + r[src] < goal) {
            acc = acc + r[src];
            ++src;
        }
        double frac = r[src] > 0.0 ? (goal - acc) / r[src] : 0.0;
        frac = fmin(fmax(frac, 0.0), 1.0);
        const double edge = __fma_rn(frac, B[src + 1] - B[src], B[src]);
        prev_edge = fmax(edge, prev_edge);
        Bn[k] = prev_edge;
    }
    Bn[nb] = 1.0;
    for (int c = 1; c < copies; ++c)
        for (int i = 0; i <= nb; ++i) Bn[(size_t)c * (nb + 1) + i] = Bn[i];
}

// One block per admitted integral: constants from the upload, then the
// uniform grid B_j[i] = i/nb (one correctly rounded division, as on the host).
constexpr int kAdmitThreads = 256;

__global__ void __launch_bounds__(kAdmitThreads)
admit_kernel(const AdmitRecord *recs, const char *upload) {
    const AdmitRecord r = recs[blockIdx.x];
    const uint32_t *src = reinterpret_cast<const uint32_t *>(upload + r.src);
    uint32_t *dst = reinterpret_cast<uint32_t *>(r.consts);
    for (int i = threadIdx.x; i < r.const_words; i += kAdmitThreads) dst[i] = src[i];
    const int row = r.nb + 1;
    const double nbd = (double)r.nb;
    for (int i = threadIdx.x; i < r.dim * row; i += kAdmitThreads) r.grid[i] = (double)(i % row) / nbd;
    for (int i = threadIdx.x; i < 4 + r.dim * r.nb; i += kAdmitThreads) r.out[i] = 0.0;
    if (threadIdx.x == 0) *r.state = kItemRunning;
}

}  // namespace

hipError_t launch_admit(const AdmitRecord *recs, int n, const char *upload, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(admit_kernel, dim3(n), dim3(kAdmitThreads), 0, stream, recs, upload);
    return hipGetLastError();
}

const void *batch_kernel(bool fp32, bool tables) {
    if (fp32)
        return tables ? reinterpret_cast<const void *>(&vsample_batch_kernel<true, true>)
                      : reinterpret_cast<const void *>(&vsample_batch_kernel<true, false>);
    return tables ? reinterpret_cast<const void *>(&vsample_batch_kernel<false, true>)
                  : reinterpret_cast<const void *>(&vsample_batch_kernel<false, false>);
}

hipError_t launch_batch(bool fp32, bool tables, int blocks, int threads, size_t lds_bytes,
                        hipStream_t stream, const BatchArgs &args) {
    const dim3 grid(blocks), block(threads);
    if (fp32) {
        if (tables)
            hipLaunchKernelGGL((vsample_batch_kernel<true, true>), grid, block, lds_bytes, stream, args);
        else
            hipLaunchKernelGGL((vsample_batch_kernel<true, false>), grid, block, lds_bytes, stream, args);
    } else {
        if (tables)
            hipLaunchKernelGGL((vsample_batch_kernel<false, true>), grid, block, lds_bytes, stream, args);
        else
            hipLaunchKernelGGL((vsample_batch_kernel<false, false>), grid, block, lds_bytes, stream, args);
    }
    return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchArgs &args, hipStream_t stream) {
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(args.n_items), dim3(kFinThreads), 0, stream, args);
    return hipGetLastError();
}

const void *batch_refine_symbol() { return reinterpret_cast<const void *>(&batch_refine_kernel); }

hipError_t launch_batch_refine(const BatchItem *items, const int32_t *axis_item,
                               double *const *next_grid, int n_axes, int max_nb,
                               hipStream_t stream) {
    if (n_axes == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_refine_kernel, dim3(n_axes), dim3(kRefThreads),
                       sizeof(double) * (size_t)max_nb, stream, items, axis_item, next_grid);
    return hipGetLastError();
}

}  // namespace mcubes
