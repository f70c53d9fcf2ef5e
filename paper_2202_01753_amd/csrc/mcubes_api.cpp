// Host side of the m-Cubes library: validation, the sub-cube lattice, the
// workspace layout, the per-iteration host steps of Alg. 2 (weighted
// estimate, bin adjustment, convergence check) and the C ABI.
//
// Built without floating-point contraction: the bin adjustment must round
// exactly as written so that a given histogram always yields the same grid.
#include "mcubes.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "host.hpp"
#include "internal.hpp"

using namespace mcubes;
using namespace mcubes::host;

namespace {


// ------------------------------------------------------------------ launch geometry and workspace

struct Geometry {
    int64_t g, m, p;
    int threads;
    int blocks_adj, blocks_noadj;
    size_t lds_adj, lds_noadj;
    int hist_stride;          // doubles per histogram accumulator (padded)
    int hist_copies;          // LDS histogram copies in adjusting passes (1 or 2)
    size_t off_consts, off_grid, off_tables, off_partials, off_hist, off_out, off_flag, off_run, total;
};

mc_status blocks_for(const void *fn, int threads, size_t lds, int64_t m, int requested, int *out) {
    int dev = 0, cus = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(allow_lds(fn, lds));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds));
    if (per_cu < 1) return MC_EINVAL;
    // Where several workgroups share a CU, launch more than fit at once: the
    // workgroups are smaller, and CUs that were handed fewer of them take more
    // later, instead of idling for the rest of the launch (four times as many:
    // 12% faster at d = 8 with two 768-thread workgroups per CU; one 1024-thread
    // workgroup per CU gains nothing and keeps the resident count).  Every
    // workgroup also ends with a flush of its histogram, so four times is
    // taken only where each lane still has at least 100 sub-cubes to do,
    // twice otherwise (the FP32 d = 6 tables pass: 60 per lane at twice;
    // once, twice and four times measured 0.632, 0.615 and 0.616 ms).
    const int64_t resident = (int64_t)per_cu * cus;
    int64_t want = resident;
    if (requested > 0)
        want = requested;
    else if (per_cu > 1)
        want = m >= (int64_t)100 * 4 * resident * threads ? 4 * resident : 2 * resident;
    const int64_t useful = (m + threads - 1) / threads;
    if (requested <= 0) want = std::min(want, useful);
    *out = (int)std::max<int64_t>(1, std::min<int64_t>(want, 1 << 20));
    return MC_OK;
}

// Workgroup size when the problem leaves it open: of 1024, 768, 512 and 256
// threads (whole multiples of four waves, so each of a CU's four SIMDs holds
// the same number of every workgroup's waves), the one that keeps the most
// waves resident per CU given the kernel's registers and the adjusting pass's
// LDS; on a tie the larger, which means fewer workgroups and so fewer
// histogram flushes.  768 is the d = 8 case: two 64 KB workgroups
// of 12 waves fit where one of 16 did.
mc_status pick_threads(const void *fn, size_t lds, int *out) {
    HIP_TRY(allow_lds(fn, lds));
    int best = 0, best_waves = -1;
    for (int t : {1024, 768, 512, 256}) {
        int per_cu = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, t, lds));
        const int waves = per_cu * t / 64;
        if (waves > best_waves) {
            best_waves = waves;
            best = t;
        }
    }
    if (best_waves < 1) return MC_EINVAL;
    *out = best;
    return MC_OK;
}

mc_status geometry(const mc_problem *pr, Geometry *geo) {
    mc_status st = validate(pr);
    if (st != MC_OK) return st;
    Geometry G{};
    lattice(pr->dim, pr->maxcalls, &G.g, &G.m, &G.p);
    const int d = pr->dim, nb = pr->nbins;
    const bool f32 = is_fp32(pr);
    G.lds_adj = lds_bytes_of(d, nb, true, f32);
    G.lds_noadj = lds_bytes_of(d, nb, false, f32);
    const void *fn = sample_kernel(pr->integrand, d, false, f32);
    if (!fn) return MC_EINVAL;
    if (pr->threads) {
        G.threads = pr->threads;
    } else {
        st = pick_threads(fn, G.lds_adj, &G.threads);
        if (st != MC_OK) return st;
    }
    // A second LDS copy of the histogram, for the upper half of each wave,
    // halves the lanes that add into one bin at once (lanes of a wave share
    // the strata of all but the fastest axes, so many fall into the same few
    // bins); taken where the extra LDS keeps as many workgroups resident.
    G.hist_copies = 1;
    {
        const size_t lds2 = G.lds_adj + sizeof(double) * d * (size_t)nb;
        if (lds2 <= kLdsDynamicLimit) {
            int per1 = 0, per2 = 0;
            HIP_TRY(allow_lds(fn, lds2));
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per1, fn, G.threads, G.lds_adj));
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per2, fn, G.threads, lds2));
            if (per2 >= per1 && per2 > 0) {
                G.hist_copies = 2;
                G.lds_adj = lds2;
            }
        }
    }
    st = blocks_for(fn, G.threads, G.lds_adj, G.m, pr->blocks, &G.blocks_adj);
    if (st != MC_OK) return st;
    st = blocks_for(fn, G.threads, G.lds_noadj, G.m, pr->blocks, &G.blocks_noadj);
    if (st != MC_OK) return st;
    G.hist_stride = (int)((d * (size_t)nb + 31) / 32 * 32);
    const size_t part_adj = 4 * (size_t)G.blocks_adj;
    const size_t part_noadj = 4 * (size_t)G.blocks_noadj;
    size_t off = 0;
    const size_t real = f32 ? sizeof(float) : sizeof(double);
    G.off_consts = off;
    off = align_up(off + real * kConstStride * d);
    G.off_grid = off;
    off = align_up(off + sizeof(double) * d * (nb + 1));
    G.off_tables = off;
    if (pr->integrand == MC_F_GAUSS_TABLES) off = align_up(off + real * (f32 ? kTablesLen32 : kTablesLen));
    G.off_partials = off;
    off = align_up(off + sizeof(double) * std::max(part_adj, part_noadj));
    // the kHistAcc histogram accumulators of adjusting passes, kept zero
    // between passes
    G.off_hist = off;
    off = align_up(off + sizeof(double) * kHistAcc * (size_t)G.hist_stride);
    G.off_out = off;
    off = align_up(off + sizeof(double) * (4 + (size_t)d * nb));
    G.off_flag = off;
    off = align_up(off + sizeof(uint32_t));
    // a device-steps run's state and its per-iteration (I, var)
    G.off_run = off;
    off = align_up(off + sizeof(RunState) + sizeof(double) * 2 * (size_t)pr->itmax);
    G.total = off;
    *geo = G;
    return MC_OK;
}

// ------------------------------------------------------------------ one sampling pass

void fill_args(const mc_problem *pr, const Geometry &G, char *ws, uint32_t iter, bool adjust,
               int blocks, SampleArgs *a) {
    const double *grid = reinterpret_cast<const double *>(ws + G.off_grid);
    const void *tables = pr->integrand == MC_F_GAUSS_TABLES ? ws + G.off_tables : nullptr;
    sample_args(pr, G.g, G.m, G.p, iter, adjust, ws + G.off_consts, grid, tables, a);
    a->partials = reinterpret_cast<double *>(ws + G.off_partials);
    a->hist_acc = reinterpret_cast<double *>(ws + G.off_hist);
    a->flag = reinterpret_cast<uint32_t *>(ws + G.off_flag);
    a->stride = (int64_t)blocks * G.threads;
    a->hist_stride = G.hist_stride;
    a->hist_copies = adjust ? G.hist_copies : 1;
    // the per-lane stride in base g (only d digits are used: a lane that
    // overflows the top digit has left the lattice)
    int64_t rest = a->stride;
    for (int j = 0; j < pr->dim; ++j) {
        a->sdig[j] = (int32_t)(rest % G.g);
        rest /= G.g;
    }
}

struct Events {
    hipEvent_t e[3] = {nullptr, nullptr, nullptr};
    bool ok = false;
    ~Events() {
        for (auto &x : e)
            if (x) (void)hipEventDestroy(x);
    }
    hipError_t create() {
        for (auto &x : e) {
            hipError_t err = hipEventCreate(&x);
            if (err != hipSuccess) return err;
        }
        ok = true;
        return hipSuccess;
    }
};

// Page-locked staging for the calling thread's passes (grid up, results
// down), grown on demand and kept until the process ends, so that both copies
// are direct DMA rather than staged through pageable memory.
hipError_t pass_stage(size_t bytes, char **out) {
    thread_local char *buf = nullptr;
    thread_local size_t cap = 0;
    if (bytes > cap) {
        if (buf) {
            const hipError_t e = hipHostFree(buf);
            buf = nullptr;
            cap = 0;
            if (e != hipSuccess) return e;
        }
        const size_t want = std::max(bytes, size_t(1) << 20);
        const hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&buf), want, hipHostMallocDefault);
        if (e != hipSuccess) return e;
        cap = want;
    }
    *out = buf;
    return hipSuccess;
}

// One pass with the steps on the host: sampling + finalize, and the result
// read back into out_host (4 + d*nb doubles).  pinned: stage the grid and
// the results through page-locked memory (direct DMA; allocated on first
// use); otherwise copy from and to the caller's pageable buffers, which
// allocates nothing.
mc_status run_pass(const mc_problem *pr, const Geometry &G, char *ws, hipStream_t stream,
                   uint32_t iter, bool adjust, const double *h_grid, double *out_host,
                   double *trace, int64_t t0, int64_t t1, Events *ev, double *ms_sample,
                   double *ms_fin, int spin_us = 0, bool pinned = true) {
    const int d = pr->dim, nb = pr->nbins;
    const int blocks = adjust ? G.blocks_adj : G.blocks_noadj;
    const size_t lds = adjust ? G.lds_adj : G.lds_noadj;
    SampleArgs a;
    fill_args(pr, G, ws, iter, adjust, blocks, &a);
    a.trace = trace;
    a.t0 = t0;
    a.t1 = t1;
    const size_t grid_bytes = sizeof(double) * d * (nb + 1);
    const size_t nout = 4 + (adjust ? (size_t)d * nb : 0);
    char *stage = nullptr;
    double *out_stage = out_host;
    if (pinned) {
        HIP_TRY(pass_stage(align_up(grid_bytes) + sizeof(double) * nout, &stage));
        std::memcpy(stage, h_grid, grid_bytes);
        out_stage = reinterpret_cast<double *>(stage + align_up(grid_bytes));
    }
    HIP_TRY(hipMemcpyAsync(ws + G.off_grid, pinned ? stage : static_cast<const void *>(h_grid),
                           grid_bytes, hipMemcpyHostToDevice, stream));
    if (ev) HIP_TRY(hipEventRecord(ev->e[0], stream));
    HIP_TRY(allow_lds(sample_kernel(pr->integrand, d, trace != nullptr, is_fp32(pr)), lds));
    HIP_TRY(launch_sample(pr->integrand, d, blocks, G.threads, lds, stream, a));
    if (ev) HIP_TRY(hipEventRecord(ev->e[1], stream));
    double *out_dev = reinterpret_cast<double *>(ws + G.off_out);
    HIP_TRY(launch_finalize(a.partials, a.hist_acc, blocks, d * nb, G.hist_stride, adjust ? 1 : 0, a.flag,
                            out_dev, stream));
    if (ev) HIP_TRY(hipEventRecord(ev->e[2], stream));
    if (adjust && d > 1 && !pr->one_d) AxisPool::get().prime(spin_us);
    HIP_TRY(hipMemcpyAsync(out_stage, out_dev, sizeof(double) * nout, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (pinned) std::memcpy(out_host, out_stage, sizeof(double) * nout);
    if (ev) {
        float a_ms = 0.f, b_ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&a_ms, ev->e[0], ev->e[1]));
        HIP_TRY(hipEventElapsedTime(&b_ms, ev->e[1], ev->e[2]));
        *ms_sample += a_ms;
        *ms_fin += b_ms;
    }
    return out_host[2] != 0.0 ? MC_ENONFINITE : MC_OK;
}

mc_status prepare(const mc_problem *pr, const Geometry &G, char *ws, hipStream_t stream) {
    const std::vector<double> consts = axis_constants(pr);
    if (is_fp32(pr)) {
        // FP32 evaluation: every constant and table value rounded once to float
        const std::vector<float> c32(consts.begin(), consts.end());
        HIP_TRY(hipMemcpyAsync(ws + G.off_consts, c32.data(), sizeof(float) * c32.size(),
                               hipMemcpyHostToDevice, stream));
        if (pr->integrand == MC_F_GAUSS_TABLES) {
            std::vector<float> t32(kTablesLen32);
            tables_f32(pr->tables, t32.data());
            HIP_TRY(hipMemcpyAsync(ws + G.off_tables, t32.data(), sizeof(float) * kTablesLen32,
                                   hipMemcpyHostToDevice, stream));
            HIP_TRY(hipStreamSynchronize(stream));  // t32 is about to go out of scope
        }
        HIP_TRY(hipStreamSynchronize(stream));
    } else {
        HIP_TRY(hipMemcpyAsync(ws + G.off_consts, consts.data(), sizeof(double) * consts.size(),
                               hipMemcpyHostToDevice, stream));
        if (pr->integrand == MC_F_GAUSS_TABLES)
            HIP_TRY(hipMemcpyAsync(ws + G.off_tables, pr->tables, sizeof(double) * kTablesLen,
                                   hipMemcpyHostToDevice, stream));
    }
    HIP_TRY(launch_clear_flag(reinterpret_cast<uint32_t *>(ws + G.off_flag), stream));
    // the histogram accumulators start at zero; the finalize or steps kernel
    // of each adjusting pass clears them again after reading them
    HIP_TRY(launch_zero(reinterpret_cast<double *>(ws + G.off_hist),
                        (size_t)kHistAcc * G.hist_stride, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return MC_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

const char *mc_status_string(mc_status s) {
    switch (s) {
    case MC_OK: return "ok";
    case MC_EINVAL: return "invalid problem or argument";
    case MC_EWORKSPACE: return "workspace too small";
    case MC_ENONFINITE: return "integrand produced a non-finite value";
    case MC_EDEVICE: return "HIP device error";
    default: return "unknown status";
    }
}

mc_status mc_shape(int32_t dim, int64_t maxcalls, int64_t *g, int64_t *m, int64_t *p) {
    if (!g || !m || !p) return MC_EINVAL;
    int64_t gg, mm, pp;
    mc_status st = lattice(dim, maxcalls, &gg, &mm, &pp);
    if (st != MC_OK) return st;
    *g = gg;
    *m = mm;
    *p = pp;
    return MC_OK;
}

mc_status mc_workspace_bytes(const mc_problem *prob, size_t *bytes) {
    if (!bytes) return MC_EINVAL;
    Geometry G;
    mc_status st = geometry(prob, &G);
    if (st != MC_OK) return st;
    *bytes = G.total;
    return MC_OK;
}

mc_status mc_launch_shape(const mc_problem *prob, int32_t adjust, int32_t *blocks, int32_t *threads,
                          int32_t *lds_bytes) {
    if (!blocks || !threads || !lds_bytes) return MC_EINVAL;
    Geometry G;
    mc_status st = geometry(prob, &G);
    if (st != MC_OK) return st;
    *blocks = adjust ? G.blocks_adj : G.blocks_noadj;
    *threads = G.threads;
    *lds_bytes = (int32_t)(adjust ? G.lds_adj : G.lds_noadj);
    return MC_OK;
}

mc_status mc_prepare(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream) {
    Geometry G;
    mc_status st = geometry(prob, &G);
    if (st != MC_OK) return st;
    if (!d_ws || ws_bytes < G.total) return MC_EWORKSPACE;
    return prepare(prob, G, static_cast<char *>(d_ws), static_cast<hipStream_t>(stream));
}

mc_status mc_sample_iteration(const mc_problem *prob, uint32_t iter, int32_t adjust,
                              const double *h_grid, void *d_ws, size_t ws_bytes, void *stream,
                              double *h_out, double *h_hist, void *d_trace, size_t trace_bytes,
                              int64_t t0, int64_t t1) {
    Geometry G;
    mc_status st = geometry(prob, &G);
    if (st != MC_OK) return st;
    if (!h_grid || !h_out || (!adjust && h_hist)) return MC_EINVAL;
    const int d = prob->dim, nb = prob->nbins;
    if (d_trace) {
        if (t0 < 0 || t1 < t0 || t1 > G.m) return MC_EINVAL;
        const size_t need = sizeof(double) * ((size_t)(t1 - t0) * G.p * (3 * d + 2) + 2 * (size_t)(t1 - t0));
        if (trace_bytes < need) return MC_EINVAL;
    }
    if (!d_ws || ws_bytes < G.total) return MC_EWORKSPACE;
    std::vector<double> out(4 + (size_t)d * nb);
    st = run_pass(prob, G, static_cast<char *>(d_ws), static_cast<hipStream_t>(stream), iter,
                  adjust != 0, h_grid, out.data(), static_cast<double *>(d_trace),
                  d_trace ? t0 : 0, d_trace ? t1 : 0, nullptr, nullptr, nullptr);
    if (st != MC_OK) return st;
    h_out[0] = out[0];
    h_out[1] = out[1];
    if (h_hist) std::copy(out.begin() + 4, out.end(), h_hist);
    return MC_OK;
}

mc_status mc_refine_grid(int32_t dim, int32_t nbins, double alpha, const double *h_hist,
                         double *h_grid) {
    if (dim < 1 || dim > MC_MAX_DIM || nbins < 2 || !(alpha > 0.0) || !h_hist || !h_grid)
        return MC_EINVAL;
    refine(dim, nbins, alpha, h_hist, h_grid);
    return MC_OK;
}

mc_status mc_refine_grid_1d(int32_t dim, int32_t nbins, double alpha, const double *h_hist,
                            double *h_grid) {
    if (dim < 1 || dim > MC_MAX_DIM || nbins < 2 || !(alpha > 0.0) || !h_hist || !h_grid)
        return MC_EINVAL;
    refine_1d(dim, nbins, alpha, h_hist, h_grid);
    return MC_OK;
}

mc_status mc_refine_grid_device(int32_t dim, int32_t nbins, double alpha, int32_t one_d,
                                const double *d_hist, double *d_grid, void *stream) {
    if (dim < 1 || dim > MC_MAX_DIM || nbins < 2 || nbins > kDeviceStepsMaxBins ||
        !(alpha > 0.0) || !std::isfinite(alpha) || (one_d != 0 && one_d != 1) || !d_hist || !d_grid)
        return MC_EINVAL;
    HIP_TRY(launch_refine(d_grid, d_hist, dim, nbins, one_d, alpha, static_cast<hipStream_t>(stream)));
    return MC_OK;
}

mc_status mc_init_grid(int32_t dim, int32_t nbins, double *h_grid) {
    if (dim < 1 || dim > MC_MAX_DIM || nbins < 2 || !h_grid) return MC_EINVAL;
    init_grid(dim, nbins, h_grid);
    return MC_OK;
}

mc_status mc_weighted_estimate(int32_t k, const double *h_I, const double *h_var, double *h_out) {
    if (k < 1 || !h_I || !h_var || !h_out) return MC_EINVAL;
    weighted(k, h_I, h_var, h_out);
    return MC_OK;
}

}  // extern "C"

namespace {

// The calling thread's page-locked host mirror of a device-steps run, mapped
// for the device (bytes, grown on demand and kept until the process ends):
// its RunState, then 2 * itmax doubles of per-iteration results, then the
// grid.
hipError_t run_mirror(size_t bytes, char **host, char **dev) {
    thread_local char *buf = nullptr;
    thread_local size_t cap = 0;
    if (bytes > cap) {
        if (buf) {
            const hipError_t e = hipHostFree(buf);
            buf = nullptr;
            cap = 0;
            if (e != hipSuccess) return e;
        }
        const size_t want = std::max(bytes, size_t(1) << 16);
        const hipError_t e = hipHostMalloc(reinterpret_cast<void **>(&buf), want,
                                           hipHostMallocMapped | hipHostMallocPortable |
                                               hipHostMallocCoherent);
        if (e != hipSuccess) return e;
        cap = want;
    }
    void *d = nullptr;
    const hipError_t e = hipHostGetDevicePointer(&d, buf, 0);
    if (e != hipSuccess) return e;
    *host = buf;
    *dev = static_cast<char *>(d);
    return hipSuccess;
}

// The calling thread's markers for timed device-steps runs on the current
// device, created once (and again after a change of device) and kept until
// the process ends.  Per pass two: after the sampling kernel, and "done"
// after the pass's last kernel.  Three slots each, since the next passes are
// queued before a pass is read.
struct RunEvents {
    int device = -1;
    hipEvent_t start = nullptr, sampled[3] = {}, done[3] = {};
};

hipError_t run_events(RunEvents **out) {
    thread_local RunEvents ev;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (ev.device != dev) {
        hipEvent_t *all[] = {&ev.start, &ev.sampled[0], &ev.sampled[1], &ev.sampled[2],
                             &ev.done[0], &ev.done[1], &ev.done[2]};
        for (hipEvent_t *x : all)
            if (*x) {
                (void)hipEventDestroy(*x);
                *x = nullptr;
            }
        ev.device = -1;
        for (hipEvent_t *x : all)
            if ((e = hipEventCreate(x)) != hipSuccess) return e;
        ev.device = dev;
    }
    *out = &ev;
    return hipSuccess;
}

// Alg. 2 with its steps between passes on the device: Init-Bins and the run
// state, then per pass the sampling kernel and one steps launch (totals,
// Weighted-Estimates, Check-Convergence and, while adjusting, the bin
// adjustment), all on the stream.  The sampling kernel of the next pass is
// always queued before the host waits for a pass, so the device never waits
// for the host; the steps of that pass are queued once the decision of the
// pass before is known, so a run that converges leaves only one sampling
// launch queued behind it, which does nothing.  The decisions, the
// per-iteration results and the grid come back through the mapped mirror.
mc_status integrate_device(const mc_problem *prob, const Geometry &G, char *ws, hipStream_t s,
                           mc_result *out, double *h_iters, double *h_grid, mc_timing *timing) {
    const int d = prob->dim, nb = prob->nbins, itmax = prob->itmax;
    const size_t grid_len = (size_t)d * (nb + 1);
    char *hbuf = nullptr, *dbuf = nullptr;
    HIP_TRY(run_mirror(sizeof(RunState) + sizeof(double) * (2 * (size_t)itmax + grid_len), &hbuf, &dbuf));
    RunEvents *ev = nullptr;
    if (timing) HIP_TRY(run_events(&ev));
    RunState *hm = reinterpret_cast<RunState *>(hbuf), *hm_dev = reinterpret_cast<RunState *>(dbuf);
    double *h_its = reinterpret_cast<double *>(hm + 1), *h_its_dev = reinterpret_cast<double *>(hm_dev + 1);
    double *h_gr = h_its + 2 * (size_t)itmax, *h_gr_dev = h_its_dev + 2 * (size_t)itmax;
    double *mirror_grid = h_grid ? h_gr_dev : nullptr;
    std::memset(static_cast<void *>(hm), 0, sizeof(RunState));
    hm->last = itmax - 1;
    RunState *dst = reinterpret_cast<RunState *>(ws + G.off_run);
    double *iters = reinterpret_cast<double *>(dst + 1);
    double *grid = reinterpret_cast<double *>(ws + G.off_grid);
    double *partials = reinterpret_cast<double *>(ws + G.off_partials);
    double *hist_acc = reinterpret_cast<double *>(ws + G.off_hist);
    uint32_t *flag = reinterpret_cast<uint32_t *>(ws + G.off_flag);
    hipEvent_t *done = timing ? ev->done : nullptr;
    const void *fn = sample_kernel(prob->integrand, d, false, is_fp32(prob));
    auto pass_blocks = [&](int it) { return it < prob->ita ? G.blocks_adj : G.blocks_noadj; };
    // the sampling kernel of pass it (and its marker)
    auto head = [&](int it) -> hipError_t {
        const bool adjust = it < prob->ita;
        const size_t lds = adjust ? G.lds_adj : G.lds_noadj;
        SampleArgs a;
        fill_args(prob, G, ws, (uint32_t)it, adjust, pass_blocks(it), &a);
        a.run_last = &dst->last;
        hipError_t e;
        if (timing && it == 0 && (e = hipEventRecord(ev->start, s)) != hipSuccess) return e;
        if ((e = allow_lds(fn, lds)) != hipSuccess) return e;
        if ((e = launch_sample(prob->integrand, d, pass_blocks(it), G.threads, lds, s, a)) != hipSuccess)
            return e;
        return timing ? hipEventRecord(ev->sampled[it % 3], s) : hipSuccess;
    };
    // the rest of pass it: totals, decision and bin adjustment in one launch,
    // and with timing the done marker
    auto tail = [&](int it) -> hipError_t {
        const bool adjust = it < prob->ita;
        StepsArgs sa{};
        sa.ctl = RunCtl{dst, iters, hm_dev, h_its_dev, it, itmax, prob->tau_rel, prob->chi2_max};
        sa.partials = partials;
        sa.blocks = pass_blocks(it);
        sa.hist_stride = G.hist_stride;
        sa.hist_acc = hist_acc;
        sa.flag = flag;
        sa.grid = grid;
        sa.host_grid = mirror_grid;
        sa.alpha = prob->alpha;
        sa.d = d;
        sa.nb = nb;
        sa.one_d = prob->one_d;
        sa.nref = adjust ? (prob->one_d ? 1 : d) : 0;
        const hipError_t e = launch_steps(sa, s);
        if (e != hipSuccess) return e;
        return timing ? hipEventRecord(done[it % 3], s) : hipSuccess;
    };
    // until pass it's decision is in the mirror: with timing, the pass's done
    // marker; otherwise the mirror's pass count, which the steps kernel writes
    // last (no marker, which would hold the stream for a few microseconds),
    // with a look at the stream now and then, so that an error or a stream
    // that has run dry ends the wait
    auto wait_pass = [&](int it) -> hipError_t {
        if (timing) return hipEventSynchronize(done[it % 3]);
        const volatile int32_t *kk = &reinterpret_cast<volatile RunState *>(hm)->k;
        for (unsigned spin = 1;; ++spin) {
            if (*kk > it) break;
            if (spin % 1024 == 0) {
                const hipError_t q = hipStreamQuery(s);
                if (q == hipSuccess && *kk <= it) return hipErrorUnknown;  // drained, no decision
                if (q != hipSuccess && q != hipErrorNotReady) return q;
            }
        }
        std::atomic_thread_fence(std::memory_order_acquire);
        return hipSuccess;
    };
    double ms_s = 0.0, ms_f = 0.0;
    int k = 0;
    hipError_t err = launch_run_init(dst, grid, mirror_grid, d, nb, itmax, s);
    if (err == hipSuccess) err = head(0);
    if (err == hipSuccess) err = tail(0);
    if (err == hipSuccess && itmax > 1) err = head(1);
    for (int it = 0; err == hipSuccess && it < itmax; ++it) {
        if ((err = wait_pass(it)) != hipSuccess) break;
        k = it + 1;
        if (timing) {
            float a_ms = 0.f, b_ms = 0.f;
            hipEvent_t from = it == 0 ? ev->start : done[(it - 1) % 3];
            if ((err = hipEventElapsedTime(&a_ms, from, ev->sampled[it % 3])) != hipSuccess ||
                (err = hipEventElapsedTime(&b_ms, ev->sampled[it % 3], done[it % 3])) != hipSuccess)
                break;
            ms_s += a_ms;
            ms_f += b_ms;
        }
        if (reinterpret_cast<volatile RunState *>(hm)->last <= it) break;  // pass it ended the run
        // the run goes on: the rest of pass it + 1, whose sampling kernel is
        // running, and the sampling kernel after it
        if ((err = tail(it + 1)) != hipSuccess) break;
        if (it + 2 < itmax && (err = head(it + 2)) != hipSuccess) break;
    }
    // a sampling launch queued after the last pass does nothing; wait for it too
    const hipError_t err2 = hipStreamSynchronize(s);
    HIP_TRY(err);
    HIP_TRY(err2);
    const volatile RunState *v = hm;
    if (v->status == kRunNonFinite) return MC_ENONFINITE;
    if (h_grid) std::memcpy(h_grid, h_gr, sizeof(double) * grid_len);
    out->estimate = v->est[0];
    out->error = v->est[1];
    out->chi2_dof = v->est[2];
    out->iterations = k;
    out->converged = v->status == kRunConverged ? 1 : 0;
    out->calls = (int64_t)k * G.m * G.p;
    if (h_iters)
        for (int i = 0; i < k; ++i) {
            h_iters[2 * i] = h_its[i];
            h_iters[2 * i + 1] = h_its[itmax + i];
        }
    if (timing) {
        timing->sample_ms = ms_s;
        timing->finalize_ms = ms_f;
        timing->launches = k;
        timing->blocks = prob->ita > 0 ? G.blocks_adj : G.blocks_noadj;
        timing->threads = G.threads;
        timing->lds_bytes = (int32_t)(prob->ita > 0 ? G.lds_adj : G.lds_noadj);
    }
    return MC_OK;
}

// Whether a run keeps the steps between passes on the device: asked for, and
// the bin adjustment's LDS holds nb.
bool steps_on_device(const mc_problem *prob) {
    return prob->device_steps == 1 && prob->nbins <= kDeviceStepsMaxBins;
}

// Alg. 2 on a workspace; upload: copy the constants and tables first
// (otherwise a previous mc_prepare() of the same problem left them there).
mc_status integrate(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream, bool upload,
                    mc_result *out, double *h_iters, double *h_grid, mc_timing *timing,
                    bool pinned = true) {
    if (!out) return MC_EINVAL;
    Geometry G;
    mc_status st = geometry(prob, &G);
    if (st != MC_OK) return st;
    if (!d_ws || ws_bytes < G.total) return MC_EWORKSPACE;
    char *ws = static_cast<char *>(d_ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (upload) {
        st = prepare(prob, G, ws, s);
        if (st != MC_OK) return st;
    }
    if (pinned && steps_on_device(prob)) return integrate_device(prob, G, ws, s, out, h_iters, h_grid, timing);

    const int d = prob->dim, nb = prob->nbins;
    std::vector<double> grid((size_t)d * (nb + 1)), buf(4 + (size_t)d * nb);
    std::vector<double> Is(prob->itmax), Vs(prob->itmax);
    init_grid(d, nb, grid.data());
    Events ev;
    if (timing) HIP_TRY(ev.create());
    double ms_s = 0.0, ms_f = 0.0, est[3] = {0.0, 0.0, NAN};
    int k = 0, converged = 0;
    int spin_us = 0;  // how long primed refinement threads spin: about one pass
    for (int it = 0; it < prob->itmax; ++it) {
        const bool adjust = it < prob->ita;
        const auto pass_start = std::chrono::steady_clock::now();
        st = run_pass(prob, G, ws, s, (uint32_t)it, adjust, grid.data(), buf.data(), nullptr, 0, 0,
                      timing ? &ev : nullptr, &ms_s, &ms_f, spin_us, pinned);
        if (st != MC_OK) return st;
        const double pass_us = std::chrono::duration<double, std::micro>(
                                   std::chrono::steady_clock::now() - pass_start).count();
        spin_us = (int)std::min(2.0 * pass_us + 200.0, 20000.0);
        Is[it] = buf[0];
        Vs[it] = buf[1];
        k = it + 1;
        weighted(k, Is.data(), Vs.data(), est);
        if (adjust) {
            if (prob->one_d)
                refine_1d(d, nb, prob->alpha, buf.data() + 4, grid.data());
            else
                refine(d, nb, prob->alpha, buf.data() + 4, grid.data());
        }
        if (check_convergence(prob, k, est)) {
            converged = 1;
            break;
        }
    }
    out->estimate = est[0];
    out->error = est[1];
    out->chi2_dof = est[2];
    out->iterations = k;
    out->converged = converged;
    out->calls = (int64_t)k * G.m * G.p;
    if (h_iters)
        for (int i = 0; i < k; ++i) {
            h_iters[2 * i] = Is[i];
            h_iters[2 * i + 1] = Vs[i];
        }
    if (h_grid) std::copy(grid.begin(), grid.end(), h_grid);
    if (timing) {
        timing->sample_ms = ms_s;
        timing->finalize_ms = ms_f;
        timing->launches = k;
        timing->blocks = prob->ita > 0 ? G.blocks_adj : G.blocks_noadj;
        timing->threads = G.threads;
        timing->lds_bytes = (int32_t)(prob->ita > 0 ? G.lds_adj : G.lds_noadj);
    }
    return MC_OK;
}

}  // namespace

extern "C" {

mc_status mc_integrate(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream,
                       mc_result *out, double *h_iters, double *h_grid, mc_timing *timing) {
    return integrate(prob, d_ws, ws_bytes, stream, true, out, h_iters, h_grid, timing);
}

mc_status mc_integrate_prepared(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream,
                                mc_result *out, double *h_iters, double *h_grid,
                                mc_timing *timing) {
    return integrate(prob, d_ws, ws_bytes, stream, false, out, h_iters, h_grid, timing);
}

}  // extern "C"

namespace mcubes {
namespace host {

mc_status integrate_unpinned(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream,
                             mc_result *out, double *h_iters, double *h_grid) {
    return integrate(prob, d_ws, ws_bytes, stream, true, out, h_iters, h_grid, nullptr, false);
}

}  // namespace host
}  // namespace mcubes
