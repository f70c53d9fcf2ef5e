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

#include "internal.hpp"

using namespace mcubes;

namespace {

constexpr int kDefaultThreads = 512;
constexpr size_t kAlign = 256;
constexpr size_t kLdsLimit = 160 * 1024;   // gfx950 LDS per workgroup
constexpr int64_t kTablesLen = 2 * kTableN * kTableN;
constexpr int64_t kMaxIntervals = int64_t(1) << 30;  // g; keeps digit arithmetic in 32 bits

#define HIP_TRY(expr)                               \
    do {                                            \
        if ((expr) != hipSuccess) return MC_EDEVICE; \
    } while (0)

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// ------------------------------------------------------------------ lattice

// 1 if b^d <= lim (no overflow).
bool pow_le(int64_t b, int d, int64_t lim) {
    __int128 acc = 1;
    for (int i = 0; i < d; ++i) {
        acc *= b;
        if (acc > lim) return false;
    }
    return true;
}

mc_status lattice(int d, int64_t maxcalls, int64_t *g, int64_t *m, int64_t *p) {
    if (d < 1 || d > MC_MAX_DIM || maxcalls < 4 || maxcalls > (int64_t(1) << 62)) return MC_EINVAL;
    const int64_t half = maxcalls / 2;
    // binary search for the largest gg with gg^d <= half
    int64_t lo = 1, hi = 2;
    while (pow_le(hi, d, half)) hi *= 2;
    while (hi - lo > 1) {
        const int64_t mid = lo + (hi - lo) / 2;
        if (pow_le(mid, d, half)) lo = mid; else hi = mid;
    }
    int64_t mm = 1;
    for (int i = 0; i < d; ++i) mm *= lo;
    *g = lo;
    *m = mm;
    *p = maxcalls / mm;
    return MC_OK;
}

int expected_params(int integrand, int d) {
    switch (integrand) {
    case MC_F_CONST: return 1;
    case MC_F_GAUSS_PRODUCT: return 2 * d;
    case MC_F_CORNER_PEAK: return d;
    case MC_F_GAUSS_TABLES: return 2 * d;
    default: return -1;
    }
}

int threads_of(const mc_problem *pr) { return pr->threads ? pr->threads : kDefaultThreads; }

size_t lds_bytes_of(int d, int nb, bool hist) {
    return sizeof(double) * ((size_t)kConstStride * d + (size_t)d * (nb + 1) + (hist ? (size_t)d * nb : 0));
}

mc_status validate(const mc_problem *pr) {
    if (!pr) return MC_EINVAL;
    const int d = pr->dim;
    if (d < 1 || d > MC_MAX_DIM) return MC_EINVAL;
    const int np = expected_params(pr->integrand, d);
    if (np < 0 || pr->n_params != np || !pr->params) return MC_EINVAL;
    if (pr->integrand == MC_F_GAUSS_TABLES) {
        if (d < 4 || !pr->tables || pr->n_tables != kTablesLen) return MC_EINVAL;
    } else if (pr->n_tables != 0) {
        return MC_EINVAL;
    }
    if (!pr->lo || !pr->hi) return MC_EINVAL;
    for (int j = 0; j < d; ++j)
        if (!std::isfinite(pr->lo[j]) || !std::isfinite(pr->hi[j]) || !(pr->lo[j] < pr->hi[j]))
            return MC_EINVAL;
    int64_t g, m, p;
    if (lattice(d, pr->maxcalls, &g, &m, &p) != MC_OK) return MC_EINVAL;
    if (g > kMaxIntervals) return MC_EINVAL;
    if (pr->nbins < 2 || pr->nbins > (1 << 20)) return MC_EINVAL;
    if (lds_bytes_of(d, pr->nbins, true) > kLdsLimit) return MC_EINVAL;
    if (pr->itmax < 1 || pr->ita < 0 || pr->ita > pr->itmax) return MC_EINVAL;
    if (pr->precision != MC_FP64) return MC_EINVAL;
    if (!(pr->alpha > 0.0) || !std::isfinite(pr->alpha)) return MC_EINVAL;
    if (!(pr->tau_rel >= 0.0) || !std::isfinite(pr->tau_rel)) return MC_EINVAL;
    const int th = threads_of(pr);
    if (pr->blocks < 0 || th < 64 || th > kMaxBlock || th % 64 != 0) return MC_EINVAL;
    return MC_OK;
}

// ------------------------------------------------------------------ launch geometry and workspace

struct Geometry {
    int64_t g, m, p;
    int threads;
    int blocks_adj, blocks_noadj;
    size_t lds_adj, lds_noadj;
    int hist_stride;          // doubles per workgroup histogram (padded)
    size_t off_consts, off_grid, off_tables, off_partials, off_out, off_flag, total;
};

std::mutex g_attr_mu;
std::vector<std::pair<const void *, size_t>> g_attr_set;  // largest LDS size set per kernel

hipError_t allow_lds(const void *fn, size_t bytes) {
    if (bytes <= 64 * 1024) return hipSuccess;
    std::lock_guard<std::mutex> lock(g_attr_mu);
    for (auto &e : g_attr_set)
        if (e.first == fn && e.second >= bytes) return hipSuccess;
    hipError_t err = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
    if (err != hipSuccess) return err;
    g_attr_set.emplace_back(fn, bytes);
    return hipSuccess;
}

mc_status blocks_for(const void *fn, int threads, size_t lds, int64_t m, int requested, int *out) {
    int dev = 0, cus = 0, per_cu = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    HIP_TRY(allow_lds(fn, lds));
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, lds));
    if (per_cu < 1) return MC_EINVAL;
    int64_t want = requested > 0 ? requested : (int64_t)per_cu * cus;
    const int64_t useful = (m + threads - 1) / threads;
    if (requested <= 0) want = std::min(want, useful);
    *out = (int)std::max<int64_t>(1, std::min<int64_t>(want, 1 << 20));
    return MC_OK;
}

mc_status geometry(const mc_problem *pr, Geometry *geo) {
    mc_status st = validate(pr);
    if (st != MC_OK) return st;
    Geometry G{};
    lattice(pr->dim, pr->maxcalls, &G.g, &G.m, &G.p);
    const int d = pr->dim, nb = pr->nbins;
    G.threads = threads_of(pr);
    G.lds_adj = lds_bytes_of(d, nb, true);
    G.lds_noadj = lds_bytes_of(d, nb, false);
    const void *fn = sample_kernel(pr->integrand, d, false);
    if (!fn) return MC_EINVAL;
    st = blocks_for(fn, G.threads, G.lds_adj, G.m, pr->blocks, &G.blocks_adj);
    if (st != MC_OK) return st;
    st = blocks_for(fn, G.threads, G.lds_noadj, G.m, pr->blocks, &G.blocks_noadj);
    if (st != MC_OK) return st;
    G.hist_stride = (int)((d * (size_t)nb + 31) / 32 * 32);
    const size_t part_adj = (4 + (size_t)G.hist_stride) * G.blocks_adj;
    const size_t part_noadj = 4 * (size_t)G.blocks_noadj;
    size_t off = 0;
    G.off_consts = off;
    off = align_up(off + sizeof(double) * kConstStride * d);
    G.off_grid = off;
    off = align_up(off + sizeof(double) * d * (nb + 1));
    G.off_tables = off;
    if (pr->integrand == MC_F_GAUSS_TABLES) off = align_up(off + sizeof(double) * kTablesLen);
    G.off_partials = off;
    off = align_up(off + sizeof(double) * std::max(part_adj, part_noadj));
    G.off_out = off;
    off = align_up(off + sizeof(double) * (4 + (size_t)d * nb));
    G.off_flag = off;
    off = align_up(off + sizeof(uint32_t));
    G.total = off;
    *geo = G;
    return MC_OK;
}

// ------------------------------------------------------------------ host worker threads

// A few host threads that take the axes of one bin adjustment in parallel
// (axes are independent, so the result does not depend on the split).  The
// jobs are short (tens of microseconds), so the driver primes the pool while
// it waits for the GPU: primed workers spin for a bounded time instead of
// sleeping, and a job is picked up within microseconds.  Tasks are tickets
// (generation << 32 | index), so a worker that wakes late for an old job can
// never take a task of a newer one.  One job at a time; a caller that finds
// the pool busy runs its job alone.
class AxisPool {
  public:
    static AxisPool &get() {
        static AxisPool pool;
        return pool;
    }

    // Workers spin (rather than sleep) for the next `us` microseconds.
    void prime(int us) {
        if (!start_workers()) return;
        spin_until_.store(now_ns() + (int64_t)us * 1000, std::memory_order_release);
        std::lock_guard<std::mutex> lk(mu_);
        cv_.notify_all();
    }

    void run(int n, const std::function<void(int)> &fn) {
        std::unique_lock<std::mutex> job_lock(job_mu_, std::try_to_lock);
        if (n < 2 || !job_lock.owns_lock() || !start_workers()) {
            for (int i = 0; i < n; ++i) fn(i);
            return;
        }
        const uint64_t gen = gen_.load(std::memory_order_relaxed) + 1;
        job_.store(&fn, std::memory_order_relaxed);
        n_.store(n, std::memory_order_relaxed);
        remaining_.store(n, std::memory_order_relaxed);
        ticket_.store(gen << 32, std::memory_order_relaxed);
        {
            std::lock_guard<std::mutex> lk(mu_);
            gen_.store(gen, std::memory_order_release);
        }
        cv_.notify_all();
        drain(gen);
        while (remaining_.load(std::memory_order_acquire) > 0) std::this_thread::yield();
    }

    ~AxisPool() {
        {
            std::lock_guard<std::mutex> lk(mu_);
            stop_.store(true);
        }
        cv_.notify_all();
        for (auto &t : workers_) t.join();
    }

  private:
    static int64_t now_ns() {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(
                   std::chrono::steady_clock::now().time_since_epoch()).count();
    }

    bool start_workers() {
        std::lock_guard<std::mutex> lk(start_mu_);
        if (!workers_.empty()) return true;
        const unsigned hw = std::thread::hardware_concurrency();
        const int count = (int)std::min<unsigned>(hw > 1 ? hw - 1 : 0, 7);
        try {
            for (int i = 0; i < count; ++i) workers_.emplace_back([this] { loop(); });
        } catch (...) {
        }
        return !workers_.empty();
    }

    void drain(uint64_t gen) {
        for (;;) {
            uint64_t t = ticket_.load(std::memory_order_acquire);
            if ((t >> 32) != gen) return;
            const uint32_t i = (uint32_t)t;
            if ((int)i >= n_.load(std::memory_order_relaxed)) return;
            if (!ticket_.compare_exchange_weak(t, t + 1, std::memory_order_acq_rel)) continue;
            (*job_.load(std::memory_order_relaxed))((int)i);
            remaining_.fetch_sub(1, std::memory_order_release);
        }
    }

    void loop() {
        uint64_t seen = gen_.load(std::memory_order_acquire);
        for (;;) {
            uint64_t g = gen_.load(std::memory_order_acquire);
            while (g == seen && !stop_.load() && now_ns() < spin_until_.load(std::memory_order_acquire)) {
                std::this_thread::yield();
                g = gen_.load(std::memory_order_acquire);
            }
            if (g == seen) {
                std::unique_lock<std::mutex> lk(mu_);
                cv_.wait(lk, [&] {
                    return stop_.load() || gen_.load(std::memory_order_acquire) != seen ||
                           now_ns() < spin_until_.load(std::memory_order_acquire);
                });
                if (stop_.load()) return;
                continue;
            }
            if (stop_.load()) return;
            seen = g;
            drain(g);
        }
    }

    std::mutex job_mu_, mu_, start_mu_;
    std::condition_variable cv_;
    std::vector<std::thread> workers_;
    // job_ and n_ are read by workers only after they acquire the generation that
    // published them; a worker still holding an older generation may read them
    // too, but its ticket compare-exchange then fails.
    std::atomic<const std::function<void(int)> *> job_{nullptr};
    std::atomic<int> n_{0};
    std::atomic<int> remaining_{0};
    std::atomic<uint64_t> gen_{0}, ticket_{0};
    std::atomic<int64_t> spin_until_{0};
    std::atomic<bool> stop_{false};
};

// ------------------------------------------------------------------ one sampling pass

void fill_args(const mc_problem *pr, const Geometry &G, char *ws, uint32_t iter, bool adjust,
               int blocks, SampleArgs *a) {
    std::memset(a, 0, sizeof(*a));
    const int d = pr->dim, nb = pr->nbins;
    a->grid = reinterpret_cast<const double *>(ws + G.off_grid);
    a->tables = pr->integrand == MC_F_GAUSS_TABLES ? reinterpret_cast<const double *>(ws + G.off_tables)
                                                   : nullptr;
    a->partials = reinterpret_cast<double *>(ws + G.off_partials);
    a->flag = reinterpret_cast<uint32_t *>(ws + G.off_flag);
    a->consts = reinterpret_cast<const double *>(ws + G.off_consts);
    a->trace = nullptr;
    a->m = G.m;
    a->stride = (int64_t)blocks * G.threads;
    a->seed = pr->seed;
    a->iter = iter;
    a->p = (int32_t)G.p;
    a->nb = nb;
    a->g = (int32_t)G.g;
    a->hist = adjust ? 1 : 0;
    a->hist_stride = G.hist_stride;
    a->s = (double)nb / (double)G.g;
    a->nb_minus1 = (double)(nb - 1);
    a->inv = 1.0 / (double)(G.m * G.p);
    a->pd = (double)G.p;
    a->inv_pm1 = 1.0 / (a->pd - 1.0);
    if (pr->integrand == MC_F_CONST) a->cval = pr->params[0];
    // the per-lane stride in base g (only d digits are used: a lane that
    // overflows the top digit has left the lattice)
    int64_t rest = a->stride;
    for (int j = 0; j < d; ++j) {
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

// Runs sampling + finalize and reads the result back.  out_host holds
// 4 + d*nb doubles.
mc_status run_pass(const mc_problem *pr, const Geometry &G, char *ws, hipStream_t stream,
                   uint32_t iter, bool adjust, const double *h_grid, double *out_host,
                   double *trace, int64_t t0, int64_t t1, Events *ev, double *ms_sample,
                   double *ms_fin, int spin_us = 0) {
    const int d = pr->dim, nb = pr->nbins;
    const int blocks = adjust ? G.blocks_adj : G.blocks_noadj;
    const size_t lds = adjust ? G.lds_adj : G.lds_noadj;
    SampleArgs a;
    fill_args(pr, G, ws, iter, adjust, blocks, &a);
    a.trace = trace;
    a.t0 = t0;
    a.t1 = t1;
    HIP_TRY(hipMemcpyAsync(ws + G.off_grid, h_grid, sizeof(double) * d * (nb + 1),
                           hipMemcpyHostToDevice, stream));
    if (ev) HIP_TRY(hipEventRecord(ev->e[0], stream));
    HIP_TRY(allow_lds(sample_kernel(pr->integrand, d, trace != nullptr), lds));
    HIP_TRY(launch_sample(pr->integrand, d, blocks, G.threads, lds, stream, a));
    if (ev) HIP_TRY(hipEventRecord(ev->e[1], stream));
    double *out_dev = reinterpret_cast<double *>(ws + G.off_out);
    HIP_TRY(launch_finalize(a.partials, blocks, d * nb, G.hist_stride, adjust ? 1 : 0, a.flag,
                            out_dev, stream));
    if (ev) HIP_TRY(hipEventRecord(ev->e[2], stream));
    if (adjust && d > 1) AxisPool::get().prime(spin_us);
    const size_t nout = 4 + (adjust ? (size_t)d * nb : 0);
    HIP_TRY(hipMemcpyAsync(out_host, out_dev, sizeof(double) * nout, hipMemcpyDeviceToHost, stream));
    HIP_TRY(hipStreamSynchronize(stream));
    if (ev) {
        float a_ms = 0.f, b_ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&a_ms, ev->e[0], ev->e[1]));
        HIP_TRY(hipEventElapsedTime(&b_ms, ev->e[1], ev->e[2]));
        *ms_sample += a_ms;
        *ms_fin += b_ms;
    }
    return out_host[2] != 0.0 ? MC_ENONFINITE : MC_OK;
}

// Per-axis constants in the layout the sampling kernel keeps in LDS.
std::vector<double> axis_constants(const mc_problem *pr) {
    const int d = pr->dim, nb = pr->nbins;
    std::vector<double> c((size_t)kConstStride * d, 0.0);
    for (int j = 0; j < d; ++j) {
        double *cj = c.data() + (size_t)kConstStride * j;
        cj[0] = pr->lo[j];
        cj[1] = pr->hi[j] - pr->lo[j];
        cj[2] = (double)nb * cj[1];
        switch (pr->integrand) {
        case MC_F_GAUSS_PRODUCT:
        case MC_F_GAUSS_TABLES:
            cj[3] = pr->params[j];
            cj[4] = 1.0 / pr->params[d + j];
            break;
        case MC_F_CORNER_PEAK:
            cj[3] = pr->params[j];
            break;
        }
    }
    return c;
}

mc_status prepare(const mc_problem *pr, const Geometry &G, char *ws, hipStream_t stream) {
    const std::vector<double> consts = axis_constants(pr);
    HIP_TRY(hipMemcpyAsync(ws + G.off_consts, consts.data(), sizeof(double) * consts.size(),
                           hipMemcpyHostToDevice, stream));
    if (pr->integrand == MC_F_GAUSS_TABLES)
        HIP_TRY(hipMemcpyAsync(ws + G.off_tables, pr->tables, sizeof(double) * kTablesLen,
                               hipMemcpyHostToDevice, stream));
    HIP_TRY(launch_clear_flag(reinterpret_cast<uint32_t *>(ws + G.off_flag), stream));
    HIP_TRY(hipStreamSynchronize(stream));
    return MC_OK;
}

// ------------------------------------------------------------------ host steps of Alg. 2

void init_grid(int d, int nb, double *grid) {
    for (int j = 0; j < d; ++j) {
        double *row = grid + (size_t)j * (nb + 1);
        for (int i = 0; i <= nb; ++i) row[i] = (double)i / (double)nb;
    }
}

// Bin adjustment of one axis; returns without change when the contributions
// carry no usable weight.
void refine_axis(int nb, double alpha, const double *C, double *B, std::vector<double> &sm,
                 std::vector<double> &r, std::vector<double> &prev) {
    sm[0] = (C[0] + C[1]) / 2.0;
    for (int i = 1; i + 1 < nb; ++i) sm[i] = ((C[i - 1] + C[i]) + C[i + 1]) / 3.0;
    sm[nb - 1] = (C[nb - 2] + C[nb - 1]) / 2.0;
    double total = 0.0;
    for (int i = 0; i < nb; ++i) total = total + sm[i];
    if (!(total > 0.0) || !std::isfinite(total)) return;
    double rsum = 0.0;
    for (int i = 0; i < nb; ++i) {
        double v;
        if (sm[i] == 0.0) v = 0.0;
        else if (sm[i] == total) v = 1.0;
        else v = std::pow((1.0 - sm[i] / total) / std::log(total / sm[i]), alpha);
        r[i] = v;
        rsum = rsum + v;
    }
    if (!(rsum > 0.0)) return;
    std::copy(B, B + nb + 1, prev.begin());
    const double per_bin = rsum / (double)nb;
    int src = 0;
    double acc = 0.0;
    for (int k = 1; k < nb; ++k) {
        const double goal = (double)k * per_bin;
        while (src < nb - 1 && acc + r[src] < goal) {
            acc = acc + r[src];
            ++src;
        }
        double frac = r[src] > 0.0 ? (goal - acc) / r[src] : 0.0;
        frac = std::min(std::max(frac, 0.0), 1.0);
        const double edge = std::fma(frac, prev[src + 1] - prev[src], prev[src]);
        B[k] = std::max(edge, B[k - 1]);
    }
    B[0] = 0.0;
    B[nb] = 1.0;
}

void refine(int d, int nb, double alpha, const double *hist, double *grid) {
    AxisPool::get().run(d, [&](int j) {
        std::vector<double> sm(nb), r(nb), prev(nb + 1);
        refine_axis(nb, alpha, hist + (size_t)j * nb, grid + (size_t)j * (nb + 1), sm, r, prev);
    });
}

void weighted(int k, const double *I, const double *var, double *out) {
    int zeros = 0;
    double zsum = 0.0;
    for (int i = 0; i < k; ++i)
        if (var[i] == 0.0) {
            ++zeros;
            zsum = zsum + I[i];
        }
    if (zeros) {
        out[0] = zsum / (double)zeros;
        out[1] = 0.0;
        out[2] = k > 1 ? 0.0 : NAN;
        return;
    }
    double wsum = 0.0, wisum = 0.0;
    for (int i = 0; i < k; ++i) {
        const double w = 1.0 / var[i];
        wsum = wsum + w;
        wisum = wisum + w * I[i];
    }
    const double mean = wisum / wsum;
    double chi = 0.0;
    for (int i = 0; i < k; ++i) {
        const double dv = I[i] - mean;
        chi = chi + (dv * dv) / var[i];
    }
    out[0] = mean;
    out[1] = 1.0 / std::sqrt(wsum);
    out[2] = k > 1 ? chi / (double)(k - 1) : NAN;
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

mc_status mc_integrate(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream,
                       mc_result *out, double *h_iters, double *h_grid, mc_timing *timing) {
    if (!out) return MC_EINVAL;
    Geometry G;
    mc_status st = geometry(prob, &G);
    if (st != MC_OK) return st;
    if (!d_ws || ws_bytes < G.total) return MC_EWORKSPACE;
    char *ws = static_cast<char *>(d_ws);
    hipStream_t s = static_cast<hipStream_t>(stream);
    st = prepare(prob, G, ws, s);
    if (st != MC_OK) return st;

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
                      timing ? &ev : nullptr, &ms_s, &ms_f, spin_us);
        if (st != MC_OK) return st;
        const double pass_us = std::chrono::duration<double, std::micro>(
                                   std::chrono::steady_clock::now() - pass_start).count();
        spin_us = (int)std::min(2.0 * pass_us + 200.0, 20000.0);
        Is[it] = buf[0];
        Vs[it] = buf[1];
        k = it + 1;
        weighted(k, Is.data(), Vs.data(), est);
        if (adjust) refine(d, nb, prob->alpha, buf.data() + 4, grid.data());
        if (k >= 2 && prob->tau_rel > 0.0 && est[1] <= prob->tau_rel * std::fabs(est[0])) {
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

}  // extern "C"
