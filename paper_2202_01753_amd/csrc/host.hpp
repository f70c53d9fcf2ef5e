// Host-side helpers shared by the single-integral driver (mcubes_api.cpp)
// and the batched driver and server (mcubes_batch.cpp).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <functional>
#include <mutex>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "mcubes.h"

namespace mcubes {
namespace host {

constexpr int kDefaultThreads = 512;
constexpr size_t kAlign = 256;
constexpr size_t kLdsLimit = 160 * 1024;   // gfx950 LDS per workgroup
// Dynamic LDS a sampling kernel may ask for: the workgroup's LDS less a
// reserve for the kernels' static arrays (the reduction scratch, 520 bytes).
constexpr size_t kLdsDynamicLimit = kLdsLimit - 1024;
constexpr int64_t kTablesLen = 2 * kTableN * kTableN;
// floats of the two tables in the FP32-eval device layout (row pairs)
constexpr int64_t kTablesLen32 = 2 * kTablesLen;
constexpr int64_t kMaxIntervals = int64_t(1) << 30;  // g; keeps digit arithmetic in 32 bits

// On failure the runtime's last-error state is cleared as well, so that the
// caller's next HIP call does not see this error again.
#define HIP_TRY(expr)                      \
    do {                                   \
        if ((expr) != hipSuccess) {        \
            (void)hipGetLastError();       \
            return MC_EDEVICE;             \
        }                                  \
    } while (0)


size_t align_up(size_t v);

// Sub-cube lattice of Alg. 2: the largest g with g^d <= maxcalls/2, m = g^d,
// p = maxcalls/m (integer arithmetic throughout).
mc_status lattice(int d, int64_t maxcalls, int64_t *g, int64_t *m, int64_t *p);
bool is_fp32(const mc_problem *pr);
inline int threads_of(const mc_problem *pr) { return pr->threads ? pr->threads : kDefaultThreads; }
// LDS of one sampling workgroup (grid, optional FP64 histogram).
size_t lds_bytes_of(int d, int nb, bool hist, bool fp32);
// Checks a problem before any device work; MC_OK or MC_EINVAL.
mc_status validate(const mc_problem *pr);
// Lets a kernel use more than 64 KB of dynamic LDS (once per kernel and size).
hipError_t allow_lds(const void *fn, size_t bytes);
// Per-axis constants (kConstStride doubles per axis) in the layout the kernels read.
std::vector<double> axis_constants(const mc_problem *pr);
// The per-integral part of the sampling-kernel arguments (lattice, scales,
// iteration, pointers into device memory); launch-specific fields are zero.
void sample_args(const mc_problem *pr, int64_t g, int64_t m, int64_t p, uint32_t iter, bool adjust,
                 const void *consts, const double *grid, const void *tables, SampleArgs *a);
// Init-Bins: nb equal bins per axis.
void init_grid(int d, int nb, double *grid);
// The two tables (kTablesLen doubles, row-major) in the FP32-eval device
// layout: kTablesLen32 floats, each value rounded once.
void tables_f32(const double *tables, float *out);
// Adjust-Bin-Bounds of one axis (scratch vectors of nb, nb, nb+1 doubles).
void refine_axis(int nb, double alpha, const double *C, double *B, std::vector<double> &sm,
                 std::vector<double> &r, std::vector<double> &prev);
// Adjust-Bin-Bounds of all axes, the axes on the host pool.
void refine(int d, int nb, double alpha, const double *hist, double *grid);
// m-Cubes1D adjustment: axis 0 from hist row 0, then copied to every axis.
void refine_1d(int d, int nb, double alpha, const double *hist, double *grid);
// Weighted-Estimates over k iterations: out = [mean, sigma, chi2/dof].
void weighted(int k, const double *I, const double *var, double *out);
// Check-Convergence with the chi^2 condition: k >= 2 iterations, est[1] <=
// tau_rel |est[0]| and est[2] (chi^2/dof) within the problem's bound.
bool check_convergence(const mc_problem *pr, int k, const double *est);

// mc_integrate on the given device buffer with the per-pass host copies made
// from and to pageable memory: no page-locked staging is allocated (the
// entry point that allocates nothing runs on this).
mc_status integrate_unpinned(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream,
                             mc_result *out, double *h_iters, double *h_grid);

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


}  // namespace host
}  // namespace mcubes
