// Batched m-Cubes and the serving loop.
//
// An Engine owns a caller-provided device workspace split into an arena and
// a step area.  The arena holds each admitted integral's persistent device
// state (per-axis constants, tables, two grid buffers, and the latest pass's
// [I, var, flag, 0, histogram]); a first-fit allocator hands it out, and an
// integral is admitted only when its block and its share of the step area
// fit ("admission by device memory").  Every step:
//   1. admits queued integrals that fit (tables are copied once; constants
//      travel with the step's upload and the starting grid is written on the
//      device);
//   2. groups the active integrals by precision and by how many workgroups
//      per CU their LDS footprint allows, splits each group's sub-cubes into
//      contiguous segments of bounded work, orders them largest first, and
//      uploads the step's small tables (items, segments, queue order and
//      counters, item indices, admissions) in one copy;
//   3. runs one persistent batched sampling launch per group present (its
//      workgroups draw segments from a counter), the in-order merge of each
//      integral's segment totals, and the bin adjustment of the integrals
//      still adjusting — on the device, so grids and histograms stay
//      resident;
//   4. after the merge, Weighted-Estimates and Check-Convergence run on the
//      device for every integral, which stops it there (its later segments
//      do nothing) once it has converged or run out of iterations;
//   5. reads back kResStride doubles per integral.
// The steps are pipelined by one: a call launches the next step first and
// only then waits for the previous one and retires the integrals it
// stopped, so the device never waits for the host's bookkeeping, and the
// upload, table staging and read-back buffers alternate between two copies.
#include <cmath>
#include <algorithm>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <unordered_map>

#include "batch_plan.hpp"
#include "estimate.hpp"
#include "host.hpp"
#include "internal.hpp"
#include "mcubes.h"

using namespace mcubes;
using namespace mcubes::host;
using mcubes::plan::Arena;

namespace {

// Page-locked host memory (hipHostMalloc), grown on demand, so that a step's
// upload and read-back are asynchronous copies.  Only resized between steps,
// when no copy from or to it is in flight.
class Pinned {
  public:
    Pinned() = default;
    Pinned(const Pinned &) = delete;
    Pinned &operator=(const Pinned &) = delete;
    ~Pinned() {
        if (p_) (void)hipHostFree(p_);
    }
    hipError_t reserve(size_t bytes) {
        if (bytes <= cap_) return hipSuccess;
        const size_t prev = cap_;
        if (p_) {
            const hipError_t e = hipHostFree(p_);
            p_ = nullptr;
            cap_ = 0;
            if (e != hipSuccess) return e;
        }
        const size_t want = std::max({bytes, 2 * prev, size_t(1) << 20});  // geometric growth
        const hipError_t e = hipHostMalloc(&p_, want, hipHostMallocDefault);
        if (e == hipSuccess) cap_ = want;
        return e;
    }
    char *data() const { return static_cast<char *>(p_); }

  private:
    void *p_ = nullptr;
    size_t cap_ = 0;
};

struct Request {
    int64_t id = 0;
    mc_problem prob{};
    std::vector<double> params, tables, lo, hi;
    std::vector<char> consts_img;  // per-axis constants in the device precision, until admitted
    int64_t g = 0, m = 0, p = 0;
    int32_t state = MC_REQ_QUEUED;
    mc_status status = MC_OK;
    size_t block_off = 0, block_bytes = 0;
    size_t off_consts = 0, off_tables = 0, off_grid[2] = {0, 0}, off_out = 0;  // in the workspace
    size_t off_iters = 0, off_state = 0;
    int cur = 0;     // current grid buffer
    int it = 0;      // iterations whose results the host has seen
    int launched = 0;  // iterations launched (it, or one more while a step is in flight)
    std::vector<double> Is, Vs;
    double est[3] = {0.0, 0.0, NAN};
    int converged = 0;
    mc_result result{};
    double cost = 0;  // relative work per sub-cube (for the work split)
    int group = 0;    // launch group of the current step
    int skipped = 0;  // consecutive steps left out under a step budget
};

bool fp32_of(const Request &r) { return is_fp32(&r.prob); }

int dnb(const Request &r) { return r.prob.dim * r.prob.nbins; }

// Relative work of one sub-cube (p samples), from the per-sample operation
// counts of the sampling kernel: Philox blocks, the map, the integrand.
double cube_cost(const mc_problem &pr, int64_t p) {
    const int d = pr.dim;
    const int blocks = is_fp32(&pr) ? (d + 3) / 4 : (d + 1) / 2;
    double f = 0.0;
    if (pr.integrand == MC_F_GAUSS_PRODUCT) f = 3.0 * d + 20;
    if (pr.integrand == MC_F_CORNER_PEAK) f = d + 16;
    if (pr.integrand == MC_F_GAUSS_TABLES) f = 3.0 * d + 64;
    return (double)p * (35.0 * blocks + 25.0 * d + f + 10.0) + 20.0 + 5.0 * d;
}

// Bytes of an integral's persistent block and the offsets inside it.
size_t block_layout(const Request &r, size_t *o_consts, size_t *o_tables, size_t *o_grid0,
                    size_t *o_grid1, size_t *o_out, size_t *o_iters = nullptr,
                    size_t *o_state = nullptr) {
    const int d = r.prob.dim, nb = r.prob.nbins;
    const size_t real = fp32_of(r) ? sizeof(float) : sizeof(double);
    size_t off = 0;
    *o_consts = off;
    off = align_up(off + real * kConstStride * d);
    *o_tables = off;
    if (r.prob.integrand == MC_F_GAUSS_TABLES) off = align_up(off + real * (fp32_of(r) ? kTablesLen32 : kTablesLen));
    *o_grid0 = off;
    off = align_up(off + sizeof(double) * d * (nb + 1));
    *o_grid1 = off;
    off = align_up(off + sizeof(double) * d * (nb + 1));
    *o_out = off;
    off = align_up(off + sizeof(double) * (4 + (size_t)d * nb));
    if (o_iters) *o_iters = off;
    off = align_up(off + sizeof(double) * 2 * (size_t)r.prob.itmax);
    if (o_state) *o_state = off;
    off = align_up(off + sizeof(uint32_t));
    return off;
}

// What the step area must hold for a set of integrals: n items, the sum and
// maximum of d*nb and the sum of d over them (all counted as adjusting).
struct StepNeed {
    int64_t n = 0, sum_dnb = 0, max_dnb = 0, sum_d = 0;
    void add(const Request &r) {
        ++n;
        sum_dnb += dnb(r);
        max_dnb = std::max<int64_t>(max_dnb, dnb(r));
        sum_d += r.prob.dim;
    }
};

struct StepLayout {
    size_t items, item_first, flags, queue, order, segs, axis_item, next_grid, admit_recs, admit_data,
        upload_end;
    size_t res, seg_tot, total;
    int64_t nseg;  // segments the layout has room for
};

// Batched kernels: precision x integrand family (closed forms, tables).
constexpr int kKernels = 4;
int kernel_of(const Request &r) {
    return 2 * (fp32_of(r) ? 1 : 0) + (r.prob.integrand == MC_F_GAUSS_TABLES ? 1 : 0);
}
bool kernel_fp32(int kern) { return kern >= 2; }
bool kernel_tables(int kern) { return kern % 2 == 1; }
// Workgroups of kBatchBlock threads a CU can hold at the kernels' register use.
constexpr int kMaxWgsPerCu = 4;
// Launch groups per step: kernel x {integrals whose LDS footprint leaves the
// kernel's register-limited occupancy, the rest}.
constexpr int kGroups = 2 * kKernels;
// Upper bound of one integral's constants in bytes (kConstStride doubles per
// axis at the batch's largest dimension).
constexpr size_t kConstsMax = sizeof(double) * kConstStride * kBatchMaxDim;

// Segments per workgroup of a launch: the queue balances the workgroups to
// within about one segment.
constexpr int kSegsPerWg = 8;
// Sub-cubes a segment should at least hold (one per thread of a workgroup, twice).
constexpr int64_t kMinSegCubes = 2 * kBatchMaxBlock;

// Element counts of one step's tables.
struct StepCounts {
    int64_t n = 0;      // integrals
    int64_t nseg = 0;   // segments
    int64_t axes = 0;   // (integral, axis) pairs to adjust
    int64_t admit = 0;  // integrals admitted in the step
};

// The most a step over these integrals can need: every integral admitted and
// adjusting, and each launch group's split cutting kSegsPerWg * gcap (+1 for
// rounding) times.  Admission keeps this within the step area.
StepCounts worst_counts(const StepNeed &s, int gcap) {
    return StepCounts{s.n, s.n + kGroups * ((int64_t)kSegsPerWg * gcap + 1), s.sum_d, s.n};
}

// The step area's regions for the given counts.  Everything up to upload_end
// is written on the host and uploaded in one copy; the regions whose size
// depends on the number of segments come last, so that a step uploads only
// what it uses.
StepLayout step_layout(const StepCounts &c) {
    StepLayout L{};
    L.nseg = c.nseg;
    size_t off = 0;
    L.items = off;
    off = align_up(off + sizeof(BatchItem) * c.n);
    L.item_first = off;
    off = align_up(off + sizeof(int32_t) * (c.n + 1));
    L.flags = off;
    off = align_up(off + sizeof(uint32_t) * c.n);
    L.queue = off;
    off = align_up(off + sizeof(uint32_t) * kGroups);
    L.axis_item = off;
    off = align_up(off + sizeof(int32_t) * 2 * c.axes);
    L.next_grid = off;
    off = align_up(off + sizeof(double *) * c.n);
    L.admit_recs = off;
    off = align_up(off + sizeof(AdmitRecord) * c.admit);
    L.admit_data = off;
    off = align_up(off + kConstsMax * c.admit);
    L.order = off;
    off = align_up(off + sizeof(int32_t) * c.nseg);
    L.segs = off;
    off = align_up(off + sizeof(BatchSegment) * c.nseg);
    L.upload_end = off;
    L.res = off;
    off = align_up(off + sizeof(double) * kResStride * c.n);
    L.seg_tot = off;
    off = align_up(off + sizeof(double) * 4 * c.nseg);
    L.total = off;
    return L;
}

mc_status validate_batch(const mc_problem *pr) {
    mc_status st = validate(pr);
    if (st != MC_OK) return st;
    if (pr->dim > MC_BATCH_MAX_DIM) return MC_EINVAL;
    return MC_OK;
}

}  // namespace

// ====================================================================== engine

// Occupancy answers of the batched kernels, shared by every server of the
// process: (device, kernel, threads, LDS bytes rounded up) -> workgroups per CU.
constexpr size_t kOccLdsGranule = 512;
static std::mutex g_occ_mu;
static std::map<std::tuple<int, int, int, size_t>, int> g_occ;

struct mc_server {
    char *ws = nullptr;
    size_t ws_bytes = 0, arena_bytes = 0, step_cap = 0;
    int32_t max_active = 0;
    hipStream_t stream = nullptr;
    int dev = 0, cus = 0, gcap = 0;
    std::unique_ptr<Arena> arena;
    int64_t next_id = 1;
    std::unordered_map<int64_t, std::unique_ptr<Request>> all;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::vector<int64_t> last_finished;  // ids finished in the last step
    std::vector<Request *> admitted;     // admitted in this step, constants and grid pending
    int occ_full[kKernels] = {};  // the register-limited occupancy (256-thread workgroups)
    int64_t step_budget = 0;      // samples per step (0: every active request in every step)
    int32_t max_skip = 0;         // steps a request may be left out in a row under the budget
    StepNeed need;  // of the active set
    // Two of each, alternating between steps: the host fills one for the step
    // it launches while the previous step may still read the other.
    Pinned staging[2];    // the step's upload
    Pinned tab_stage[2];  // tables of the integrals admitted in the step
    Pinned res_buf[2];    // the step's read-back: kResStride doubles per integral
    hipEvent_t ev[2][3] = {};  // per buffer: sampling start and end, step done
    int buf = 0;               // the buffer of the next step launched
    // The step launched and not yet read back: its buffer, the ids of the
    // integrals it lists (in the order of its results) and its host time.
    struct InFlight {
        bool valid = false;
        int buf = 0;
        std::vector<int64_t> ids;
        double host_ms = 0.0;
    } inflight;
    mc_batch_stats stats{};

    ~mc_server() {
        for (auto &b : ev)
            for (auto &e : b)
                if (e) (void)hipEventDestroy(e);
    }

    mc_status init() {
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        gcap = cus * kMaxWgsPerCu;
        for (auto &b : ev)
            for (auto &e : b) HIP_TRY(hipEventCreate(&e));
        for (int k = 0; k < kKernels; ++k) {
            HIP_TRY(allow_lds(batch_kernel(kernel_fp32(k), kernel_tables(k)), kLdsDynamicLimit));
            mc_status st = occupancy(k, kBatchBlock, 0, &occ_full[k]);
            if (st != MC_OK) return st;
        }
        arena = std::make_unique<Arena>(arena_bytes);
        return MC_OK;
    }

    // Workgroups of a batched kernel that fit on a CU with the given
    // workgroup size and dynamic LDS (cached: the kernels do not change).
    // The LDS size is rounded up to kOccLdsGranule before the query, which can
    // only under-state the occupancy, and the answers are kept for the whole
    // process: a batch has thousands of distinct footprints, a query costs
    // microseconds.
    mc_status occupancy(int kern, int threads, size_t lds, int *out) {
        const size_t lds_q = (lds + kOccLdsGranule - 1) / kOccLdsGranule * kOccLdsGranule;
        const auto key = std::make_tuple(dev, kern, threads, lds_q);
        {
            std::lock_guard<std::mutex> lk(g_occ_mu);
            auto it = g_occ.find(key);
            if (it != g_occ.end()) {
                *out = it->second;
                return *out >= 1 ? MC_OK : MC_EINVAL;
            }
        }
        int per_cu = 0;
        HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &per_cu, batch_kernel(kernel_fp32(kern), kernel_tables(kern)), threads, lds_q));
        per_cu = std::min(per_cu, gcap / cus);
        {
            std::lock_guard<std::mutex> lk(g_occ_mu);
            g_occ.emplace(key, per_cu);
        }
        *out = per_cu;
        return per_cu >= 1 ? MC_OK : MC_EINVAL;
    }

    mc_status submit(const mc_problem *pr, int64_t *id) {
        mc_status st = validate_batch(pr);
        if (st != MC_OK) return st;
        auto r = std::make_unique<Request>();
        r->id = next_id++;
        r->prob = *pr;
        const int d = pr->dim;
        r->params.assign(pr->params, pr->params + pr->n_params);
        if (pr->tables) r->tables.assign(pr->tables, pr->tables + pr->n_tables);
        r->lo.assign(pr->lo, pr->lo + d);
        r->hi.assign(pr->hi, pr->hi + d);
        r->prob.params = r->params.data();
        r->prob.tables = r->tables.empty() ? nullptr : r->tables.data();
        r->prob.lo = r->lo.data();
        r->prob.hi = r->hi.data();
        lattice(d, pr->maxcalls, &r->g, &r->m, &r->p);
        r->cost = cube_cost(r->prob, r->p);
        size_t a, b, c, e, f;
        r->block_bytes = block_layout(*r, &a, &b, &c, &e, &f);
        StepNeed one;
        one.add(*r);
        if (r->block_bytes > arena_bytes || step_layout(worst_counts(one, gcap)).total > step_cap) return MC_EWORKSPACE;
        *id = r->id;
        queue.push_back(r.get());
        all.emplace(r->id, std::move(r));
        return MC_OK;
    }

    void finish(Request *r, int32_t state, mc_status status) {
        last_finished.push_back(r->id);
        r->state = state;
        r->status = status;
        arena->release(r->block_off, r->block_bytes);
        if (state == MC_REQ_DONE) {
            r->result.estimate = r->est[0];
            r->result.error = r->est[1];
            r->result.chi2_dof = r->est[2];
            r->result.iterations = r->it;
            r->result.converged = r->converged;
            r->result.calls = (int64_t)r->it * r->m * r->p;
        }
    }

    // Admits queued integrals in arrival order while their blocks and the
    // step area fit.
    mc_status admit() {
        const size_t first_new = admitted.size();
        while (!queue.empty() && (int32_t)active.size() < max_active) {
            Request *r = queue.front();
            StepNeed grown = need;
            grown.add(*r);
            if (step_layout(worst_counts(grown, gcap)).total > step_cap) break;
            size_t off;
            if (!arena->alloc(r->block_bytes, &off)) break;
            size_t oc, ot, og0, og1, oo, oi, os;
            block_layout(*r, &oc, &ot, &og0, &og1, &oo, &oi, &os);
            r->block_off = off;
            r->off_consts = off + oc;
            r->off_tables = off + ot;
            r->off_grid[0] = off + og0;
            r->off_grid[1] = off + og1;
            r->off_out = off + oo;
            r->off_iters = off + oi;
            r->off_state = off + os;
            // constants and the starting grid travel with the step's upload
            // (admit_kernel); the tables are copied below
            const std::vector<double> c = axis_constants(&r->prob);
            if (fp32_of(*r)) {
                const std::vector<float> c32(c.begin(), c.end());
                r->consts_img.assign(reinterpret_cast<const char *>(c32.data()),
                                     reinterpret_cast<const char *>(c32.data() + c32.size()));
            } else {
                r->consts_img.assign(reinterpret_cast<const char *>(c.data()),
                                     reinterpret_cast<const char *>(c.data() + c.size()));
            }
            admitted.push_back(r);
            r->cur = 0;
            r->state = MC_REQ_RUNNING;
            queue.pop_front();
            active.push_back(r);
            need = grown;
        }
        // the new integrals' tables (in their device precision), packed into
        // page-locked memory and copied from there
        size_t tab_bytes = 0;
        for (size_t k = first_new; k < admitted.size(); ++k)
            if (!admitted[k]->tables.empty())
                tab_bytes += align_up(fp32_of(*admitted[k]) ? sizeof(float) * kTablesLen32 : sizeof(double) * kTablesLen);
        if (tab_bytes) {
            // this step's copy of the staging buffer: its last copies were two
            // steps ago, which the previous call has waited for
            Pinned &tab = tab_stage[buf];
            HIP_TRY(tab.reserve(tab_bytes));
            size_t off = 0;
            for (size_t k = first_new; k < admitted.size(); ++k) {
                const Request *r = admitted[k];
                if (r->tables.empty()) continue;
                char *dst = tab.data() + off;
                size_t bytes;
                if (fp32_of(*r)) {
                    tables_f32(r->tables.data(), reinterpret_cast<float *>(dst));
                    bytes = sizeof(float) * kTablesLen32;
                } else {
                    std::memcpy(dst, r->tables.data(), sizeof(double) * kTablesLen);
                    bytes = sizeof(double) * kTablesLen;
                }
                HIP_TRY(hipMemcpyAsync(ws + r->off_tables, dst, bytes, hipMemcpyHostToDevice, stream));
                off += align_up(bytes);
            }
        }
        return MC_OK;
    }

    // Under a step budget: keeps in active the requests this step runs
    // (plan::select_for_step over their estimated remaining work, cost per
    // iteration times plan::expected_iterations) and moves the others to idle.
    void select_for_step(std::vector<Request *> &idle) {
        std::vector<plan::Candidate> cand;
        cand.reserve(active.size());
        for (const Request *r : active) {
            const double iters =
                plan::expected_iterations(r->it, r->prob.itmax, r->prob.tau_rel, r->est[0], r->est[1]);
            cand.push_back(plan::Candidate{r->cost * (double)r->m * iters, r->m * r->p, r->skipped, r->id});
        }
        const std::vector<char> run = plan::select_for_step(cand, step_budget, max_skip);
        std::vector<Request *> now;
        for (size_t i = 0; i < active.size(); ++i) {
            Request *r = active[i];
            if (run[i]) {
                r->skipped = 0;
                now.push_back(r);
            } else {
                r->skipped += 1;
                idle.push_back(r);
            }
        }
        active.swap(now);
    }

    mc_status step(int32_t *n_finished) {
        *n_finished = 0;
        last_finished.clear();
        const auto t_start = std::chrono::steady_clock::now();
        mc_status st = admit();
        if (st != MC_OK) return st;
        InFlight next;
        // integrals whose last iteration is in flight have certainly stopped:
        // they wait for the read-back outside this step
        std::vector<Request *> idle;  // not run in this step
        {
            std::vector<Request *> runnable;
            for (Request *r : active) (r->launched < r->prob.itmax ? runnable : idle).push_back(r);
            active.swap(runnable);
        }
        if (!active.empty()) {
            if (step_budget > 0) select_for_step(idle);
            st = launch_step(next);
        }
        active.insert(active.end(), idle.begin(), idle.end());
        if (st != MC_OK) return st;
        const auto t_launched = std::chrono::steady_clock::now();
        // the previous step's results, while the device runs this one
        double collect_host_ms = 0.0;
        if (inflight.valid) {
            st = collect(inflight, n_finished, &collect_host_ms);
            if (st != MC_OK) return st;
        }
        inflight = std::move(next);
        if (inflight.valid) buf ^= 1;
        need = StepNeed{};
        for (Request *r : active) need.add(*r);
        const auto t_end = std::chrono::steady_clock::now();
        stats.step_ms += std::chrono::duration<double, std::milli>(t_end - t_start).count();
        stats.host_ms +=
            std::chrono::duration<double, std::milli>(t_launched - t_start).count() + collect_host_ms;
        return MC_OK;
    }

    // Waits for a launched step, then retires what it stopped: the
    // integrals the device found converged, out of iterations or non-finite.
    // (Integrals retired by an earlier step may be listed; they did nothing.)
    mc_status collect(InFlight &f, int32_t *n_finished, double *host_ms) {
        HIP_TRY(hipEventSynchronize(ev[f.buf][2]));
        const auto t0 = std::chrono::steady_clock::now();
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[f.buf][0], ev[f.buf][1]));
        const double *res = reinterpret_cast<const double *>(res_buf[f.buf].data());
        bool worked = false;  // whether any integral listed still ran in this step
        for (size_t k = 0; k < f.ids.size(); ++k) {
            auto found = all.find(f.ids[k]);
            if (found == all.end()) continue;  // released by the caller
            Request *r = found->second.get();
            if (r->state != MC_REQ_RUNNING) continue;
            const double *q = res + (size_t)kResStride * k;
            if (q[6] == kResSkipped) continue;
            worked = true;
            stats.calls += r->m * r->p;
            r->it += 1;
            r->Is.push_back(q[0]);
            r->Vs.push_back(q[1]);
            r->est[0] = q[3];
            r->est[1] = q[4];
            r->est[2] = q[5];
            if (q[6] == (double)kItemFailed) {
                finish(r, MC_REQ_FAILED, MC_ENONFINITE);
                ++*n_finished;
            } else if (q[6] == (double)kItemDone) {
                r->converged = q[7] != 0.0 ? 1 : 0;
                finish(r, MC_REQ_DONE, MC_OK);
                ++*n_finished;
            }
        }
        active.erase(std::remove_if(active.begin(), active.end(),
                                    [](const Request *r) { return r->state != MC_REQ_RUNNING; }),
                     active.end());
        if (worked) stats.steps += 1;
        stats.sample_ms += ms;
        f.valid = false;
        *host_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        return MC_OK;
    }

    // Launches one step over the requests in active (nothing waits for it):
    // the upload, admissions, sampling launches, merge and decision, bin
    // adjustment and the read-back into this step's buffer; next describes it.
    mc_status launch_step(InFlight &next) {
        mc_status st = MC_OK;
        // launch groups: the kernel, then whether the integral's LDS footprint
        // still allows the kernel's register-limited workgroups per CU
        for (Request *r : active) {
            const int kern = kernel_of(*r);
            const size_t lds = lds_bytes_of(r->prob.dim, r->prob.nbins, r->launched < r->prob.ita, kernel_fp32(kern));
            int o = 0;
            st = occupancy(kern, kBatchBlock, lds, &o);
            if (st != MC_OK) return st;
            r->group = 2 * kern + (o < occ_full[kern] ? 1 : 0);
        }
        std::stable_sort(active.begin(), active.end(),
                         [](const Request *x, const Request *y) { return x->group < y->group; });
        const int n = (int)active.size();

        char *step_base = ws + arena_bytes;
        // per integral: the launch group's LDS, the group ranges, the axes to adjust
        int n_axes = 0, max_nb = 2;
        size_t lds[kGroups] = {};
        int first[kGroups + 1] = {};
        for (int i = 0; i < n; ++i) {
            const Request *r = active[i];
            const bool adjust = r->launched < r->prob.ita;
            if (adjust) {
                n_axes += r->prob.one_d ? 1 : r->prob.dim;  // m-Cubes1D: axis 0, then copied
                max_nb = std::max(max_nb, r->prob.nbins);
            }
            const int grp = r->group;
            lds[grp] = std::max(lds[grp], lds_bytes_of(r->prob.dim, r->prob.nbins, adjust, kernel_fp32(grp / 2)));
            first[grp + 1] = i + 1;
        }
        for (int grp = 1; grp <= kGroups; ++grp) first[grp] = std::max(first[grp], first[grp - 1]);
        // work split per group, each group one launch filling the GPU; its
        // segments go to the queue largest first
        std::vector<plan::Piece> segs;
        std::vector<int32_t> item_first(n, -1), order;
        std::vector<int64_t> cubes_of(n);
        std::vector<double> costs(n);
        for (int i = 0; i < n; ++i) {
            cubes_of[i] = active[i]->m;
            costs[i] = active[i]->cost;
        }
        int G[kGroups] = {}, T[kGroups] = {}, seg_lo[kGroups + 1] = {};
        for (int grp = 0; grp < kGroups; ++grp) {
            seg_lo[grp] = (int)segs.size();
            if (first[grp] == first[grp + 1]) continue;
            const int kern = grp / 2;
            int per_cu = 0;
            st = occupancy(kern, kBatchBlock, lds[grp], &per_cu);
            if (st != MC_OK) return st;
            T[grp] = kBatchBlock;
            if (grp % 2 == 1) {  // LDS-limited: larger workgroups keep more waves per CU
                int wide = 0;
                if (occupancy(kern, kBatchMaxBlock, lds[grp], &wide) == MC_OK &&
                    wide * kBatchMaxBlock > per_cu * kBatchBlock) {
                    per_cu = wide;
                    T[grp] = kBatchMaxBlock;
                }
            }
            G[grp] = per_cu * cus;
            int64_t cubes = 0;
            for (int i = first[grp]; i < first[grp + 1]; ++i) cubes += active[i]->m;
            const int64_t parts =
                std::max<int64_t>(1, std::min<int64_t>((int64_t)kSegsPerWg * G[grp], cubes / kMinSegCubes));
            plan::split_work(cubes_of.data(), costs.data(), first[grp], first[grp + 1], parts, segs,
                             item_first.data());
            plan::largest_first(segs, costs.data(), seg_lo[grp], (int)segs.size(), order);
        }
        seg_lo[kGroups] = (int)segs.size();

        // this step's tables, packed for the counts it actually has (within
        // the worst case that admission reserved)
        const StepCounts counts{n, (int64_t)segs.size(), n_axes, (int64_t)admitted.size()};
        const StepLayout L = step_layout(counts);
        if (L.total > step_cap || (int64_t)segs.size() > worst_counts(need, gcap).nseg)
            return MC_EWORKSPACE;  // cannot happen: admission keeps the worst case within the area
        HIP_TRY(staging[buf].reserve(L.upload_end));
        char *up = staging[buf].data();
        std::memset(up + L.flags, 0, L.axis_item - L.flags);  // flags and queue counters start at 0
        BatchItem *items = reinterpret_cast<BatchItem *>(up + L.items);
        int32_t *item_first_h = reinterpret_cast<int32_t *>(up + L.item_first);
        double **next_grid = reinterpret_cast<double **>(up + L.next_grid);
        int32_t *axis_item = reinterpret_cast<int32_t *>(up + L.axis_item);
        int ax = 0;
        for (int i = 0; i < n; ++i) {
            Request *r = active[i];
            const bool adjust = r->launched < r->prob.ita;
            BatchItem &b = items[i];
            std::memset(&b, 0, sizeof(b));
            double *grid = reinterpret_cast<double *>(ws + r->off_grid[r->cur]);
            sample_args(&r->prob, r->g, r->m, r->p, (uint32_t)r->launched, adjust, ws + r->off_consts,
                        grid, r->tables.empty() ? nullptr : ws + r->off_tables, &b.a);
            b.grid = grid;
            b.out = reinterpret_cast<double *>(ws + r->off_out);
            b.iters = reinterpret_cast<double *>(ws + r->off_iters);
            b.state = reinterpret_cast<uint32_t *>(ws + r->off_state);
            b.alpha = r->prob.alpha;
            b.tau_rel = r->prob.tau_rel;
            b.chi2_max = r->prob.chi2_max;
            b.itmax = r->prob.itmax;
            b.refine = adjust ? 1 : 0;
            next_grid[i] = reinterpret_cast<double *>(ws + r->off_grid[1 - r->cur]);
            if (adjust) {
                const int axes = r->prob.one_d ? 1 : r->prob.dim;
                for (int j = 0; j < axes; ++j) {
                    axis_item[2 * ax] = i;
                    axis_item[2 * ax + 1] = j;
                    ++ax;
                }
            }
            item_first_h[i] = item_first[i];
        }
        item_first_h[n] = (int32_t)segs.size();
        BatchSegment *segs_h = reinterpret_cast<BatchSegment *>(up + L.segs);
        for (size_t k = 0; k < segs.size(); ++k)
            segs_h[k] = BatchSegment{segs[k].item, 0, segs[k].t0, segs[k].t1};
        std::memcpy(up + L.order, order.data(), sizeof(int32_t) * order.size());
        // admissions of this step: constants into the upload, records for admit_kernel
        AdmitRecord *recs = reinterpret_cast<AdmitRecord *>(up + L.admit_recs);
        for (size_t k = 0; k < admitted.size(); ++k) {
            Request *r = admitted[k];
            const size_t src = L.admit_data + k * kConstsMax;
            std::memcpy(up + src, r->consts_img.data(), r->consts_img.size());
            AdmitRecord &rec = recs[k];
            std::memset(&rec, 0, sizeof(rec));
            rec.consts = ws + r->off_consts;
            rec.grid = reinterpret_cast<double *>(ws + r->off_grid[0]);
            rec.out = reinterpret_cast<double *>(ws + r->off_out);
            rec.state = reinterpret_cast<uint32_t *>(ws + r->off_state);
            rec.src = (int64_t)src;
            rec.const_words = (int32_t)(r->consts_img.size() / 4);
            rec.dim = r->prob.dim;
            rec.nb = r->prob.nbins;
            std::vector<char>().swap(r->consts_img);
        }
        HIP_TRY(hipMemcpyAsync(step_base, up, L.upload_end, hipMemcpyHostToDevice, stream));
        HIP_TRY(launch_admit(reinterpret_cast<const AdmitRecord *>(step_base + L.admit_recs),
                             (int)admitted.size(), step_base, stream));
        admitted.clear();

        BatchArgs A{};
        A.items = reinterpret_cast<const BatchItem *>(step_base + L.items);
        A.segs = reinterpret_cast<const BatchSegment *>(step_base + L.segs);
        A.item_first = reinterpret_cast<const int32_t *>(step_base + L.item_first);
        A.seg_tot = reinterpret_cast<double *>(step_base + L.seg_tot);
        A.order = reinterpret_cast<const int32_t *>(step_base + L.order);
        A.flags = reinterpret_cast<uint32_t *>(step_base + L.flags);
        A.res = reinterpret_cast<double *>(step_base + L.res);
        A.n_items = n;
        HIP_TRY(hipEventRecord(ev[buf][0], stream));
        for (int grp = 0; grp < kGroups; ++grp) {
            if (!G[grp]) continue;
            A.queue = reinterpret_cast<uint32_t *>(step_base + L.queue) + grp;
            A.lo = seg_lo[grp];
            A.hi = seg_lo[grp + 1];
            HIP_TRY(launch_batch(kernel_fp32(grp / 2), kernel_tables(grp / 2), G[grp], T[grp], lds[grp], stream,
                                 A));
        }
        HIP_TRY(hipEventRecord(ev[buf][1], stream));
        HIP_TRY(launch_batch_finalize(A, stream));
        HIP_TRY(allow_lds(batch_refine_symbol(), sizeof(double) * max_nb));
        HIP_TRY(launch_batch_refine(A.items, reinterpret_cast<const int32_t *>(step_base + L.axis_item),
                                    reinterpret_cast<double *const *>(step_base + L.next_grid), n_axes,
                                    max_nb, stream));
        HIP_TRY(res_buf[buf].reserve(sizeof(double) * kResStride * (size_t)n));
        HIP_TRY(hipMemcpyAsync(res_buf[buf].data(), A.res, sizeof(double) * kResStride * n,
                               hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipEventRecord(ev[buf][2], stream));
        // the iterations launched, the grids the device adjusts into
        next.valid = true;
        next.buf = buf;
        next.ids.resize(n);
        for (int i = 0; i < n; ++i) {
            Request *r = active[i];
            next.ids[i] = r->id;
            if (r->launched < r->prob.ita) r->cur = 1 - r->cur;
            r->launched += 1;
        }
        stats.max_active = std::max<int32_t>(stats.max_active, n);
        return MC_OK;
    }
};

// ====================================================================== C ABI

extern "C" {

mc_status mc_server_create(void *d_ws, size_t ws_bytes, size_t arena_bytes, int32_t max_active,
                           void *stream, mc_server **out) {
    if (!out || !d_ws || max_active < 1 || arena_bytes >= ws_bytes) return MC_EINVAL;
    auto s = std::make_unique<mc_server>();
    s->ws = static_cast<char *>(d_ws);
    s->ws_bytes = ws_bytes;
    s->arena_bytes = align_up(arena_bytes);
    if (s->arena_bytes >= ws_bytes) return MC_EINVAL;
    s->step_cap = ws_bytes - s->arena_bytes;
    s->max_active = max_active;
    s->stream = static_cast<hipStream_t>(stream);
    mc_status st = s->init();
    if (st != MC_OK) return st;
    *out = s.release();
    return MC_OK;
}

mc_status mc_server_set_step_budget(mc_server *srv, int64_t samples, int32_t max_skip) {
    if (!srv || samples < 0 || max_skip < 0) return MC_EINVAL;
    srv->step_budget = samples;
    srv->max_skip = max_skip;
    return MC_OK;
}

mc_status mc_server_submit(mc_server *srv, const mc_problem *prob, int64_t *id) {
    if (!srv || !id) return MC_EINVAL;
    return srv->submit(prob, id);
}

mc_status mc_server_step(mc_server *srv, int32_t *active, int32_t *queued, int32_t *finished) {
    if (!srv) return MC_EINVAL;
    int32_t fin = 0;
    mc_status st = srv->step(&fin);
    if (st != MC_OK) return st;
    if (active) *active = (int32_t)srv->active.size();
    if (queued) *queued = (int32_t)srv->queue.size();
    if (finished) *finished = fin;
    return MC_OK;
}

mc_status mc_server_poll(mc_server *srv, int64_t id, int32_t *state, mc_result *out,
                         mc_status *status) {
    if (!srv || !state) return MC_EINVAL;
    auto it = srv->all.find(id);
    if (it == srv->all.end()) return MC_EINVAL;
    const Request &r = *it->second;
    *state = r.state;
    if (status) *status = r.status;
    if (out && r.state == MC_REQ_DONE) *out = r.result;
    return MC_OK;
}

mc_status mc_server_finished(mc_server *srv, int64_t *ids, int32_t cap, int32_t *n) {
    if (!srv || !n || (cap > 0 && !ids)) return MC_EINVAL;
    const int32_t k = std::min<int32_t>(cap, (int32_t)srv->last_finished.size());
    for (int32_t i = 0; i < k; ++i) ids[i] = srv->last_finished[i];
    *n = k;
    return MC_OK;
}

mc_status mc_server_release(mc_server *srv, int64_t id) {
    if (!srv) return MC_EINVAL;
    auto it = srv->all.find(id);
    if (it == srv->all.end()) return MC_EINVAL;
    if (it->second->state != MC_REQ_DONE && it->second->state != MC_REQ_FAILED) return MC_EINVAL;
    srv->all.erase(it);
    return MC_OK;
}

mc_status mc_server_stats(mc_server *srv, mc_batch_stats *stats) {
    if (!srv || !stats) return MC_EINVAL;
    *stats = srv->stats;
    return MC_OK;
}

mc_status mc_server_destroy(mc_server *srv) {
    if (!srv) return MC_EINVAL;
    if (srv->stream) (void)hipStreamSynchronize(srv->stream);
    delete srv;
    return MC_OK;
}

mc_status mc_batch_workspace_bytes(const mc_problem *probs, int32_t n, size_t *bytes) {
    if (!probs || n < 1 || !bytes) return MC_EINVAL;
    size_t arena = 0;
    StepNeed need;
    for (int32_t i = 0; i < n; ++i) {
        mc_status st = validate_batch(&probs[i]);
        if (st != MC_OK) return st;
        Request r;
        r.prob = probs[i];
        size_t a, b, c, e, f;
        arena += block_layout(r, &a, &b, &c, &e, &f);
        need.add(r);
    }
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    *bytes = align_up(arena) + step_layout(worst_counts(need, cus * kMaxWgsPerCu)).total;
    return MC_OK;
}

mc_status mc_batch_integrate(const mc_problem *probs, int32_t n, void *d_ws, size_t ws_bytes,
                             void *stream, mc_result *results, mc_status *statuses,
                             mc_batch_stats *stats) {
    if (!probs || n < 1 || !results || !statuses) return MC_EINVAL;
    size_t need = 0;
    mc_status st = mc_batch_workspace_bytes(probs, n, &need);
    if (st != MC_OK) return st;
    if (!d_ws || ws_bytes < need) return MC_EWORKSPACE;
    size_t arena = 0;
    for (int32_t i = 0; i < n; ++i) {
        Request r;
        r.prob = probs[i];
        size_t a, b, c, e, f;
        arena += block_layout(r, &a, &b, &c, &e, &f);
    }
    mc_server *srv = nullptr;
    st = mc_server_create(d_ws, ws_bytes, arena, n, stream, &srv);
    if (st != MC_OK) return st;
    std::unique_ptr<mc_server> hold(srv);
    std::vector<int64_t> ids(n);
    for (int32_t i = 0; i < n; ++i) {
        st = srv->submit(&probs[i], &ids[i]);
        if (st != MC_OK) return st;
    }
    while (!srv->active.empty() || !srv->queue.empty() || srv->inflight.valid) {
        int32_t fin = 0;
        st = srv->step(&fin);
        if (st != MC_OK) return st;
        if (srv->active.empty() && !srv->queue.empty() && !srv->inflight.valid)
            return MC_EWORKSPACE;  // cannot admit
    }
    for (int32_t i = 0; i < n; ++i) {
        const Request &r = *srv->all[ids[i]];
        statuses[i] = r.status;
        if (r.state == MC_REQ_DONE) results[i] = r.result;
    }
    if (stats) *stats = srv->stats;
    return MC_OK;
}

}  // extern "C"
