// Batched m-Cubes and the serving loop.
//
// An Engine owns a caller-provided device workspace split into an arena and
// a step area.  The arena holds each admitted integral's persistent device
// state (per-axis constants, tables, two grid buffers, and the latest pass's
// [I, var, flag, 0, histogram]); a first-fit allocator hands it out, and an
// integral is admitted only when its block and its share of the step area
// fit ("admission by device memory").  Every step:
//   1. admits queued integrals that fit (constants, tables and the initial
//      grid are uploaded once);
//   2. splits the active integrals' sub-cubes into contiguous segments of
//      roughly equal work, one run of segments per workgroup, and uploads the
//      step's small tables (items, segments, workgroup and item indices);
//   3. runs one persistent batched sampling launch per precision present,
//      the in-order merge of each integral's segments, and the bin adjustment
//      of the integrals still adjusting — on the device, so grids and
//      histograms stay resident;
//   4. reads back 4 doubles per integral and runs Weighted-Estimates and
//      Check-Convergence on the host; finished integrals release their block.
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <unordered_map>

#include "host.hpp"
#include "internal.hpp"
#include "mcubes.h"

using namespace mcubes;
using namespace mcubes::host;

namespace {

// First-fit allocator over [0, cap) with coalescing of neighbours.
class Arena {
  public:
    explicit Arena(size_t cap) {
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = align_up(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes, next = it->first + bytes;
            free_.erase(it);
            if (rest) free_[next] = rest;
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = align_up(bytes);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }

  private:
    std::map<size_t, size_t> free_;
};

struct Request {
    int64_t id = 0;
    mc_problem prob{};
    std::vector<double> params, tables, lo, hi;
    int64_t g = 0, m = 0, p = 0;
    int32_t state = MC_REQ_QUEUED;
    mc_status status = MC_OK;
    size_t block_off = 0, block_bytes = 0;
    size_t off_consts = 0, off_tables = 0, off_grid[2] = {0, 0}, off_out = 0;  // in the workspace
    int cur = 0;     // current grid buffer
    int it = 0;      // iterations done
    std::vector<double> Is, Vs;
    double est[3] = {0.0, 0.0, NAN};
    int converged = 0;
    mc_result result{};
    double cost = 0;  // relative work per sub-cube (for the work split)
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
    return (double)p * (51.0 * blocks + 25.0 * d + f + 10.0) + 20.0 + 5.0 * d;
}

// Bytes of an integral's persistent block and the offsets inside it.
size_t block_layout(const Request &r, size_t *o_consts, size_t *o_tables, size_t *o_grid0,
                    size_t *o_grid1, size_t *o_out) {
    const int d = r.prob.dim, nb = r.prob.nbins;
    const size_t real = fp32_of(r) ? sizeof(float) : sizeof(double);
    size_t off = 0;
    *o_consts = off;
    off = align_up(off + real * kConstStride * d);
    *o_tables = off;
    if (r.prob.integrand == MC_F_GAUSS_TABLES) off = align_up(off + real * 2 * kTableN * kTableN);
    *o_grid0 = off;
    off = align_up(off + sizeof(double) * d * (nb + 1));
    *o_grid1 = off;
    off = align_up(off + sizeof(double) * d * (nb + 1));
    *o_out = off;
    off = align_up(off + sizeof(double) * (4 + (size_t)d * nb));
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
    size_t items, item_first, flags, wg_first, segs, axis_item, next_grid, upload_end;
    size_t res, seg_tot, seg_hist, total;
};

StepLayout step_layout(const StepNeed &s, int gcap) {
    StepLayout L{};
    const int64_t nseg = s.n + 2 * (int64_t)gcap;
    size_t off = 0;
    L.items = off;
    off = align_up(off + sizeof(BatchItem) * s.n);
    L.item_first = off;
    off = align_up(off + sizeof(int32_t) * (s.n + 1));
    L.flags = off;
    off = align_up(off + sizeof(uint32_t) * s.n);
    L.wg_first = off;
    off = align_up(off + sizeof(int32_t) * 2 * (gcap + 1));
    L.segs = off;
    off = align_up(off + sizeof(BatchSegment) * nseg);
    L.axis_item = off;
    off = align_up(off + sizeof(int32_t) * 2 * s.sum_d);
    L.next_grid = off;
    off = align_up(off + sizeof(double *) * s.n);
    L.upload_end = off;
    L.res = off;
    off = align_up(off + sizeof(double) * 4 * s.n);
    L.seg_tot = off;
    off = align_up(off + sizeof(double) * 4 * nseg);
    L.seg_hist = off;
    off = align_up(off + sizeof(double) * (s.sum_dnb + 2 * (int64_t)gcap * s.max_dnb));
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

struct mc_server {
    char *ws = nullptr;
    size_t ws_bytes = 0, arena_bytes = 0, step_cap = 0;
    int32_t max_active = 0;
    hipStream_t stream = nullptr;
    int cus = 0, gcap = 0;
    std::unique_ptr<Arena> arena;
    int64_t next_id = 1;
    std::unordered_map<int64_t, std::unique_ptr<Request>> all;
    std::deque<Request *> queue;
    std::vector<Request *> active;
    std::vector<int64_t> last_finished;  // ids finished in the last step
    StepNeed need;  // of the active set
    std::vector<char> staging;
    std::vector<double> res;
    hipEvent_t ev[2] = {nullptr, nullptr};
    mc_batch_stats stats{};

    ~mc_server() {
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }

    mc_status init() {
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        gcap = cus * 4;  // 256-thread workgroups: at most 4 per CU at the kernels' register use
        for (auto &e : ev) HIP_TRY(hipEventCreate(&e));
        arena = std::make_unique<Arena>(arena_bytes);
        return MC_OK;
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
        if (r->block_bytes > arena_bytes || step_layout(one, gcap).total > step_cap) return MC_EWORKSPACE;
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
        while (!queue.empty() && (int32_t)active.size() < max_active) {
            Request *r = queue.front();
            StepNeed grown = need;
            grown.add(*r);
            if (step_layout(grown, gcap).total > step_cap) break;
            size_t off;
            if (!arena->alloc(r->block_bytes, &off)) break;
            size_t oc, ot, og0, og1, oo;
            block_layout(*r, &oc, &ot, &og0, &og1, &oo);
            r->block_off = off;
            r->off_consts = off + oc;
            r->off_tables = off + ot;
            r->off_grid[0] = off + og0;
            r->off_grid[1] = off + og1;
            r->off_out = off + oo;
            const int d = r->prob.dim, nb = r->prob.nbins;
            // constants, tables and the initial grid; host copies live in the Request
            const std::vector<double> c = axis_constants(&r->prob);
            std::vector<double> grid((size_t)d * (nb + 1));
            init_grid(d, nb, grid.data());
            if (fp32_of(*r)) {
                const std::vector<float> c32(c.begin(), c.end());
                HIP_TRY(hipMemcpyAsync(ws + r->off_consts, c32.data(), sizeof(float) * c32.size(),
                                       hipMemcpyHostToDevice, stream));
                if (!r->tables.empty()) {
                    const std::vector<float> t32(r->tables.begin(), r->tables.end());
                    HIP_TRY(hipMemcpyAsync(ws + r->off_tables, t32.data(), sizeof(float) * t32.size(),
                                           hipMemcpyHostToDevice, stream));
                    HIP_TRY(hipStreamSynchronize(stream));
                }
                HIP_TRY(hipStreamSynchronize(stream));
            } else {
                HIP_TRY(hipMemcpyAsync(ws + r->off_consts, c.data(), sizeof(double) * c.size(),
                                       hipMemcpyHostToDevice, stream));
                if (!r->tables.empty())
                    HIP_TRY(hipMemcpyAsync(ws + r->off_tables, r->tables.data(),
                                           sizeof(double) * r->tables.size(), hipMemcpyHostToDevice,
                                           stream));
            }
            HIP_TRY(hipMemcpyAsync(ws + r->off_grid[0], grid.data(), sizeof(double) * grid.size(),
                                   hipMemcpyHostToDevice, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            r->cur = 0;
            r->state = MC_REQ_RUNNING;
            queue.pop_front();
            active.push_back(r);
            need = grown;
        }
        return MC_OK;
    }

    // Splits the items [first, last) of one precision into segments of
    // roughly equal work over G workgroups; appends to segs and wg_first.
    void split(const std::vector<Request *> &items, int first, int last, int G,
               std::vector<BatchSegment> &segs, std::vector<int32_t> &wg_first,
               std::vector<int32_t> &item_first, int64_t &hist_cursor) {
        double W = 0.0;
        std::vector<double> start(last - first + 1);
        for (int i = first; i < last; ++i) {
            start[i - first] = W;
            W += (double)items[i]->m * items[i]->cost;
        }
        start[last - first] = W;
        auto bound = [&](int i, int k) -> int64_t {
            const double x = W * (double)k / (double)G;
            const double c = std::llround((x - start[i - first]) / items[i]->cost);
            return std::min<int64_t>(std::max<int64_t>((int64_t)c, 0), items[i]->m);
        };
        int i0 = first;
        for (int k = 0; k < G; ++k) {
            wg_first.push_back((int32_t)segs.size());
            const double x0 = W * (double)k / (double)G, x1 = W * (double)(k + 1) / (double)G;
            while (i0 < last && start[i0 + 1 - first] <= x0 && bound(i0, k) >= items[i0]->m) ++i0;
            for (int i = i0; i < last && start[i - first] <= x1; ++i) {
                const int64_t t0 = bound(i, k), t1 = bound(i, k + 1);
                if (t1 <= t0) continue;
                if (item_first[i] < 0) item_first[i] = (int32_t)segs.size();
                BatchSegment sg{};
                sg.item = i;
                sg.t0 = t0;
                sg.t1 = t1;
                if (items[i]->it < items[i]->prob.ita) {
                    sg.hist_off = hist_cursor;
                    hist_cursor += dnb(*items[i]);
                }
                segs.push_back(sg);
            }
        }
    }

    mc_status step(int32_t *n_finished) {
        *n_finished = 0;
        last_finished.clear();
        mc_status st = admit();
        if (st != MC_OK) return st;
        if (active.empty()) return MC_OK;
        const auto t_start = std::chrono::steady_clock::now();
        // FP64 integrals first, then FP32: one launch per precision present
        std::stable_partition(active.begin(), active.end(), [](Request *r) { return !fp32_of(*r); });
        const int n = (int)active.size();
        int n64 = 0;
        while (n64 < n && !fp32_of(*active[n64])) ++n64;

        char *step_base = ws + arena_bytes;
        const StepLayout L = step_layout(need, gcap);
        staging.assign(L.upload_end, 0);
        BatchItem *items = reinterpret_cast<BatchItem *>(staging.data() + L.items);
        int32_t *item_first_h = reinterpret_cast<int32_t *>(staging.data() + L.item_first);
        double **next_grid = reinterpret_cast<double **>(staging.data() + L.next_grid);
        int32_t *axis_item = reinterpret_cast<int32_t *>(staging.data() + L.axis_item);
        int n_axes = 0, max_nb = 2;
        size_t lds[2] = {0, 0};
        for (int i = 0; i < n; ++i) {
            Request *r = active[i];
            const bool adjust = r->it < r->prob.ita;
            BatchItem &b = items[i];
            double *grid = reinterpret_cast<double *>(ws + r->off_grid[r->cur]);
            sample_args(&r->prob, r->g, r->m, r->p, (uint32_t)r->it, adjust, ws + r->off_consts, grid,
                        r->tables.empty() ? nullptr : ws + r->off_tables, &b.a);
            b.grid = grid;
            b.out = reinterpret_cast<double *>(ws + r->off_out);
            b.alpha = r->prob.alpha;
            b.refine = adjust ? 1 : 0;
            next_grid[i] = reinterpret_cast<double *>(ws + r->off_grid[1 - r->cur]);
            if (adjust) {
                const int axes = r->prob.one_d ? 1 : r->prob.dim;  // m-Cubes1D: axis 0, then copied
                for (int j = 0; j < axes; ++j) {
                    axis_item[2 * n_axes] = i;
                    axis_item[2 * n_axes + 1] = j;
                    ++n_axes;
                }
                max_nb = std::max(max_nb, r->prob.nbins);
            }
            const int grp = fp32_of(*r) ? 1 : 0;
            lds[grp] = std::max(lds[grp], lds_bytes_of(r->prob.dim, r->prob.nbins, adjust, grp == 1));
        }
        // work split per precision group
        std::vector<BatchSegment> segs;
        std::vector<int32_t> wg_first, item_first(n, -1);
        int64_t hist_cursor = 0;
        int G[2] = {0, 0};
        for (int grp = 0; grp < 2; ++grp) {
            const int first = grp == 0 ? 0 : n64, last = grp == 0 ? n64 : n;
            if (first == last) continue;
            const void *fn = batch_kernel(grp == 1);
            HIP_TRY(allow_lds(fn, lds[grp]));
            int per_cu = 0;
            HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBatchBlock, lds[grp]));
            if (per_cu < 1) return MC_EINVAL;
            G[grp] = std::min(per_cu * cus, gcap);
            split(active, first, last, G[grp], segs, wg_first, item_first, hist_cursor);
            wg_first.push_back((int32_t)segs.size());
        }
        for (int i = 0; i < n; ++i) item_first_h[i] = item_first[i];
        item_first_h[n] = (int32_t)segs.size();
        std::memcpy(staging.data() + L.segs, segs.data(), sizeof(BatchSegment) * segs.size());
        std::memcpy(staging.data() + L.wg_first, wg_first.data(), sizeof(int32_t) * wg_first.size());
        HIP_TRY(hipMemcpyAsync(step_base, staging.data(), L.upload_end, hipMemcpyHostToDevice, stream));

        BatchArgs A{};
        A.items = reinterpret_cast<const BatchItem *>(step_base + L.items);
        A.segs = reinterpret_cast<const BatchSegment *>(step_base + L.segs);
        A.item_first = reinterpret_cast<const int32_t *>(step_base + L.item_first);
        A.seg_tot = reinterpret_cast<double *>(step_base + L.seg_tot);
        A.seg_hist = reinterpret_cast<double *>(step_base + L.seg_hist);
        A.flags = reinterpret_cast<uint32_t *>(step_base + L.flags);
        A.res = reinterpret_cast<double *>(step_base + L.res);
        A.n_items = n;
        const int32_t *wg_dev = reinterpret_cast<const int32_t *>(step_base + L.wg_first);
        HIP_TRY(hipEventRecord(ev[0], stream));
        int wg_base = 0;
        for (int grp = 0; grp < 2; ++grp) {
            if (!G[grp]) continue;
            A.wg_first = wg_dev + wg_base;
            HIP_TRY(launch_batch(grp == 1, G[grp], kBatchBlock, lds[grp], stream, A));
            wg_base += G[grp] + 1;
        }
        HIP_TRY(hipEventRecord(ev[1], stream));
        HIP_TRY(launch_batch_finalize(A, stream));
        HIP_TRY(allow_lds(batch_refine_symbol(), sizeof(double) * max_nb));
        HIP_TRY(launch_batch_refine(A.items, reinterpret_cast<const int32_t *>(step_base + L.axis_item),
                                    reinterpret_cast<double *const *>(step_base + L.next_grid), n_axes,
                                    max_nb, stream));
        res.resize(4 * (size_t)n);
        HIP_TRY(hipMemcpyAsync(res.data(), A.res, sizeof(double) * 4 * n, hipMemcpyDeviceToHost, stream));
        HIP_TRY(hipStreamSynchronize(stream));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, ev[0], ev[1]));

        // host steps of Alg. 2 per integral
        std::vector<Request *> still;
        still.reserve(n);
        for (int i = 0; i < n; ++i) {
            Request *r = active[i];
            const bool adjust = r->it < r->prob.ita;
            stats.calls += r->m * r->p;
            if (res[4 * i + 2] != 0.0) {
                finish(r, MC_REQ_FAILED, MC_ENONFINITE);
                ++*n_finished;
                continue;
            }
            r->Is.push_back(res[4 * i]);
            r->Vs.push_back(res[4 * i + 1]);
            r->it += 1;
            weighted(r->it, r->Is.data(), r->Vs.data(), r->est);
            if (adjust) r->cur = 1 - r->cur;
            const bool conv = r->it >= 2 && r->prob.tau_rel > 0.0 &&
                              r->est[1] <= r->prob.tau_rel * std::fabs(r->est[0]);
            if (conv || r->it >= r->prob.itmax) {
                r->converged = conv ? 1 : 0;
                finish(r, MC_REQ_DONE, MC_OK);
                ++*n_finished;
            } else {
                still.push_back(r);
            }
        }
        active.swap(still);
        need = StepNeed{};
        for (Request *r : active) need.add(*r);
        stats.steps += 1;
        stats.max_active = std::max<int32_t>(stats.max_active, n);
        stats.sample_ms += ms;
        stats.step_ms += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
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
    *bytes = align_up(arena) + step_layout(need, cus * 4).total;
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
    while (!srv->active.empty() || !srv->queue.empty()) {
        int32_t fin = 0;
        st = srv->step(&fin);
        if (st != MC_OK) return st;
        if (srv->active.empty() && !srv->queue.empty()) return MC_EWORKSPACE;  // cannot admit
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
