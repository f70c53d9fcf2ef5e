// Host-side planning of a batched step, free of any device call, so that the
// CPU test suite can compile and check it on its own:
//   * Arena: first-fit allocation of the integrals' persistent blocks in the
//     device workspace (offsets only), with coalescing of free neighbours;
//   * split_work: cutting a group of integrals' sub-cubes into segments of
//     bounded work;
//   * largest_first: the order in which a launch's workgroups take them;
//   * expected_iterations, select_for_step: which requests a serving step
//     runs under a step budget.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>
#include <iterator>
#include <map>
#include <numeric>
#include <vector>

namespace mcubes {
namespace plan {

constexpr size_t kArenaAlign = 256;

inline size_t arena_round(size_t v) { return (v + kArenaAlign - 1) / kArenaAlign * kArenaAlign; }

// First-fit allocator over [0, cap) in kArenaAlign units; freed ranges merge
// with free neighbours.
class Arena {
  public:
    explicit Arena(size_t cap) {
        cap = cap / kArenaAlign * kArenaAlign;
        if (cap) free_[0] = cap;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = arena_round(bytes);
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
        bytes = arena_round(bytes);
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
    size_t free_bytes() const {
        size_t s = 0;
        for (const auto &kv : free_) s += kv.second;
        return s;
    }
    size_t free_ranges() const { return free_.size(); }

  private:
    std::map<size_t, size_t> free_;  // offset -> length
};

// A contiguous range [t0, t1) of integral `item`'s sub-cubes.
struct Piece {
    int32_t item;
    int64_t t0, t1;
};

// Cuts the work of integrals first..last-1 (m[i] sub-cubes of cost[i] each)
// into `parts` equal shares laid end to end, and every integral into the
// pieces the cuts leave (an integral smaller than a share stays whole).
// Appends the pieces in integral order, each integral's in sub-cube order;
// first_piece[i] is set to the index of integral i's first piece.  At most
// (last - first) + parts + 1 pieces are appended.
inline void split_work(const int64_t *m, const double *cost, int first, int last, int64_t parts,
                       std::vector<Piece> &out, int32_t *first_piece) {
    double W = 0.0;
    std::vector<double> start(last - first + 1);
    for (int i = first; i < last; ++i) {
        start[i - first] = W;
        W += (double)m[i] * cost[i];
    }
    start[last - first] = W;
    const double share = W / (double)std::max<int64_t>(parts, 1);
    for (int i = first; i < last; ++i) {
        first_piece[i] = (int32_t)out.size();
        const double a = start[i - first], b = start[i + 1 - first];
        int64_t t0 = 0;
        if (share > 0.0) {
            for (double x = std::ceil(a / share) * share; x < b; x += share) {
                const int64_t t = std::min<int64_t>((int64_t)std::llround((x - a) / cost[i]), m[i]);
                if (t <= t0) continue;
                out.push_back(Piece{i, t0, t});
                t0 = t;
            }
        }
        if (t0 < m[i]) out.push_back(Piece{i, t0, m[i]});
    }
}

// Indices lo..hi-1 of `pieces`, appended to order from the largest work to
// the smallest, by a counting sort on the work quantised to 1/kOrderBuckets
// of the largest piece's (equal buckets keep index order): linear in the
// number of pieces, and within one bucket of the exact order, which is all
// that taking the large pieces first needs.
constexpr int kOrderBuckets = 256;

inline void largest_first(const std::vector<Piece> &pieces, const double *cost, int lo, int hi,
                          std::vector<int32_t> &order) {
    if (hi <= lo) return;
    std::vector<double> work(hi - lo);
    double top = 0.0;
    for (int k = lo; k < hi; ++k) {
        work[k - lo] = (double)(pieces[k].t1 - pieces[k].t0) * cost[pieces[k].item];
        top = std::max(top, work[k - lo]);
    }
    std::vector<int32_t> bucket(hi - lo);
    std::vector<int64_t> count(kOrderBuckets + 1, 0);
    for (int k = 0; k < hi - lo; ++k) {
        const int b = top > 0.0 ? std::min(kOrderBuckets - 1, (int)(work[k] / top * kOrderBuckets)) : 0;
        bucket[k] = kOrderBuckets - 1 - b;  // largest first
        ++count[bucket[k] + 1];
    }
    for (int b = 0; b < kOrderBuckets; ++b) count[b + 1] += count[b];
    const size_t o0 = order.size();
    order.resize(o0 + (hi - lo));
    for (int k = 0; k < hi - lo; ++k) order[o0 + count[bucket[k]]++] = lo + k;
}

// Iterations a request of the serving loop is still expected to need, after
// `it` of at most itmax, with target relative error tau and weighted estimate
// and error so far.  The error of the weighted average falls as 1/sqrt(k) for
// a settled grid, so after k >= 2 iterations with relative error e the target
// needs about k (e/tau)^2 in all.  Before two iterations (no usable error
// yet) a target-driven request is taken to need only the two the convergence
// test requires, so that new requests get their first iterations soon;
// without a target (tau = 0) it runs to itmax.  At least 1, at most what is
// left.
inline double expected_iterations(int it, int itmax, double tau, double estimate, double error) {
    const int left = itmax - it;
    if (left <= 0) return 1.0;
    if (tau <= 0.0) return left;
    if (it < 2 || !(error > 0.0) || !std::isfinite(error) || !(std::fabs(estimate) > 0.0))
        return std::min(std::max(2 - it, 1), left);
    const double ratio = error / (tau * std::fabs(estimate));
    const double need = std::ceil((double)it * ratio * ratio) - it;
    return std::min<double>(std::max(need, 1.0), left);
}

// One active request as the step budget sees it.
struct Candidate {
    double work;      // estimated remaining work (any unit common to all)
    int64_t samples;  // samples of its next iteration
    int32_t skipped;  // steps it has been left out in a row
    int64_t id;       // arrival order
};

// Which candidates run in this step under a budget of `budget` samples: every
// one left out max_skip steps in a row, and then, by least remaining work
// (ties: arrival order), each that keeps the others' samples within the
// budget (the overdue ones do not count against it, so they delay no one);
// if that leaves the step empty, the first by that order.  run[i] is 1 for a
// candidate that runs.
inline std::vector<char> select_for_step(const std::vector<Candidate> &c, int64_t budget,
                                         int32_t max_skip) {
    std::vector<int> idx(c.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int x, int y) {
        if (c[x].work != c[y].work) return c[x].work < c[y].work;
        return c[x].id < c[y].id;
    });
    std::vector<char> run(c.size(), 0);
    int64_t used = 0;
    bool any = false;
    for (int i : idx) {
        if (c[i].skipped >= max_skip) {
            run[i] = 1;
            any = true;
        } else if (used + c[i].samples <= budget) {
            run[i] = 1;
            used += c[i].samples;
            any = true;
        }
    }
    if (!any && !idx.empty()) run[idx[0]] = 1;
    return run;
}

}  // namespace plan
}  // namespace mcubes
