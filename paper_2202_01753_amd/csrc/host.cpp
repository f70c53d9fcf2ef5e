// Host-side helpers: lattice, validation, constants, Init-Bins, bin
// adjustment and weighted estimates.  Built without floating-point
// contraction: the bin adjustment must round exactly as written so that a
// given histogram always yields the same grid.
#include "host.hpp"

#include "estimate.hpp"

#include <cmath>
#include <cstring>

namespace mcubes {
namespace host {

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

bool is_fp32(const mc_problem *pr) { return pr->precision == MC_FP32_EVAL; }

// LDS of one sampling workgroup: the grid (FP64: nb+1 boundaries per axis;
// FP32: a float (left, width) pair per bin) and, when collecting bin
// contributions, the FP64 histogram.
size_t lds_bytes_of(int d, int nb, bool hist, bool fp32) {
    const size_t grid = fp32 ? (size_t)d * nb * 2 * sizeof(float) : (size_t)d * (nb + 1) * sizeof(double);
    return grid + (hist ? (size_t)d * nb * sizeof(double) : 0);
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
    if (pr->precision != MC_FP64 && pr->precision != MC_FP32_EVAL) return MC_EINVAL;
    if (pr->one_d != 0 && pr->one_d != 1) return MC_EINVAL;
    if (pr->device_steps != 0 && pr->device_steps != 1) return MC_EINVAL;
    if (is_fp32(pr) && g > (int64_t(1) << 24)) return MC_EINVAL;  // digits exact in float
    if (pr->nbins < 2 || pr->nbins > (1 << 20)) return MC_EINVAL;
    if (lds_bytes_of(d, pr->nbins, true, is_fp32(pr)) > kLdsDynamicLimit) return MC_EINVAL;
    if (pr->itmax < 1 || pr->ita < 0 || pr->ita > pr->itmax) return MC_EINVAL;
    if (!(pr->alpha > 0.0) || !std::isfinite(pr->alpha)) return MC_EINVAL;
    if (!(pr->tau_rel >= 0.0) || !std::isfinite(pr->tau_rel)) return MC_EINVAL;
    if (std::isnan(pr->chi2_max)) return MC_EINVAL;
    const int th = threads_of(pr);
    if (pr->blocks < 0 || th < 64 || th > kMaxBlock || th % 64 != 0) return MC_EINVAL;
    return MC_OK;
}

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

// Per-axis constants in the layout the sampling kernels read.
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

// ------------------------------------------------------------------ host steps of Alg. 2

void init_grid(int d, int nb, double *grid) {
    for (int j = 0; j < d; ++j) {
        double *row = grid + (size_t)j * (nb + 1);
        for (int i = 0; i <= nb; ++i) row[i] = (double)i / (double)nb;
    }
}

void tables_f32(const double *tables, float *out) {
    for (int t = 0; t < 2; ++t) {
        const double *T = tables + (size_t)t * kTableN * kTableN;
        float *P = out + (size_t)t * 2 * kTableN * kTableN;
        for (int a = 0; a < kTableN; ++a)
            for (int b = 0; b < kTableN; ++b) {
                P[2 * (a * kTableN + b)] = (float)T[a * kTableN + b];
                P[2 * (a * kTableN + b) + 1] = a + 1 < kTableN ? (float)T[(a + 1) * kTableN + b] : 0.0f;
            }
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

void refine_1d(int d, int nb, double alpha, const double *hist, double *grid) {
    std::vector<double> sm(nb), r(nb), prev(nb + 1);
    refine_axis(nb, alpha, hist, grid, sm, r, prev);
    for (int j = 1; j < d; ++j) std::copy(grid, grid + nb + 1, grid + (size_t)j * (nb + 1));
}

void weighted(int k, const double *I, const double *var, double *out) {
    weighted_estimate(k, I, var, out);
}

bool check_convergence(const mc_problem *pr, int k, const double *est) {
    return converged_after(k, est, pr->tau_rel, pr->chi2_max);
}

void sample_args(const mc_problem *pr, int64_t g, int64_t m, int64_t p, uint32_t iter, bool adjust,
                 const void *consts, const double *grid, const void *tables, SampleArgs *a) {
    std::memset(a, 0, sizeof(*a));
    const int nb = pr->nbins;
    a->grid = grid;
    a->tables = tables;
    a->consts = consts;
    a->fp32 = is_fp32(pr) ? 1 : 0;
    a->m = m;
    a->seed = pr->seed;
    a->iter = iter;
    a->p = (int32_t)p;
    a->nb = nb;
    a->g = (int32_t)g;
    a->hist = adjust ? 1 : 0;
    a->kind = pr->integrand * 32 + pr->dim;
    a->one_d = pr->one_d ? 1 : 0;
    a->hist_copies = 1;
    a->s = (double)nb / (double)g;
    a->s32 = (float)a->s;
    a->inv = 1.0 / (double)(m * p);
    a->pd = (double)p;
    a->inv_pm1 = 1.0 / (a->pd - 1.0);
    if (pr->integrand == MC_F_CONST) a->cval = pr->params[0];
}

}  // namespace host
}  // namespace mcubes
