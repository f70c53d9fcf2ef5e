/*
 * m-Cubes VEGAS oracle: a plain, sequential, FP64 implementation of the
 * method of Sakiotis et al., "m-Cubes: An Efficient and Portable
 * Implementation of Multi-Dimensional Integration for GPUs" (arXiv 2202.01753).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no
 * source, header, table or constant generator with the GPU library; the two
 * meet only in the seeded input generators and in the tests.
 *
 * What it follows:
 *   Alg. 1 (one VEGAS iteration): per sub-cube, p samples; each sample is a
 *       point y in (0,1)^d mapped to x, evaluated, and its contribution is
 *       added to one bin per axis; the bins then drive the boundary update.
 *   Alg. 2 (m-Cubes driver): g = (maxcalls/2)^(1/d) intervals per axis,
 *       m = g^d sub-cubes, p = maxcalls/m samples per sub-cube, equal initial
 *       bins, "ita" adjusting iterations followed by non-adjusting ones, a
 *       weighted estimate and a convergence check every iteration.
 *   Alg. 3 (V-Sample): per sub-cube sums I_t and E_t of the sample estimates,
 *       the bin contributions I_k^2, a per-cube variance, and the totals (I, E).
 *
 * Readings where the paper is silent or refers to Lepage (1978) for the
 * formula (the same readings the GPU library implements):
 *   - g is the largest integer with g^d <= floor(maxcalls/2), found by integer
 *     arithmetic; m = g^d; p = floor(maxcalls/m); maxcalls < 4 is rejected.
 *   - Sub-cube t has digits c_j = floor(t / g^j) mod g, j = 0..d-1.
 *   - Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = seed and
 *     counter (k*nblk + blk, iteration, t_lo, t_hi), nblk = ceil(d/2); the
 *     sample's words are w[4*blk + r].
 *   - Uniform for axis j: X = (w[j] << 20) | (w[d+j] >> 12), u = (2X+1) 2^-53.
 *   - VEGAS map (Lepage 1978): y_j = (c_j + u_j)/g, bin i = floor(y_j nb),
 *     x_j = L_j + (H_j - L_j)(B_j[i] + (y_j nb - i)(B_j[i+1] - B_j[i])), and
 *     Jacobian J = prod_j nb (B_j[i+1] - B_j[i]) (H_j - L_j).
 *   - I_k = f(x) J / (m p); per-cube variance (p sum I_k^2 - (sum I_k)^2)/(p-1)
 *     from shifted sums; totals are compensated sums in ascending t.
 *   - Bin contributions are reset every iteration.
 *   - Bin adjustment: three-point smoothing, Lepage's compression
 *     ((1 - s_i/S) / ln(S/s_i))^alpha, and equal-share rebinning.
 *   - Weighted estimate: inverse-variance weights over the iterations so far
 *     that carry information, chi^2 per degree of freedom about the weighted
 *     mean.  An iteration whose estimate and variance are both zero (no
 *     sample saw a non-zero value) carries none and is left out.
 *   - Convergence (Sec. V counts a run as converged only with a small
 *     chi^2): at least two iterations, sigma <= tau_rel |I| and
 *     chi^2/dof <= chi2_max (5 unless the problem sets another bound; a
 *     negative bound leaves chi^2 unchecked).
 *   - FP32-eval mode (precision 1): the uniform u = (2 (w[j] >> 9) + 1) 2^-24
 *     from the same words, the map and the integrand in single precision
 *     (constants, each bin's left boundary and width, and the tables rounded
 *     to float from FP64), then I_k and everything after it in FP64 as above.
 *   - m-Cubes1D variant (Sec. V, "The m-Cubes1D variant"): the bin
 *     contributions are collected for the first axis only, its boundaries are
 *     adjusted from them, and every axis takes those boundaries, so all axes
 *     share one grid (meant for fully symmetric integrands).
 *
 * Build with -ffp-contract=off: every rounding below is the one written.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENONFINITE 3

#define ORC_F_CONST 0
#define ORC_F_GAUSS_PRODUCT 1
#define ORC_F_CORNER_PEAK 2
#define ORC_F_GAUSS_TABLES 3

#define ORC_TABLE_N 256

typedef struct {
    int32_t integrand;
    const double *params;   /* integrand parameters, layout per integrand id */
    const double *tables;   /* two 256x256 row-major tables (GAUSS_TABLES) */
    int32_t dim;
    const double *lo, *hi;  /* integration bounds, length dim */
    int64_t maxcalls;
    int32_t nbins;
    int32_t itmax, ita;
    double alpha, tau_rel;
    uint64_t seed;
    int32_t precision;      /* 0: FP64, 1: FP32 evaluation with FP64 accumulation */
    int32_t one_d;          /* 1: the m-Cubes1D variant */
    double chi2_max;        /* convergence bound on chi^2/dof: 0 = 5, negative = none */
} orc_problem;

#define ORC_CHI2_DOF_DEFAULT 5.0

/* ------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the
 * published multipliers, the Weyl key increments applied between rounds.   */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t prod_a = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t prod_b = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi_a = (uint32_t)(prod_a >> 32), lo_a = (uint32_t)prod_a;
        uint32_t hi_b = (uint32_t)(prod_b >> 32), lo_b = (uint32_t)prod_b;
        uint32_t y0 = hi_b ^ x1 ^ k0;
        uint32_t y1 = lo_b;
        uint32_t y2 = hi_a ^ x3 ^ k1;
        uint32_t y3 = lo_a;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform on the open interval (0,1) from 52 random bits: (2X+1) 2^-53.    */
double orc_uniform64(uint32_t whi, uint32_t wlo)
{
    uint64_t X = ((uint64_t)whi << 20) | (uint64_t)(wlo >> 12);
    uint64_t odd = 2u * X + 1u;            /* < 2^53: exact in a double */
    return (double)odd * 0x1p-53;
}

/* Single-precision uniform on (0,1) from the top 23 bits: (2 (w >> 9) + 1) 2^-24. */
float orc_uniform24(uint32_t w)
{
    uint32_t odd = 2u * (w >> 9) + 1u;     /* < 2^24: exact in a float */
    return (float)odd * 0x1p-24f;
}

/* ------------------------------------------------------------------ */
/* Sub-cube lattice (Alg. 2): g, m = g^d, p = floor(maxcalls/m).            */

/* 1 if b^d <= lim, computed without overflow. */
static int pow_at_most(int64_t b, int d, int64_t lim)
{
    __int128 acc = 1;
    for (int i = 0; i < d; ++i) {
        acc *= b;
        if (acc > lim) return 0;
    }
    return 1;
}

int orc_shape(int32_t d, int64_t maxcalls, int64_t *g_out, int64_t *m_out, int64_t *p_out)
{
    if (d < 1 || maxcalls < 4) return ORC_EINVAL;
    int64_t half = maxcalls / 2;
    /* start from a floating estimate, then settle it with exact integer checks */
    int64_t g = (int64_t)floor(pow((double)half, 1.0 / (double)d));
    if (g < 1) g = 1;
    while (g > 1 && !pow_at_most(g, d, half)) --g;
    while (pow_at_most(g + 1, d, half)) ++g;
    int64_t m = 1;
    for (int i = 0; i < d; ++i) m *= g;
    *g_out = g;
    *m_out = m;
    *p_out = maxcalls / m;
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Neumaier's compensated summation.                                         */

typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double v)
{
    double t = a->s + v;
    if (fabs(a->s) >= fabs(v))
        a->c += (a->s - t) + v;
    else
        a->c += (v - t) + a->s;
    a->s = t;
}

static double nsum_value(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Integrands.                                                                */

static int params_expected(int integrand, int d)
{
    switch (integrand) {
    case ORC_F_CONST: return 1;
    case ORC_F_GAUSS_PRODUCT: return 2 * d;
    case ORC_F_CORNER_PEAK: return d;
    case ORC_F_GAUSS_TABLES: return 2 * d;
    default: return -1;
    }
}

/* linear interpolation between a and b at fraction t */
static double lerp(double a, double b, double t) { return fma(t, b - a, a); }

/* Bilinear interpolation in a 256x256 table T[a][b] whose node (a,b) sits at
 * (a/255, b/255).  Outside the unit square the edge cell is extended.       */
static double table_bilinear(const double *T, double x, double y)
{
    double ux = x * 255.0, uy = y * 255.0;
    double fa = floor(ux), fb = floor(uy);
    if (fa < 0.0) fa = 0.0;
    if (fa > 254.0) fa = 254.0;
    if (fb < 0.0) fb = 0.0;
    if (fb > 254.0) fb = 254.0;
    double tx = ux - fa, ty = uy - fb;
    int a = (int)fa, b = (int)fb;
    double t00 = T[a * ORC_TABLE_N + b];
    double t10 = T[(a + 1) * ORC_TABLE_N + b];
    double t01 = T[a * ORC_TABLE_N + b + 1];
    double t11 = T[(a + 1) * ORC_TABLE_N + b + 1];
    double along0 = lerp(t00, t10, tx);
    double along1 = lerp(t01, t11, tx);
    return lerp(along0, along1, ty);
}

/* exp(-sum_j ((x_j - c_j) / w_j)^2) with 1/w_j rounded once */
static double gaussian_product(int d, const double *params, const double *x)
{
    double acc = 0.0;
    for (int j = 0; j < d; ++j) {
        double inv_w = 1.0 / params[d + j];
        double t = (x[j] - params[j]) * inv_w;
        acc = fma(t, t, acc);
    }
    return exp(-acc);
}

/* (1 + sum_j a_j x_j)^-(d+1), the power by left-to-right binary powering */
static double corner_peak(int d, const double *params, const double *x)
{
    double S = 1.0;
    for (int j = 0; j < d; ++j) S = fma(params[j], x[j], S);
    unsigned e = (unsigned)(d + 1);
    int top = 31;
    while (!((e >> top) & 1u)) --top;
    double pw = S;
    for (int bit = top - 1; bit >= 0; --bit) {
        pw = pw * pw;
        if ((e >> bit) & 1u) pw = pw * S;
    }
    return 1.0 / pw;
}

static double integrand_value(const orc_problem *P, const double *x)
{
    int d = P->dim;
    switch (P->integrand) {
    case ORC_F_CONST:
        return P->params[0];
    case ORC_F_GAUSS_PRODUCT:
        return gaussian_product(d, P->params, x);
    case ORC_F_CORNER_PEAK:
        return corner_peak(d, P->params, x);
    case ORC_F_GAUSS_TABLES: {
        double G = gaussian_product(d, P->params, x);
        double T1 = table_bilinear(P->tables, x[0], x[1]);
        double T2 = table_bilinear(P->tables + ORC_TABLE_N * ORC_TABLE_N, x[2], x[3]);
        return (G * T1) * T2;
    }
    default:
        return NAN;
    }
}

/* ---- single-precision evaluation (FP32-eval mode) ---- */

typedef struct {
    float lo[16], span[16], q[16], pa[16], pb[16];
    float s, cval;
    float *grid;     /* d*nb (left boundary, width) pairs rounded to float */
    float *tables;   /* 2*256*256 rounded to float, or NULL */
} f32_consts;

static float lerpf_(float a, float b, float t) { return fmaf(t, b - a, a); }

static float table_bilinear_f(const float *T, float x, float y)
{
    float ux = x * 255.0f, uy = y * 255.0f;
    float fa = floorf(ux), fb = floorf(uy);
    if (fa < 0.0f) fa = 0.0f;
    if (fa > 254.0f) fa = 254.0f;
    if (fb < 0.0f) fb = 0.0f;
    if (fb > 254.0f) fb = 254.0f;
    float tx = ux - fa, ty = uy - fb;
    int a = (int)fa, b = (int)fb;
    float t00 = T[a * ORC_TABLE_N + b];
    float t10 = T[(a + 1) * ORC_TABLE_N + b];
    float t01 = T[a * ORC_TABLE_N + b + 1];
    float t11 = T[(a + 1) * ORC_TABLE_N + b + 1];
    return lerpf_(lerpf_(t00, t10, tx), lerpf_(t01, t11, tx), ty);
}

static float integrand_value_f(const orc_problem *P, const f32_consts *K, const float *x)
{
    int d = P->dim;
    if (P->integrand == ORC_F_CONST) return K->cval;
    if (P->integrand == ORC_F_CORNER_PEAK) {
        float S = 1.0f;
        for (int j = 0; j < d; ++j) S = fmaf(K->pa[j], x[j], S);
        unsigned e = (unsigned)(d + 1);
        int top = 31;
        while (!((e >> top) & 1u)) --top;
        float pw = S;
        for (int bit = top - 1; bit >= 0; --bit) {
            pw = pw * pw;
            if ((e >> bit) & 1u) pw = pw * S;
        }
        return 1.0f / pw;
    }
    float acc = 0.0f;
    for (int j = 0; j < d; ++j) {
        float t = (x[j] - K->pa[j]) * K->pb[j];
        acc = fmaf(t, t, acc);
    }
    float G = expf(-acc);
    if (P->integrand == ORC_F_GAUSS_PRODUCT) return G;
    float T1 = table_bilinear_f(K->tables, x[0], x[1]);
    float T2 = table_bilinear_f(K->tables + ORC_TABLE_N * ORC_TABLE_N, x[2], x[3]);
    return (G * T1) * T2;
}

static int validate(const orc_problem *P)
{
    int d = P->dim;
    if (d < 1 || d > 16) return ORC_EINVAL;
    if (P->nbins < 2) return ORC_EINVAL;
    if (P->maxcalls < 4) return ORC_EINVAL;
    if (P->itmax < 1 || P->ita < 0 || P->ita > P->itmax) return ORC_EINVAL;
    if (!(P->alpha > 0.0) || !(P->tau_rel >= 0.0)) return ORC_EINVAL;
    if (isnan(P->chi2_max)) return ORC_EINVAL;
    if (P->precision != 0 && P->precision != 1) return ORC_EINVAL;
    if (P->one_d != 0 && P->one_d != 1) return ORC_EINVAL;
    if (params_expected(P->integrand, d) < 0) return ORC_EINVAL;
    if (P->integrand == ORC_F_GAUSS_TABLES && (d < 4 || P->tables == NULL)) return ORC_EINVAL;
    for (int j = 0; j < d; ++j)
        if (!isfinite(P->lo[j]) || !isfinite(P->hi[j]) || !(P->lo[j] < P->hi[j])) return ORC_EINVAL;
    return ORC_OK;
}

/* Evaluate the integrand at one point (lets tests integrate it by quadrature). */
double orc_integrand(const orc_problem *P, const double *x)
{
    return integrand_value(P, x);
}

/* Evaluate the integrand at n points (row-major n x d), for quadrature tests. */
void orc_integrand_many(const orc_problem *P, int64_t n, const double *xs, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = integrand_value(P, xs + i * P->dim);
}

/* ------------------------------------------------------------------ */
/* VEGAS map for one point given z_j = y_j * nb per axis: bin index, point in
 * the integration domain and Jacobian.  grid holds d rows of nb+1 boundaries
 * in unit coordinates.                                                       */

static double map_point(int d, int nb, const double *grid, const double *lo,
                        const double *span, const double *q, const double *z,
                        double *x, int64_t *bin)
{
    double J = 1.0;
    for (int j = 0; j < d; ++j) {
        double fz = floor(z[j]);
        int64_t i = (int64_t)fz;
        double frac;
        if (i > nb - 1) {
            i = nb - 1;
            frac = 1.0;
        } else {
            frac = z[j] - fz;
        }
        const double *B = grid + (size_t)j * (nb + 1);
        double left = B[i];
        double width = B[i + 1] - left;
        double xu = fma(frac, width, left);
        x[j] = fma(span[j], xu, lo[j]);
        J = J * (width * q[j]);
        bin[j] = i;
    }
    return J;
}

/* The map evaluated at a point y in (0,1)^d (z = y * nb), for quadrature tests. */
double orc_map(int32_t d, int32_t nb, const double *grid, const double *lo, const double *hi,
               const double *y, double *x, int64_t *bin)
{
    double span[16], q[16], z[16];
    for (int j = 0; j < d; ++j) {
        span[j] = hi[j] - lo[j];
        q[j] = (double)nb * span[j];
        z[j] = y[j] * (double)nb;
    }
    return map_point(d, nb, grid, lo, span, q, z, x, bin);
}

/* ------------------------------------------------------------------ */
/* One V-Sample pass (Alg. 3) over sub-cubes [t0, t1) of iteration `iter`.
 *
 * grid      d*(nb+1) bin boundaries in unit coordinates (row j = axis j)
 * out_I     sum over the sub-cubes of I_t
 * out_var   sum over the sub-cubes of the per-cube variance
 * hist      if non-NULL, d*nb bin contributions sum I_k^2 (overwritten)
 * strace    if non-NULL, (t1-t0)*p records of 3d+2 doubles:
 *           u[0..d), bin[0..d), x[0..d), J, f
 * ctrace    if non-NULL, (t1-t0) records of 2 doubles: I_t, var_t
 */
int orc_vsample(const orc_problem *P, uint32_t iter, const double *grid, int64_t t0, int64_t t1,
                double *out_I, double *out_var, double *hist, double *strace, double *ctrace)
{
    int rc = validate(P);
    if (rc != ORC_OK) return rc;
    int64_t g, m, p;
    rc = orc_shape(P->dim, P->maxcalls, &g, &m, &p);
    if (rc != ORC_OK) return rc;
    if (t0 < 0 || t1 > m || t0 > t1) return ORC_EINVAL;

    const int d = P->dim, nb = P->nbins;
    const double s = (double)nb / (double)g;
    const double inv = 1.0 / (double)(m * p);
    const double pd = (double)p;
    const double inv_pm1 = 1.0 / (pd - 1.0);
    const int nblk = (d + 1) / 2;
    const uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
    double span[16], q[16];
    for (int j = 0; j < d; ++j) {
        span[j] = P->hi[j] - P->lo[j];
        q[j] = (double)nb * span[j];
    }

    const int fp32 = P->precision == 1;
    if (fp32 && g > (1 << 24)) return ORC_EINVAL; /* cube digits must be exact floats */
    f32_consts K;
    memset(&K, 0, sizeof(K));
    if (fp32) {
        K.s = (float)s;
        for (int j = 0; j < d; ++j) {
            K.lo[j] = (float)P->lo[j];
            K.span[j] = (float)span[j];
            K.q[j] = (float)q[j];
        }
        if (P->integrand == ORC_F_CONST) K.cval = (float)P->params[0];
        if (P->integrand == ORC_F_CORNER_PEAK)
            for (int j = 0; j < d; ++j) K.pa[j] = (float)P->params[j];
        if (P->integrand == ORC_F_GAUSS_PRODUCT || P->integrand == ORC_F_GAUSS_TABLES)
            for (int j = 0; j < d; ++j) {
                K.pa[j] = (float)P->params[j];
                K.pb[j] = (float)(1.0 / P->params[d + j]);
            }
        /* per bin: left boundary and width, each rounded once from FP64 */
        K.grid = (float *)malloc(sizeof(float) * 2 * d * nb);
        for (int j = 0; j < d; ++j)
            for (int i = 0; i < nb; ++i) {
                const double *B = grid + (size_t)j * (nb + 1);
                K.grid[2 * ((size_t)j * nb + i)] = (float)B[i];
                K.grid[2 * ((size_t)j * nb + i) + 1] = (float)(B[i + 1] - B[i]);
            }
        if (P->integrand == ORC_F_GAUSS_TABLES) {
            K.tables = (float *)malloc(sizeof(float) * 2 * ORC_TABLE_N * ORC_TABLE_N);
            for (int i = 0; i < 2 * ORC_TABLE_N * ORC_TABLE_N; ++i) K.tables[i] = (float)P->tables[i];
        }
    }
    /* FP32 needs one word per axis, FP64 two; the counter layout is the same */
    const int blocks_used = fp32 ? (d + 3) / 4 : nblk;

    nsum *bins = NULL;
    if (hist) {
        bins = (nsum *)calloc((size_t)d * nb, sizeof(nsum));
        if (!bins) return ORC_EINVAL;
    }
    nsum total_I = {0, 0}, total_V = {0, 0};
    int nonfinite = 0;
    const int rec = 3 * d + 2;

    for (int64_t t = t0; t < t1; ++t) {
        int64_t digit[16];
        int64_t rest = t;
        for (int j = 0; j < d; ++j) {
            digit[j] = rest % g;
            rest /= g;
        }
        double I0 = 0.0, S1 = 0.0, S2 = 0.0;
        for (int64_t k = 0; k < p; ++k) {
            uint32_t w[32];
            for (int blk = 0; blk < blocks_used; ++blk) {
                uint32_t ctr[4] = {(uint32_t)(k * nblk + blk), iter, (uint32_t)t, (uint32_t)((uint64_t)t >> 32)};
                orc_philox4x32_10(ctr, key, w + 4 * blk);
            }
            double u[16], z[16], x[16];
            int64_t bin[16];
            double J, f;
            if (!fp32) {
                for (int j = 0; j < d; ++j) {
                    u[j] = orc_uniform64(w[j], w[d + j]);
                    double v = (double)digit[j] + u[j];
                    z[j] = v * s;
                }
                J = map_point(d, nb, grid, P->lo, span, q, z, x, bin);
                f = integrand_value(P, x);
            } else {
                float xf[16], Jf = 1.0f;
                for (int j = 0; j < d; ++j) {
                    float uf = orc_uniform24(w[j]);
                    float zf = ((float)digit[j] + uf) * K.s;
                    float fz = floorf(zf);
                    int64_t i = (int64_t)fz;
                    float frac;
                    if (i > nb - 1) {
                        i = nb - 1;
                        frac = 1.0f;
                    } else {
                        frac = zf - fz;
                    }
                    const float *cell = K.grid + 2 * ((size_t)j * nb + i);
                    float left = cell[0];
                    float width = cell[1];
                    float xu = fmaf(frac, width, left);
                    xf[j] = fmaf(K.span[j], xu, K.lo[j]);
                    Jf = Jf * (width * K.q[j]);
                    bin[j] = i;
                    u[j] = (double)uf;
                    x[j] = (double)xf[j];
                }
                J = (double)Jf;
                f = (double)integrand_value_f(P, &K, xf);
            }
            double F = f * J;
            if (!isfinite(F)) nonfinite = 1;
            double Ik = F * inv;
            if (k == 0) {
                I0 = Ik;
            } else {
                double dev = Ik - I0;
                S1 = S1 + dev;
                S2 = fma(dev, dev, S2);
            }
            if (bins) {
                double sq = Ik * Ik;
                int axes = P->one_d ? 1 : d;
                for (int j = 0; j < axes; ++j) nsum_add(&bins[(size_t)j * nb + bin[j]], sq);
            }
            if (strace) {
                double *r = strace + ((t - t0) * p + k) * rec;
                for (int j = 0; j < d; ++j) {
                    r[j] = u[j];
                    r[d + j] = (double)bin[j];
                    r[2 * d + j] = x[j];
                }
                r[3 * d] = J;
                r[3 * d + 1] = f;
            }
        }
        double It = fma(pd, I0, S1);
        double num = fma(-S1, S1, pd * S2);
        double vt = num * inv_pm1;
        if (vt < 0.0) vt = 0.0;
        nsum_add(&total_I, It);
        nsum_add(&total_V, vt);
        if (ctrace) {
            ctrace[2 * (t - t0)] = It;
            ctrace[2 * (t - t0) + 1] = vt;
        }
    }
    free(K.grid);
    free(K.tables);
    *out_I = nsum_value(&total_I);
    *out_var = nsum_value(&total_V);
    if (bins) {
        for (size_t i = 0; i < (size_t)d * nb; ++i) hist[i] = nsum_value(&bins[i]);
        free(bins);
    }
    return nonfinite ? ORC_ENONFINITE : ORC_OK;
}

/* ------------------------------------------------------------------ */
/* Init-Bins (Alg. 2): nb equal bins per axis, boundaries i/nb.              */
void orc_init_grid(int32_t d, int32_t nb, double *grid)
{
    for (int j = 0; j < d; ++j)
        for (int i = 0; i <= nb; ++i) grid[(size_t)j * (nb + 1) + i] = (double)i / (double)nb;
}

/* Adjust-Bin-Bounds: bins with large contributions become smaller
 * (Alg. 1 and the text after it).  Per axis: three-point smoothing of the
 * contributions, Lepage's damped compression with exponent alpha, then new
 * boundaries placed so that every new bin holds an equal share of the
 * compressed weight, assuming the weight is spread evenly inside each old bin.
 * An axis with no positive finite weight keeps its boundaries.              */
void orc_refine(int32_t d, int32_t nb, double alpha, const double *hist, double *grid)
{
    double *sm = (double *)malloc(sizeof(double) * nb);
    double *wt = (double *)malloc(sizeof(double) * nb);
    double *old = (double *)malloc(sizeof(double) * (nb + 1));
    for (int j = 0; j < d; ++j) {
        const double *C = hist + (size_t)j * nb;
        double *B = grid + (size_t)j * (nb + 1);
        sm[0] = (C[0] + C[1]) / 2.0;
        for (int i = 1; i < nb - 1; ++i) sm[i] = ((C[i - 1] + C[i]) + C[i + 1]) / 3.0;
        sm[nb - 1] = (C[nb - 2] + C[nb - 1]) / 2.0;
        double S = 0.0;
        for (int i = 0; i < nb; ++i) S = S + sm[i];
        if (!(S > 0.0) || !isfinite(S)) continue;
        double R = 0.0;
        for (int i = 0; i < nb; ++i) {
            if (sm[i] == 0.0)
                wt[i] = 0.0;
            else if (sm[i] == S)
                wt[i] = 1.0;
            else
                wt[i] = pow((1.0 - sm[i] / S) / log(S / sm[i]), alpha);
            R = R + wt[i];
        }
        if (!(R > 0.0)) continue;
        memcpy(old, B, sizeof(double) * (nb + 1));
        double share = R / (double)nb;
        int i = 0;
        double cum = 0.0;
        for (int k = 1; k < nb; ++k) {
            double target = (double)k * share;
            while (i < nb - 1 && cum + wt[i] < target) {
                cum = cum + wt[i];
                ++i;
            }
            double frac = wt[i] > 0.0 ? (target - cum) / wt[i] : 0.0;
            if (frac < 0.0) frac = 0.0;
            if (frac > 1.0) frac = 1.0;
            double edge = fma(frac, old[i + 1] - old[i], old[i]);
            B[k] = edge > B[k - 1] ? edge : B[k - 1];
        }
        B[0] = 0.0;
        B[nb] = 1.0;
    }
    free(sm);
    free(wt);
    free(old);
}

/* m-Cubes1D bin adjustment: the first axis's boundaries adjusted from its
 * contributions, then copied to every axis. */
void orc_refine_1d(int32_t d, int32_t nb, double alpha, const double *hist, double *grid)
{
    orc_refine(1, nb, alpha, hist, grid);
    for (int j = 1; j < d; ++j) memcpy(grid + (size_t)j * (nb + 1), grid, sizeof(double) * (nb + 1));
}

/* Weighted-Estimates: inverse-variance weighted mean of the iteration
 * estimates, its standard deviation and chi^2 per degree of freedom
 * (n - 1 degrees of freedom for n informative iterations).
 * An iteration with estimate 0 and variance 0 saw no non-zero sample: it
 * says nothing about the integral and is left out.  If an informative
 * iteration has variance 0 (the integrand is constant on every sub-cube,
 * so the iteration is exact), the mean of those iterations is the estimate,
 * with standard deviation 0 and chi^2/dof 0.  Without any informative
 * iteration the estimate is 0 with an infinite standard deviation.        */
void orc_weighted(int32_t k, const double *I, const double *var, double *Ibar, double *sigma,
                  double *chi2_dof)
{
    int n = 0, nzero = 0;
    double zsum = 0.0;
    for (int i = 0; i < k; ++i) {
        if (var[i] == 0.0 && I[i] == 0.0) continue;
        ++n;
        if (var[i] == 0.0) {
            ++nzero;
            zsum = zsum + I[i];
        }
    }
    if (n == 0) {
        *Ibar = 0.0;
        *sigma = INFINITY;
        *chi2_dof = NAN;
        return;
    }
    if (nzero > 0) {
        *Ibar = zsum / (double)nzero;
        *sigma = 0.0;
        *chi2_dof = n > 1 ? 0.0 : NAN;
        return;
    }
    double W = 0.0, WI = 0.0;
    for (int i = 0; i < k; ++i) {
        if (var[i] == 0.0) continue;   /* only the uninformative ones are left */
        double w = 1.0 / var[i];
        W = W + w;
        WI = WI + w * I[i];
    }
    double mean = WI / W;
    double chi = 0.0;
    for (int i = 0; i < k; ++i) {
        if (var[i] == 0.0) continue;
        double dev = I[i] - mean;
        chi = chi + (dev * dev) / var[i];
    }
    *Ibar = mean;
    *sigma = 1.0 / sqrt(W);
    *chi2_dof = n > 1 ? chi / (double)(n - 1) : NAN;
}

/* The convergence test of Alg. 2 (Check-Convergence) with the chi^2
 * condition of Sec. V: at least two iterations, the standard deviation at
 * most tau_rel times the estimate's magnitude, and chi^2/dof at most the
 * problem's bound.                                                          */
static int orc_converged(const orc_problem *P, int k, double Ibar, double sigma, double chi2)
{
    if (k < 2 || !(P->tau_rel > 0.0)) return 0;
    if (!(sigma <= P->tau_rel * fabs(Ibar))) return 0;
    if (P->chi2_max < 0.0) return 1;
    double bound = P->chi2_max > 0.0 ? P->chi2_max : ORC_CHI2_DOF_DEFAULT;
    return chi2 <= bound;
}

/* The whole m-Cubes run (Alg. 2).
 * it_I, it_var: itmax doubles each (per-iteration estimates), may be NULL.
 * grid_out: d*(nb+1) doubles, the final boundaries, may be NULL.
 * res: estimate, error, chi2/dof;  ires: iterations, converged;  calls.     */
int orc_integrate(const orc_problem *P, double *res, int64_t *ires, double *it_I, double *it_var,
                  double *grid_out)
{
    int rc = validate(P);
    if (rc != ORC_OK) return rc;
    int64_t g, m, p;
    rc = orc_shape(P->dim, P->maxcalls, &g, &m, &p);
    if (rc != ORC_OK) return rc;
    const int d = P->dim, nb = P->nbins;
    double *grid = (double *)malloc(sizeof(double) * d * (nb + 1));
    double *hist = (double *)malloc(sizeof(double) * d * nb);
    double *Is = (double *)malloc(sizeof(double) * P->itmax);
    double *Vs = (double *)malloc(sizeof(double) * P->itmax);
    orc_init_grid(d, nb, grid);
    double Ibar = 0.0, sigma = 0.0, chi2 = NAN;
    int k = 0, converged = 0;
    for (int it = 0; it < P->itmax; ++it) {
        int adjust = it < P->ita;
        rc = orc_vsample(P, (uint32_t)it, grid, 0, m, &Is[it], &Vs[it], adjust ? hist : NULL, NULL, NULL);
        if (rc != ORC_OK) break;
        k = it + 1;
        orc_weighted(k, Is, Vs, &Ibar, &sigma, &chi2);
        if (adjust) {
            if (P->one_d)
                orc_refine_1d(d, nb, P->alpha, hist, grid);
            else
                orc_refine(d, nb, P->alpha, hist, grid);
        }
        if (orc_converged(P, k, Ibar, sigma, chi2)) {
            converged = 1;
            break;
        }
    }
    if (rc == ORC_OK) {
        res[0] = Ibar;
        res[1] = sigma;
        res[2] = chi2;
        ires[0] = k;
        ires[1] = converged;
        ires[2] = (int64_t)k * m * p;
        for (int i = 0; i < k; ++i) {
            if (it_I) it_I[i] = Is[i];
            if (it_var) it_var[i] = Vs[i];
        }
        if (grid_out) memcpy(grid_out, grid, sizeof(double) * d * (nb + 1));
    }
    free(grid);
    free(hist);
    free(Is);
    free(Vs);
    return rc;
}
