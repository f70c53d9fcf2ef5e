// V-Sample / V-Sample-No-Adjust (Alg. 3) for gfx950: the per-iteration
// sampling pass of m-Cubes.
//
// Work mapping: one lane per sub-cube at a time, persistent workgroups that
// stride through the g^d sub-cubes.  Because every random number is keyed by
// (seed; iteration, sub-cube, sample) rather than by thread, the mapping of
// sub-cubes to lanes does not change any sample point.
//
// Per sample (FP64, or FP32 for the map and the integrand in the FP32-eval
// path; no implicit contraction, fma only where written):
//   Philox4x32-10 blocks -> 52-bit uniforms -> stratified coordinate in bins
//   -> bin index, boundary and width from the LDS copy of the grid -> point
//   and Jacobian -> integrand -> I_k = f J / (m p) -> shifted per-cube sums
//   -> (V-Sample only) I_k^2 added to one LDS bin per axis.
// Per sub-cube: I_t and the unbiased variance estimate, accumulated per lane
// with error-free transformations.  Per workgroup: a fixed-order wave and
// workgroup reduction, then the totals go to this workgroup's slot of the
// partials array and the LDS histogram is added into one of the histogram
// accumulators, both merged after the pass (finalize or steps kernel).
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace mcubes {

// Read-only data reached through the constant address space: uniform loads
// become scalar loads, which the compiler may repeat instead of keeping every
// value in registers.  Only for memory that nothing writes while the kernel
// runs.
template <typename T>
using Const = __attribute__((address_space(4))) const T;


// The constants of axis j.  The single-integral kernel passes a volatile
// pointer: the compiler then reloads each constant where it is used instead of
// holding every axis's constants in scalar registers (which spilled them).
// With BATCH the pointer is instead made opaque once per axis, by an empty asm
// that the loads through it cannot move above: they still stay inside the
// loops, but they are no longer volatile, so the compiler merges the axis's
// loads and waits for them once rather than once per value (each wait also
// drains the LDS reads in flight).  That is 2-3% faster for the FP64
// Gaussian and table kernels and up to 2% slower for the others (more scalar
// spills), so those keep the per-use loads.
template <bool BATCH, typename CP>
__device__ __forceinline__ auto axis_consts(CP base, int j) {
    using P = std::remove_pointer_t<CP>;
    if constexpr (BATCH && std::is_volatile_v<P>) {
        auto p = const_cast<std::remove_volatile_t<P> *>(base + kConstStride * j);
        asm volatile("" : "+s"(p));
        return p;
    } else {
        return base + kConstStride * j;
    }
}

// ---------------------------------------------------------------- Philox4x32-10
// Salmon et al., SC'11: ten rounds of two 32x32->64 products, with the key
// advanced by the Weyl constants between rounds.  The key is uniform across
// the wavefront, so its schedule stays in scalar registers.  Each round's two
// three-way XORs are single v_bitop3_b32 instructions (truth table 0x96 is
// a ^ b ^ c); in the first round the counter words x1, x3 are uniform or fixed
// per sub-cube, so there the compiler folds their XOR with the key instead.
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
    return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}

__device__ __forceinline__ void philox4x32_10(uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                              uint32_t &x3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)x0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        const uint32_t y0 = r == 0 ? (uint32_t)(pb >> 32) ^ (x1 ^ k0) : xor3((uint32_t)(pb >> 32), x1, k0);
        const uint32_t y2 = r == 0 ? (uint32_t)(pa >> 32) ^ (x3 ^ k1) : xor3((uint32_t)(pa >> 32), x3, k1);
        x1 = (uint32_t)pb;
        x3 = (uint32_t)pa;
        x0 = y0;
        x2 = y2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// (2X+1) 2^-53 for the 52-bit X = (whi << 20) | (wlo >> 12): the double with
// exponent 0 and mantissa X is 1 + X 2^-52; subtracting 1 - 2^-53 is exact
// (Sterbenz), so the result is exactly the open-interval uniform.
__device__ __forceinline__ double uniform53(uint32_t whi, uint32_t wlo) {
    // both words are funnel shifts of a 64-bit pair: {0x3FF, whi} >> 12 is
    // 0x3FF00000 | (whi >> 12), and {whi, wlo} >> 12 is (whi << 20) | (wlo >> 12)
    const uint32_t hi = __builtin_amdgcn_alignbit(0x3FFu, whi, 12);
    const uint32_t lo = __builtin_amdgcn_alignbit(whi, wlo, 12);
    return __hiloint2double((int)hi, (int)lo) - 0x1.fffffffffffffp-1;
}

// ---------------------------------------------------------------- FP32-eval helpers

// (2 (w >> 9) + 1) 2^-24: the float with exponent 0 and mantissa w >> 9 is
// 1 + (w >> 9) 2^-23; subtracting 1 - 2^-24 is exact (Sterbenz).
__device__ __forceinline__ float uniform24(uint32_t w) {
    // {0x7F, w} >> 9 is 0x3F800000 | (w >> 9)
    return __uint_as_float(__builtin_amdgcn_alignbit(0x7Fu, w, 9)) - 0x1.fffffep-1f;
}

// Arithmetic of the evaluation precision R (double for the FP64 path, float
// for FP32 evaluation): each is a single correctly rounded IEEE operation.
__device__ __forceinline__ double rfma(double a, double b, double c) { return __fma_rn(a, b, c); }
__device__ __forceinline__ float rfma(float a, float b, float c) { return __fmaf_rn(a, b, c); }
__device__ __forceinline__ double rfloor(double a) { return floor(a); }
__device__ __forceinline__ float rfloor(float a) { return floorf(a); }
__device__ __forceinline__ double rmin(double a, double b) { return fmin(a, b); }
__device__ __forceinline__ float rmin(float a, float b) { return fminf(a, b); }
__device__ __forceinline__ double rmax(double a, double b) { return fmax(a, b); }
__device__ __forceinline__ float rmax(float a, float b) { return fmaxf(a, b); }
__device__ __forceinline__ double rexp(double a) { return exp(a); }
__device__ __forceinline__ float rexp(float a) { return expf(a); }

// ---------------------------------------------------------------- integrands

template <typename R>
__device__ __forceinline__ R lerp(R a, R b, R t) {
    return rfma(t, b - a, a);
}

// Bilinear interpolation in one 256x256 table, node (a,b) at (a/255, b/255),
// the edge cell extended outside the unit square, in two parts: table_cell
// finds the cell of (x, y) and loads its four nodes, interpolate combines
// them.  The integrand fetches each table's cell as soon as its two
// coordinates are known, so the loads are in flight while the remaining axes
// and the exponential are computed; the arithmetic is that of one bilinear
// interpolation, in the same order.
template <typename R>
struct TableCell {
    R t00, t01, t10, t11, tx, ty;
};

// Device layout of the two tables, one after the other.  FP64: row-major,
// node (a, b) at a * 256 + b; the two nodes of a cell's row are adjacent, so
// a cell is two 16-byte loads.  FP32-eval: row pairs, element 2 (a * 256 + b)
// holding node (a, b) and the next one node (a + 1, b) (0 for a = 255), so a
// cell's four nodes are four consecutive floats, one 16-byte load instead of
// two 8-byte ones (2% faster; the same layout in FP64 measured 0.5% slower).
template <typename R>
constexpr int kTableStride = std::is_same<R, float>::value ? 2 * kTableN * kTableN : kTableN * kTableN;

template <typename R>
__device__ __forceinline__ TableCell<R> table_cell(const R *__restrict__ T, R x, R y) {
    const R ux = x * R(255), uy = y * R(255);
    const R fa = rmin(rmax(rfloor(ux), R(0)), R(254));
    const R fb = rmin(rmax(rfloor(uy), R(0)), R(254));
    const int cell = (int)fa * kTableN + (int)fb;
    TableCell<R> c;
    c.tx = ux - fa;
    c.ty = uy - fb;
    if constexpr (std::is_same<R, float>::value) {
        // two 8-byte-aligned pairs, which the compiler merges into one load
        const float2 *q = reinterpret_cast<const float2 *>(T + 2 * cell);
        const float2 lo = q[0], hi = q[1];
        c.t00 = lo.x;
        c.t10 = lo.y;
        c.t01 = hi.x;
        c.t11 = hi.y;
    } else {
        c.t00 = T[cell];
        c.t01 = T[cell + 1];
        c.t10 = T[cell + kTableN];
        c.t11 = T[cell + kTableN + 1];
    }
    return c;
}

template <typename R>
__device__ __forceinline__ R interpolate(const TableCell<R> &c) {
    return lerp(lerp(c.t00, c.t10, c.tx), lerp(c.t01, c.t11, c.tx), c.ty);
}

// The integrand, accumulated axis by axis in ascending order so that the
// point itself need not stay in registers:
//   Gaussian product  acc = sum_j t_j^2 by fma, t_j = (x_j - c_j) * (1/w_j); f = exp(-acc)
//   corner peak       S = 1 + sum_j a_j x_j by fma; f = 1 / S^(D+1), the power by
//                     left-to-right binary powering, one correctly rounded division
//   tables            the Gaussian product times T1(x_1, x_2) times T2(x_3, x_4)
// EARLY (tables only): fetch each table's cell as soon as its coordinates are
// known rather than at the end; the loads then overlap the remaining axes and
// the exponential, at the price of registers for the eight nodes.  Kernels
// that inline many cases into one register allocation leave it off.
template <int F, int D, typename R, bool EARLY>
struct Integrand {
    R acc;
    R x0, x1, x2, x3;        // table coordinates (tables only)
    TableCell<R> c1, c2;     // the two tables' cells (tables, EARLY only)
    const R *T;              // the two tables, one after the other (tables only)

    __device__ __forceinline__ explicit Integrand(const void *tables)
        : acc(F == 2 ? R(1) : R(0)), x0(0), x1(0), x2(0), x3(0), c1(), c2(),
          T(static_cast<const R *>(tables)) {}

    template <typename CP>
    __device__ __forceinline__ void axis(int j, R xj, CP cj) {
        if constexpr (F == 1 || F == 3) {
            const R t = (xj - cj[3]) * cj[4];
            acc = rfma(t, t, acc);
        } else if constexpr (F == 2) {
            acc = rfma(cj[3], xj, acc);
        }
        if constexpr (F == 3) {
            if (j == 0) x0 = xj;
            if (j == 1) x1 = xj;
            if (j == 2) x2 = xj;
            if (j == 3) x3 = xj;
            if constexpr (EARLY) {
                if (j == 1) c1 = table_cell(T, x0, x1);
                if (j == 3) c2 = table_cell(T + kTableStride<R>, x2, x3);
            }
        }
    }

    template <typename A>
    __device__ __forceinline__ R value(const A &a) const {
        if constexpr (F == 0) {
            return R(a.cval);
        } else if constexpr (F == 1) {
            return rexp(-acc);
        } else if constexpr (F == 2) {
            constexpr unsigned e = (unsigned)(D + 1);
            constexpr int top = 31 - __builtin_clz(e);
            R pw = acc;
#pragma unroll
            for (int bit = top - 1; bit >= 0; --bit) {
                pw = pw * pw;
                if ((e >> bit) & 1u) pw = pw * acc;
            }
            return R(1) / pw;
        } else {
            static_assert(D >= 4, "table integrand needs four axes");
            const R G = rexp(-acc);
            const R T1 = interpolate(EARLY ? c1 : table_cell(T, x0, x1));
            const R T2 = interpolate(EARLY ? c2 : table_cell(T + kTableStride<R>, x2, x3));
            return (G * T1) * T2;
        }
    }
};

// ---------------------------------------------------------------- compensated sums

// s + c += v with the exact rounding error of s + v kept in c (Knuth's TwoSum).
__device__ __forceinline__ void two_sum_add(double &s, double &c, double v) {
    const double t = s + v;
    const double bp = t - s;
    const double e = (s - (t - bp)) + (v - bp);
    s = t;
    c += e;
}

__device__ __forceinline__ void two_sum_merge(double &s, double &c, double s2, double c2) {
    const double t = s + s2;
    const double bp = t - s;
    const double e = (s - (t - bp)) + (s2 - bp);
    s = t;
    c = (c + c2) + e;
}

// ---------------------------------------------------------------- LDS layout

// Per workgroup: the grid, then (V-Sample only) the d x nb histogram.  FP64
// keeps each axis's nb+1 boundaries; FP32 keeps per bin its left boundary and
// width, each rounded once from FP64.  (The per-axis constants are read with
// scalar loads from device memory; see Const.)
template <bool F32>
__host__ __device__ constexpr size_t lds_grid_bytes(int d, int nb) {
    return F32 ? (size_t)d * nb * 2 * sizeof(float) : (size_t)d * (nb + 1) * sizeof(double);
}

// ---------------------------------------------------------------- building blocks

template <bool F32>
using real_t = typename std::conditional<F32, float, double>::type;

// The workgroup's LDS regions for an integral of dimension d with nb bins.
template <bool F32>
struct LdsView {
    real_t<F32> *grid;
    double *hist;
    __device__ LdsView(double *lds, int d, int nb) {
        char *base = reinterpret_cast<char *>(lds);
        grid = reinterpret_cast<real_t<F32> *>(base);
        hist = reinterpret_cast<double *>(base + lds_grid_bytes<F32>(d, nb));
    }
};

// Copies the integral's grid into LDS and clears the histogram.  Callers
// synchronise the workgroup afterwards.  (A is SampleArgs, possibly in the
// constant address space: see the batched kernel.)
template <int D, bool F32, typename A>
__device__ __forceinline__ void load_lds(const A &a, const LdsView<F32> &v) {
    const int nb = a.nb, row = nb + 1, tid = threadIdx.x, nthr = blockDim.x;
    if constexpr (F32) {
        for (int i = tid; i < D * nb; i += nthr) {
            const int j = i / nb, b = i - j * nb;
            const double *B = a.grid + j * row + b;
            v.grid[2 * i] = (float)B[0];
            v.grid[2 * i + 1] = (float)(B[1] - B[0]);
        }
    } else {
        for (int i = tid; i < D * row; i += nthr) v.grid[i] = a.grid[i];
    }
    if (a.hist)
        for (int i = tid; i < D * nb * a.hist_copies; i += nthr) v.hist[i] = 0.0;
}

// Whether the one-sample path computes every axis's bin and issues every
// grid read before the rest of the sample (GF in cube_pass).  Each axis's
// constants are scalar loads whose wait also waits for the LDS reads in
// flight, so axis by axis every grid read was waited for on its own; in two
// phases they overlap.  Taken for the FP64 Gaussian and table kernels where
// the values held across the phases keep the occupancy and add no spill:
// 3-4% faster at d = 4, 2-3% at d = 6 to 8 (the d = 6 table kernel 1.024 ->
// 0.993 ms), 1% for the tables at d = 7, and for the FP32-eval table kernel
// at d = 6 together with the priority hint of cube_pass held until the
// integrand value (1.5%; 3% slower without the hint); the corner-peak
// kernels lose occupancy (d = 8: 9% slower; 4% with the hint), and d >= 10
// would spill.
template <int F, int D, bool F32>
constexpr bool kGridFirst =
    (!F32 && ((F == 1 && (D == 3 || D == 4 || (D >= 6 && D <= 9))) || (F == 3 && D >= 4 && D <= 7))) ||
    (F32 && F == 3 && D == 6);

// Whether cube_pass evaluates the samples of a sub-cube two at a time.  Two
// independent evaluations interleave and hide each other's LDS and
// transcendental latency, but both must fit in registers: in FP32 evaluation
// they do (up to d = 11, d = 8 with tables); in FP64 the pair spills to
// scratch memory (over 1 GB of HBM writes per launch at d = 6), so FP64
// keeps one sample at a time.  The FP32 table kernel at d = 6 also keeps one:
// the pair needs 86 VGPRs, which allows one 1024-thread workgroup per CU (4
// waves per SIMD), one sample at a time 69, which allows two 768-thread
// workgroups (6 waves per SIMD, the LDS limit) and is 11% faster; the pair
// had been 6% faster at the 4-wave shape.
template <int F, int D, bool F32>
constexpr bool kPairSamples = F32 && (F == 3 ? D <= 8 && D != 6 : D <= 11);

// Whether the single-integral kernel keeps each axis's lower bound in vector
// registers for the whole launch.  The point x = lo + span xu is one fma with
// two scalar operands otherwise, which the hardware cannot read in one
// instruction, so every sample moved lo into a vector register first (two
// moves per axis in FP64, one in FP32).  Taken for the FP64 Gaussian and
// table kernels of d = 6..8 (5% fewer VALU instructions at d = 6 and 8,
// 1.5-1.7% faster) and the FP32 table kernel at d = 6 (1.4% faster), which
// keep their waves per SIMD; at lower d the extra registers cost waves, at
// higher d they spill, and the d = 8 corner-peak and FP32 d = 8 kernels
// would lose the two workgroups per CU they run at.
template <int F, int D, bool F32>
constexpr bool kLowInVgpr = F32 ? (F == 3 && D == 6) : ((F == 1 || F == 3) && D >= 6 && D <= 8);

// The waves per SIMD the compiler is told a kernel runs at, where that is
// fixed by its launch (amdgpu_waves_per_eu(w, w)), so that it schedules for
// that occupancy rather than for a higher one the kernel cannot reach; 0: the
// compiler's own range (1 to 8 waves, which compiles to the same code as no
// attribute).  4 for the FP64 Gaussian kernels of d = 6..8 and table kernels
// of d = 6, 7 (108-128 VGPRs, one 1024-thread workgroup per CU either way):
// 0.6% faster at d = 6 with the tables, 0.8% at d = 8 with the Gaussian (at
// d = 8 with the tables it would spill 12 bytes).  6 for the FP32 table
// kernel at d = 6 (two 72 KB workgroups of 768 threads per CU): 0.6% faster;
// the d = 8 corner-peak kernels, also at 6 by their LDS, measured 0.5-1.5%
// slower with it.
template <int F, int D, bool TRACE, bool F32>
constexpr int kFixedWaves =
    TRACE ? 0
          : (!F32 && ((F == 1 && D >= 6 && D <= 8) || (F == 3 && (D == 6 || D == 7)))) ? 4
          : (F32 && F == 3 && D == 6) ? 6
                                      : 0;

// All p samples of sub-cube t (digits dig): returns I_t and var_t, adds the bin
// contributions to the LDS histogram when collecting them, and records the
// cube in the trace when tracing.  PAIR: evaluate the samples two at a time
// (kPairSamples for a kernel of its own; kernels that inline many cases into
// one register allocation leave it off).  EARLY: see Integrand.  LOV: lov
// holds the axes' lower bounds in vector registers (kLowInVgpr); otherwise
// they are read with the other constants.  (A compile-time choice: a null
// pointer tested at run time, though folded away, changed the FP32 d = 8
// kernels' register allocation from 72 to 90.)  GF: see kGridFirst.  PRIO:
// the one-sample path raises the wave's priority for the first part of each
// sample (the pair path always does).
template <int F, int D, bool TRACE, bool F32, bool PAIR, bool EARLY, bool LOV = false, bool GF = false,
          bool PRIO = false, typename A, typename CP>
__device__ __forceinline__ void cube_pass(const A &a, const LdsView<F32> &v, CP sC, uint64_t t,
                                          const uint32_t (&dig)[D], double &It, double &vt,
                                          bool &bad, const real_t<F32> *lov = nullptr) {
    using R = real_t<F32>;
    constexpr bool kBatchConsts = !F32 && (F == 1 || F == 3);  // see axis_consts
    constexpr int NBLK = (D + 1) / 2;                      // blocks in the counter layout
    constexpr int NUSED = F32 ? (D + 3) / 4 : NBLK;        // blocks this precision needs
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const int nb = a.nb, row = nb + 1, rec = 3 * D + 2;
    const R s = R(F32 ? a.s32 : a.s);
    const R last = R(nb - 1);
    const R *sG = v.grid;
    // with two histogram copies the upper half of each wave adds into the
    // second, so at most half as many lanes add into one bin at once
    double *sH = v.hist + (a.hist_copies > 1 && (threadIdx.x & 32) ? D * a.nb : 0);

    R cd[D];
#pragma unroll
    for (int j = 0; j < D; ++j) cd[j] = R(dig[j]);
    const uint32_t tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
    const bool traced = TRACE && (int64_t)t >= a.t0 && (int64_t)t < a.t1;

    double I0 = 0.0, S1 = 0.0, S2 = 0.0;
    if constexpr (PAIR) {
        // One sample: its value I_k and its bin on every axis (and its trace record).
        auto point = [&](int k, int (&bin)[D]) -> double {
            // raised wave priority while the sample's random words, bins and
            // grid reads are formed, back to normal before its integrand
            // value (see the one-sample path below; FP32-eval Gaussian and
            // corner-peak kernels 2-3% faster)
            __builtin_amdgcn_s_setprio(1);
            uint32_t w[4 * NUSED];
#pragma unroll
            for (int b = 0; b < NUSED; ++b) {
                uint32_t x0 = (uint32_t)(k * NBLK + b), x1 = a.iter, x2 = tlo, x3 = thi;
                philox4x32_10(x0, x1, x2, x3, k0, k1);
                w[4 * b] = x0;
                w[4 * b + 1] = x1;
                w[4 * b + 2] = x2;
                w[4 * b + 3] = x3;
            }
            Integrand<F, D, R, EARLY> fx(a.tables);
            R J = R(1);
#pragma unroll
            for (int j = 0; j < D; ++j) {
                R u;
                if constexpr (F32) u = uniform24(w[j]);
                else u = uniform53(w[j], w[D + j]);
                const R z = (cd[j] + u) * s;
                // bin index, clamped to the last bin with fraction 1 there: once
                // floor(z) > nb-1 we have z >= nb, so z - (nb-1) >= 1 and the min
                // gives exactly 1; otherwise z - floor(z) < 1 is exact.
                const R fz = rmin(rfloor(z), last);
                const int i = (int)fz;
                const R frac = rmin(z - fz, R(1));
                R left, width;
                if constexpr (F32) {
                    const float2 cell = reinterpret_cast<const float2 *>(sG)[j * nb + i];
                    left = cell.x;
                    width = cell.y;
                } else {
                    const R *B = sG + j * row + i;
                    left = B[0];
                    width = B[1] - left;
                }
                const R xu = rfma(frac, width, left);
                const auto cj = axis_consts<kBatchConsts>(sC, j);
                R xj;
                if constexpr (LOV)
                    xj = rfma(cj[1], xu, lov[j]);
                else
                    xj = rfma(cj[1], xu, cj[0]);
                J = J * (width * cj[2]);
                bin[j] = i;
                fx.axis(j, xj, cj);
                if (traced) {
                    double *r = a.trace + ((t - a.t0) * (uint64_t)a.p + k) * rec;
                    r[j] = (double)u;
                    r[D + j] = (double)i;
                    r[2 * D + j] = (double)xj;
                }
            }
            __builtin_amdgcn_s_setprio(0);
            const R f = fx.value(a);
            if (traced) {
                double *r = a.trace + ((t - a.t0) * (uint64_t)a.p + k) * rec;
                r[3 * D] = (double)J;
                r[3 * D + 1] = (double)f;
            }
            // f J, not f alone: in FP32 evaluation the Jacobian can overflow
            const double Fv = (double)f * (double)J;
            bad |= !isfinite(Fv);
            return Fv * a.inv;
        };
        // shifted sums in sample order
        // (for k == 0 the deviation is exactly +0 and leaves S1 = S2 = +0)
        auto accumulate = [&](int k, double Ik) {
            if (k == 0) I0 = Ik;
            const double dev = Ik - I0;
            S1 = S1 + dev;
            S2 = __fma_rn(dev, dev, S2);
        };
        auto add_bins = [&](const int (&bin)[D], double Ik) {
            if (a.hist) {
                const double sq = Ik * Ik;
                const int axes = a.one_d ? 1 : D;
#pragma unroll
                for (int j = 0; j < D; ++j)
                    if (j < axes) atomicAdd(&sH[j * nb + bin[j]], sq);
            }
        };
        {
            // both points (grid reads included) before either sample's histogram
            // atomics, so that the two evaluations can interleave
            int k = 0;
            for (; k + 1 < a.p; k += 2) {
                int bin0[D], bin1[D];
                const double Ia = point(k, bin0);
                const double Ib = point(k + 1, bin1);
                accumulate(k, Ia);
                accumulate(k + 1, Ib);
                add_bins(bin0, Ia);
                add_bins(bin1, Ib);
            }
            if (k < a.p) {
                int bin0[D];
                const double Ia = point(k, bin0);
                accumulate(k, Ia);
                add_bins(bin0, Ia);
            }
        }
    } else {
        // the same steps one sample at a time, written out in the loop: the
        // batched kernel, which inlines every case, allocates fewer registers
        // for this form than for the lambda one
        for (int k = 0; k < a.p; ++k) {
            // PRIO: the wave runs at raised priority from the start of a
            // sample until its integrand value.  s_setprio only orders issue
            // among the waves of a SIMD; favouring the waves that are still on
            // their way to their grid reads and table loads puts more of them
            // in flight while the others compute.  Taken with the two phases
            // (FP64 table and Gaussian kernels 2-5% faster), where phase 1
            // runs a level higher still (another 0.3-1.2%), and in the
            // batched kernel (FP32-eval 1%); the one-phase single-integral
            // kernels of this path, FP64 corner peak and FP32-eval tables at
            // d = 6, gained nothing or lost up to 2%.
            if constexpr (PRIO) __builtin_amdgcn_s_setprio(GF ? 2 : 1);
            uint32_t w[4 * NUSED];
#pragma unroll
            for (int b = 0; b < NUSED; ++b) {
                uint32_t x0 = (uint32_t)(k * NBLK + b), x1 = a.iter, x2 = tlo, x3 = thi;
                philox4x32_10(x0, x1, x2, x3, k0, k1);
                w[4 * b] = x0;
                w[4 * b + 1] = x1;
                w[4 * b + 2] = x2;
                w[4 * b + 3] = x3;
            }
            Integrand<F, D, R, EARLY> fx(a.tables);
            int bin[D];
            R J = R(1);
            // GF: every axis's bin and grid read first, then the rest axis by
            // axis, so that the grid reads are in flight together rather
            // than each waited for before the next is issued (see kGridFirst)
            R gf_frac[GF ? D : 1], gf_left[GF ? D : 1], gf_right[GF ? D : 1];
            int gf_bin[GF ? D : 1];
            if constexpr (GF) {
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    R uj;
                    if constexpr (F32) uj = uniform24(w[j]);
                    else uj = uniform53(w[j], w[D + j]);
                    const R z = (cd[j] + uj) * s;
                    const R fz = rmin(rfloor(z), last);
                    gf_bin[j] = (int)fz;
                    gf_frac[j] = rmin(z - fz, R(1));
                    if constexpr (F32) {
                        const float2 cell = reinterpret_cast<const float2 *>(sG)[j * nb + gf_bin[j]];
                        gf_left[j] = cell.x;
                        gf_right[j] = cell.y;  // FP32-eval grids hold the width here
                    } else {
                        const R *B = sG + j * row + gf_bin[j];
                        gf_left[j] = B[0];
                        gf_right[j] = B[1];
                    }
                }
                __builtin_amdgcn_sched_barrier(0);  // keep the reads ahead of their uses
                if constexpr (PRIO) __builtin_amdgcn_s_setprio(1);
            }
#pragma unroll
            for (int j = 0; j < D; ++j) {
                R u = R(0), frac, left, width;
                int i;
                if constexpr (GF) {
                    if (traced) {
                        if constexpr (F32) u = uniform24(w[j]);
                        else u = uniform53(w[j], w[D + j]);
                    }
                    i = gf_bin[j];
                    frac = gf_frac[j];
                    left = gf_left[j];
                    if constexpr (F32) width = gf_right[j];
                    else width = gf_right[j] - left;
                } else {
                    if constexpr (F32) u = uniform24(w[j]);
                    else u = uniform53(w[j], w[D + j]);
                    const R z = (cd[j] + u) * s;
                    // bin index, clamped to the last bin with fraction 1 there: once
                    // floor(z) > nb-1 we have z >= nb, so z - (nb-1) >= 1 and the min
                    // gives exactly 1; otherwise z - floor(z) < 1 is exact.
                    const R fz = rmin(rfloor(z), last);
                    i = (int)fz;
                    frac = rmin(z - fz, R(1));
                    if constexpr (F32) {
                        const float2 cell = reinterpret_cast<const float2 *>(sG)[j * nb + i];
                        left = cell.x;
                        width = cell.y;
                    } else {
                        const R *B = sG + j * row + i;
                        left = B[0];
                        width = B[1] - left;
                    }
                }
                const R xu = rfma(frac, width, left);
                const auto cj = axis_consts<kBatchConsts>(sC, j);
                R xj;
                if constexpr (LOV)
                    xj = rfma(cj[1], xu, lov[j]);
                else
                    xj = rfma(cj[1], xu, cj[0]);
                J = J * (width * cj[2]);
                bin[j] = i;
                fx.axis(j, xj, cj);
                if (traced) {
                    double *r = a.trace + ((t - a.t0) * (uint64_t)a.p + k) * rec;
                    r[j] = (double)u;
                    r[D + j] = (double)i;
                    r[2 * D + j] = (double)xj;
                }
            }
            if constexpr (PRIO) __builtin_amdgcn_s_setprio(0);
            const R f = fx.value(a);
            const double Fv = (double)f * (double)J;
            bad |= !isfinite(Fv);
            const double Ik = Fv * a.inv;
            if (k == 0) I0 = Ik;
            {
                const double dev = Ik - I0;  // exactly +0 for k == 0: S1, S2 stay +0
                S1 = S1 + dev;
                S2 = __fma_rn(dev, dev, S2);
            }
            if (a.hist) {
                const double sq = Ik * Ik;
                const int axes = a.one_d ? 1 : D;
#pragma unroll
                for (int j = 0; j < D; ++j)
                    if (j < axes) atomicAdd(&sH[j * nb + bin[j]], sq);
            }
            if (traced) {
                double *r = a.trace + ((t - a.t0) * (uint64_t)a.p + k) * rec;
                r[3 * D] = (double)J;
                r[3 * D + 1] = (double)f;
            }
        }
    }
    It = __fma_rn(a.pd, I0, S1);
    const double num = __fma_rn(-S1, S1, a.pd * S2);
    vt = num * a.inv_pm1;
    if (vt < 0.0) vt = 0.0;
    if (traced) {
        double *r = a.trace + (uint64_t)(a.t1 - a.t0) * (uint64_t)a.p * rec + (t - a.t0) * 2;
        r[0] = It;
        r[1] = vt;
    }
}

// dig += step digit by digit in base g (the carry out of the top digit is
// dropped: the caller's cube index tells whether the lane is done).
template <int D>
__device__ __forceinline__ void odometer_add(uint32_t (&dig)[D], const int32_t *step, uint32_t g) {
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const uint32_t v = dig[j] + (uint32_t)step[j] + carry;  // < 2g + 1 <= 2^31 + 1
        carry = v >= g ? 1u : 0u;
        dig[j] = carry ? v - g : v;
    }
}

template <int D>
__device__ __forceinline__ void digits_of(uint64_t t, uint32_t g, uint32_t (&dig)[D]) {
#pragma unroll
    for (int j = 0; j < D; ++j) {
        dig[j] = (uint32_t)(t % (uint64_t)g);
        t /= (uint64_t)g;
    }
}

// Workgroup reduction of the lanes' compensated (I, var) sums: a butterfly in
// each wavefront, then the wavefronts in order.  Thread 0 writes the four
// doubles (sum and compensation of I and var) to out and raises *flag if any
// lane saw a non-finite integrand value.  Ends with a workgroup barrier.
__device__ __forceinline__ void block_totals(double sI, double cI, double sV, double cV, bool bad,
                                             double *out, uint32_t *flag) {
    __shared__ double wave_tot[kMaxBlock / 64][4];
    __shared__ uint32_t wave_bad;
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (tid == 0) wave_bad = 0u;
    __syncthreads();
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double s2 = __shfl_xor(sI, off, 64), c2 = __shfl_xor(cI, off, 64);
        const double v2 = __shfl_xor(sV, off, 64), e2 = __shfl_xor(cV, off, 64);
        two_sum_merge(sI, cI, s2, c2);
        two_sum_merge(sV, cV, v2, e2);
    }
    const int wave = tid >> 6;
    if ((tid & 63) == 0) {
        wave_tot[wave][0] = sI;
        wave_tot[wave][1] = cI;
        wave_tot[wave][2] = sV;
        wave_tot[wave][3] = cV;
    }
    if (__any(bad) && (tid & 63) == 0) atomicOr(&wave_bad, 1u);
    __syncthreads();
    if (tid == 0) {
        double s0 = wave_tot[0][0], c0 = wave_tot[0][1], v0 = wave_tot[0][2], e0 = wave_tot[0][3];
        for (int wv = 1; wv < nthr / 64; ++wv) {
            two_sum_merge(s0, c0, wave_tot[wv][0], wave_tot[wv][1]);
            two_sum_merge(v0, e0, wave_tot[wv][2], wave_tot[wv][3]);
        }
        out[0] = s0;
        out[1] = c0;
        out[2] = v0;
        out[3] = e0;
        if (wave_bad) atomicOr(flag, 1u);
    }
    __syncthreads();
}

// ---------------------------------------------------------------- the kernel

// One integral: persistent workgroups stride through all m sub-cubes.
// TRACE instantiations additionally write per-sample and per-cube records for
// the sub-cubes [t0, t1); F32 instantiations evaluate the map and the
// integrand in single precision.  Everything from I_k on is FP64 in both.
template <int F, int D, bool TRACE, bool F32>
__global__ void __launch_bounds__(kMaxBlock)
    __attribute__((amdgpu_waves_per_eu(kFixedWaves<F, D, TRACE, F32> ? kFixedWaves<F, D, TRACE, F32> : 1,
                                       kFixedWaves<F, D, TRACE, F32> ? kFixedWaves<F, D, TRACE, F32> : 8)))
    vsample_kernel(const SampleArgs a) {
    if (a.run_last && (int64_t)a.iter > (int64_t)*a.run_last) return;  // the run has ended
    extern __shared__ double lds[];
    const LdsView<F32> v(lds, D, a.nb);
    load_lds<D, F32>(a, v);
    __syncthreads();
    // the per-axis constants are the same for every lane: read them with
    // scalar loads (constant address space) rather than from LDS, whose
    // bandwidth the grid reads and histogram atomics need.  volatile makes
    // the compiler load each where it is used instead of holding all of them
    // in scalar registers, which spilled them to VGPR lanes and cost a VALU
    // read-back per use.
    volatile Const<real_t<F32>> *sC = (volatile Const<real_t<F32>> *)a.consts;

    uint64_t t = (uint64_t)blockIdx.x * (uint64_t)blockDim.x + (uint64_t)threadIdx.x;
    uint32_t dig[D];
    digits_of<D>(t, (uint32_t)a.g, dig);
    double sI = 0.0, cI = 0.0, sV = 0.0, cV = 0.0;
    bool bad = false;
    // the lower bounds, copied once into vector registers (the empty asm keeps
    // the copies there rather than reloading them as scalars)
    real_t<F32> lov[D];
    if constexpr (kLowInVgpr<F, D, F32>) {
#pragma unroll
        for (int j = 0; j < D; ++j) {
            lov[j] = sC[kConstStride * j];
            asm volatile("" : "+v"(lov[j]));
        }
    }
    while (t < (uint64_t)a.m) {
        double It, vt;
        cube_pass<F, D, TRACE, F32, kPairSamples<F, D, F32>, true, kLowInVgpr<F, D, F32>,
                  kGridFirst<F, D, F32>, kGridFirst<F, D, F32>>(
            a, v, sC, t, dig, It, vt, bad, lov);
        two_sum_add(sI, cI, It);
        two_sum_add(sV, cV, vt);
        // next sub-cube of this lane: t += stride, digit by digit
        t += (uint64_t)a.stride;
        odometer_add<D>(dig, a.sdig, (uint32_t)a.g);
    }
    block_totals(sI, cI, sV, cV, bad, a.partials + 4 * (size_t)blockIdx.x, a.flag);
    if (a.hist) {
        // into accumulator blockIdx % kHistAcc (ordinary device memory, so the
        // hardware FP64 atomic add applies); bins it never reached are skipped
        const int n = D * a.nb;
        double *acc = a.hist_acc + (size_t)(blockIdx.x % kHistAcc) * a.hist_stride;
        for (int i = threadIdx.x; i < n; i += blockDim.x) {
            const double h = a.hist_copies > 1 ? v.hist[i] + v.hist[n + i] : v.hist[i];
            if (h != 0.0) unsafeAtomicAdd(acc + i, h);
        }
    }
}

template <int F, int D>
hipError_t launch_sample_fd(int blocks, int threads, size_t lds_bytes, hipStream_t stream,
                            const SampleArgs &args) {
    const dim3 grid(blocks), block(threads);
    if (args.fp32) {
        if (args.trace)
            hipLaunchKernelGGL((vsample_kernel<F, D, true, true>), grid, block, lds_bytes, stream, args);
        else
            hipLaunchKernelGGL((vsample_kernel<F, D, false, true>), grid, block, lds_bytes, stream, args);
    } else {
        if (args.trace)
            hipLaunchKernelGGL((vsample_kernel<F, D, true, false>), grid, block, lds_bytes, stream, args);
        else
            hipLaunchKernelGGL((vsample_kernel<F, D, false, false>), grid, block, lds_bytes, stream, args);
    }
    return hipGetLastError();
}

}  // namespace mcubes
