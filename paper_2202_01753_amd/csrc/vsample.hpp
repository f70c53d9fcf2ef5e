// V-Sample / V-Sample-No-Adjust (Alg. 3) for gfx950: the per-iteration
// sampling pass of m-Cubes.
//
// Work mapping: one lane per sub-cube at a time, persistent workgroups that
// stride through the g^d sub-cubes.  Because every random number is keyed by
// (seed; iteration, sub-cube, sample) rather than by thread, the mapping of
// sub-cubes to lanes does not change any sample point.
//
// Per sample (all FP64, no implicit contraction; fma only where written):
//   Philox4x32-10 blocks -> 52-bit uniforms -> stratified coordinate in bins
//   -> bin index, boundary and width from the LDS copy of the grid -> point
//   and Jacobian -> integrand -> I_k = f J / (m p) -> shifted per-cube sums
//   -> (V-Sample only) I_k^2 added to one LDS bin per axis.
// Per sub-cube: I_t and the unbiased variance estimate, accumulated per lane
// with error-free transformations.  Per workgroup: a fixed-order wave and
// workgroup reduction, then the totals and the LDS histogram go to this
// workgroup's slot of the partials array for the finalize kernel.
#pragma once

#include "internal.hpp"

namespace mcubes {

// ---------------------------------------------------------------- Philox4x32-10
// Salmon et al., SC'11: ten rounds of two 32x32->64 products, with the key
// advanced by the Weyl constants between rounds.  The key is uniform across
// the wavefront, so its schedule stays in scalar registers.
__device__ __forceinline__ void philox4x32_10(uint32_t &x0, uint32_t &x1, uint32_t &x2,
                                              uint32_t &x3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa = (uint64_t)0xD2511F53u * (uint64_t)x0;
        const uint64_t pb = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        const uint32_t y0 = (uint32_t)(pb >> 32) ^ x1 ^ k0;
        const uint32_t y2 = (uint32_t)(pa >> 32) ^ x3 ^ k1;
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
    const uint32_t hi = 0x3FF00000u | (whi >> 12);
    const uint32_t lo = (whi << 20) | (wlo >> 12);
    return __hiloint2double((int)hi, (int)lo) - 0x1.fffffffffffffp-1;
}

// ---------------------------------------------------------------- integrands

__device__ __forceinline__ double lerp(double a, double b, double t) {
    return __fma_rn(t, b - a, a);
}

// Bilinear interpolation in one 256x256 table, node (a,b) at (a/255, b/255),
// the edge cell extended outside the unit square.
__device__ __forceinline__ double bilinear(const double *__restrict__ T, double x, double y) {
    const double ux = x * 255.0, uy = y * 255.0;
    const double fa = fmin(fmax(floor(ux), 0.0), 254.0);
    const double fb = fmin(fmax(floor(uy), 0.0), 254.0);
    const double tx = ux - fa, ty = uy - fb;
    const int cell = (int)fa * kTableN + (int)fb;
    const double t00 = T[cell];
    const double t01 = T[cell + 1];
    const double t10 = T[cell + kTableN];
    const double t11 = T[cell + kTableN + 1];
    return lerp(lerp(t00, t10, tx), lerp(t01, t11, tx), ty);
}

template <int D>
__device__ __forceinline__ double gauss_product(const double *sC, const double (&x)[D]) {
    double acc = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        const double t = (x[j] - sC[kConstStride * j + 3]) * sC[kConstStride * j + 4];
        acc = __fma_rn(t, t, acc);
    }
    return exp(-acc);
}

// S^(D+1) by left-to-right binary powering, then one correctly rounded division.
template <int D>
__device__ __forceinline__ double corner_peak(const double *sC, const double (&x)[D]) {
    double S = 1.0;
#pragma unroll
    for (int j = 0; j < D; ++j) S = __fma_rn(sC[kConstStride * j + 3], x[j], S);
    constexpr unsigned e = (unsigned)(D + 1);
    constexpr int top = 31 - __builtin_clz(e);
    double pw = S;
#pragma unroll
    for (int bit = top - 1; bit >= 0; --bit) {
        pw = pw * pw;
        if ((e >> bit) & 1u) pw = pw * S;
    }
    return 1.0 / pw;
}

template <int F, int D>
__device__ __forceinline__ double integrand(const SampleArgs &a, const double *sC,
                                            const double (&x)[D]) {
    if constexpr (F == 0) {
        return a.cval;
    } else if constexpr (F == 1) {
        return gauss_product<D>(sC, x);
    } else if constexpr (F == 2) {
        return corner_peak<D>(sC, x);
    } else {
        static_assert(D >= 4, "table integrand needs four axes");
        const double G = gauss_product<D>(sC, x);
        const double T1 = bilinear(a.tables, x[0], x[1]);
        const double T2 = bilinear(a.tables + kTableN * kTableN, x[2], x[3]);
        return (G * T1) * T2;
    }
}

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

// ---------------------------------------------------------------- the kernel

// TRACE instantiations additionally write per-sample and per-cube records for
// the sub-cubes [t0, t1); everything else is the same code.
template <int F, int D, bool TRACE>
__global__ void __launch_bounds__(kMaxBlock) vsample_kernel(const SampleArgs a) {
    extern __shared__ double lds[];
    __shared__ double wave_tot[kMaxBlock / 64][4];
    __shared__ uint32_t wave_bad;

    const int nb = a.nb;
    const int row = nb + 1;
    double *sC = lds;                       // D blocks of per-axis constants
    double *sB = lds + kConstStride * D;    // D rows of nb+1 boundaries
    double *sH = sB + D * row;              // D rows of nb bin contributions
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;

    for (int i = tid; i < kConstStride * D; i += nthr) sC[i] = a.consts[i];
    for (int i = tid; i < D * row; i += nthr) sB[i] = a.grid[i];
    if (a.hist)
        for (int i = tid; i < D * nb; i += nthr) sH[i] = 0.0;
    if (tid == 0) wave_bad = 0u;
    __syncthreads();

    constexpr int NBLK = (D + 1) / 2;
    const uint32_t k0 = (uint32_t)a.seed, k1 = (uint32_t)(a.seed >> 32);
    const uint32_t g = (uint32_t)a.g;

    uint64_t t = (uint64_t)blockIdx.x * (uint64_t)nthr + (uint64_t)tid;
    uint32_t dig[D];
    {
        uint64_t rest = t;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            dig[j] = (uint32_t)(rest % (uint64_t)g);
            rest /= (uint64_t)g;
        }
    }

    double sI = 0.0, cI = 0.0, sV = 0.0, cV = 0.0;
    bool bad = false;
    const int rec = 3 * D + 2;

    while (t < (uint64_t)a.m) {
        double cd[D];
#pragma unroll
        for (int j = 0; j < D; ++j) cd[j] = (double)dig[j];
        const uint32_t tlo = (uint32_t)t, thi = (uint32_t)(t >> 32);
        const bool traced = TRACE && (int64_t)t >= a.t0 && (int64_t)t < a.t1;

        double I0 = 0.0, S1 = 0.0, S2 = 0.0;
        for (int k = 0; k < a.p; ++k) {
            uint32_t w[4 * NBLK];
#pragma unroll
            for (int b = 0; b < NBLK; ++b) {
                uint32_t x0 = (uint32_t)(k * NBLK + b), x1 = a.iter, x2 = tlo, x3 = thi;
                philox4x32_10(x0, x1, x2, x3, k0, k1);
                w[4 * b] = x0;
                w[4 * b + 1] = x1;
                w[4 * b + 2] = x2;
                w[4 * b + 3] = x3;
            }
            double x[D];
            int bin[D];
            double J = 1.0;
#pragma unroll
            for (int j = 0; j < D; ++j) {
                const double u = uniform53(w[j], w[D + j]);
                const double z = (cd[j] + u) * a.s;
                // bin index, clamped to the last bin with fraction 1 there: once
                // floor(z) > nb-1 we have z >= nb, so z - (nb-1) >= 1 and the min
                // gives exactly 1; otherwise z - floor(z) < 1 is exact.
                const double fz = fmin(floor(z), a.nb_minus1);
                const int i = (int)fz;
                const double frac = fmin(z - fz, 1.0);
                const double *B = sB + j * row + i;
                const double left = B[0];
                const double width = B[1] - left;
                const double xu = __fma_rn(frac, width, left);
                const double *cj = sC + kConstStride * j;
                x[j] = __fma_rn(cj[1], xu, cj[0]);
                J = J * (width * cj[2]);
                bin[j] = i;
                if (traced) {
                    double *r = a.trace + ((t - a.t0) * (uint64_t)a.p + k) * rec;
                    r[j] = u;
                    r[D + j] = (double)i;
                    r[2 * D + j] = x[j];
                }
            }
            const double f = integrand<F, D>(a, sC, x);
            bad |= !isfinite(f);
            const double Fv = f * J;
            const double Ik = Fv * a.inv;
            if (k == 0) {
                I0 = Ik;
            } else {
                const double dev = Ik - I0;
                S1 = S1 + dev;
                S2 = __fma_rn(dev, dev, S2);
            }
            if (a.hist) {
                const double sq = Ik * Ik;
#pragma unroll
                for (int j = 0; j < D; ++j) atomicAdd(&sH[j * nb + bin[j]], sq);
            }
            if (traced) {
                double *r = a.trace + ((t - a.t0) * (uint64_t)a.p + k) * rec;
                r[3 * D] = J;
                r[3 * D + 1] = f;
            }
        }
        const double It = __fma_rn(a.pd, I0, S1);
        const double num = __fma_rn(-S1, S1, a.pd * S2);
        double vt = num * a.inv_pm1;
        if (vt < 0.0) vt = 0.0;
        two_sum_add(sI, cI, It);
        two_sum_add(sV, cV, vt);
        if (traced) {
            double *r = a.trace + (uint64_t)(a.t1 - a.t0) * (uint64_t)a.p * rec + (t - a.t0) * 2;
            r[0] = It;
            r[1] = vt;
        }
        // next sub-cube of this lane: t += stride, digit by digit
        t += (uint64_t)a.stride;
        uint32_t carry = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const uint32_t v = dig[j] + (uint32_t)a.sdig[j] + carry;  // < 2g + 1 <= 2^31 + 1
            carry = v >= g ? 1u : 0u;
            dig[j] = carry ? v - g : v;
        }
    }

    // lane -> wave: butterfly with compensated merges (every lane ends equal)
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

    double *part = a.partials;
    if (tid == 0) {
        double s0 = wave_tot[0][0], c0 = wave_tot[0][1], v0 = wave_tot[0][2], e0 = wave_tot[0][3];
        for (int wv = 1; wv < nthr / 64; ++wv) {
            two_sum_merge(s0, c0, wave_tot[wv][0], wave_tot[wv][1]);
            two_sum_merge(v0, e0, wave_tot[wv][2], wave_tot[wv][3]);
        }
        double *o = part + 4 * (size_t)blockIdx.x;
        o[0] = s0;
        o[1] = c0;
        o[2] = v0;
        o[3] = e0;
        if (wave_bad) atomicOr(a.flag, 1u);
    }
    if (a.hist) {
        double *ph = part + 4 * (size_t)gridDim.x + (size_t)blockIdx.x * a.hist_stride;
        for (int i = tid; i < D * nb; i += nthr) ph[i] = sH[i];
    }
}

template <int F, int D>
hipError_t launch_sample_fd(int blocks, int threads, size_t lds_bytes, hipStream_t stream,
                            const SampleArgs &args) {
    if (args.trace)
        hipLaunchKernelGGL((vsample_kernel<F, D, true>), dim3(blocks), dim3(threads), lds_bytes,
                           stream, args);
    else
        hipLaunchKernelGGL((vsample_kernel<F, D, false>), dim3(blocks), dim3(threads), lds_bytes,
                           stream, args);
    return hipGetLastError();
}

}  // namespace mcubes
