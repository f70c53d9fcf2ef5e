// Weighted-Estimates and Check-Convergence (Alg. 2), written once for the
// host driver and for the batched engine's device-side decision, so that both
// decide from the same iteration results with the same roundings (the
// library is built without floating-point contraction; division and square
// root are correctly rounded on both sides).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "mcubes.h"

namespace mcubes {

// Inverse-variance weighted mean of k iteration results, its standard
// deviation and chi^2 per degree of freedom: out = [mean, sigma, chi2/dof].
// Iterations with I = 0 and var = 0 saw no non-zero sample and carry no
// information, so they take no part; among the others an exact iteration
// (var = 0) decides the mean alone; with none left the result is 0 with an
// infinite standard deviation.
__host__ __device__ inline void weighted_estimate(int k, const double *I, const double *var,
                                                  double *out) {
    int used = 0, exact = 0;
    double exact_sum = 0.0;
    for (int i = 0; i < k; ++i) {
        if (var[i] == 0.0 && I[i] == 0.0) continue;
        ++used;
        if (var[i] == 0.0) {
            ++exact;
            exact_sum = exact_sum + I[i];
        }
    }
    if (used == 0) {
        out[0] = 0.0;
        out[1] = INFINITY;
        out[2] = NAN;
        return;
    }
    if (exact) {
        out[0] = exact_sum / (double)exact;
        out[1] = 0.0;
        out[2] = used > 1 ? 0.0 : NAN;
        return;
    }
    double wsum = 0.0, wisum = 0.0;
    for (int i = 0; i < k; ++i) {
        if (var[i] == 0.0) continue;
        const double w = 1.0 / var[i];
        wsum = wsum + w;
        wisum = wisum + w * I[i];
    }
    const double mean = wisum / wsum;
    double chi = 0.0;
    for (int i = 0; i < k; ++i) {
        if (var[i] == 0.0) continue;
        const double dv = I[i] - mean;
        chi = chi + (dv * dv) / var[i];
    }
    out[0] = mean;
    out[1] = 1.0 / sqrt(wsum);
    out[2] = used > 1 ? chi / (double)(used - 1) : NAN;
}

// Check-Convergence with the chi^2 condition of Sec. V: k >= 2 iterations,
// est[1] <= tau_rel |est[0]| and chi^2/dof within chi2_max (0: the default
// bound, negative: not checked).
__host__ __device__ inline bool converged_after(int k, const double *est, double tau_rel,
                                                double chi2_max) {
    if (k < 2 || !(tau_rel > 0.0)) return false;
    if (!(est[1] <= tau_rel * fabs(est[0]))) return false;
    if (chi2_max < 0.0) return true;
    const double bound = chi2_max > 0.0 ? chi2_max : MC_CHI2_DOF_DEFAULT;
    return est[2] <= bound;  // false for NaN (fewer than two informative iterations)
}

}  // namespace mcubes
