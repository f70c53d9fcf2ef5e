// Internal interface between the host driver (mcubes_api.cpp) and the HIP
// kernels (vsample_*.hip, finalize.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mcubes {

constexpr int kMaxDim = 16;
constexpr int kTableN = 256;
constexpr int kMaxBlock = 1024;

// Everything the sampling kernel needs, passed by value so that the per-axis
// constants arrive in scalar registers.
struct SampleArgs {
    const double *grid;     // dim*(nb+1) boundaries, unit coordinates
    const double *tables;   // 2*256*256 (gauss-tables integrand) or nullptr
    double *partials;       // per workgroup: 4 totals, then (optional) dim*nb bins
    uint32_t *flag;         // set to nonzero when the integrand is not finite
    double *trace;          // optional per-sample / per-cube records
    int64_t m;              // sub-cubes
    int64_t t0, t1;         // traced sub-cube range
    int64_t stride;         // sub-cubes advanced per lane step (= grid size in threads)
    uint64_t seed;
    uint32_t iter;
    int32_t p;              // samples per sub-cube
    int32_t nb;             // bins per axis
    int32_t g;              // intervals per axis
    int32_t hist;           // nonzero: collect bin contributions (V-Sample)
    int32_t hist_stride;    // doubles between two workgroups' histograms in partials
    double s;               // nb / g
    double nb_minus1;       // nb - 1
    double inv;             // 1 / (m p)
    double pd;              // p
    double inv_pm1;         // 1 / (p - 1)
    double cval;            // constant integrand value
    const double *consts;   // kConstStride doubles per axis, see below
    int32_t sdig[kMaxDim];  // stride in base g, least significant digit first
};

// Per-axis constants, copied to LDS by every workgroup:
//   [0] lo   [1] span = hi - lo   [2] q = nb * span
//   [3] Gaussian centre or corner-peak coefficient   [4] Gaussian 1/width   [5] 0
constexpr int kConstStride = 6;

// Returns the sampling kernel for (integrand, dim) and its tracing variant, or nullptr.
const void *sample_kernel(int integrand, int dim, bool trace);

// Launches the sampling kernel; lds_bytes is the dynamic LDS size.
hipError_t launch_sample(int integrand, int dim, int blocks, int threads, size_t lds_bytes,
                         hipStream_t stream, const SampleArgs &args);

// Reduces per-workgroup partials in a fixed order into out = [I, var, flag, 0, hist...]
// and clears the flag.
hipError_t launch_finalize(const double *partials, int blocks, int nhist, int hist_stride,
                           int with_hist, uint32_t *flag, double *out, hipStream_t stream);

hipError_t launch_clear_flag(uint32_t *flag, hipStream_t stream);

}  // namespace mcubes
