// Internal interface between the host driver (mcubes_api.cpp) and the HIP
// kernels (vsample_*.hip, finalize.hip, steps.hip).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mcubes.h"

namespace mcubes {

constexpr int kMaxDim = 16;
constexpr int kTableN = 256;
constexpr int kMaxBlock = 1024;
constexpr int kBatchBlock = 256;     // threads per workgroup of the batched kernel (or twice that)
constexpr int kBatchMaxBlock = 512;
constexpr int kBatchMaxDim = 10;     // dimensions the batched kernel supports

// Everything the sampling kernel needs, passed by value so that the per-axis
// constants arrive in scalar registers.
struct SampleArgs {
    const double *grid;     // dim*(nb+1) boundaries, unit coordinates
    const void *tables;     // the two tables in the device layout of the evaluation precision
                            // (see table_cell), or nullptr
    double *partials;       // per workgroup 4 totals
    double *hist_acc;       // kHistAcc histogram accumulators, hist_stride doubles apart
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
    int32_t hist_stride;    // doubles between two histogram accumulators
    int32_t kind;           // integrand id * 32 + dim (dispatch in the batched kernel)
    int32_t one_d;          // nonzero: collect bin contributions of the first axis only
    int32_t hist_copies;    // LDS histogram copies: 2 = lanes 32-63 of a wave add into a second
    double s;               // nb / g
    float s32;              // nb / g rounded to float (FP32 evaluation)
    int32_t fp32;           // nonzero: FP32 evaluation
    double inv;             // 1 / (m p)
    double pd;              // p
    double inv_pm1;         // 1 / (p - 1)
    double cval;            // constant integrand value
    const void *consts;     // kConstStride values of the evaluation precision per axis
    const int32_t *run_last;  // nullptr, or the last iteration of a run whose steps run on the
                              // device: a pass with iter beyond it does nothing
    int32_t sdig[kMaxDim];  // stride in base g, least significant digit first
};

// Per-axis constants, in device memory (the kernels read them with scalar loads):
//   [0] lo   [1] span = hi - lo   [2] q = nb * span
//   [3] Gaussian centre or corner-peak coefficient   [4] Gaussian 1/width   [5] 0
constexpr int kConstStride = 6;

// Returns the sampling kernel for (integrand, dim, trace, FP32 evaluation), or nullptr.
const void *sample_kernel(int integrand, int dim, bool trace, bool fp32);

// Launches the sampling kernel; lds_bytes is the dynamic LDS size.
hipError_t launch_sample(int integrand, int dim, int blocks, int threads, size_t lds_bytes,
                         hipStream_t stream, const SampleArgs &args);

// Histogram accumulators of a V-Sample pass (a region of their own, so that
// the totals of a pass with more workgroups never reach them): workgroup b
// adds its LDS histogram into accumulator b % kHistAcc with device-scope
// FP64 atomics.  Eight copies cut the atomics that meet on one address
// eightfold (workgroups are dispatched round-robin over the chip's eight
// XCDs, so the copies also split by XCD); they are summed in order after the
// pass, by the finalize or by the steps kernel.
constexpr int kHistAcc = 8;

// Reduces the per-workgroup totals in a fixed order and sums the histogram
// accumulators in order into out = [I, var, flag, 0, hist...]; clears the
// accumulators (for the next pass) and the flag.  (Runs whose steps between
// passes are on the host.)
hipError_t launch_finalize(const double *partials, double *hist_acc, int blocks, int nhist, int hist_stride,
                           int with_hist, uint32_t *flag, double *out, hipStream_t stream);

// A run whose steps between sampling passes (Weighted-Estimates,
// Check-Convergence, Adjust-Bin-Bounds of Alg. 2) run on the device: its
// state in the workspace, mirrored after every pass into page-locked host
// memory that the host reads once the pass is over.  last is the index of
// the run's last iteration: itmax - 1 until a pass ends the run earlier
// (converged, or a non-finite value); every kernel of a later pass then does
// nothing.
struct RunState {
    int32_t last;
    int32_t status;   // kRunGoing, kRunConverged or kRunNonFinite
    int32_t k;        // passes finished
    int32_t pad;
    double est[3];    // weighted estimate, its standard deviation, chi^2/dof after k passes
    double pad2;
};
constexpr int32_t kRunGoing = 0, kRunConverged = 1, kRunNonFinite = 2;

// The decision after pass it of such a run.  iters holds I_0 .. I_{itmax-1},
// then var_0 .. var_{itmax-1}, on the device; host_iters the same in the host
// mirror (host, host_iters: mapped page-locked memory).
struct RunCtl {
    RunState *state;
    double *iters;
    RunState *host;
    double *host_iters;
    int32_t it, itmax;
    double tau_rel, chi2_max;
};

// Start of a device-steps run: the state (last = itmax - 1, nothing done) and
// Init-Bins (boundaries i/nb on every axis) in the workspace, and in
// host_grid (mapped host memory) unless it is null.
hipError_t launch_run_init(RunState *state, double *grid, double *host_grid, int d, int nb, int itmax,
                           hipStream_t stream);

// Everything between pass ctl.it and the next of a device-steps run, one
// launch: the totals merged and the decision taken (ctl), and in an
// adjusting pass (nref = d, or 1 for m-Cubes1D; 0 otherwise) the grid
// adjusted from the histogram accumulators, one workgroup per axis.
struct StepsArgs {
    RunCtl ctl;
    const double *partials;   // the pass's per-workgroup totals
    int32_t blocks;           // workgroups of the pass
    int32_t hist_stride;
    double *hist_acc;         // kHistAcc accumulators (cleared as they are read)
    uint32_t *flag;           // non-finite flag (read and cleared)
    double *grid;             // d*(nb+1) boundaries, adjusted in place
    double *host_grid;        // mapped host copy of the boundaries, or null
    double alpha;
    int32_t d, nb, one_d, nref;
};
hipError_t launch_steps(const StepsArgs &args, hipStream_t stream);

// Adjust-Bin-Bounds on the device (mc_refine_grid_device): one workgroup per
// axis (m-Cubes1D: axis 0, then copied to every axis), the host's steps with
// sums in a fixed order of its own and the device library's pow and log: the
// host's result to rounding.  Reads the histogram hist (d*nb), rewrites grid
// in place.
hipError_t launch_refine(double *grid, const double *hist, int d, int nb, int one_d, double alpha,
                         hipStream_t stream);
// LDS of one adjusting workgroup, and the largest nb it takes.
size_t refine_lds_bytes(int nb);
constexpr int kDeviceStepsMaxBins = MC_DEVICE_STEPS_MAX_BINS;

// Zeroes n doubles (the histogram accumulators, before a workspace's first pass).
hipError_t launch_zero(double *p, size_t n, hipStream_t stream);

hipError_t launch_clear_flag(uint32_t *flag, hipStream_t stream);

// ---- batched sampling: many integrals in one persistent launch ----

// One integral of a batch.  a carries its constants, grid and table pointers,
// lattice, iteration and whether this pass collects bin contributions (its
// trace, partials and stride fields are unused).  out holds [I, var, flag, 0,
// d*nb bin contributions] of the integral's latest pass: the segments add
// their bin contributions into it (zero at admission and after every bin
// adjustment); when refine is set, the grid is adjusted on the device from
// that histogram after the pass.
//
// Each integral also keeps on the device the results of all its iterations
// (iters: I_0.. I_{itmax-1}, then var_0 .. var_{itmax-1}) and a state word:
// the merge kernel runs Weighted-Estimates and Check-Convergence after every
// pass and sets the state once the integral stops (converged, out of
// iterations, or a non-finite value).  Later steps may still list it (the
// host learns of the stop one step later); its segments then do no work.
struct BatchItem {
    SampleArgs a;
    double *grid;       // the integral's grid (a.grid, writable)
    double *out;
    double *iters;      // 2 * itmax doubles
    uint32_t *state;    // kItemRunning until the integral stops
    double alpha;
    double tau_rel;     // Check-Convergence: target relative error (0: never converged)
    double chi2_max;    //   and bound on chi^2/dof (0: default, negative: unchecked)
    int32_t itmax;
    int32_t refine;
};

// Item states, and the merge kernel's per-step results (kResStride doubles
// per listed integral: I, var, non-finite flag, weighted estimate, its
// standard deviation, chi^2/dof, state after the pass or kResSkipped, 1 if
// converged).
constexpr uint32_t kItemRunning = 0, kItemDone = 1, kItemFailed = 2;
constexpr int kResStride = 8;
constexpr double kResSkipped = -1.0;

// A contiguous range of one integral's sub-cubes, processed by one workgroup.
struct BatchSegment {
    int32_t item;       // integral (index into the items array)
    int32_t pad;
    int64_t t0, t1;     // sub-cubes [t0, t1)
};

// The device arrays of one batched step.  An integral's segments are
// contiguous, [item_first[i], item_first[i+1]).  The workgroups of one
// launch take the segments order[lo], order[lo+1], ... one at a time from the
// launch's counter *queue (zero before the step) until it reaches hi.
struct BatchArgs {
    const BatchItem *items;
    const BatchSegment *segs;
    const int32_t *order;
    const int32_t *item_first;
    double *seg_tot;          // 4 doubles per segment
    uint32_t *flags;          // per item, zero before the step
    double *res;              // per item: kResStride doubles (packed for one read-back)
    uint32_t *queue;          // this launch's segment counter
    int32_t lo, hi;           // this launch's range of order
    int32_t n_items;
};

// Admission of one integral into a batch: its per-axis constants are copied
// from the step's upload into its block, its starting grid (Init-Bins,
// uniform boundaries i/nb on every axis) is written there and its output
// (totals and bin contributions) is cleared.
struct AdmitRecord {
    char *consts;         // destination of the constants in the integral's block
    double *grid;         // destination of the d*(nb+1) starting boundaries
    double *out;          // the integral's 4 + d*nb output doubles
    uint32_t *state;      // the integral's state word (set to kItemRunning)
    int64_t src;          // byte offset of the constants in the upload (4-byte aligned)
    int32_t const_words;  // 4-byte words of constants
    int32_t dim, nb, pad;
};
hipError_t launch_admit(const AdmitRecord *recs, int n, const char *upload, hipStream_t stream);

// Launches the batched sampling kernel of one precision and integrand family
// (tables: the Gaussian-times-tables integrand; otherwise the closed-form
// ones) over the segments order[args.lo .. args.hi) (args.queue is this
// launch's counter).  threads is kBatchBlock or kBatchMaxBlock.
hipError_t launch_batch(bool fp32, bool tables, int blocks, int threads, size_t lds_bytes,
                        hipStream_t stream, const BatchArgs &args);
const void *batch_kernel(bool fp32, bool tables);
// Merges every running integral's segment totals in order into its out and
// res, clears its flag, appends (I, var) to its iterations and decides
// whether it stops (Weighted-Estimates, Check-Convergence, itmax).
hipError_t launch_batch_finalize(const BatchArgs &args, hipStream_t stream);
// Adjust-Bin-Bounds on the device for n_axes (integral, axis) pairs
// (axis_item[2a], axis_item[2a+1]): reads the integral's histogram row from its
// out (and clears it for the next collecting pass) and its boundaries from
// a.grid, writes the new ones to next_grid[integral].
hipError_t launch_batch_refine(const BatchItem *items, const int32_t *axis_item,
                               double *const *next_grid, int n_axes, int max_nb,
                               hipStream_t stream);
const void *batch_refine_symbol();

}  // namespace mcubes
