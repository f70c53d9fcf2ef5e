/*
 * mcubes.h - C ABI of the MI355X (gfx950) m-Cubes VEGAS integrator.
 *
 * The library implements the method of Sakiotis et al., "m-Cubes: An
 * Efficient and Portable Implementation of Multi-Dimensional Integration for
 * GPUs" (arXiv 2202.01753): the m-Cubes driver (Alg. 2) on the host and the
 * V-Sample / V-Sample-No-Adjust sampling pass (Alg. 3, Sec. IV) as HIP kernels.
 *
 * Conventions for every entry point:
 *   - All functions return an mc_status; nothing else crosses the boundary on
 *     error, and output arguments are left untouched when the status is not
 *     MC_OK.
 *   - "host" pointers are ordinary CPU memory, borrowed for the duration of
 *     the call (the library copies what it keeps).  "device" pointers are
 *     GPU memory on the current HIP device, owned by the caller.
 *   - The library never allocates device memory: the caller provides a
 *     workspace of at least mc_workspace_bytes() bytes.  Streams are
 *     hipStream_t values passed as void* (NULL = the default stream).
 *   - Calls are reentrant across distinct workspaces; two calls that share a
 *     workspace must not overlap.
 *   - Integration domains are boxes [lo_j, hi_j]; the adaptive grid lives in
 *     unit coordinates and is d rows of nbins+1 boundaries (row j = axis j,
 *     boundary 0 is 0.0 and boundary nbins is 1.0).
 */
#ifndef MCUBES_H
#define MCUBES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mc_status;
#define MC_OK 0
#define MC_EINVAL 1      /* invalid problem or argument; checked before any device work */
#define MC_EWORKSPACE 2  /* workspace smaller than mc_workspace_bytes() */
#define MC_ENONFINITE 3  /* the integrand produced a NaN or an infinity */
#define MC_EDEVICE 4     /* a HIP runtime error (no device, launch failure, ...) */

/* Integrand ids.  Parameter layouts (n_params doubles):
 *   MC_F_CONST          [v]                   f = v
 *   MC_F_GAUSS_PRODUCT  [c_1..c_d, w_1..w_d]  f = exp(-sum_j ((x_j - c_j)/w_j)^2)
 *   MC_F_CORNER_PEAK    [a_1..a_d]            f = (1 + sum_j a_j x_j)^-(d+1)
 *   MC_F_GAUSS_TABLES   [c_1..c_d, w_1..w_d]  f = gauss_product * T1(x_1,x_2) * T2(x_3,x_4)
 * The last one needs d >= 4 and two 256x256 row-major FP64 tables (n_tables =
 * 131072), node (a,b) at (a/255, b/255), bilinear inside a cell and extended
 * from the edge cell outside the unit square.  The Gaussian and corner-peak
 * forms are the product-peak / Gaussian and corner-peak families of the
 * paper's test suite (Sec. V, eqs. 3-4). */
#define MC_F_CONST 0
#define MC_F_GAUSS_PRODUCT 1
#define MC_F_CORNER_PEAK 2
#define MC_F_GAUSS_TABLES 3

#define MC_FP64 0      /* all arithmetic in FP64 */
#define MC_FP32_EVAL 1 /* the map and the integrand in FP32 (uniforms from the top 23 bits of
                          the same random words; constants, bin edges and widths, and tables
                          rounded to float); I_k, per-cube and per-bin sums, the weighted
                          estimate and the bin adjustment in FP64.  Needs g <= 2^24. */

#define MC_MAX_DIM 16

/* An integration problem: the inputs of the m-Cubes procedure (Alg. 2:
 * f, d, nb, maxcalls, L, H, itmax, ita) plus the damping exponent of the bin
 * adjustment, the target relative error of the convergence check (Sec. V) and
 * the seed of the counter-based random numbers. */
typedef struct mc_problem {
    int32_t integrand;       /* MC_F_* */
    int32_t dim;             /* d, 1..MC_MAX_DIM */
    const double *params;    /* host, n_params doubles (layout above) */
    int64_t n_params;
    const double *tables;    /* host, n_tables doubles, or NULL */
    int64_t n_tables;
    const double *lo;        /* host, dim doubles, finite */
    const double *hi;        /* host, dim doubles, finite, hi > lo */
    int64_t maxcalls;        /* samples per iteration budget, >= 4 */
    int32_t nbins;           /* nb, bins per axis, >= 2 */
    int32_t itmax;           /* iterations, >= 1 */
    int32_t ita;             /* adjusting iterations, 0..itmax */
    int32_t precision;       /* MC_FP64 or MC_FP32_EVAL */
    double alpha;            /* damping exponent of the bin adjustment, > 0 */
    double tau_rel;          /* target relative error; 0 runs all itmax iterations */
    uint64_t seed;           /* random-number key */
    int32_t blocks;          /* workgroups of the sampling kernel; 0 = fill the device */
    int32_t threads;         /* threads per workgroup, a multiple of 64 in 64..1024; 0: of 1024,
                                768, 512 and 256 the one keeping the most waves resident per
                                CU (ties to the larger) */
    int32_t one_d;           /* 1: the m-Cubes1D variant (Sec. V): bin contributions of the first
                                axis only, and its adjusted boundaries shared by every axis; meant
                                for fully symmetric integrands.  0: separate grids per axis */
    double chi2_max;         /* the convergence check also requires chi^2/dof <= chi2_max (Sec. V
                                counts a run as converged only with a small chi^2); 0 selects
                                MC_CHI2_DOF_DEFAULT, a negative value leaves chi^2 unchecked;
                                not NaN */
    int32_t device_steps;    /* 1: mc_integrate and mc_integrate_prepared run the steps of Alg. 2
                                between sampling passes (Weighted-Estimates, Check-Convergence,
                                Adjust-Bin-Bounds) on the device, so the passes of a run follow
                                each other with no host round trip.  The bin adjustment takes the
                                host's steps with its sums in a fixed order of its own and the
                                device library's pow and log, so its boundaries agree with
                                mc_refine_grid's to rounding, not bit for bit.  Taken for
                                nbins <= MC_DEVICE_STEPS_MAX_BINS; above that, and in
                                mc_integrate_noalloc, the host runs the steps.  0: the host runs
                                them (the grid is then exactly mc_refine_grid's). */
} mc_problem;

#define MC_DEVICE_STEPS_MAX_BINS 4000

#define MC_CHI2_DOF_DEFAULT 5.0

typedef struct mc_result {
    double estimate;   /* weighted estimate over the iterations run (see mc_weighted_estimate) */
    double error;      /* its standard deviation; +inf when no iteration saw a non-zero sample */
    double chi2_dof;   /* chi^2 per degree of freedom (NaN with fewer than two informative
                          iterations) */
    int32_t iterations;
    int32_t converged; /* 1 if, after >= 2 iterations, error <= tau_rel |estimate| and
                          chi2_dof <= the problem's bound */
    int64_t calls;     /* integrand evaluations: iterations * m * p */
} mc_result;

/* Optional timing of mc_integrate, measured with HIP events on the call's
 * stream around each kernel launch. */
typedef struct mc_timing {
    double sample_ms;    /* sum over iterations of the sampling kernel */
    double finalize_ms;  /* sum over iterations of the reduction kernel (with device_steps:
                            of everything after the sampling kernel, the decision and the
                            bin adjustment included) */
    int32_t launches;    /* sampling-kernel launches */
    int32_t blocks;      /* workgroups per sampling launch */
    int32_t threads;     /* threads per workgroup */
    int32_t lds_bytes;   /* LDS per workgroup */
} mc_timing;

/* Human-readable text for a status (static storage). */
const char *mc_status_string(mc_status status);

/* Sub-cube lattice of Alg. 2: g = the largest integer with g^d <= maxcalls/2
 * (integer division), m = g^d sub-cubes, p = maxcalls / m samples per
 * sub-cube.  Host only.  MC_EINVAL for dim outside 1..MC_MAX_DIM, maxcalls < 4
 * or maxcalls beyond 2^62.  (Problems additionally need g <= 2^30.) */
mc_status mc_shape(int32_t dim, int64_t maxcalls, int64_t *g, int64_t *m, int64_t *p);

/* Bytes of device workspace the problem needs on the current device.
 * MC_EINVAL for an invalid problem, MC_EDEVICE if no device is usable. */
mc_status mc_workspace_bytes(const mc_problem *prob, size_t *bytes);

/* The sampling kernel's launch for the problem on the current device:
 * workgroups, threads per workgroup and bytes of LDS per workgroup of a
 * V-Sample pass (adjust != 0) or a V-Sample-No-Adjust pass (adjust == 0), as
 * mc_integrate and mc_sample_iteration launch it.  Host query; no kernel
 * runs.  MC_EINVAL for an invalid problem or a NULL output, MC_EDEVICE
 * without a usable device. */
mc_status mc_launch_shape(const mc_problem *prob, int32_t adjust, int32_t *blocks, int32_t *threads,
                          int32_t *lds_bytes);

/* Copies the problem's parameters and tables into the workspace and prepares
 * it for mc_sample_iteration().  mc_integrate() does this itself. */
mc_status mc_prepare(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream);

/* One sampling pass, V-Sample (adjust != 0) or V-Sample-No-Adjust (adjust
 * == 0) of Alg. 3, on a workspace prepared by mc_prepare() for the same
 * problem.  Synchronous.
 *   iter       iteration number (part of the random-number counter)
 *   h_grid     host, dim*(nbins+1) boundaries
 *   h_out      host, 2 doubles: the iteration estimate I and its variance
 *   h_hist     host, dim*nbins bin contributions sum I_k^2, or NULL; must be
 *              NULL when adjust == 0
 *   d_trace    device or NULL.  When not NULL, the sampling kernel also
 *              records the sub-cubes t in [t0, t1): first (t1-t0)*p records
 *              of 3*dim+2 doubles (u_1..u_d, bin_1..bin_d, x_1..x_d, J, f)
 *              in the order (t, k), then (t1-t0) records of 2 doubles (I_t,
 *              var_t).  trace_bytes must hold them. */
mc_status mc_sample_iteration(const mc_problem *prob, uint32_t iter, int32_t adjust,
                              const double *h_grid, void *d_ws, size_t ws_bytes, void *stream,
                              double *h_out, double *h_hist, void *d_trace, size_t trace_bytes,
                              int64_t t0, int64_t t1);

/* Adjust-Bin-Bounds (Alg. 2; Alg. 1 and the text after it): rebuilds the
 * boundaries so that bins with large contributions become smaller.  Per
 * axis: three-point smoothing of the contributions, Lepage's damped
 * compression ((1 - s_i/S) / ln(S/s_i))^alpha, then equal shares of the
 * compressed weight per new bin.  An axis without positive finite weight is
 * left unchanged.  Host only; h_grid is updated in place. */
mc_status mc_refine_grid(int32_t dim, int32_t nbins, double alpha, const double *h_hist,
                         double *h_grid);

/* The m-Cubes1D adjustment (Sec. V): the first axis's boundaries adjusted
 * from the first axis's contributions (h_hist row 0), then copied to every
 * axis.  Host only; h_grid is updated in place. */
mc_status mc_refine_grid_1d(int32_t dim, int32_t nbins, double alpha, const double *h_hist,
                            double *h_grid);

/* mc_refine_grid (one_d == 0) or mc_refine_grid_1d (one_d == 1) on the
 * device, as runs with device_steps take it: the same steps, one workgroup
 * per axis, with the sums formed in a fixed order of its own and the device
 * library's pow and log, so the boundaries agree with the host call's to
 * rounding (deterministic: the same input gives the same output).
 *   d_hist   device, dim*nbins contributions (row 0 only when one_d)
 *   d_grid   device, dim*(nbins+1) boundaries, updated in place
 * Queued on the stream; returns without waiting.  MC_EINVAL for dim outside
 * 1..MC_MAX_DIM, nbins outside 2..MC_DEVICE_STEPS_MAX_BINS, alpha not
 * positive and finite, one_d not 0 or 1, or a NULL pointer; MC_EDEVICE if the
 * launch fails. */
mc_status mc_refine_grid_device(int32_t dim, int32_t nbins, double alpha, int32_t one_d,
                                const double *d_hist, double *d_grid, void *stream);

/* Init-Bins (Alg. 2): nbins equal bins per axis.  Host only. */
mc_status mc_init_grid(int32_t dim, int32_t nbins, double *h_grid);

/* Weighted-Estimates (Alg. 2): inverse-variance weighted mean of k iteration
 * results, its standard deviation and chi^2 per degree of freedom, written
 * to h_out[0..2].  An iteration with estimate 0 and variance 0 (no sample saw
 * a non-zero value) carries no information and is left out; chi^2/dof has
 * n-1 degrees of freedom for n informative iterations (NaN for n < 2).
 * Informative iterations with zero variance (an integrand constant on every
 * sub-cube is estimated exactly), if any, decide the mean alone, with
 * standard deviation 0 and chi^2/dof 0.  With no informative iteration the
 * result is 0 with standard deviation +inf.  Host only. */
mc_status mc_weighted_estimate(int32_t k, const double *h_I, const double *h_var, double *h_out);

/* The whole m-Cubes run (Alg. 2): iterations of sampling, weighting, bin
 * adjustment (first ita iterations) and the convergence check, on the given
 * stream.  Synchronous.
 *   h_iters  host, 2*itmax doubles or NULL: per-iteration (I_i, var_i)
 *   h_grid   host, dim*(nbins+1) doubles or NULL: the final boundaries
 *   timing   host or NULL */
mc_status mc_integrate(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream,
                       mc_result *out, double *h_iters, double *h_grid, mc_timing *timing);

/* mc_integrate() on a workspace that mc_prepare() has already filled for the
 * same problem (same integrand, parameters, tables, bounds and precision):
 * nothing of the problem is uploaded again, so repeated runs, e.g. with other
 * seeds or iteration counts, start with their inputs resident in device
 * memory.  Arguments, results and errors as for mc_integrate().  On a
 * workspace prepared for a different problem the result is meaningless (all
 * accesses stay inside the workspace). */
mc_status mc_integrate_prepared(const mc_problem *prob, void *d_ws, size_t ws_bytes, void *stream,
                                mc_result *out, double *h_iters, double *h_grid,
                                mc_timing *timing);

/* For callers that cannot allocate device memory (code under stream capture,
 * serving loops that must not allocate): mc_integrate() without a
 * workspace.  The library runs the problem in a device scratch array of
 * MC_NOALLOC_SCRATCH_BYTES that it holds on every GPU it is loaded on until
 * the process ends; nothing is allocated, neither on the device nor as
 * page-locked host memory (the per-iteration copies go through the caller's
 * pageable memory).  Arguments, results and errors as for mc_integrate(),
 * plus MC_EWORKSPACE when mc_workspace_bytes() of the problem exceeds the
 * scratch size (fewer workgroups, prob->blocks, need less).  All calls on one
 * device share its array and are serialised by the library (a call waits for
 * the previous one to finish); the array keeps the last call's contents,
 * which the next call overwrites before reading. */
#define MC_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
mc_status mc_integrate_noalloc(const mc_problem *prob, void *stream, mc_result *out,
                               double *h_iters, double *h_grid);

/* ---------------------------------------------------------------- batches and serving
 *
 * Many independent integrals advanced together.  Every step runs one sampling
 * pass (V-Sample or V-Sample-No-Adjust, per integral) of every active
 * integral in one persistent launch per group present (precision, and
 * whether the integral's LDS footprint limits workgroups per CU), merges each
 * integral's pieces in a fixed order, adjusts the grids of the integrals
 * still in their adjusting iterations on the device (the same steps as
 * mc_refine_grid, with the device library's pow and log), and then runs
 * Weighted-Estimates and Check-Convergence per integral on the host.  Grids,
 * histograms and tables stay in device memory.  Each integral's random
 * numbers depend only on its own seed, iteration, cube and sample, so an
 * integral gets the same samples alone and in any mix.
 *
 * Integrals in a batch or a server have dim <= MC_BATCH_MAX_DIM; everything
 * else is as for mc_integrate. */
#define MC_BATCH_MAX_DIM 10

#define MC_REQ_QUEUED 0   /* submitted, waiting for device memory */
#define MC_REQ_RUNNING 1  /* admitted: iterating */
#define MC_REQ_DONE 2     /* converged or ran itmax iterations; result available */
#define MC_REQ_FAILED 3   /* stopped with an error status (e.g. MC_ENONFINITE) */

typedef struct mc_batch_stats {
    int32_t steps;       /* persistent sampling steps */
    int32_t max_active;  /* most integrals in one step */
    double sample_ms;    /* sampling-launch time summed over steps (HIP events) */
    double step_ms;      /* host wall time of the steps */
    int64_t calls;       /* integrand evaluations over all integrals */
    double host_ms;      /* host work of the steps: admission and step set-up before the
                            launches, and the per-integral host steps after the read-back */
} mc_batch_stats;

/* Device workspace for running the n problems together with
 * mc_batch_integrate.  MC_EINVAL for an invalid problem or dim above
 * MC_BATCH_MAX_DIM; MC_EDEVICE without a usable device. */
mc_status mc_batch_workspace_bytes(const mc_problem *probs, int32_t n, size_t *bytes);

/* Runs the n problems to completion together (one persistent sampling launch
 * per step).  Synchronous.  results[i] is written when statuses[i] is MC_OK;
 * statuses[i] is MC_ENONFINITE for an integral whose integrand produced a
 * non-finite value (the others are unaffected).  The return value is MC_OK
 * unless the whole batch failed (invalid input, workspace, device). */
mc_status mc_batch_integrate(const mc_problem *probs, int32_t n, void *d_ws, size_t ws_bytes,
                             void *stream, mc_result *results, mc_status *statuses,
                             mc_batch_stats *stats);

/* A serving loop with continuous batching over a caller-owned workspace.
 * The first arena_bytes of the workspace hold admitted integrals' persistent
 * state (constants, tables, two grids and the latest histogram per
 * integral); the rest holds one step's work tables.  Requests are admitted
 * in arrival order when both fit, at most max_active at a time.  One server
 * must not be used from two threads at once.  Device memory is only the
 * caller's workspace; the server keeps its host copies of the requests and a
 * page-locked host buffer for each step's upload and read-back. */
typedef struct mc_server mc_server;

mc_status mc_server_create(void *d_ws, size_t ws_bytes, size_t arena_bytes, int32_t max_active,
                           void *stream, mc_server **out);
/* Bounds the work of one step (not in the paper: a scheduling policy of the
 * serving loop).  samples: the step's budget of integrand samples (m p per
 * iteration of each request it runs); 0, the default, runs every active
 * request in every step.  Under a budget a step takes every request left out
 * max_skip steps in a row, and then, by least estimated remaining work (cost
 * per iteration times the iterations still expected from the current error
 * and the target, or 2 before an error estimate exists), each that keeps the
 * other requests' samples within the budget; an empty step takes the first by
 * that order.  Short requests then finish in a few short steps instead of
 * waiting for every long one's iteration, and no request is left out more
 * than max_skip steps in a row.  Each request's result is the same as without
 * a budget (its samples do not depend on the schedule; sums may be formed in
 * another order).  MC_EINVAL for a null server or a negative argument.  Takes
 * effect from the next step. */
mc_status mc_server_set_step_budget(mc_server *srv, int64_t samples, int32_t max_skip);
/* Copies the problem (host arrays included) and queues it.  MC_EWORKSPACE if
 * it could never fit, even alone. */
mc_status mc_server_submit(mc_server *srv, const mc_problem *prob, int64_t *id);
/* Admits what fits, runs one step over the active requests, retires the
 * finished ones.  active/queued/finished (each may be NULL) report the counts
 * after the step. */
mc_status mc_server_step(mc_server *srv, int32_t *active, int32_t *queued, int32_t *finished);
/* State (MC_REQ_*) of a request; out is written when it is MC_REQ_DONE and
 * status (may be NULL) holds its final status. */
mc_status mc_server_poll(mc_server *srv, int64_t id, int32_t *state, mc_result *out,
                         mc_status *status);
/* Ids of the requests that finished (done or failed) in the last step, up to
 * cap of them; *n is how many were written. */
mc_status mc_server_finished(mc_server *srv, int64_t *ids, int32_t cap, int32_t *n);
/* Forgets a finished request. */
mc_status mc_server_release(mc_server *srv, int64_t id);
mc_status mc_server_stats(mc_server *srv, mc_batch_stats *stats);
mc_status mc_server_destroy(mc_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* MCUBES_H */
