/* A plain C99 consumer of include/mcubes.h: takes the address of every
 * entry point (so each prototype must be valid C) and calls the host-only
 * ones, linked straight against libmcubes.so with no Python in between.
 * Prints one line per check; exits non-zero on the first failure. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "mcubes.h"

#define CHECK(cond)                                                   \
    do {                                                              \
        if (!(cond)) {                                                \
            printf("FAIL %s (line %d)\n", #cond, __LINE__);           \
            return 1;                                                 \
        }                                                             \
    } while (0)

int main(void) {
    /* every entry point (a link error if one is missing) */
    typedef void (*entry_fn)(void);
    const entry_fn entry[] = {
        (entry_fn)mc_status_string, (entry_fn)mc_shape, (entry_fn)mc_workspace_bytes,
        (entry_fn)mc_launch_shape, (entry_fn)mc_prepare, (entry_fn)mc_sample_iteration,
        (entry_fn)mc_refine_grid, (entry_fn)mc_refine_grid_1d, (entry_fn)mc_refine_grid_device,
        (entry_fn)mc_init_grid,
        (entry_fn)mc_weighted_estimate, (entry_fn)mc_integrate, (entry_fn)mc_integrate_prepared,
        (entry_fn)mc_integrate_noalloc, (entry_fn)mc_batch_workspace_bytes,
        (entry_fn)mc_batch_integrate, (entry_fn)mc_server_create, (entry_fn)mc_server_submit,
        (entry_fn)mc_server_step, (entry_fn)mc_server_poll, (entry_fn)mc_server_finished,
        (entry_fn)mc_server_release, (entry_fn)mc_server_stats, (entry_fn)mc_server_destroy,
        (entry_fn)mc_server_set_step_budget,
    };
    for (size_t i = 0; i < sizeof entry / sizeof entry[0]; ++i) CHECK(entry[i] != NULL);
    printf("entry points %u\n", (unsigned)(sizeof entry / sizeof entry[0]));

    CHECK(mc_status_string(MC_OK) != NULL);
    CHECK(mc_status_string(MC_EINVAL) != NULL);

    /* the d = 6 tables lattice at 1e8 samples: 19^6 sub-cubes, 2 samples each */
    int64_t g = 0, m = 0, p = 0;
    CHECK(mc_shape(6, 100000000, &g, &m, &p) == MC_OK);
    CHECK(g == 19 && m == 47045881 && p == 2);
    CHECK(mc_shape(0, 100, &g, &m, &p) == MC_EINVAL);
    printf("shape %lld %lld %lld\n", (long long)g, (long long)m, (long long)p);

    /* Init-Bins, then an adjustment from a histogram that puts all weight
     * in the first half of each axis: boundaries stay in [0, 1], ordered,
     * and move towards 0 */
    enum { D = 2, NB = 8 };
    double grid[D * (NB + 1)], hist[D * NB];
    CHECK(mc_init_grid(D, NB, grid) == MC_OK);
    for (int j = 0; j < D; ++j)
        for (int i = 0; i <= NB; ++i) CHECK(grid[j * (NB + 1) + i] == (double)i / NB);
    for (int j = 0; j < D; ++j)
        for (int i = 0; i < NB; ++i) hist[j * NB + i] = i < NB / 2 ? 1.0 : 1e-6;
    CHECK(mc_refine_grid(D, NB, 1.5, hist, grid) == MC_OK);
    for (int j = 0; j < D; ++j) {
        const double *B = grid + j * (NB + 1);
        CHECK(B[0] == 0.0 && B[NB] == 1.0);
        for (int i = 0; i < NB; ++i) CHECK(B[i] <= B[i + 1]);
        CHECK(B[NB / 2] < 0.5);
    }
    printf("refined middle boundary %.6f\n", grid[NB / 2]);

    /* Weighted-Estimates of two iterations with equal variance: the mean,
     * sigma / sqrt(2), and chi^2 of their spread */
    const double I[2] = {1.0, 3.0}, var[2] = {4.0, 4.0};
    double est[3];
    CHECK(mc_weighted_estimate(2, I, var, est) == MC_OK);
    CHECK(est[0] == 2.0 && fabs(est[1] - sqrt(2.0)) < 1e-15 && est[2] == 0.5);
    printf("weighted %.3f %.6f %.3f\n", est[0], est[1], est[2]);
    printf("ok\n");
    return 0;
}
