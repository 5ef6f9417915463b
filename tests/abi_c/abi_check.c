/*
 * abi_check.c -- drives the RTLBFS library through its C ABI alone (no torch,
 * no Python): library-owned workspace, the null stream, a 2D cavity and a
 * batch of two cavities.  Prints one JSON object; exit status 0 on success.
 * Test infrastructure (run by tests/test_c_abi_gpu.py).
 *
 * usage: abi_check N RA STEPS OUT_T_FILE
 *   writes the N*N absolute temperature field (double, x-fastest) of the
 *   single-domain run to OUT_T_FILE.
 */
#include <stdio.h>
#include <stdlib.h>

#include "rtlbfs.h"

#define CHECK(call)                                                                             \
    do {                                                                                        \
        int rc_ = (call);                                                                       \
        if (rc_ != RTLBFS_OK) {                                                                 \
            fprintf(stderr, "%s failed: %s (%s)\n", #call, rtlbfs_strerror(rc_), detail());     \
            return 1;                                                                           \
        }                                                                                       \
    } while (0)

static rtlbfs_t g_h = NULL;
static const char *detail(void) { return rtlbfs_last_error(g_h); }

int main(int argc, char **argv) {
    if (argc != 5) {
        fprintf(stderr, "usage: %s N RA STEPS OUT_T_FILE\n", argv[0]);
        return 2;
    }
    const int n = atoi(argv[1]);
    const double Ra = atof(argv[2]);
    const long steps = atol(argv[3]);

    rtlbfs_mesh mesh = {0};
    mesh.dim = 2;
    mesh.n[0] = mesh.n[1] = n;
    mesh.n[2] = 1;
    rtlbfs_bc bc = {0};
    bc.kind[0] = bc.kind[1] = RTLBFS_WALL_ISOTHERMAL;
    bc.kind[2] = bc.kind[3] = RTLBFS_WALL_ADIABATIC;
    bc.Tdev[0] = 0.5;
    bc.Tdev[1] = -0.5;
    bc.gravity_axis = 1;
    rtlbfs_opts opts;
    CHECK(rtlbfs_opts_init(&opts));
    opts.noise_amp = 1e-6;
    opts.seed = 1;

    /* single domain: library-owned workspace, null stream */
    CHECK(rtlbfs_create(&mesh, Ra, 0.71, 0.1, &bc, &opts, NULL, NULL, 0, &g_h));
    CHECK(rtlbfs_step(g_h, steps));
    double ru = 0, rT = 0;
    CHECK(rtlbfs_residual(g_h, &ru, &rT));
    rtlbfs_nu nu;
    CHECK(rtlbfs_nusselt(g_h, &nu));
    rtlbfs_info info;
    CHECK(rtlbfs_get_info(g_h, &info));
    double *T = (double *)malloc(sizeof(double) * (size_t)n * n);
    if (!T) return 1;
    CHECK(rtlbfs_get_field(g_h, 3, T, (size_t)n * n));
    FILE *f = fopen(argv[4], "wb");
    if (!f || fwrite(T, sizeof(double), (size_t)n * n, f) != (size_t)n * n) return 1;
    fclose(f);
    /* misuse is reported, not fatal */
    const int bad_field = rtlbfs_get_field(g_h, 9, T, (size_t)n * n);
    free(T);
    CHECK(rtlbfs_destroy(g_h));
    g_h = NULL;

    /* a batch of two cavities of different sizes */
    rtlbfs_mesh meshes[2] = {mesh, mesh};
    meshes[1].n[0] = meshes[1].n[1] = n / 2;
    const double Ras[2] = {Ra, 10.0 * Ra}, Prs[2] = {0.71, 7.0};
    rtlbfs_bc bcs[2] = {bc, bc};
    rtlbfs_batch_t b = NULL;
    CHECK(rtlbfs_batch_create(2, meshes, Ras, Prs, 0.1, bcs, &opts, NULL, NULL, 0, &b));
    CHECK(rtlbfs_batch_step(b, steps));
    int flags[2] = {-1, -1};
    CHECK(rtlbfs_batch_diverged(b, flags));
    rtlbfs_nu nub;
    CHECK(rtlbfs_batch_nusselt(b, 0, &nub));
    CHECK(rtlbfs_batch_destroy(b));

    printf("{\"steps\": %ld, \"res_u\": %.17g, \"res_T\": %.17g, \"nu_hot\": %.17g, \"nu_volume\": %.17g, "
           "\"tile\": [%d, %d, %d], \"bad_field_rc\": %d, \"batch_diverged\": [%d, %d], "
           "\"batch_nu_hot0\": %.17g}\n",
           steps, ru, rT, nu.hot_avg, nu.volume, info.tile_x, info.tile_y, info.steps_per_launch, bad_field,
           flags[0], flags[1], nub.hot_avg);
    return 0;
}
