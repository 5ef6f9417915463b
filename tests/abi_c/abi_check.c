/*
 * abi_check.c -- drives the RTLBFS library through its C ABI alone (no torch,
 * no Python): library-owned workspace, the null stream, a 2D cavity and a
 * batch of two cavities.  Prints one JSON object; exit status 0 on success.
 * Test infrastructure (run by tests/test_c_abi_gpu.py).
 *
 * usage: abi_check N RA STEPS OUT_T_FILE
 *   writes the N*N absolute temperature field (double, x-fastest) of the
 *   single-domain run to OUT_T_FILE, and the vertex arrays of the two
 *   body-fitted runs (a 2D O-mesh annulus with a heated wall and far field,
 *   a 3D annulus wedge closed by a rotation) to OUT_T_FILE.cx/.cy and
 *   OUT_T_FILE.c3x/.c3y/.c3z.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

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

static int write_doubles(const char *base, const char *ext, const double *v, size_t n) {
    char name[4096];
    snprintf(name, sizeof(name), "%s%s", base, ext);
    FILE *f = fopen(name, "wb");
    if (!f) return 1;
    const int ok = fwrite(v, sizeof(double), n, f) == n;
    fclose(f);
    return !ok;
}

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

    /* body-fitted 2D: an O-mesh annulus, periodic around, heated inner wall,
     * far field outside with an upward stream, aiding buoyancy */
    const int ni = 36, nj = 14;
    double *cx = (double *)malloc(sizeof(double) * (ni + 1) * (nj + 1));
    double *cy = (double *)malloc(sizeof(double) * (ni + 1) * (nj + 1));
    if (!cx || !cy) return 1;
    for (int j = 0; j <= nj; ++j)
        for (int i = 0; i <= ni; ++i) {
            const double r = 25.0 * pow(1.15, j), th = 2.0 * 3.14159265358979323846 * (i % ni) / ni;
            cx[j * (ni + 1) + i] = r * cos(th);
            cy[j * (ni + 1) + i] = r * sin(th);
        }
    if (write_doubles(argv[4], ".cx", cx, (size_t)(ni + 1) * (nj + 1)) ||
        write_doubles(argv[4], ".cy", cy, (size_t)(ni + 1) * (nj + 1)))
        return 1;
    rtlbfs_curv_mesh cm = {{ni, nj}, cx, cy};
    rtlbfs_curv_bc cb;
    memset(&cb, 0, sizeof(cb));
    cb.kind[0] = cb.kind[1] = RTLBFS_PERIODIC;
    cb.kind[2] = RTLBFS_WALL_ISOTHERMAL;
    cb.kind[3] = RTLBFS_FARFIELD;
    cb.Tw[2] = 1.0;
    cb.up[1] = 1.0;
    cb.u_inf[1] = 0.04;
    rtlbfs_opts copts;
    CHECK(rtlbfs_opts_init(&copts));
    copts.dt = 0.5;
    CHECK(rtlbfs_curv_create(&cm, 0.08, 0.11, 4e-5, &cb, &copts, NULL, NULL, 0, &g_h));
    CHECK(rtlbfs_step(g_h, steps));
    double wh[2];
    CHECK(rtlbfs_wall_heat(g_h, 2, wh));
    rtlbfs_nu nu_curv;
    const int curv_nusselt_rc = rtlbfs_nusselt(g_h, &nu_curv); /* not defined on body-fitted meshes */
    CHECK(rtlbfs_destroy(g_h));
    g_h = NULL;
    free(cx);
    free(cy);

    /* body-fitted 3D: an annulus wedge of one azimuthal cell */
    const int nr = 8, nz = 10, nv = (nr + 1) * 2 * (nz + 1);
    const double dth = 0.1;
    double *x3 = (double *)malloc(sizeof(double) * nv), *y3 = (double *)malloc(sizeof(double) * nv);
    double *z3 = (double *)malloc(sizeof(double) * nv);
    if (!x3 || !y3 || !z3) return 1;
    for (int k = 0; k <= nz; ++k)
        for (int j = 0; j <= 1; ++j)
            for (int i = 0; i <= nr; ++i) {
                const int v = (k * 2 + j) * (nr + 1) + i;
                const double r = 10.0 + i, th = (j - 0.5) * dth;
                x3[v] = r * cos(th);
                y3[v] = r * sin(th);
                z3[v] = k;
            }
    if (write_doubles(argv[4], ".c3x", x3, nv) || write_doubles(argv[4], ".c3y", y3, nv) ||
        write_doubles(argv[4], ".c3z", z3, nv))
        return 1;
    rtlbfs_curv3_mesh m3 = {{nr, 1, nz}, x3, y3, z3};
    rtlbfs_curv3_bc b3;
    memset(&b3, 0, sizeof(b3));
    b3.kind[0] = b3.kind[1] = RTLBFS_WALL_ISOTHERMAL;
    b3.kind[2] = b3.kind[3] = RTLBFS_PERIODIC;
    b3.kind[4] = b3.kind[5] = RTLBFS_WALL_ADIABATIC;
    b3.rot[1] = dth;
    b3.Tw[0] = 1.0;
    b3.up[2] = 1.0;
    b3.T_ref = 0.5;
    CHECK(rtlbfs_curv3_create(&m3, 0.06, 0.08, 5e-4, &b3, &copts, NULL, NULL, 0, &g_h));
    CHECK(rtlbfs_step(g_h, steps));
    double wh3[2];
    CHECK(rtlbfs_wall_heat(g_h, 0, wh3));
    CHECK(rtlbfs_destroy(g_h));
    g_h = NULL;
    free(x3);
    free(y3);
    free(z3);

    printf("{\"steps\": %ld, \"res_u\": %.17g, \"res_T\": %.17g, \"nu_hot\": %.17g, \"nu_volume\": %.17g, "
           "\"tile\": [%d, %d, %d], \"bad_field_rc\": %d, \"batch_diverged\": [%d, %d], "
           "\"batch_nu_hot0\": %.17g, \"curv_wall_heat\": [%.17g, %.17g], \"curv_nusselt_rc\": %d, "
           "\"curv3_wall_heat\": [%.17g, %.17g]}\n",
           steps, ru, rT, nu.hot_avg, nu.volume, info.tile_x, info.tile_y, info.steps_per_launch, bad_field,
           flags[0], flags[1], nub.hot_avg, wh[0], wh[1], curv_nusselt_rc, wh3[0], wh3[1]);
    return 0;
}
