/* Drives every entry point of the C oracle on small cases, for a build with
 * AddressSanitizer and UndefinedBehaviorSanitizer: 2D and 3D Cartesian runs
 * (walls, periodic axes, stretched meshes, plain and deviation storage, both
 * interior-face fluxes), the single-face fluxes, and the body-fitted 2D and
 * 3D runs.  Exits 0 when every call succeeds and every value is finite; the
 * sanitizers abort on any invalid access or undefined operation. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "curv3_oracle.h"
#include "curv_oracle.h"
#include "rtlbfs_oracle.h"

static int fail(const char *what) {
    fprintf(stderr, "asan driver: %s\n", what);
    return 1;
}

static int finite_all(const double *v, long n) {
    for (long i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static int run_cartesian(int dim, const int *n, const double *stretch, const int *bc, int dev, int method) {
    orc_cfg c = {0};
    c.dim = dim;
    for (int a = 0; a < 3; ++a) {
        c.n[a] = n[a];
        c.stretch[a] = stretch[a];
    }
    for (int k = 0; k < 6; ++k) c.bc[k] = bc[k];
    c.Tw[0] = 0.5;
    c.Tw[1] = -0.5;
    c.gravity_axis = dim - 1;
    c.nu = 0.05;
    c.chi = 0.07;
    c.beta_g = 1e-3;
    c.dtl = 1.0;
    c.dt = 0.5;
    c.deviation = dev;
    c.force_in_predictor = 1;
    c.init = ORC_INIT_CONDUCTION;
    c.seed = 7;
    c.noise_amp = 1e-3;
    c.method = method;
    orc_state *s = NULL;
    if (orc_create(&c, &s) != 0 || !s) return fail("orc_create");
    const long N = orc_cells(s);
    double *buf = malloc(sizeof(double) * N * 3), *rho = malloc(sizeof(double) * N),
           *T = malloc(sizeof(double) * N);
    double out[8];
    if (orc_step(s, 5) != 0) return fail("orc_step");
    for (int f = 0; f < dim + 2; ++f) {
        if (orc_get_stored(s, f, buf) != 0 || !finite_all(buf, N)) return fail("orc_get_stored");
        if (orc_set_stored(s, f, buf) != 0) return fail("orc_set_stored");
        if (orc_get_prim(s, f, buf) != 0 || !finite_all(buf, N)) return fail("orc_get_prim");
    }
    orc_get_prim(s, 0, rho);
    orc_get_prim(s, dim + 1, T);
    for (int a = 0; a < dim; ++a) orc_get_prim(s, 1 + a, buf + (long)a * N);
    if (orc_set_prim(s, rho, buf, T) != 0) return fail("orc_set_prim");
    for (int a = 0; a < dim; ++a)
        if (orc_axis(s, a, rho, T) != 0) return fail("orc_axis");
    if (orc_step(s, 3) != 0 || orc_steps_done(s) != 8) return fail("orc_step count");
    orc_residual(s, out);
    if (!finite_all(out, 2)) return fail("orc_residual");
    if (orc_nusselt(s, out) == 0 && !finite_all(out, 5)) return fail("orc_nusselt");
    orc_integrals(s, out);
    orc_taus(s, out);
    if (!finite_all(out, 2)) return fail("orc_taus");
    orc_destroy(s);
    free(buf);
    free(rho);
    free(T);
    return 0;
}

static int run_faces(void) {
    for (int dim = 2; dim <= 3; ++dim)
        for (int method = 0; method < 2; ++method)
            for (int dev = 0; dev < 2; ++dev) {
                orc_cfg c = {0};
                c.dim = dim;
                c.nu = 0.05;
                c.chi = 0.07;
                c.beta_g = 1e-3;
                c.gravity_axis = 1;
                c.dtl = 0.8;
                c.deviation = dev;
                c.force_in_predictor = 1;
                c.method = method;
                double pL[5] = {dev ? 0.01 : 1.01, 0.02, -0.01, 0.005, dev ? 0.1 : 0.6};
                double pR[5] = {dev ? -0.02 : 0.98, 0.01, 0.02, -0.004, dev ? -0.05 : 0.45};
                double gL[15], gR[15], flux[5], pred[5];
                for (int k = 0; k < 15; ++k) {
                    gL[k] = 1e-3 * (k % 7 - 3);
                    gR[k] = -1e-3 * (k % 5 - 2);
                }
                for (int axis = 0; axis < dim; ++axis) {
                    orc_face_flux(&c, axis, pL, gL, pR, gR, 0.6, 0.9, flux, pred);
                    if (!finite_all(flux, dim + 2) || !finite_all(pred, dim + 2)) return fail("orc_face_flux");
                }
                const double xSL[3] = {0.6, 0.1, -0.05}, xSR[3] = {-0.9, -0.2, 0.03}, fdir[3] = {0.0, 1.0, 0.0};
                orc_face_flux_frame(&c, pL, gL, pR, gR, xSL, xSR, fdir, 0.5, flux, pred);
                if (!finite_all(flux, dim + 2)) return fail("orc_face_flux_frame");
            }
    return 0;
}

static int run_curv2d(int dev, int method) {
    const int ni = 7, nj = 5;
    double *x = malloc(sizeof(double) * (ni + 1) * (nj + 1)), *y = malloc(sizeof(double) * (ni + 1) * (nj + 1));
    for (int j = 0; j <= nj; ++j)
        for (int i = 0; i <= ni; ++i) {
            x[j * (ni + 1) + i] = i + 0.15 * sin(0.7 * j);
            y[j * (ni + 1) + i] = j + 0.1 * sin(0.9 * i);
        }
    orc_curv_cfg c = {0};
    c.ni = ni;
    c.nj = nj;
    c.bc[0] = ORC_WALL_ISOTHERMAL;
    c.bc[1] = ORC_FARFIELD;
    c.bc[2] = ORC_WALL_ADIABATIC;
    c.bc[3] = ORC_WALL_ISOTHERMAL;
    c.Tw[0] = 1.0;
    c.up[1] = 1.0;
    c.Tb = 0.5;
    c.u_inf[0] = 0.02;
    c.T_inf = 0.5;
    c.nu = 0.06;
    c.chi = 0.08;
    c.beta_g = 1e-3;
    c.dtl = 1.0;
    c.dt = 0.5;
    c.deviation = dev;
    c.force_in_predictor = 1;
    c.method = method;
    orc_curv *s = NULL;
    if (orc_curv_create(&c, x, y, &s) != 0 || !s) return fail("orc_curv_create");
    const long N = (long)ni * nj;
    double *buf = malloc(sizeof(double) * N * 3), out[8];
    if (orc_curv_step(s, 5) != 0) return fail("orc_curv_step");
    for (int f = 0; f < 4; ++f)
        if (orc_curv_get_prim(s, f, buf) != 0 || !finite_all(buf, N) || orc_curv_get_stored(s, f, buf) != 0)
            return fail("orc_curv_get_prim");
    orc_curv_cells(s, buf, buf + N, buf + 2 * N);
    orc_curv_residual(s, out);
    if (orc_curv_wall_heat(s, 0, out) != 0 || !finite_all(out, 2)) return fail("orc_curv_wall_heat");
    orc_curv_integrals(s, out);
    double *rho = malloc(sizeof(double) * N), *u = calloc(2 * N, sizeof(double)), *T = malloc(sizeof(double) * N);
    for (long k = 0; k < N; ++k) {
        rho[k] = 1.0;
        T[k] = 0.5;
    }
    if (orc_curv_set_prim(s, rho, u, T) != 0 || orc_curv_step(s, 2) != 0) return fail("orc_curv_set_prim");
    orc_curv_destroy(s);
    free(x);
    free(y);
    free(buf);
    free(rho);
    free(u);
    free(T);
    return 0;
}

static int run_curv3d(int dev, int method) {
    const int ni = 4, nj = 2, nk = 3;
    const double dth = 0.15, ri = 8.0;
    const long nv = (long)(ni + 1) * (nj + 1) * (nk + 1);
    double *x = malloc(sizeof(double) * nv), *y = malloc(sizeof(double) * nv), *z = malloc(sizeof(double) * nv);
    for (int k = 0; k <= nk; ++k)
        for (int j = 0; j <= nj; ++j)
            for (int i = 0; i <= ni; ++i) {
                const long v = ((long)k * (nj + 1) + j) * (ni + 1) + i;
                x[v] = (ri + i) * cos(j * dth);
                y[v] = (ri + i) * sin(j * dth);
                z[v] = k;
            }
    orc_curv3_cfg c = {0};
    c.n[0] = ni;
    c.n[1] = nj;
    c.n[2] = nk;
    c.bc[0] = ORC_WALL_ISOTHERMAL;
    c.bc[1] = ORC_WALL_ISOTHERMAL;
    c.bc[2] = c.bc[3] = ORC_PERIODIC;
    c.bc[4] = c.bc[5] = ORC_WALL_ADIABATIC;
    c.rot[1] = nj * dth;
    c.Tw[0] = 1.0;
    c.up[2] = 1.0;
    c.Tb = 0.5;
    c.nu = 0.06;
    c.chi = 0.08;
    c.beta_g = 1e-3;
    c.dtl = 1.0;
    c.dt = 0.5;
    c.deviation = dev;
    c.force_in_predictor = 1;
    c.method = method;
    orc_curv3 *s = NULL;
    if (orc_curv3_create(&c, x, y, z, &s) != 0 || !s) return fail("orc_curv3_create");
    const long N = (long)ni * nj * nk;
    double *buf = malloc(sizeof(double) * N * 4), out[8];
    if (orc_curv3_step(s, 4) != 0) return fail("orc_curv3_step");
    for (int f = 0; f < 5; ++f)
        if (orc_curv3_get_prim(s, f, buf) != 0 || !finite_all(buf, N)) return fail("orc_curv3_get_prim");
    orc_curv3_cells(s, buf, buf + N, buf + 2 * N, buf + 3 * N);
    orc_curv3_residual(s, out);
    if (orc_curv3_wall_heat(s, 0, out) != 0 || !finite_all(out, 2)) return fail("orc_curv3_wall_heat");
    orc_curv3_integrals(s, out);
    double *rho = malloc(sizeof(double) * N), *u = calloc(3 * N, sizeof(double)), *T = malloc(sizeof(double) * N);
    for (long k = 0; k < N; ++k) {
        rho[k] = 1.0;
        T[k] = 0.5;
    }
    if (orc_curv3_set_prim(s, rho, u, T) != 0 || orc_curv3_step(s, 2) != 0) return fail("orc_curv3_set_prim");
    orc_curv3_destroy(s);
    free(x);
    free(y);
    free(z);
    free(buf);
    free(rho);
    free(u);
    free(T);
    return 0;
}

int main(void) {
    double x[33], phys[3];
    if (!(orc_mesh_nodes(32, 1.5, x) > 32.0)) return fail("orc_mesh_nodes");
    orc_physics_from_ra(1e5, 0.71, 0.1, 64.0, phys);
    if (!finite_all(phys, 3) || !isfinite(orc_splitmix_uniform(1, 5))) return fail("helpers");
    const int walls[6] = {ORC_WALL_ISOTHERMAL, ORC_WALL_ISOTHERMAL, ORC_WALL_ADIABATIC,
                          ORC_WALL_ADIABATIC, ORC_WALL_ADIABATIC, ORC_WALL_ADIABATIC};
    const int per_x[6] = {ORC_PERIODIC, ORC_PERIODIC, ORC_WALL_ISOTHERMAL, ORC_WALL_ISOTHERMAL,
                          ORC_WALL_ADIABATIC, ORC_WALL_ADIABATIC};
    const int n2[3] = {9, 7, 1}, n3[3] = {5, 4, 6};
    const double st[3] = {1.4, 1.2, 1.6}, flat[3] = {0.0, 1.2, 1.6};
    for (int dev = 0; dev < 2; ++dev)
        for (int method = 0; method < 2; ++method) {
            if (run_cartesian(2, n2, st, walls, dev, method) || run_cartesian(2, n2, flat, per_x, dev, method) ||
                run_cartesian(3, n3, st, walls, dev, method) || run_cartesian(3, n3, flat, per_x, dev, method) ||
                run_curv2d(dev, method) || run_curv3d(dev, method))
                return 1;
        }
    if (run_faces()) return 1;
    printf("oracle sanitizer run: ok\n");
    return 0;
}
