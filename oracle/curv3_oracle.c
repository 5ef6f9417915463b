/*
 * curv3_oracle.c -- plain FP64 CPU oracle of the RTLBFS step on a 3D
 * body-fitted hexahedral mesh (Sec. 4.5: the concentric annulus, run with
 * one azimuthal cell layer).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, never by the product
 * path; it shares no code with the GPU library.
 *
 * The step of Sec. 3.2 on arbitrary hexahedra, written cell by cell: for
 * every cell, each of its six faces is visited, the neighbour across it found
 * (a cell of the mesh, the rotated image of a cell across a periodic pair, or
 * a wall), and
 *   - Eq. 55: (1/dV) sum_faces phi_S S_out with Eq. 56 face values;
 *   - the interior-face flux of Sec. 3.2 (or Sec. 2.2) in the face frame
 *     (n, t1, t2), the D3Q19 lattice of Fig. 1 aligned with it;
 *   - forward Euler (Eqs. 41-43) with the Eq. 64 body force.
 * A face shared by two cells is evaluated once from each of them, with the
 * same inputs in the same order, so both see the same flux.
 *
 * Readings (listed in the design notes):
 *   - face (corners q0..q3 in the cyclic order of the two axes spanning it):
 *     centre = vertex mean, area vector S = (q2 - q0) x (q3 - q1) / 2,
 *     normal n = S/|S| towards the higher index, t1 = the first edge
 *     q1 - q0 without its normal part, normalised, t2 = n x t1;
 *   - cell volume and centroid: the 24 tetrahedra formed by the cell's vertex
 *     mean and the four triangles (face centre, two consecutive corners) of
 *     each face;
 *   - wall distance d = (x_S - x_P) . n_out; walls as in the 2D oracle;
 *   - a periodic pair closed by a rotation alpha about z: the neighbour
 *     across the high side is the low-side cell rotated by +alpha (its
 *     centroid, velocity and gradients), across the low side by -alpha.
 */
#include "curv3_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define CS2 (1.0 / 3.0)
#define T0 0.5

struct orc_curv3 {
    orc_curv3_cfg c;
    orc_cfg fc;
    int n[3];
    long N;
    double orient;
    double *vx, *vy, *vz;
    double *cx, *cy, *cz, *vol;
    double *U[5], *Unew[5], *prim[5], *grad[5][3], *rhs[5];
    double res_u, res_T;
};

static long vid(const orc_curv3 *s, int i, int j, int k)
{
    return ((long)k * (s->n[1] + 1) + j) * (s->n[0] + 1) + i;
}
static long cid(const orc_curv3 *s, int i, int j, int k) { return ((long)k * s->n[1] + j) * s->n[0] + i; }

static void vert(const orc_curv3 *s, const int *p, double *q)
{
    long v = vid(s, p[0], p[1], p[2]);
    q[0] = s->vx[v];
    q[1] = s->vy[v];
    q[2] = s->vz[v];
}

static void cross(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double dot(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Corners of the face normal to `axis` at vertex index p, in the cyclic
 * order of the spanning axes a1 = axis+1, a2 = axis+2. */
static void face_corners(const orc_curv3 *s, int axis, const int *p, double q[4][3])
{
    int a1 = (axis + 1) % 3, a2 = (axis + 2) % 3;
    int r[4][3];
    for (int m = 0; m < 4; ++m)
        for (int a = 0; a < 3; ++a) r[m][a] = p[a];
    r[1][a1] += 1;
    r[2][a1] += 1;
    r[2][a2] += 1;
    r[3][a2] += 1;
    for (int m = 0; m < 4; ++m) vert(s, r[m], q[m]);
}

typedef struct {
    double xs[3], S[3], dS, n[3], t1[3], t2[3];
} face3;

static void face_geom(const orc_curv3 *s, int axis, const int *p, face3 *f)
{
    double q[4][3], d1[3], d2[3], e[3];
    face_corners(s, axis, p, q);
    for (int a = 0; a < 3; ++a) {
        f->xs[a] = 0.25 * (q[0][a] + q[1][a] + q[2][a] + q[3][a]);
        d1[a] = q[2][a] - q[0][a];
        d2[a] = q[3][a] - q[1][a];
        e[a] = q[1][a] - q[0][a];
    }
    cross(d1, d2, f->S);
    for (int a = 0; a < 3; ++a) f->S[a] *= 0.5 * s->orient;
    f->dS = sqrt(dot(f->S, f->S));
    for (int a = 0; a < 3; ++a) f->n[a] = f->S[a] / f->dS;
    double en = dot(e, f->n);
    for (int a = 0; a < 3; ++a) f->t1[a] = e[a] - en * f->n[a];
    double l = sqrt(dot(f->t1, f->t1));
    for (int a = 0; a < 3; ++a) f->t1[a] /= l;
    cross(f->n, f->t1, f->t2);
}

/* Signed volume and centroid of cell (i, j, k) from 24 tetrahedra. */
static double cell_shape(const orc_curv3 *s, int i, int j, int k, double *c)
{
    int p0[3] = {i, j, k};
    double O[3] = {0, 0, 0};
    for (int m = 0; m < 8; ++m) {
        int p[3] = {i + (m & 1), j + ((m >> 1) & 1), k + ((m >> 2) & 1)};
        double q[3];
        vert(s, p, q);
        for (int a = 0; a < 3; ++a) O[a] += 0.125 * q[a];
    }
    double V = 0.0, M[3] = {0, 0, 0};
    for (int axis = 0; axis < 3; ++axis)
        for (int hi = 0; hi < 2; ++hi) {
            int p[3] = {p0[0], p0[1], p0[2]};
            p[axis] += hi;
            double q[4][3], cf[3];
            face_corners(s, axis, p, q);
            for (int a = 0; a < 3; ++a) cf[a] = 0.25 * (q[0][a] + q[1][a] + q[2][a] + q[3][a]);
            for (int m = 0; m < 4; ++m) {
                const double *qa = q[m], *qb = q[(m + 1) % 4];
                double u[3], w[3], A[3], h[3];
                for (int a = 0; a < 3; ++a) {
                    u[a] = qa[a] - cf[a];
                    w[a] = qb[a] - cf[a];
                    h[a] = cf[a] - O[a];
                }
                cross(u, w, A); /* twice the triangle area vector, towards +axis */
                double vt = (hi ? 1.0 : -1.0) * dot(h, A) / 6.0;
                V += vt;
                for (int a = 0; a < 3; ++a) M[a] += vt * 0.25 * (O[a] + cf[a] + qa[a] + qb[a]);
            }
        }
    for (int a = 0; a < 3; ++a) c[a] = M[a] / V;
    return V;
}

static void rotz(double ang, const double *v, double *o)
{
    double c = cos(ang), sn = sin(ang);
    double x = c * v[0] - sn * v[1], y = sn * v[0] + c * v[1];
    o[0] = x;
    o[1] = y;
    o[2] = v[2];
}

static double store_T(const orc_curv3 *s, double Tabs) { return s->c.deviation ? Tabs - T0 : Tabs; }

/* A cell as seen from a face: primitives, gradients [p][axis] and centroid,
 * possibly the rotated image of a mesh cell. */
typedef struct {
    double p[5], g[5][3], x[3];
} cellv;

static void cell_view(const orc_curv3 *s, long c, double ang, int with_grad, cellv *v)
{
    double x[3] = {s->cx[c], s->cy[c], s->cz[c]};
    double u[3] = {s->prim[1][c], s->prim[2][c], s->prim[3][c]};
    rotz(ang, x, v->x);
    v->p[0] = s->prim[0][c];
    rotz(ang, u, v->p + 1);
    v->p[4] = s->prim[4][c];
    if (!with_grad) return;
    for (int p = 0; p < 5; ++p) {
        double g[3] = {s->grad[p][0][c], s->grad[p][1][c], s->grad[p][2][c]};
        if (p == 0 || p == 4) {
            rotz(ang, g, v->g[p]);
        }
    }
    /* velocity gradient G[a][b] = d_b u_a rotates as R G R^T */
    double G[3][3], RG[3][3], R[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) G[a][b] = s->grad[1 + a][b][c];
    double cs = cos(ang), sn = sin(ang);
    double Rm[3][3] = {{cs, -sn, 0}, {sn, cs, 0}, {0, 0, 1}};
    memcpy(R, Rm, sizeof(R));
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t = 0.0;
            for (int m = 0; m < 3; ++m) t += R[a][m] * G[m][b];
            RG[a][b] = t;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t = 0.0;
            for (int m = 0; m < 3; ++m) t += RG[a][m] * R[b][m];
            v->g[1 + a][b] = t;
        }
}

/* Neighbour of cell (i, j, k) across its face `axis`, side hi: returns the
 * mesh cell index and the rotation of its image, or -1 for a wall. */
static long neighbour(const orc_curv3 *s, const int *ijk, int axis, int hi, double *ang)
{
    int q[3] = {ijk[0], ijk[1], ijk[2]};
    q[axis] += hi ? 1 : -1;
    *ang = 0.0;
    if (q[axis] < 0 || q[axis] >= s->n[axis]) {
        if (s->c.bc[2 * axis] != ORC_PERIODIC) return -1;
        if (q[axis] < 0) {
            q[axis] += s->n[axis];
            *ang = -s->c.rot[axis];
        } else {
            q[axis] -= s->n[axis];
            *ang = s->c.rot[axis];
        }
    }
    return cid(s, q[0], q[1], q[2]);
}

static void compute_primitives(orc_curv3 *s)
{
    for (long c = 0; c < s->N; ++c) {
        double r = s->U[0][c];
        double dens = s->c.deviation ? 1.0 + r : r;
        s->prim[0][c] = r;
        for (int p = 1; p < 5; ++p) s->prim[p][c] = s->U[p][c] / dens;
    }
}

static void compute_gradients(orc_curv3 *s)
{
    for (int k = 0; k < s->n[2]; ++k)
        for (int j = 0; j < s->n[1]; ++j)
            for (int i = 0; i < s->n[0]; ++i) {
                long c = cid(s, i, j, k);
                int ijk[3] = {i, j, k};
                double acc[5][3];
                memset(acc, 0, sizeof(acc));
                for (int axis = 0; axis < 3; ++axis)
                    for (int hi = 0; hi < 2; ++hi) {
                        int p[3] = {i, j, k};
                        p[axis] += hi;
                        face3 f;
                        face_geom(s, axis, p, &f);
                        double so = hi ? 1.0 : -1.0;
                        double ang;
                        long nb = neighbour(s, ijk, axis, hi, &ang);
                        double phi[5];
                        if (nb < 0) {
                            int kind = s->c.bc[2 * axis + hi];
                            phi[0] = s->prim[0][c];
                            phi[1] = phi[2] = phi[3] = 0.0;
                            phi[4] = kind == ORC_WALL_ISOTHERMAL ? store_T(s, s->c.Tw[2 * axis + hi]) : s->prim[4][c];
                        } else {
                            cellv nv;
                            cell_view(s, nb, ang, 0, &nv);
                            double xP[3] = {s->cx[c], s->cy[c], s->cz[c]}, dP[3], dN[3];
                            for (int a = 0; a < 3; ++a) {
                                dP[a] = xP[a] - f.xs[a];
                                dN[a] = nv.x[a] - f.xs[a];
                            }
                            double lP = sqrt(dot(dP, dP)), lN = sqrt(dot(dN, dN));
                            for (int q = 0; q < 5; ++q) phi[q] = (s->prim[q][c] * lN + nv.p[q] * lP) / (lP + lN);
                        }
                        for (int q = 0; q < 5; ++q)
                            for (int a = 0; a < 3; ++a) acc[q][a] += phi[q] * so * f.S[a];
                    }
                for (int q = 0; q < 5; ++q)
                    for (int a = 0; a < 3; ++a) s->grad[q][a][c] = acc[q][a] / s->vol[c];
            }
}

/* Interior-face flux along +n times dS (global components) between the low
 * side A and the high side B. */
static void interior_flux(const orc_curv3 *s, const face3 *f, const cellv *A, const cellv *B, double *F)
{
    const double *e[3] = {f->n, f->t1, f->t2};
    double pA[5], pB[5], gA[15], gB[15], xSL[3], xSR[3], fdir[3], Fl[5];
    const cellv *sides[2] = {A, B};
    double *pp[2] = {pA, pB}, *gg[2] = {gA, gB};
    for (int m = 0; m < 2; ++m) {
        const cellv *v = sides[m];
        pp[m][0] = v->p[0];
        pp[m][4] = v->p[4];
        for (int q = 0; q < 3; ++q) pp[m][1 + q] = dot(v->p + 1, e[q]);
        for (int k = 0; k < 3; ++k) {
            gg[m][0 * 3 + k] = dot(v->g[0], e[k]);
            gg[m][4 * 3 + k] = dot(v->g[4], e[k]);
            for (int q = 0; q < 3; ++q) { /* d_k u_q = e_q . (grad u) e_k */
                double t = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) t += e[q][a] * v->g[1 + a][b] * e[k][b];
                gg[m][(1 + q) * 3 + k] = t;
            }
        }
    }
    double rL[3], rR[3];
    for (int a = 0; a < 3; ++a) {
        rL[a] = f->xs[a] - A->x[a];
        rR[a] = f->xs[a] - B->x[a];
    }
    for (int k = 0; k < 3; ++k) {
        xSL[k] = dot(rL, e[k]);
        xSR[k] = dot(rR, e[k]);
        fdir[k] = dot(s->c.up, e[k]);
    }
    orc_face_flux_frame(&s->fc, pA, gA, pB, gB, xSL, xSR, fdir, s->c.Tb, Fl, NULL);
    F[0] = Fl[0] * f->dS;
    for (int a = 0; a < 3; ++a) F[1 + a] = (Fl[1] * e[0][a] + Fl[2] * e[1][a] + Fl[3] * e[2][a]) * f->dS;
    F[4] = Fl[4] * f->dS;
}

static void accumulate_fluxes(orc_curv3 *s)
{
    for (int p = 0; p < 5; ++p) memset(s->rhs[p], 0, sizeof(double) * s->N);
    for (int k = 0; k < s->n[2]; ++k)
        for (int j = 0; j < s->n[1]; ++j)
            for (int i = 0; i < s->n[0]; ++i) {
                long c = cid(s, i, j, k);
                int ijk[3] = {i, j, k};
                for (int axis = 0; axis < 3; ++axis)
                    for (int hi = 0; hi < 2; ++hi) {
                        int p[3] = {i, j, k};
                        p[axis] += hi;
                        face3 f;
                        face_geom(s, axis, p, &f);
                        double ang, F[5];
                        long nb = neighbour(s, ijk, axis, hi, &ang);
                        if (nb < 0) { /* wall: outward flux, outward normal so n */
                            double so = hi ? 1.0 : -1.0, no[3], xP[3] = {s->cx[c], s->cy[c], s->cz[c]}, rP[3];
                            for (int a = 0; a < 3; ++a) {
                                no[a] = so * f.n[a];
                                rP[a] = f.xs[a] - xP[a];
                            }
                            double d = dot(rP, no);
                            int kind = s->c.bc[2 * axis + hi];
                            double r = s->U[0][c];
                            double dens = s->c.deviation ? 1.0 + r : r;
                            double m[3] = {s->U[1][c], s->U[2][c], s->U[3][c]};
                            double mn = dot(m, no);
                            double Fo[5];
                            Fo[0] = 0.0;
                            for (int a = 0; a < 3; ++a)
                                Fo[1 + a] = CS2 * r * no[a] + s->c.nu * (m[a] + 2.0 * mn * no[a]) / d;
                            Fo[4] = kind == ORC_WALL_ISOTHERMAL
                                        ? -s->c.chi * (dens * store_T(s, s->c.Tw[2 * axis + hi]) - s->U[4][c]) / d
                                        : 0.0;
                            for (int q = 0; q < 5; ++q) s->rhs[q][c] -= Fo[q] * f.dS;
                            continue;
                        }
                        cellv P, Nb;
                        cell_view(s, c, 0.0, 1, &P);
                        cell_view(s, nb, ang, 1, &Nb);
                        if (hi) {
                            interior_flux(s, &f, &P, &Nb, F);
                            for (int q = 0; q < 5; ++q) s->rhs[q][c] -= F[q];
                        } else {
                            interior_flux(s, &f, &Nb, &P, F);
                            for (int q = 0; q < 5; ++q) s->rhs[q][c] += F[q];
                        }
                    }
            }
}

static void update(orc_curv3 *s)
{
    const int dev = s->c.deviation;
    double du = 0.0, su = 0.0, dT = 0.0, sT = 0.0;
    for (long c = 0; c < s->N; ++c) {
        for (int p = 0; p < 5; ++p) s->Unew[p][c] = s->U[p][c] + s->c.dt / s->vol[c] * s->rhs[p][c];
        double r = s->U[0][c];
        double dens = dev ? 1.0 + r : r;
        double Tm = dev ? s->prim[4][c] + (T0 - s->c.Tb) : s->prim[4][c] - s->c.Tb;
        for (int a = 0; a < 3; ++a)
            if (s->c.up[a] != 0.0) s->Unew[1 + a][c] += s->c.dt * s->c.beta_g * dens * Tm * s->c.up[a];
        double rn = s->Unew[0][c];
        double densn = dev ? 1.0 + rn : rn;
        double uo = 0.0, un = 0.0;
        for (int a = 0; a < 3; ++a) {
            double vo = s->prim[1 + a][c], vn = s->Unew[1 + a][c] / densn;
            uo += vo * vo;
            un += vn * vn;
        }
        uo = sqrt(uo);
        un = sqrt(un);
        double To = s->prim[4][c] + (dev ? T0 : 0.0);
        double Tn = s->Unew[4][c] / densn + (dev ? T0 : 0.0);
        du += fabs(un - uo);
        su += un;
        dT += fabs(Tn - To);
        sT += Tn;
    }
    s->res_u = su > 0.0 ? du / su : 0.0;
    s->res_T = sT != 0.0 ? dT / sT : 0.0;
    for (int p = 0; p < 5; ++p) {
        double *t = s->U[p];
        s->U[p] = s->Unew[p];
        s->Unew[p] = t;
    }
}

/* ----------------------------------------------------------------- API -- */

void orc_curv3_destroy(orc_curv3 *s)
{
    if (!s) return;
    free(s->vx);
    free(s->vy);
    free(s->vz);
    free(s->cx);
    free(s->cy);
    free(s->cz);
    free(s->vol);
    for (int p = 0; p < 5; ++p) {
        free(s->U[p]);
        free(s->Unew[p]);
        free(s->prim[p]);
        free(s->rhs[p]);
        for (int a = 0; a < 3; ++a) free(s->grad[p][a]);
    }
    free(s);
}

int orc_curv3_create(const orc_curv3_cfg *cfg, const double *x, const double *y, const double *z, orc_curv3 **out)
{
    if (!cfg || !x || !y || !z || !out) return -1;
    for (int a = 0; a < 3; ++a) {
        if (cfg->n[a] < 1) return -1;
        if ((cfg->bc[2 * a] == ORC_PERIODIC) != (cfg->bc[2 * a + 1] == ORC_PERIODIC)) return -1;
        if (cfg->bc[2 * a] != ORC_PERIODIC && cfg->n[a] < 2) return -1;
    }
    for (int k = 0; k < 6; ++k)
        if (cfg->bc[k] < 0 || cfg->bc[k] > ORC_WALL_ADIABATIC) return -1;
    orc_curv3 *s = (orc_curv3 *)calloc(1, sizeof(orc_curv3));
    if (!s) return -1;
    s->c = *cfg;
    for (int a = 0; a < 3; ++a) s->n[a] = cfg->n[a];
    s->N = (long)s->n[0] * s->n[1] * s->n[2];
    long NV = (long)(s->n[0] + 1) * (s->n[1] + 1) * (s->n[2] + 1);
    s->vx = (double *)malloc(sizeof(double) * NV);
    s->vy = (double *)malloc(sizeof(double) * NV);
    s->vz = (double *)malloc(sizeof(double) * NV);
    s->cx = (double *)malloc(sizeof(double) * s->N);
    s->cy = (double *)malloc(sizeof(double) * s->N);
    s->cz = (double *)malloc(sizeof(double) * s->N);
    s->vol = (double *)malloc(sizeof(double) * s->N);
    int ok = s->vx && s->vy && s->vz && s->cx && s->cy && s->cz && s->vol;
    for (int p = 0; p < 5 && ok; ++p) {
        s->U[p] = (double *)calloc(s->N, sizeof(double));
        s->Unew[p] = (double *)calloc(s->N, sizeof(double));
        s->prim[p] = (double *)calloc(s->N, sizeof(double));
        s->rhs[p] = (double *)calloc(s->N, sizeof(double));
        ok = s->U[p] && s->Unew[p] && s->prim[p] && s->rhs[p];
        for (int a = 0; a < 3 && ok; ++a) ok = (s->grad[p][a] = (double *)calloc(s->N, sizeof(double))) != NULL;
    }
    if (!ok) {
        orc_curv3_destroy(s);
        return -1;
    }
    memcpy(s->vx, x, sizeof(double) * NV);
    memcpy(s->vy, y, sizeof(double) * NV);
    memcpy(s->vz, z, sizeof(double) * NV);
    double scale = 0.0;
    for (long v = 0; v < NV; ++v) scale = fmax(scale, fmax(fabs(x[v]), fmax(fabs(y[v]), fabs(z[v]))));
    /* periodic pairs close the mesh, up to the stated rotation */
    for (int a = 0; a < 3; ++a) {
        if (cfg->bc[2 * a] != ORC_PERIODIC) continue;
        int lim[3] = {s->n[0], s->n[1], s->n[2]};
        lim[a] = 0;
        for (int k = 0; k <= lim[2]; ++k)
            for (int j = 0; j <= lim[1]; ++j)
                for (int i = 0; i <= lim[0]; ++i) {
                    int p0[3] = {i, j, k}, p1[3] = {i, j, k};
                    p1[a] = s->n[a];
                    double q0[3], q1[3], r0[3];
                    vert(s, p0, q0);
                    vert(s, p1, q1);
                    rotz(cfg->rot[a], q0, r0);
                    for (int b = 0; b < 3; ++b)
                        if (fabs(r0[b] - q1[b]) > 1e-9 * scale) {
                            orc_curv3_destroy(s);
                            return -1;
                        }
                }
    }
    s->orient = 1.0;
    int npos = 0;
    for (int k = 0; k < s->n[2]; ++k)
        for (int j = 0; j < s->n[1]; ++j)
            for (int i = 0; i < s->n[0]; ++i) {
                long c = cid(s, i, j, k);
                double cc[3];
                double V = cell_shape(s, i, j, k, cc);
                if (!(V != 0.0)) {
                    orc_curv3_destroy(s);
                    return -1;
                }
                npos += V > 0.0;
                s->cx[c] = cc[0];
                s->cy[c] = cc[1];
                s->cz[c] = cc[2];
                s->vol[c] = fabs(V);
            }
    if (npos != 0 && npos != s->N) {
        orc_curv3_destroy(s);
        return -1;
    }
    s->orient = npos ? 1.0 : -1.0;
    memset(&s->fc, 0, sizeof(s->fc));
    s->fc.dim = 3;
    s->fc.nu = cfg->nu;
    s->fc.chi = cfg->chi;
    s->fc.beta_g = cfg->beta_g;
    s->fc.dtl = cfg->dtl;
    s->fc.dt = cfg->dt;
    s->fc.deviation = cfg->deviation;
    s->fc.force_in_predictor = cfg->force_in_predictor;
    s->fc.method = cfg->method;
    s->fc.gravity_axis = -1;
    for (long c = 0; c < s->N; ++c) s->U[0][c] = cfg->deviation ? 0.0 : 1.0;
    for (long c = 0; c < s->N; ++c) s->U[4][c] = store_T(s, T0);
    *out = s;
    return 0;
}

int orc_curv3_step(orc_curv3 *s, long nsteps)
{
    for (long k = 0; k < nsteps; ++k) {
        compute_primitives(s);
        compute_gradients(s);
        accumulate_fluxes(s);
        update(s);
    }
    return 0;
}

int orc_curv3_set_prim(orc_curv3 *s, const double *rho, const double *u, const double *T)
{
    for (long c = 0; c < s->N; ++c) {
        s->U[0][c] = s->c.deviation ? rho[c] - 1.0 : rho[c];
        for (int a = 0; a < 3; ++a) s->U[1 + a][c] = rho[c] * u[a * s->N + c];
        s->U[4][c] = rho[c] * store_T(s, T[c]);
    }
    return 0;
}

int orc_curv3_get_prim(const orc_curv3 *s, int f, double *out)
{
    if (f < 0 || f > 4) return -1;
    for (long c = 0; c < s->N; ++c) {
        double r = s->U[0][c];
        double dens = s->c.deviation ? 1.0 + r : r;
        if (f == 0) out[c] = dens;
        else if (f < 4) out[c] = s->U[f][c] / dens;
        else out[c] = s->U[4][c] / dens + (s->c.deviation ? T0 : 0.0);
    }
    return 0;
}

void orc_curv3_cells(const orc_curv3 *s, double *cx, double *cy, double *cz, double *vol)
{
    memcpy(cx, s->cx, sizeof(double) * s->N);
    memcpy(cy, s->cy, sizeof(double) * s->N);
    memcpy(cz, s->cz, sizeof(double) * s->N);
    memcpy(vol, s->vol, sizeof(double) * s->N);
}

void orc_curv3_residual(const orc_curv3 *s, double *out)
{
    out[0] = s->res_u;
    out[1] = s->res_T;
}

int orc_curv3_wall_heat(const orc_curv3 *s, int side, double *out)
{
    if (side < 0 || side > 5 || s->c.bc[side] != ORC_WALL_ISOTHERMAL) return -1;
    int axis = side / 2, hi = side & 1;
    double q = 0.0, A = 0.0;
    for (int k = 0; k < s->n[2]; ++k)
        for (int j = 0; j < s->n[1]; ++j)
            for (int i = 0; i < s->n[0]; ++i) {
                int ijk[3] = {i, j, k};
                if (ijk[axis] != (hi ? s->n[axis] - 1 : 0)) continue;
                long c = cid(s, i, j, k);
                int p[3] = {i, j, k};
                p[axis] += hi;
                face3 f;
                face_geom(s, axis, p, &f);
                double so = hi ? 1.0 : -1.0;
                double d = so * ((f.xs[0] - s->cx[c]) * f.n[0] + (f.xs[1] - s->cy[c]) * f.n[1] +
                                 (f.xs[2] - s->cz[c]) * f.n[2]);
                double r = s->U[0][c];
                double dens = s->c.deviation ? 1.0 + r : r;
                double TP = s->U[4][c] / dens + (s->c.deviation ? T0 : 0.0);
                q += (s->c.Tw[side] - TP) / d * f.dS;
                A += f.dS;
            }
    out[0] = q;
    out[1] = A;
    return 0;
}

void orc_curv3_integrals(const orc_curv3 *s, double *out)
{
    double mdev = 0.0, mass = 0.0, en = 0.0, vol = 0.0;
    for (long c = 0; c < s->N; ++c) {
        double r = s->c.deviation ? s->U[0][c] : s->U[0][c] - 1.0;
        double dens = 1.0 + r;
        double e = s->c.deviation ? s->U[4][c] + T0 * dens : s->U[4][c];
        mdev += r * s->vol[c];
        mass += (s->c.deviation ? dens : s->U[0][c]) * s->vol[c];
        en += e * s->vol[c];
        vol += s->vol[c];
    }
    out[0] = mdev;
    out[1] = mass;
    out[2] = en;
    out[3] = vol;
}
