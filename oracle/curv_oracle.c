/*
 * curv_oracle.c -- plain FP64 CPU oracle of the RTLBFS step on a 2D
 * body-fitted quadrilateral mesh (the meshes of Secs. 4.3 and 4.5).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, never by the product
 * path; it shares no code with the GPU library.
 *
 * One step, in the order of Sec. 3.2:
 *   1. primitives of every cell;
 *   2. Eq. 55 cell gradients, (1/dV) sum_k phi_S n_k dS_k over the four faces
 *      with the outward normal, and Eq. 56 inverse-distance face values;
 *   3. for every interior face, the flux of Sec. 3.2 (or Sec. 2.2) computed in
 *      the face frame (n, t): the primitives and gradients of both cells are
 *      rotated into it, Eq. 29 places the D2Q9 nodes at x_S + h (a n + b t),
 *      and the momentum flux is rotated back;
 *   4. forward-Euler update of Eqs. 41-43 with the Eq. 64 body force.
 *
 * Readings where the paper is silent (listed in the design notes):
 *   - geometry: cell centre = centroid of the quadrilateral; face centre =
 *     edge midpoint; the wall distance d of the one-sided wall closure is the
 *     distance of the centroid from the face along its normal;
 *   - walls: the closure of the Cartesian oracle written in the face frame
 *     (zero mass flux, pressure c_s^2 r, viscous stress with V_n = -3 m_n/d,
 *     V_t = -m_t/d, conduction -chi (rho T_w - e)/d on isothermal walls);
 *   - far field: a ghost cell mirrored across the face (same normal
 *     distance, zero gradient) that holds the free-stream state Sec. 4.3
 *     prescribes (rho_inf = 1, u_inf, T_inf); the face is then an ordinary
 *     interior face;
 *   - buoyancy F = beta_g rho (T - T_b) along the given upward unit vector,
 *     with T_b the far-field temperature in mixed convection.
 */
#include "curv_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define CS2 (1.0 / 3.0)
#define T0 0.5 /* temperature offset of the deviation storage */

struct orc_curv {
    orc_curv_cfg c;
    orc_cfg fc; /* the part of the configuration the face flux reads */
    int ni, nj;
    long N;
    double orient; /* +1 if the corners run counter-clockwise, else -1 */
    double *vx, *vy;
    double *cx, *cy, *area;
    double *U[4], *Unew[4], *prim[4], *grad[4][2], *rhs[4];
    double res_u, res_T;
};

typedef struct {
    double xs[2]; /* edge midpoint */
    double n[2];  /* unit normal, pointing to +i (i-faces) or +j (j-faces) */
    double dS;    /* edge length */
    long L, R;    /* cells on the low and high side, -1 where there is none */
    int side;     /* boundary side (0 i-, 1 i+, 2 j-, 3 j+) of a face with one cell, else -1 */
} face_t;

static long vid(const orc_curv *s, int i, int j) { return (long)j * (s->ni + 1) + i; }
static long cid(const orc_curv *s, int i, int j) { return (long)j * s->ni + i; }
static int is_wall(int k) { return k == ORC_WALL_ISOTHERMAL || k == ORC_WALL_ADIABATIC; }

/* Signed area and centroid of cell (i, j) (polygon formulas, corners taken
 * relative to the first one to keep the products small). */
static double cell_shape(const orc_curv *s, int i, int j, double *cx, double *cy)
{
    long v[4] = {vid(s, i, j), vid(s, i + 1, j), vid(s, i + 1, j + 1), vid(s, i, j + 1)};
    double x[4], y[4];
    for (int k = 0; k < 4; ++k) {
        x[k] = s->vx[v[k]] - s->vx[v[0]];
        y[k] = s->vy[v[k]] - s->vy[v[0]];
    }
    double A = 0.0, Cx = 0.0, Cy = 0.0;
    for (int k = 0; k < 4; ++k) {
        int l = (k + 1) % 4;
        double cr = x[k] * y[l] - x[l] * y[k];
        A += 0.5 * cr;
        Cx += (x[k] + x[l]) * cr;
        Cy += (y[k] + y[l]) * cr;
    }
    *cx = s->vx[v[0]] + Cx / (6.0 * A);
    *cy = s->vy[v[0]] + Cy / (6.0 * A);
    return A;
}

/* Face `axis` (0: between cells (i-1, j) and (i, j); 1: between (i, j-1) and
 * (i, j)). */
static void face_of(const orc_curv *s, int axis, int i, int j, face_t *f)
{
    long a = vid(s, i, j), b = axis == 0 ? vid(s, i, j + 1) : vid(s, i + 1, j);
    double ex = s->vx[b] - s->vx[a], ey = s->vy[b] - s->vy[a];
    f->xs[0] = 0.5 * (s->vx[a] + s->vx[b]);
    f->xs[1] = 0.5 * (s->vy[a] + s->vy[b]);
    f->dS = sqrt(ex * ex + ey * ey);
    double nx = axis == 0 ? ey : -ey, ny = axis == 0 ? -ex : ex;
    f->n[0] = s->orient * nx / f->dS;
    f->n[1] = s->orient * ny / f->dS;
    int per = s->c.bc[2 * axis] == ORC_PERIODIC;
    f->side = -1;
    if (axis == 0) {
        f->R = i < s->ni ? cid(s, i, j) : -1;
        f->L = i > 0 ? cid(s, i - 1, j) : (per ? cid(s, s->ni - 1, j) : -1);
    } else {
        f->R = j < s->nj ? cid(s, i, j) : -1;
        f->L = j > 0 ? cid(s, i, j - 1) : (per ? cid(s, i, s->nj - 1) : -1);
    }
    if (f->L < 0) f->side = 2 * axis;
    if (f->R < 0) f->side = 2 * axis + 1;
}

/* Faces of one axis in a fixed order: i-faces (i, j) with i = 0..ni (ni - 1
 * when periodic: face ni is face 0), then j-faces likewise. */
static int face_count(const orc_curv *s, int axis, int *n_along, int *n_across)
{
    int per = s->c.bc[2 * axis] == ORC_PERIODIC;
    if (axis == 0) {
        *n_along = s->ni + (per ? 0 : 1);
        *n_across = s->nj;
    } else {
        *n_along = s->nj + (per ? 0 : 1);
        *n_across = s->ni;
    }
    return *n_along * *n_across;
}

static void face_at(const orc_curv *s, int axis, int along, int across, face_t *f)
{
    if (axis == 0) face_of(s, 0, along, across, f);
    else face_of(s, 1, across, along, f);
}

static double store_T(const orc_curv *s, double Tabs) { return s->c.deviation ? Tabs - T0 : Tabs; }

/* Ghost primitives (storage convention) of a far-field face: the free
 * stream. */
static void ghost_prim(const orc_curv *s, double *G)
{
    G[0] = s->c.deviation ? 0.0 : 1.0;
    G[1] = s->c.u_inf[0];
    G[2] = s->c.u_inf[1];
    G[3] = store_T(s, s->c.T_inf);
}

static void compute_primitives(orc_curv *s)
{
    for (long c = 0; c < s->N; ++c) {
        double r = s->U[0][c];
        double dens = s->c.deviation ? 1.0 + r : r;
        s->prim[0][c] = r;
        s->prim[1][c] = s->U[1][c] / dens;
        s->prim[2][c] = s->U[2][c] / dens;
        s->prim[3][c] = s->U[3][c] / dens;
    }
}

/* Eq. 55 with Eq. 56 face values, accumulated face by face. */
static void compute_gradients(orc_curv *s)
{
    for (int p = 0; p < 4; ++p)
        for (int a = 0; a < 2; ++a) memset(s->grad[p][a], 0, sizeof(double) * s->N);
    for (int axis = 0; axis < 2; ++axis) {
        int na, nc;
        face_count(s, axis, &na, &nc);
        for (int al = 0; al < na; ++al)
            for (int ac = 0; ac < nc; ++ac) {
                face_t f;
                face_at(s, axis, al, ac, &f);
                if (f.side < 0) {
                    double dL = hypot(s->cx[f.L] - f.xs[0], s->cy[f.L] - f.xs[1]);
                    double dR = hypot(s->cx[f.R] - f.xs[0], s->cy[f.R] - f.xs[1]);
                    for (int p = 0; p < 4; ++p) {
                        double phi = (s->prim[p][f.L] * dR + s->prim[p][f.R] * dL) / (dL + dR);
                        for (int a = 0; a < 2; ++a) {
                            s->grad[p][a][f.L] += phi * f.n[a] * f.dS;
                            s->grad[p][a][f.R] -= phi * f.n[a] * f.dS;
                        }
                    }
                    continue;
                }
                long P = f.L >= 0 ? f.L : f.R;
                double sg = f.L >= 0 ? 1.0 : -1.0; /* outward normal = sg * n */
                double no[2] = {sg * f.n[0], sg * f.n[1]};
                int kind = s->c.bc[f.side];
                double phi[4];
                if (is_wall(kind)) {
                    phi[0] = s->prim[0][P]; /* zero normal density gradient */
                    phi[1] = phi[2] = 0.0;  /* no slip */
                    phi[3] = kind == ORC_WALL_ISOTHERMAL ? store_T(s, s->c.Tw[f.side]) : s->prim[3][P];
                } else { /* far field: mirrored ghost, equal distances */
                    double G[4];
                    ghost_prim(s, G);
                    for (int p = 0; p < 4; ++p) phi[p] = 0.5 * (s->prim[p][P] + G[p]);
                }
                for (int p = 0; p < 4; ++p)
                    for (int a = 0; a < 2; ++a) s->grad[p][a][P] += phi[p] * no[a] * f.dS;
            }
    }
    for (long c = 0; c < s->N; ++c)
        for (int p = 0; p < 4; ++p)
            for (int a = 0; a < 2; ++a) s->grad[p][a][c] /= s->area[c];
}

/* Primitives and gradients of cell c in the frame (e0, e1). */
static void to_frame(const orc_curv *s, long c, const double *e0, const double *e1, double *pl, double *gl)
{
    const double *e[2] = {e0, e1};
    memset(gl, 0, sizeof(double) * 12);
    pl[0] = s->prim[0][c];
    pl[1] = s->prim[1][c] * e0[0] + s->prim[2][c] * e0[1];
    pl[2] = s->prim[1][c] * e1[0] + s->prim[2][c] * e1[1];
    pl[3] = s->prim[3][c];
    for (int k = 0; k < 2; ++k) {
        gl[0 * 3 + k] = s->grad[0][0][c] * e[k][0] + s->grad[0][1][c] * e[k][1];
        gl[3 * 3 + k] = s->grad[3][0][c] * e[k][0] + s->grad[3][1][c] * e[k][1];
        for (int q = 0; q < 2; ++q) { /* d_k u_q = e_q . (grad u) . e_k */
            double v = 0.0;
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) v += e[q][a] * s->grad[1 + a][b][c] * e[k][b];
            gl[(1 + q) * 3 + k] = v;
        }
    }
}

static void add_flux(orc_curv *s, long c, double sign, const double *F, const double *e0, const double *e1, double dS)
{
    s->rhs[0][c] += sign * F[0] * dS;
    s->rhs[1][c] += sign * (F[1] * e0[0] + F[2] * e1[0]) * dS;
    s->rhs[2][c] += sign * (F[1] * e0[1] + F[2] * e1[1]) * dS;
    s->rhs[3][c] += sign * F[3] * dS;
}

static void accumulate_fluxes(orc_curv *s)
{
    for (int p = 0; p < 4; ++p) memset(s->rhs[p], 0, sizeof(double) * s->N);
    for (int axis = 0; axis < 2; ++axis) {
        int na, nc;
        face_count(s, axis, &na, &nc);
        for (int al = 0; al < na; ++al)
            for (int ac = 0; ac < nc; ++ac) {
                face_t f;
                face_at(s, axis, al, ac, &f);
                if (f.side < 0) { /* interior face, frame (n, t) with n from L to R */
                    double t[2] = {-f.n[1], f.n[0]};
                    double pL[4], pR[4], gL[12], gR[12], F[4];
                    to_frame(s, f.L, f.n, t, pL, gL);
                    to_frame(s, f.R, f.n, t, pR, gR);
                    double rL[2] = {f.xs[0] - s->cx[f.L], f.xs[1] - s->cy[f.L]};
                    double rR[2] = {f.xs[0] - s->cx[f.R], f.xs[1] - s->cy[f.R]};
                    double xSL[3] = {rL[0] * f.n[0] + rL[1] * f.n[1], rL[0] * t[0] + rL[1] * t[1], 0.0};
                    double xSR[3] = {rR[0] * f.n[0] + rR[1] * f.n[1], rR[0] * t[0] + rR[1] * t[1], 0.0};
                    double fdir[3] = {s->c.up[0] * f.n[0] + s->c.up[1] * f.n[1],
                                      s->c.up[0] * t[0] + s->c.up[1] * t[1], 0.0};
                    orc_face_flux_frame(&s->fc, pL, gL, pR, gR, xSL, xSR, fdir, s->c.Tb, F, NULL);
                    add_flux(s, f.L, -1.0, F, f.n, t, f.dS);
                    add_flux(s, f.R, +1.0, F, f.n, t, f.dS);
                    continue;
                }
                long P = f.L >= 0 ? f.L : f.R;
                double sg = f.L >= 0 ? 1.0 : -1.0;
                double no[2] = {sg * f.n[0], sg * f.n[1]}, to[2] = {-no[1], no[0]};
                double rP[2] = {f.xs[0] - s->cx[P], f.xs[1] - s->cy[P]};
                double d = rP[0] * no[0] + rP[1] * no[1]; /* normal distance centroid - face */
                int kind = s->c.bc[f.side];
                double F[4];
                if (is_wall(kind)) { /* outward fluxes of the wall closure */
                    double r = s->U[0][P];
                    double dens = s->c.deviation ? 1.0 + r : r;
                    double mn = s->U[1][P] * no[0] + s->U[2][P] * no[1];
                    double mt = s->U[1][P] * to[0] + s->U[2][P] * to[1];
                    F[0] = 0.0;
                    F[1] = CS2 * r + 3.0 * s->c.nu * mn / d;
                    F[2] = s->c.nu * mt / d;
                    F[3] = kind == ORC_WALL_ISOTHERMAL
                               ? -s->c.chi * (dens * store_T(s, s->c.Tw[f.side]) - s->U[3][P]) / d
                               : 0.0;
                } else { /* far field: P on the left of the frame (no, to), the ghost on the right */
                    double pL[4], gL[12], pR[4], gR[12], G[4];
                    to_frame(s, P, no, to, pL, gL);
                    ghost_prim(s, G);
                    pR[0] = G[0];
                    pR[1] = G[1] * no[0] + G[2] * no[1];
                    pR[2] = G[1] * to[0] + G[2] * to[1];
                    pR[3] = G[3];
                    memset(gR, 0, sizeof(gR));
                    double tP = rP[0] * to[0] + rP[1] * to[1];
                    double xSL[3] = {d, tP, 0.0}, xSR[3] = {-d, tP, 0.0};
                    double fdir[3] = {s->c.up[0] * no[0] + s->c.up[1] * no[1], s->c.up[0] * to[0] + s->c.up[1] * to[1],
                                      0.0};
                    orc_face_flux_frame(&s->fc, pL, gL, pR, gR, xSL, xSR, fdir, s->c.Tb, F, NULL);
                }
                add_flux(s, P, -1.0, F, no, to, f.dS);
            }
    }
}

static void update(orc_curv *s)
{
    const int dev = s->c.deviation;
    double du = 0.0, su = 0.0, dT = 0.0, sT = 0.0;
    for (long c = 0; c < s->N; ++c) {
        for (int p = 0; p < 4; ++p) s->Unew[p][c] = s->U[p][c] + s->c.dt / s->area[c] * s->rhs[p][c];
        double r = s->U[0][c];
        double dens = dev ? 1.0 + r : r;
        double Tm = dev ? s->prim[3][c] + (T0 - s->c.Tb) : s->prim[3][c] - s->c.Tb; /* T - T_b */
        for (int a = 0; a < 2; ++a)
            if (s->c.up[a] != 0.0) s->Unew[1 + a][c] += s->c.dt * s->c.beta_g * dens * Tm * s->c.up[a];
        /* Eq. 65 terms, absolute temperature */
        double rn = s->Unew[0][c];
        double densn = dev ? 1.0 + rn : rn;
        double uo = 0.0, un = 0.0;
        for (int a = 0; a < 2; ++a) {
            double vo = s->prim[1 + a][c], vn = s->Unew[1 + a][c] / densn;
            uo += vo * vo;
            un += vn * vn;
        }
        uo = sqrt(uo);
        un = sqrt(un);
        double To = s->prim[3][c] + (dev ? T0 : 0.0);
        double Tn = s->Unew[3][c] / densn + (dev ? T0 : 0.0);
        du += fabs(un - uo);
        su += un;
        dT += fabs(Tn - To);
        sT += Tn;
    }
    s->res_u = su > 0.0 ? du / su : 0.0;
    s->res_T = sT != 0.0 ? dT / sT : 0.0;
    for (int p = 0; p < 4; ++p) {
        double *t = s->U[p];
        s->U[p] = s->Unew[p];
        s->Unew[p] = t;
    }
}

/* ----------------------------------------------------------------- API -- */

void orc_curv_destroy(orc_curv *s)
{
    if (!s) return;
    free(s->vx);
    free(s->vy);
    free(s->cx);
    free(s->cy);
    free(s->area);
    for (int p = 0; p < 4; ++p) {
        free(s->U[p]);
        free(s->Unew[p]);
        free(s->prim[p]);
        free(s->rhs[p]);
        for (int a = 0; a < 2; ++a) free(s->grad[p][a]);
    }
    free(s);
}

int orc_curv_create(const orc_curv_cfg *cfg, const double *x, const double *y, orc_curv **out)
{
    if (!cfg || !x || !y || !out) return -1;
    if (cfg->ni < 2 || cfg->nj < 2) return -1;
    for (int k = 0; k < 4; ++k)
        if (cfg->bc[k] < 0 || cfg->bc[k] > ORC_FARFIELD) return -1;
    for (int a = 0; a < 2; ++a)
        if ((cfg->bc[2 * a] == ORC_PERIODIC) != (cfg->bc[2 * a + 1] == ORC_PERIODIC)) return -1;
    orc_curv *s = (orc_curv *)calloc(1, sizeof(orc_curv));
    if (!s) return -1;
    s->c = *cfg;
    s->ni = cfg->ni;
    s->nj = cfg->nj;
    s->N = (long)s->ni * s->nj;
    long NV = (long)(s->ni + 1) * (s->nj + 1);
    s->vx = (double *)malloc(sizeof(double) * NV);
    s->vy = (double *)malloc(sizeof(double) * NV);
    s->cx = (double *)malloc(sizeof(double) * s->N);
    s->cy = (double *)malloc(sizeof(double) * s->N);
    s->area = (double *)malloc(sizeof(double) * s->N);
    int ok = s->vx && s->vy && s->cx && s->cy && s->area;
    for (int p = 0; p < 4 && ok; ++p) {
        s->U[p] = (double *)calloc(s->N, sizeof(double));
        s->Unew[p] = (double *)calloc(s->N, sizeof(double));
        s->prim[p] = (double *)calloc(s->N, sizeof(double));
        s->rhs[p] = (double *)calloc(s->N, sizeof(double));
        ok = s->U[p] && s->Unew[p] && s->prim[p] && s->rhs[p];
        for (int a = 0; a < 2 && ok; ++a) ok = (s->grad[p][a] = (double *)calloc(s->N, sizeof(double))) != NULL;
    }
    if (!ok) {
        orc_curv_destroy(s);
        return -1;
    }
    memcpy(s->vx, x, sizeof(double) * NV);
    memcpy(s->vy, y, sizeof(double) * NV);
    /* closed periodic sides */
    double scale = 0.0;
    for (long v = 0; v < NV; ++v) scale = fmax(scale, fmax(fabs(x[v]), fabs(y[v])));
    if (cfg->bc[0] == ORC_PERIODIC)
        for (int j = 0; j <= s->nj; ++j)
            if (fabs(x[vid(s, 0, j)] - x[vid(s, s->ni, j)]) > 1e-12 * scale ||
                fabs(y[vid(s, 0, j)] - y[vid(s, s->ni, j)]) > 1e-12 * scale) {
                orc_curv_destroy(s);
                return -1;
            }
    if (cfg->bc[2] == ORC_PERIODIC)
        for (int i = 0; i <= s->ni; ++i)
            if (fabs(x[vid(s, i, 0)] - x[vid(s, i, s->nj)]) > 1e-12 * scale ||
                fabs(y[vid(s, i, 0)] - y[vid(s, i, s->nj)]) > 1e-12 * scale) {
                orc_curv_destroy(s);
                return -1;
            }
    /* cells: one orientation for all */
    int npos = 0;
    for (int j = 0; j < s->nj; ++j)
        for (int i = 0; i < s->ni; ++i) {
            long c = cid(s, i, j);
            double A = cell_shape(s, i, j, &s->cx[c], &s->cy[c]);
            if (A > 0.0) ++npos;
            else if (!(A < 0.0)) {
                orc_curv_destroy(s);
                return -1;
            }
            s->area[c] = fabs(A);
        }
    if (npos != 0 && npos != s->N) {
        orc_curv_destroy(s);
        return -1;
    }
    s->orient = npos ? 1.0 : -1.0;
    memset(&s->fc, 0, sizeof(s->fc));
    s->fc.dim = 2;
    s->fc.nu = cfg->nu;
    s->fc.chi = cfg->chi;
    s->fc.beta_g = cfg->beta_g;
    s->fc.dtl = cfg->dtl;
    s->fc.dt = cfg->dt;
    s->fc.deviation = cfg->deviation;
    s->fc.force_in_predictor = cfg->force_in_predictor;
    s->fc.method = cfg->method;
    s->fc.gravity_axis = -1;
    /* far-field state everywhere */
    for (long c = 0; c < s->N; ++c) {
        s->U[0][c] = cfg->deviation ? 0.0 : 1.0;
        s->U[1][c] = cfg->u_inf[0];
        s->U[2][c] = cfg->u_inf[1];
        s->U[3][c] = store_T(s, cfg->T_inf);
    }
    *out = s;
    return 0;
}

int orc_curv_step(orc_curv *s, long nsteps)
{
    for (long k = 0; k < nsteps; ++k) {
        compute_primitives(s);
        compute_gradients(s);
        accumulate_fluxes(s);
        update(s);
    }
    return 0;
}

int orc_curv_set_prim(orc_curv *s, const double *rho, const double *u, const double *T)
{
    for (long c = 0; c < s->N; ++c) {
        s->U[0][c] = s->c.deviation ? rho[c] - 1.0 : rho[c];
        s->U[1][c] = rho[c] * u[c];
        s->U[2][c] = rho[c] * u[s->N + c];
        s->U[3][c] = rho[c] * store_T(s, T[c]);
    }
    return 0;
}

int orc_curv_get_prim(const orc_curv *s, int f, double *out)
{
    if (f < 0 || f > 3) return -1;
    for (long c = 0; c < s->N; ++c) {
        double r = s->U[0][c];
        double dens = s->c.deviation ? 1.0 + r : r;
        if (f == 0) out[c] = dens;
        else if (f < 3) out[c] = s->U[f][c] / dens;
        else out[c] = s->U[3][c] / dens + (s->c.deviation ? T0 : 0.0);
    }
    return 0;
}

int orc_curv_get_stored(const orc_curv *s, int f, double *out)
{
    if (f < 0 || f > 3) return -1;
    memcpy(out, s->U[f], sizeof(double) * s->N);
    return 0;
}

void orc_curv_cells(const orc_curv *s, double *cx, double *cy, double *area)
{
    memcpy(cx, s->cx, sizeof(double) * s->N);
    memcpy(cy, s->cy, sizeof(double) * s->N);
    memcpy(area, s->area, sizeof(double) * s->N);
}

void orc_curv_residual(const orc_curv *s, double *out)
{
    out[0] = s->res_u;
    out[1] = s->res_T;
}

int orc_curv_wall_heat(const orc_curv *s, int side, double *out)
{
    if (side < 0 || side > 3 || s->c.bc[side] != ORC_WALL_ISOTHERMAL) return -1;
    int axis = side / 2, hi = side & 1;
    int na, nc;
    face_count(s, axis, &na, &nc);
    double q = 0.0, A = 0.0;
    for (int ac = 0; ac < nc; ++ac) {
        face_t f;
        face_at(s, axis, hi ? na - 1 : 0, ac, &f);
        long P = f.L >= 0 ? f.L : f.R;
        double sg = f.L >= 0 ? 1.0 : -1.0;
        double d = (f.xs[0] - s->cx[P]) * sg * f.n[0] + (f.xs[1] - s->cy[P]) * sg * f.n[1];
        double r = s->U[0][P];
        double dens = s->c.deviation ? 1.0 + r : r;
        double TP = s->U[3][P] / dens + (s->c.deviation ? T0 : 0.0);
        q += (s->c.Tw[side] - TP) / d * f.dS;
        A += f.dS;
    }
    out[0] = q;
    out[1] = A;
    return 0;
}

void orc_curv_integrals(const orc_curv *s, double *out)
{
    double mdev = 0.0, mass = 0.0, en = 0.0, vol = 0.0;
    for (long c = 0; c < s->N; ++c) {
        double r = s->c.deviation ? s->U[0][c] : s->U[0][c] - 1.0;
        double dens = 1.0 + r;
        double e = s->c.deviation ? s->U[3][c] + T0 * dens : s->U[3][c];
        mdev += r * s->area[c];
        mass += (s->c.deviation ? dens : s->U[0][c]) * s->area[c];
        en += e * s->area[c];
        vol += s->area[c];
    }
    out[0] = mdev;
    out[1] = mass;
    out[2] = en;
    out[3] = vol;
}
