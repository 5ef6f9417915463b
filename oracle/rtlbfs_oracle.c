/*
 * rtlbfs_oracle.c -- plain FP64 CPU oracle of one RTLBFS time step.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark, never by the product path.  It shares no
 * code with the GPU library.
 *
 * What it computes (Lu, Dai & Yu, arXiv 2202.13449):
 *   Sec. 3.2(a) predictor: at every interior face a unit lattice (D2Q9 offsets
 *     in 2D, D3Q19 in 3D) is centred on the face; node values are filled by
 *     the one-sided linear reconstruction of Eq. 29 from cell gradients given
 *     by the discrete Gauss theorem (Eq. 55) with inverse-distance face values
 *     (Eq. 56); Eqs. 46-48 are evaluated by central finite differences on the
 *     lattice nodes to give rho*, (rho u)*, (rho c_p T)* at the face centre.
 *   Sec. 3.2(b) corrector: face fluxes of Eqs. 57-59 (equivalently the closed
 *     forms Eqs. 49-51 rewritten with the time-n terms) and the forward-Euler
 *     finite-volume update of Eqs. 41-43, plus the Boussinesq body force of
 *     Eq. 64.
 *   Eq. 65 residual, Eq. 69 volume Nusselt number and wall Nusselt numbers.
 *
 * Readings where the text is silent or garbled (each is listed in the design
 * notes of the repository):
 *   - finite differences: D_a f = (f(+a) - f(-a))/2h, D_aa f = (f(+a) - 2f(0)
 *     + f(-a))/h^2, D_ab f = (f(+a+b) - f(+a-b) - f(-a+b) + f(-a-b))/4h^2, with
 *     lattice spacing h = c*dtl (the referenced FD scheme is not reproduced in
 *     the paper);
 *   - Eq. 55 carries the 1/dV factor and the outward normal;
 *   - primitives rho, u, T are reconstructed and products formed per node;
 *   - time-n face values are those of the centre node, face derivatives the
 *     lattice central differences;
 *   - buoyancy F = beta_g rho (T - T_ref) along +gravity_axis, applied in the
 *     cell update and (by default) in the predicted momentum;
 *   - walls: no lattice across the wall; zero mass flux, pressure rho_P c_s^2,
 *     one-sided viscous and conductive fluxes over the half-cell distance;
 *   - Eq. 65 uses the absolute temperature.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fPIC -shared (no fast-math).
 */
#include "rtlbfs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define CS2 (1.0 / 3.0) /* lattice sound speed squared, c_s^2 = c^2/3 (Eq. 6) */
#define TREF 0.5        /* T_ref = (T_h + T_l)/2 with T_l = 0, T_h = 1 (Eq. 64) */

struct orc_state {
    orc_cfg c;
    int D;
    long N;
    double L[3];          /* domain length per axis */
    double *node[3];      /* n+1 node coordinates per axis */
    double *ctr[3];       /* cell centres */
    double *wid[3];       /* cell widths */
    double *U[5];         /* stored conserved fields */
    double *Unew[5];
    double *prim[5];      /* rho (or r), u_a, T (or T') */
    double *grad[5][3];   /* Eq. 55 cell gradients */
    double *rhs[5];       /* -sum_k F_k dS_k per cell */
    double tau_f, tau_g;
    double res_u, res_T;
    long steps;
};

/* ------------------------------------------------------------------ mesh -- */

double orc_mesh_nodes(int n, double stretch, double *x)
{
    if (stretch <= 0.0) {
        for (int i = 0; i <= n; ++i) x[i] = (double)i;
        return (double)n;
    }
    /* Eq. 74 on a unit length, then rescaled so the smallest cell is 1. */
    double tp = tanh(stretch);
    for (int i = 0; i <= n; ++i)
        x[i] = (tp + tanh(2.0 * stretch * ((double)i / n - 0.5))) / (2.0 * tp);
    double hmin = 1e300;
    for (int i = 0; i < n; ++i)
        if (x[i + 1] - x[i] < hmin) hmin = x[i + 1] - x[i];
    double L = 1.0 / hmin;
    for (int i = 0; i <= n; ++i) x[i] *= L;
    return L;
}

void orc_physics_from_ra(double Ra, double Pr, double Ma, double L, double *out)
{
    /* Eq. 63: Ra = V_c^2 L^2/(nu chi), Pr = nu/chi, V_c^2 = beta g dT L. */
    double Vc = Ma;
    double nu = Vc * L * sqrt(Pr / Ra);
    out[0] = nu;
    out[1] = nu / Pr;
    out[2] = Vc * Vc / L;
}

double orc_splitmix_uniform(uint64_t seed, uint64_t i)
{
    /* SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): the state advances by the
     * golden gamma and each output is the state passed through the mix. */
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    double u01 = (double)(z >> 11) * (1.0 / 9007199254740992.0);
    return 2.0 * u01 - 1.0;
}

/* --------------------------------------------------------------- helpers -- */

static long cell_index(const orc_state *s, const int *ijk)
{
    return ijk[0] + (long)s->c.n[0] * (ijk[1] + (long)s->c.n[1] * ijk[2]);
}

static void cell_coords(const orc_state *s, long idx, int *ijk)
{
    ijk[0] = (int)(idx % s->c.n[0]);
    ijk[1] = (int)((idx / s->c.n[0]) % s->c.n[1]);
    ijk[2] = (s->D == 3) ? (int)(idx / ((long)s->c.n[0] * s->c.n[1])) : 0;
}

static double cell_volume(const orc_state *s, const int *ijk)
{
    double v = 1.0;
    for (int a = 0; a < s->D; ++a) v *= s->wid[a][ijk[a]];
    return v;
}

static double face_area(const orc_state *s, int axis, const int *ijk)
{
    double A = 1.0;
    for (int a = 0; a < s->D; ++a)
        if (a != axis) A *= s->wid[a][ijk[a]];
    return A;
}

static int is_wall(int kind) { return kind == ORC_WALL_ISOTHERMAL || kind == ORC_WALL_ADIABATIC; }

/* ------------------------------------------------------- lattice + fluxes -- */

/* Lattice node (a, b, c) offsets from the face centre in units of h.  In 2D the
 * nine D2Q9 offsets (c = 0); in 3D the nineteen D3Q19 offsets (no corners). */
static int node_in_lattice(int D, int a, int b, int c)
{
    if (D == 2) return c == 0;
    return abs(a) + abs(b) + abs(c) <= 2;
}

typedef struct {
    double v[3][3][3]; /* value at offset (a+1, b+1, c+1) */
} nodefield;

static double nf(const nodefield *f, const int *o) { return f->v[o[0] + 1][o[1] + 1][o[2] + 1]; }

/* Central differences on the local lattice (reading of the FD discretisation
 * of Eqs. 46-48). */
static double d1(const nodefield *f, int a, double h)
{
    int p[3] = {0, 0, 0}, m[3] = {0, 0, 0};
    p[a] = 1;
    m[a] = -1;
    return (nf(f, p) - nf(f, m)) / (2.0 * h);
}

static double d2(const nodefield *f, int a, int b, double h)
{
    if (a == b) {
        int p[3] = {0, 0, 0}, m[3] = {0, 0, 0}, z[3] = {0, 0, 0};
        p[a] = 1;
        m[a] = -1;
        return (nf(f, p) - 2.0 * nf(f, z) + nf(f, m)) / (h * h);
    }
    int pp[3] = {0, 0, 0}, pm[3] = {0, 0, 0}, mp[3] = {0, 0, 0}, mm[3] = {0, 0, 0};
    pp[a] = 1; pp[b] = 1;
    pm[a] = 1; pm[b] = -1;
    mp[a] = -1; mp[b] = 1;
    mm[a] = -1; mm[b] = -1;
    return (nf(f, pp) - nf(f, pm) - nf(f, mp) + nf(f, mm)) / (4.0 * h * h);
}

/* Primitives at every node of the face lattice by Eq. 29.  Node (a, b, c)
 * sits at x_S + h (a n + b t1 + c t2), where n is the frame axis `axis` and
 * t1, t2 the remaining axes in increasing order.  xSL = x_S - x_L and xSR =
 * x_S - x_R are the face centre relative to the two cell centres (on a
 * Cartesian mesh dL n and -dR n), so the node lies at xSL + h (a, b, c)
 * from the left centre and at xSR + h (a, b, c) from the right one.  val[p]
 * is indexed by the local offsets. */
static void reconstruct_nodes(const orc_cfg *cfg, int axis, const double *primL, const double *gradL,
                              const double *primR, const double *gradR, const double *xSL, const double *xSR,
                              nodefield *val)
{
    const int D = cfg->dim;
    const int NP = D + 2;
    const double h = cfg->dtl;
    memset(val, 0, sizeof(nodefield) * 5);
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                if (!node_in_lattice(D, a, b, c)) continue;
                int off[3] = {a, b, c};
                /* off[0] is the normal offset; off[1], off[2] the tangential
                 * ones mapped to the remaining axes in increasing order. */
                double rL[3] = {0, 0, 0}, rR[3] = {0, 0, 0};
                int t = 1;
                for (int ax = 0; ax < D; ++ax) {
                    int o = ax == axis ? a : off[t++];
                    rL[ax] = xSL[ax] + o * h;
                    rR[ax] = xSR[ax] + o * h;
                }
                for (int p = 0; p < NP; ++p) {
                    double vL = primL[p], vR = primR[p];
                    for (int ax = 0; ax < D; ++ax) {
                        vL += gradL[p * 3 + ax] * rL[ax];
                        vR += gradR[p * 3 + ax] * rR[ax];
                    }
                    double v;
                    if (a < 0) v = vL;           /* node on the left cell side */
                    else if (a > 0) v = vR;      /* node on the right cell side */
                    else v = 0.5 * (vL + vR);    /* node on the interface */
                    val[p].v[a + 1][b + 1][c + 1] = v;
                }
            }
}

static void tlbfs_face_flux(const orc_cfg *cfg, int axis, const nodefield *val, const double *fdir, double Tb,
                            double *flux, double *pred);

/* The interior-face flux along +axis of the frame the arguments are given in.
 * fdir: unit vector of the buoyancy (against gravity) in that frame, or zero;
 * Tb: the absolute reference temperature of the buoyancy force. */
static void face_flux_core(const orc_cfg *cfg, int axis, const double *primL, const double *gradL,
                           const double *primR, const double *gradR, const double *xSL, const double *xSR,
                           const double *fdir, double Tb, double *flux, double *pred)
{
    const int D = cfg->dim;
    const int dev = cfg->deviation;
    const double h = cfg->dtl; /* lattice spacing c*dtl with c = 1 */
    const double dtl = cfg->dtl;
    const double tau_f = 0.5 + cfg->nu / (CS2 * dtl); /* Eq. 9 */
    const double tau_g = 0.5 + cfg->chi / (CS2 * dtl); /* Eq. 10 */

    /* Step 1: primitives at the lattice nodes (Eq. 29). */
    nodefield val[5];
    reconstruct_nodes(cfg, axis, primL, gradL, primR, gradR, xSL, xSR, val);
    if (cfg->method == 1) {
        tlbfs_face_flux(cfg, axis, val, fdir, Tb, flux, pred);
        return;
    }

    /* Step 2: node values of the conserved quantities and of the moments that
     * Eqs. 46-48 differentiate.  Index the node fields by the GLOBAL axis:
     * re-map the (normal, t1, t2) offsets to global offsets. */
    nodefield rho, rhoN /* rho or r: the part of rho carrying pressure */, m[3], P[3][3], e, q[3],
        K[3][3];
    memset(&rho, 0, sizeof(rho));
    memset(&rhoN, 0, sizeof(rhoN));
    memset(m, 0, sizeof(m));
    memset(P, 0, sizeof(P));
    memset(&e, 0, sizeof(e));
    memset(q, 0, sizeof(q));
    memset(K, 0, sizeof(K));
    int tmap[3]; /* global axis of local offset slot 0, 1, 2 */
    {
        int t = 1;
        tmap[0] = axis;
        for (int ax = 0; ax < D; ++ax)
            if (ax != axis) tmap[t++] = ax;
        if (D == 2) tmap[2] = 2;
    }
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                if (!node_in_lattice(D, a, b, c)) continue;
                int loc[3] = {a, b, c};
                int g[3] = {0, 0, 0};
                for (int k = 0; k < 3; ++k) g[tmap[k]] = loc[k];
                int gi = g[0] + 1, gj = g[1] + 1, gk = g[2] + 1;
                double r0 = val[0].v[a + 1][b + 1][c + 1];
                double dens = dev ? 1.0 + r0 : r0;
                double u[3] = {0, 0, 0};
                for (int ax = 0; ax < D; ++ax) u[ax] = val[1 + ax].v[a + 1][b + 1][c + 1];
                double T = val[D + 1].v[a + 1][b + 1][c + 1]; /* T or T' */
                rho.v[gi][gj][gk] = dens;
                rhoN.v[gi][gj][gk] = r0;
                for (int x = 0; x < D; ++x) {
                    m[x].v[gi][gj][gk] = dens * u[x];
                    q[x].v[gi][gj][gk] = dens * u[x] * T;
                    for (int y = 0; y < D; ++y) {
                        K[x][y].v[gi][gj][gk] = dens * u[x] * u[y];
                        /* Pi = rho u u + rho c_s^2 I (Eqs. 7, 14); the deviation
                         * form keeps only r c_s^2 (a constant pressure has no
                         * finite-difference derivative and no net face force). */
                        P[x][y].v[gi][gj][gk] = dens * u[x] * u[y] + (x == y ? CS2 * r0 : 0.0);
                    }
                }
                e.v[gi][gj][gk] = dens * T; /* e = rho c_p T, or theta = rho c_p T' */
            }

    /* Step 3: predictor, Eqs. 46-48 with the buoyancy in the momentum. */
    const int z[3] = {0, 0, 0};
    double rho0 = nf(&rho, z), r0 = nf(&rhoN, z), e0 = nf(&e, z);
    double m0[3] = {0, 0, 0}, u0[3] = {0, 0, 0};
    for (int x = 0; x < D; ++x) {
        m0[x] = nf(&m[x], z);
        u0[x] = m0[x] / rho0;
    }
    double T0n = e0 / rho0; /* T or T' at the face centre */

    double drho = 0.0; /* rho* - rho_0 */
    for (int x = 0; x < D; ++x) drho -= dtl * d1(&m[x], x, h);
    for (int x = 0; x < D; ++x)
        for (int y = 0; y < D; ++y) drho += 0.5 * dtl * dtl * d2(&P[x][y], x, y, h);

    double force[3] = {0, 0, 0};
    if (cfg->force_in_predictor) {
        /* T - T_b from T' = T - T0 (deviation) or the absolute T */
        double Tabs_minus_ref = dev ? T0n + (TREF - Tb) : (T0n - Tb);
        for (int x = 0; x < D; ++x)
            if (fdir[x] != 0.0) force[x] = fdir[x] * cfg->beta_g * rho0 * Tabs_minus_ref; /* Eq. 64 */
    }
    double dm[3] = {0, 0, 0}; /* (rho u)* - (rho u)_0 */
    for (int x = 0; x < D; ++x) {
        double s = 0.0;
        for (int y = 0; y < D; ++y) s -= dtl * d1(&P[x][y], y, h);
        /* 0.5 c_s^2 dt^2 d_b [d_b m_a + d_a m_b + delta_ab d_g m_g]
         *   = 0.5 c_s^2 dt^2 [lap m_a + 2 d_a (div m)] */
        double lap = 0.0, graddiv = 0.0;
        for (int y = 0; y < D; ++y) {
            lap += d2(&m[x], y, y, h);
            graddiv += d2(&m[y], x, y, h);
        }
        s += 0.5 * CS2 * dtl * dtl * (lap + 2.0 * graddiv);
        s += dtl * force[x];
        dm[x] = s;
    }
    double de = 0.0; /* (rho c_p T)* - (rho c_p T)_0, or theta* - theta_0 */
    for (int x = 0; x < D; ++x) de -= dtl * d1(&q[x], x, h);
    for (int x = 0; x < D; ++x) de += 0.5 * CS2 * dtl * dtl * d2(&e, x, x, h);

    double rhos = rho0 + drho;
    double rNs = r0 + drho;
    double ms[3] = {0, 0, 0};
    for (int x = 0; x < D; ++x) ms[x] = m0[x] + dm[x];
    double es = e0 + de;
    if (pred) {
        pred[0] = rNs;
        for (int x = 0; x < D; ++x) pred[1 + x] = ms[x];
        pred[D + 1] = es;
    }

    /* Step 4: face fluxes per unit area along +axis (Eqs. 57-59 / 49-51). */
    const int n = axis;
    flux[0] = ms[n]; /* Eq. 57 / 49 */
    double divm = 0.0;
    for (int g = 0; g < D; ++g) divm += d1(&m[g], g, h);
    for (int x = 0; x < D; ++x) {
        double Pn = rho0 * u0[x] * u0[n] + (x == n ? CS2 * r0 : 0.0);
        double Ps = ms[x] * ms[n] / rhos + (x == n ? CS2 * rNs : 0.0);
        double V = d1(&m[x], n, h) + d1(&m[n], x, h) + (x == n ? divm : 0.0);
        flux[1 + x] = Pn - cfg->nu * V - (tau_f - 1.5) * (Ps - Pn); /* Eq. 58 */
    }
    double qn = rho0 * u0[n] * T0n; /* (rho c_p u_n T)^n, or with T' */
    if (!dev) {
        flux[D + 1] = qn - cfg->chi * d1(&e, n, h) - (tau_g - 1.5) * (ms[n] * es / rhos - qn); /* Eq. 59 */
    } else {
        /* Deviation storage: theta = e - T0 rho, so the stored energy is
         * advanced with Q - T0 P.  e* = T0 rho_e* + theta*, where rho_e* is
         * the density predictor with c_s^2 d_a d_b (rho delta_ab) only:
         * rho_e* - rho* = -0.5 dt^2 d_a d_b (rho u_a u_b). */
        double drho_e = 0.0;
        for (int x = 0; x < D; ++x)
            for (int y = 0; y < D; ++y) drho_e -= 0.5 * dtl * dtl * d2(&K[x][y], x, y, h);
        double Tpart = -(tau_g - 0.5) * dm[n] - cfg->chi * d1(&rhoN, n, h)
                       - (tau_g - 1.5) * ms[n] * drho_e / rhos;
        double Dpart = qn - cfg->chi * d1(&e, n, h) - (tau_g - 1.5) * (ms[n] * es / rhos - qn);
        flux[D + 1] = TREF * Tpart + Dpart;
    }
}

void orc_face_flux(const orc_cfg *cfg, int axis, const double *primL, const double *gradL,
                   const double *primR, const double *gradR, double dL, double dR,
                   double *flux, double *pred)
{
    double xSL[3] = {0, 0, 0}, xSR[3] = {0, 0, 0}, fdir[3] = {0, 0, 0};
    xSL[axis] = dL;
    xSR[axis] = -dR;
    if (cfg->gravity_axis >= 0) fdir[cfg->gravity_axis] = 1.0;
    face_flux_core(cfg, axis, primL, gradL, primR, gradR, xSL, xSR, fdir, TREF, flux, pred);
}

void orc_face_flux_frame(const orc_cfg *cfg, const double *primL, const double *gradL, const double *primR,
                         const double *gradR, const double *xSL, const double *xSR, const double *fdir, double Tb,
                         double *flux, double *pred)
{
    face_flux_core(cfg, 0, primL, gradL, primR, gradR, xSL, xSR, fdir, Tb, flux, pred);
}

/* TLBFS interface flux (Sec. 2.2), in the paper's order:
 *   (a) primitives at x_S - e_i dt by Eq. 29 (the lattice nodes above: node
 *       offset (a, b, c) = -e_i in the face frame), and f_i^eq, g_i^eq there
 *       by Eqs. 3-4;
 *   (b) the predicted rho*, rho* u*, rho* c_p T* at x_S by Eqs. 30-32 (the
 *       buoyancy enters the predicted momentum as dt F at the face centre,
 *       the same reading as for RTLBFS), and f_i^eq, g_i^eq at x_S from them;
 *   (c) the fluxes of Eqs. 38-40 along the face normal.
 * D2Q9 / D3Q19 velocities and weights of Eqs. 5-6 (c = 1), c_p = 1.  The
 * computation is done in absolute variables; with deviation storage the
 * node values are converted first and the fluxes afterwards (the r flux is the
 * rho flux, the theta flux is Q - T0 P, and the constant pressure c_s^2 is
 * left out of the momentum flux). */
static void tlbfs_face_flux(const orc_cfg *cfg, int axis, const nodefield *val, const double *fdir, double Tb,
                            double *flux, double *pred)
{
    const int D = cfg->dim;
    const int dev = cfg->deviation;
    const double dtl = cfg->dtl;
    const double tau_f = 0.5 + cfg->nu / (CS2 * dtl); /* Eq. 9 */
    const double tau_g = 0.5 + cfg->chi / (CS2 * dtl); /* Eq. 10 */
    int tmap[3];
    {
        int t = 1;
        tmap[0] = axis;
        for (int ax = 0; ax < D; ++ax)
            if (ax != axis) tmap[t++] = ax;
        if (D == 2) tmap[2] = 2;
    }

    /* (a) the discrete velocities with their weights and the equilibria at
     * the nodes they stream from */
    int Q = 0;
    double e[19][3], w[19], fb[19], gb[19];
    double rho_c = 0.0, T_c = 0.0; /* face-centre node (e_i = 0), for the force */
    for (int a = -1; a <= 1; ++a)
        for (int b = -1; b <= 1; ++b)
            for (int c = -1; c <= 1; ++c) {
                if (!node_in_lattice(D, a, b, c)) continue;
                int loc[3] = {a, b, c};
                double eg[3] = {0.0, 0.0, 0.0};
                for (int k = 0; k < 3; ++k) eg[tmap[k]] = -(double)loc[k]; /* e_i = -offset */
                int nz = abs(a) + abs(b) + abs(c);
                double wi = D == 2 ? (nz == 0 ? 4.0 / 9.0 : nz == 1 ? 1.0 / 9.0 : 1.0 / 36.0)
                                   : (nz == 0 ? 1.0 / 3.0 : nz == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
                double r0 = val[0].v[a + 1][b + 1][c + 1];
                double rho = dev ? 1.0 + r0 : r0;
                double u[3] = {0.0, 0.0, 0.0};
                for (int ax = 0; ax < D; ++ax) u[ax] = val[1 + ax].v[a + 1][b + 1][c + 1];
                double T = val[D + 1].v[a + 1][b + 1][c + 1] + (dev ? TREF : 0.0);
                double eu = 0.0, uu = 0.0;
                for (int ax = 0; ax < D; ++ax) {
                    eu += eg[ax] * u[ax];
                    uu += u[ax] * u[ax];
                }
                for (int ax = 0; ax < 3; ++ax) e[Q][ax] = eg[ax];
                w[Q] = wi;
                fb[Q] = wi * rho * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2)); /* Eq. 3 */
                gb[Q] = wi * rho * T * (1.0 + eu / CS2);                                           /* Eq. 4 */
                if (nz == 0) {
                    rho_c = rho;
                    T_c = T;
                }
                ++Q;
            }

    /* (b) Eqs. 30-32 */
    double rhos = 0.0, ms[3] = {0.0, 0.0, 0.0}, Es = 0.0;
    for (int i = 0; i < Q; ++i) {
        rhos += fb[i];
        for (int ax = 0; ax < D; ++ax) ms[ax] += e[i][ax] * fb[i];
        Es += gb[i];
    }
    if (cfg->force_in_predictor)
        for (int ax = 0; ax < D; ++ax)
            if (fdir[ax] != 0.0) ms[ax] += fdir[ax] * dtl * cfg->beta_g * rho_c * (T_c - Tb); /* Eq. 64, face centre */
    double us[3] = {0.0, 0.0, 0.0};
    for (int ax = 0; ax < D; ++ax) us[ax] = ms[ax] / rhos;
    double Ts = Es / rhos;
    double fs[19], gs[19];
    for (int i = 0; i < Q; ++i) {
        double eu = 0.0, uu = 0.0;
        for (int ax = 0; ax < D; ++ax) {
            eu += e[i][ax] * us[ax];
            uu += us[ax] * us[ax];
        }
        fs[i] = w[i] * rhos * (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
        gs[i] = w[i] * rhos * Ts * (1.0 + eu / CS2);
    }

    /* (c) Eqs. 38-40 along n = axis */
    const int n = axis;
    double P = 0.0, Pi[3] = {0.0, 0.0, 0.0}, Qn = 0.0;
    for (int i = 0; i < Q; ++i) {
        P += e[i][n] * fs[i];
        for (int ax = 0; ax < D; ++ax)
            Pi[ax] += e[i][ax] * e[i][n] * (fs[i] + (0.5 - tau_f) * (fs[i] - fb[i]));
        Qn += e[i][n] * (gs[i] + (0.5 - tau_g) * (gs[i] - gb[i]));
    }
    flux[0] = P;
    for (int ax = 0; ax < D; ++ax) flux[1 + ax] = Pi[ax] - ((dev && ax == n) ? CS2 : 0.0);
    flux[D + 1] = dev ? Qn - TREF * P : Qn;
    if (pred) {
        pred[0] = dev ? rhos - 1.0 : rhos;
        for (int ax = 0; ax < D; ++ax) pred[1 + ax] = ms[ax];
        pred[D + 1] = dev ? Es - TREF * rhos : Es;
    }
}

/* ----------------------------------------------------------------- setup -- */

int orc_create(const orc_cfg *cfg, orc_state **out)
{
    if (!cfg || !out) return -1;
    if (cfg->dim != 2 && cfg->dim != 3) return -1;
    if (cfg->method != 0 && cfg->method != 1) return -1;
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    if (!s) return -2;
    s->c = *cfg;
    s->D = cfg->dim;
    if (s->D == 2) {
        s->c.n[2] = 1;
        s->c.bc[4] = s->c.bc[5] = ORC_PERIODIC;
    }
    s->N = 1;
    for (int a = 0; a < s->D; ++a) {
        if (s->c.n[a] < 2) { free(s); return -1; }
        if ((s->c.bc[2 * a] == ORC_PERIODIC) != (s->c.bc[2 * a + 1] == ORC_PERIODIC)) { free(s); return -1; }
        s->N *= s->c.n[a];
    }
    for (int a = 0; a < s->D; ++a) {
        int n = s->c.n[a];
        s->node[a] = (double *)malloc(sizeof(double) * (n + 1));
        s->ctr[a] = (double *)malloc(sizeof(double) * n);
        s->wid[a] = (double *)malloc(sizeof(double) * n);
        s->L[a] = orc_mesh_nodes(n, s->c.stretch[a], s->node[a]);
        for (int i = 0; i < n; ++i) {
            s->ctr[a][i] = 0.5 * (s->node[a][i] + s->node[a][i + 1]);
            s->wid[a][i] = s->node[a][i + 1] - s->node[a][i];
        }
    }
    const int NF = s->D + 2;
    for (int f = 0; f < NF; ++f) {
        s->U[f] = (double *)calloc(s->N, sizeof(double));
        s->Unew[f] = (double *)calloc(s->N, sizeof(double));
        s->prim[f] = (double *)calloc(s->N, sizeof(double));
        s->rhs[f] = (double *)calloc(s->N, sizeof(double));
        for (int a = 0; a < s->D; ++a) s->grad[f][a] = (double *)calloc(s->N, sizeof(double));
    }
    s->tau_f = 0.5 + s->c.nu / (CS2 * s->c.dtl);
    s->tau_g = 0.5 + s->c.chi / (CS2 * s->c.dtl);

    /* Initial state: rho = 1, u = 0, T' = 0 (rest) or the linear conduction
     * profile between the isothermal walls, plus seeded noise. */
    int haxis = -1;
    for (int a = 0; a < s->D; ++a)
        if (s->c.bc[2 * a] == ORC_WALL_ISOTHERMAL && s->c.bc[2 * a + 1] == ORC_WALL_ISOTHERMAL) { haxis = a; break; }
    for (long idx = 0; idx < s->N; ++idx) {
        int ijk[3];
        cell_coords(s, idx, ijk);
        double Tp = 0.0;
        if (s->c.init == ORC_INIT_CONDUCTION && haxis >= 0) {
            double xi = s->ctr[haxis][ijk[haxis]] / s->L[haxis];
            Tp = s->c.Tw[2 * haxis] + (s->c.Tw[2 * haxis + 1] - s->c.Tw[2 * haxis]) * xi;
        }
        Tp += s->c.noise_amp * orc_splitmix_uniform(s->c.seed, (uint64_t)idx);
        s->U[0][idx] = s->c.deviation ? 0.0 : 1.0;
        for (int a = 0; a < s->D; ++a) s->U[1 + a][idx] = 0.0;
        s->U[s->D + 1][idx] = s->c.deviation ? Tp : (TREF + Tp);
    }
    *out = s;
    return 0;
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    for (int f = 0; f < 5; ++f) {
        free(s->U[f]);
        free(s->Unew[f]);
        free(s->prim[f]);
        free(s->rhs[f]);
        for (int a = 0; a < 3; ++a) free(s->grad[f][a]);
    }
    for (int a = 0; a < 3; ++a) {
        free(s->node[a]);
        free(s->ctr[a]);
        free(s->wid[a]);
    }
    free(s);
}

long orc_cells(const orc_state *s) { return s->N; }
long orc_steps_done(const orc_state *s) { return s->steps; }

/* ------------------------------------------------------------------ step -- */

/* Primitives from the stored conserved state: rho (or r), u = m/rho,
 * T = e/(rho c_p) (or T' = theta/(rho c_p)), with c_p = 1. */
static void compute_primitives(orc_state *s)
{
    const int D = s->D;
    for (long i = 0; i < s->N; ++i) {
        double r = s->U[0][i];
        double dens = s->c.deviation ? 1.0 + r : r;
        s->prim[0][i] = r;
        for (int a = 0; a < D; ++a) s->prim[1 + a][i] = s->U[1 + a][i] / dens;
        s->prim[D + 1][i] = s->U[D + 1][i] / dens;
    }
}

/* Value of primitive p on the wall face of cell idx (side 2*axis + hi). */
static double wall_face_value(const orc_state *s, int p, long idx, int side)
{
    const int D = s->D;
    if (p == 0) return s->prim[0][idx];           /* density: zero normal gradient */
    if (p <= D) return 0.0;                        /* no-slip */
    if (s->c.bc[side] == ORC_WALL_ISOTHERMAL)      /* temperature */
        return s->c.deviation ? s->c.Tw[side] : TREF + s->c.Tw[side];
    return s->prim[D + 1][idx];                    /* adiabatic: zero gradient */
}

/* Eq. 55 with Eq. 56 face values: (d_a phi)_P = (phi_hi - phi_lo)/width. */
static void compute_gradients(orc_state *s)
{
    const int D = s->D, NP = D + 2;
    for (long idx = 0; idx < s->N; ++idx) {
        int ijk[3];
        cell_coords(s, idx, ijk);
        for (int a = 0; a < D; ++a) {
            int n = s->c.n[a];
            double wP = s->wid[a][ijk[a]];
            for (int p = 0; p < NP; ++p) {
                double face[2];
                for (int hi = 0; hi < 2; ++hi) {
                    int side = 2 * a + hi;
                    int nb[3] = {ijk[0], ijk[1], ijk[2]};
                    nb[a] += hi ? 1 : -1;
                    int outside = nb[a] < 0 || nb[a] >= n;
                    if (outside && is_wall(s->c.bc[side])) {
                        face[hi] = wall_face_value(s, p, idx, side);
                        continue;
                    }
                    if (outside) nb[a] = (nb[a] + n) % n; /* periodic wrap */
                    long nidx = cell_index(s, nb);
                    double wN = s->wid[a][nb[a]];
                    /* Eq. 56: inverse-distance weights; |x_P - x_S| = wP/2,
                     * |x_N - x_S| = wN/2. */
                    face[hi] = (s->prim[p][idx] * (0.5 * wN) + s->prim[p][nidx] * (0.5 * wP))
                               / (0.5 * wN + 0.5 * wP);
                }
                s->grad[p][a][idx] = (face[1] - face[0]) / wP;
            }
        }
    }
}

/* Wall flux on the wall face of cell idx, per unit area along the outward
 * normal sgn * e_axis (sgn = -1 on the low side, +1 on the high side). */
static void wall_flux(const orc_state *s, long idx, int axis, int side, double *Fout)
{
    const int D = s->D;
    const int sgn = (side & 1) ? 1 : -1;
    int ijk[3];
    cell_coords(s, idx, ijk);
    const double d = 0.5 * s->wid[axis][ijk[axis]]; /* centre-to-wall distance */
    double r = s->U[0][idx];
    double dens = s->c.deviation ? 1.0 + r : r;
    double mn = sgn * s->U[1 + axis][idx]; /* outward normal momentum */
    Fout[0] = 0.0;                          /* impermeable wall */
    for (int x = 0; x < D; ++x) {
        /* Pressure r c_s^2 (or rho c_s^2) on the normal; one-sided viscous
         * flux -nu V with V_n = -3 m_n/d and V_t = -m_t/d. */
        double F = s->c.nu * (s->U[1 + x][idx] + (x == axis ? 2.0 * mn * sgn : 0.0)) / d;
        if (x == axis) F += sgn * CS2 * r;
        Fout[1 + x] = F;
    }
    if (s->c.bc[side] == ORC_WALL_ISOTHERMAL) {
        double Tw = s->c.deviation ? s->c.Tw[side] : TREF + s->c.Tw[side];
        Fout[D + 1] = -s->c.chi * (dens * Tw - s->U[D + 1][idx]) / d;
    } else {
        Fout[D + 1] = 0.0;
    }
}

static void accumulate_fluxes(orc_state *s)
{
    const int D = s->D, NF = D + 2;
    for (int f = 0; f < NF; ++f) memset(s->rhs[f], 0, sizeof(double) * s->N);

    for (int axis = 0; axis < D; ++axis) {
        int n = s->c.n[axis];
        int periodic = s->c.bc[2 * axis] == ORC_PERIODIC;
        for (long idx = 0; idx < s->N; ++idx) {
            int ijk[3];
            cell_coords(s, idx, ijk);
            double A = face_area(s, axis, ijk);
            /* The face on the low side of this cell. */
            if (ijk[axis] == 0 && !periodic) {
                double F[5];
                wall_flux(s, idx, axis, 2 * axis, F);
                for (int f = 0; f < NF; ++f) s->rhs[f][idx] -= F[f] * A;
                continue;
            }
            int lj[3] = {ijk[0], ijk[1], ijk[2]};
            lj[axis] = (ijk[axis] - 1 + n) % n;
            long L = cell_index(s, lj), R = idx;
            double pL[5], pR[5], gL[15], gR[15];
            memset(gL, 0, sizeof(gL));
            memset(gR, 0, sizeof(gR));
            for (int p = 0; p < NF; ++p) {
                pL[p] = s->prim[p][L];
                pR[p] = s->prim[p][R];
                for (int a = 0; a < D; ++a) {
                    gL[p * 3 + a] = s->grad[p][a][L];
                    gR[p * 3 + a] = s->grad[p][a][R];
                }
            }
            double dL = 0.5 * s->wid[axis][lj[axis]], dR = 0.5 * s->wid[axis][ijk[axis]];
            double F[5];
            orc_face_flux(&s->c, axis, pL, gL, pR, gR, dL, dR, F, NULL);
            for (int f = 0; f < NF; ++f) {
                s->rhs[f][L] -= F[f] * A;
                s->rhs[f][R] += F[f] * A;
            }
        }
        if (!periodic) { /* the high wall */
            for (long idx = 0; idx < s->N; ++idx) {
                int ijk[3];
                cell_coords(s, idx, ijk);
                if (ijk[axis] != n - 1) continue;
                double A = face_area(s, axis, ijk);
                double F[5];
                wall_flux(s, idx, axis, 2 * axis + 1, F);
                for (int f = 0; f < NF; ++f) s->rhs[f][idx] -= F[f] * A;
            }
        }
    }
}

/* Eqs. 57-59 forward-Euler update with the Eq. 64 body force, then Eq. 65. */
static void update(orc_state *s)
{
    const int D = s->D, NF = D + 2;
    const int dev = s->c.deviation;
    double du = 0.0, su = 0.0, dT = 0.0, sT = 0.0;
    for (long idx = 0; idx < s->N; ++idx) {
        int ijk[3];
        cell_coords(s, idx, ijk);
        double dV = cell_volume(s, ijk);
        for (int f = 0; f < NF; ++f) s->Unew[f][idx] = s->U[f][idx] + s->c.dt / dV * s->rhs[f][idx];
        if (s->c.gravity_axis >= 0) {
            double r = s->U[0][idx];
            double dens = dev ? 1.0 + r : r;
            double Tm = dev ? s->prim[D + 1][idx] : s->prim[D + 1][idx] - TREF;
            s->Unew[1 + s->c.gravity_axis][idx] += s->c.dt * s->c.beta_g * dens * Tm;
        }
        /* Eq. 65 terms with the absolute temperature. */
        double rn = s->Unew[0][idx];
        double densn = dev ? 1.0 + rn : rn;
        double uo = 0.0, un = 0.0;
        for (int a = 0; a < D; ++a) {
            double vo = s->prim[1 + a][idx];
            double vn = s->Unew[1 + a][idx] / densn;
            uo += vo * vo;
            un += vn * vn;
        }
        uo = sqrt(uo);
        un = sqrt(un);
        double To = dev ? TREF + s->prim[D + 1][idx] : s->prim[D + 1][idx];
        double Tn = s->Unew[D + 1][idx] / densn + (dev ? TREF : 0.0);
        du += fabs(un - uo);
        su += un;
        dT += fabs(Tn - To);
        sT += Tn;
    }
    s->res_u = su > 0.0 ? du / su : 0.0;
    s->res_T = sT != 0.0 ? dT / sT : 0.0;
    for (int f = 0; f < NF; ++f) {
        double *t = s->U[f];
        s->U[f] = s->Unew[f];
        s->Unew[f] = t;
    }
}

int orc_step(orc_state *s, long nsteps)
{
    for (long k = 0; k < nsteps; ++k) {
        compute_primitives(s);
        compute_gradients(s);
        accumulate_fluxes(s);
        update(s);
        s->steps++;
    }
    return 0;
}

/* ----------------------------------------------------------- accessors -- */

int orc_get_stored(const orc_state *s, int f, double *out)
{
    if (f < 0 || f > s->D + 1) return -1;
    memcpy(out, s->U[f], sizeof(double) * s->N);
    return 0;
}

int orc_set_stored(orc_state *s, int f, const double *in)
{
    if (f < 0 || f > s->D + 1) return -1;
    memcpy(s->U[f], in, sizeof(double) * s->N);
    return 0;
}

int orc_get_prim(const orc_state *s, int f, double *out)
{
    const int D = s->D, dev = s->c.deviation;
    if (f < 0 || f > D + 1) return -1;
    for (long i = 0; i < s->N; ++i) {
        double r = s->U[0][i];
        double dens = dev ? 1.0 + r : r;
        if (f == 0) out[i] = dens;
        else if (f <= D) out[i] = s->U[f][i] / dens;
        else out[i] = s->U[D + 1][i] / dens + (dev ? TREF : 0.0);
    }
    return 0;
}

int orc_set_prim(orc_state *s, const double *rho, const double *u, const double *T)
{
    const int D = s->D, dev = s->c.deviation;
    for (long i = 0; i < s->N; ++i) {
        s->U[0][i] = dev ? rho[i] - 1.0 : rho[i];
        for (int a = 0; a < D; ++a) s->U[1 + a][i] = rho[i] * u[(long)a * s->N + i];
        s->U[D + 1][i] = dev ? rho[i] * (T[i] - TREF) : rho[i] * T[i];
    }
    return 0;
}

int orc_axis(const orc_state *s, int axis, double *centres, double *widths)
{
    if (axis < 0 || axis >= s->D) return -1;
    for (int i = 0; i < s->c.n[axis]; ++i) {
        if (centres) centres[i] = s->ctr[axis][i];
        if (widths) widths[i] = s->wid[axis][i];
    }
    return 0;
}

void orc_residual(const orc_state *s, double *out)
{
    out[0] = s->res_u;
    out[1] = s->res_T;
}

void orc_taus(const orc_state *s, double *out)
{
    out[0] = s->tau_f;
    out[1] = s->tau_g;
}

void orc_integrals(const orc_state *s, double *out)
{
    const int D = s->D, dev = s->c.deviation;
    double mdev = 0.0, mass = 0.0, en = 0.0, th = 0.0, vol = 0.0;
    for (long i = 0; i < s->N; ++i) {
        int ijk[3];
        cell_coords(s, i, ijk);
        double dV = cell_volume(s, ijk);
        double r = dev ? s->U[0][i] : s->U[0][i] - 1.0;
        double dens = 1.0 + r;
        double theta = dev ? s->U[D + 1][i] : s->U[D + 1][i] - TREF * s->U[0][i];
        double e = dev ? s->U[D + 1][i] + TREF * dens : s->U[D + 1][i];
        mdev += r * dV;
        mass += (dev ? dens : s->U[0][i]) * dV;
        en += e * dV;
        th += theta * dV;
        vol += dV;
    }
    out[0] = mdev;
    out[1] = mass;
    out[2] = en;
    out[3] = th;
    out[4] = vol;
}

/* Wall Nusselt numbers on the two isothermal walls of the heat axis and the
 * volume Nusselt number of Eq. 69 generalised to that axis:
 *   wall:   Nu_P = (L/dT) (T_w - T_P)/d (hot),  (T_P - T_w)/d (cold),
 *           average weighted by face area, maximum over the wall;
 *   volume: Nu = L/(chi dT) * <s (u_a T - chi d_a T)>, exactly the
 *           integrand of Eq. 69 (velocity times absolute temperature, no
 *           density factor), with s = +1 when the hot wall is on the low
 *           side and the Eq. 55 gradient of T. */
int orc_nusselt(const orc_state *s, double *out)
{
    const int D = s->D;
    int haxis = -1;
    for (int a = 0; a < D; ++a)
        if (s->c.bc[2 * a] == ORC_WALL_ISOTHERMAL && s->c.bc[2 * a + 1] == ORC_WALL_ISOTHERMAL) { haxis = a; break; }
    if (haxis < 0) return -1;
    double Tlo = s->c.Tw[2 * haxis], Thi = s->c.Tw[2 * haxis + 1];
    double dTw = fabs(Thi - Tlo);
    if (dTw == 0.0) return -1;
    int hot_hi = Thi > Tlo;
    double La = s->L[haxis];
    orc_state *w = (orc_state *)s; /* primitives and gradients are scratch */
    compute_primitives(w);
    compute_gradients(w);

    double hot_sum = 0, hot_area = 0, hot_max = -1e300, cold_sum = 0, cold_area = 0, cold_max = -1e300;
    double vol_sum = 0, vol = 0;
    const int dev = s->c.deviation;
    for (long idx = 0; idx < s->N; ++idx) {
        int ijk[3];
        cell_coords(s, idx, ijk);
        double Tp = s->prim[D + 1][idx] - (dev ? 0.0 : TREF); /* T' */
        int n = s->c.n[haxis];
        for (int hi = 0; hi < 2; ++hi) {
            if (ijk[haxis] != (hi ? n - 1 : 0)) continue;
            double d = 0.5 * s->wid[haxis][ijk[haxis]];
            double A = face_area(s, haxis, ijk);
            double Tw = s->c.Tw[2 * haxis + hi];
            int is_hot = (hi == hot_hi);
            double nu = La / dTw * (is_hot ? (Tw - Tp) : (Tp - Tw)) / d;
            if (is_hot) {
                hot_sum += nu * A;
                hot_area += A;
                if (nu > hot_max) hot_max = nu;
            } else {
                cold_sum += nu * A;
                cold_area += A;
                if (nu > cold_max) cold_max = nu;
            }
        }
        double dV = cell_volume(s, ijk);
        double Tabs = Tp + TREF;
        double qa = s->prim[1 + haxis][idx] * Tabs - s->c.chi * s->grad[D + 1][haxis][idx];
        vol_sum += (hot_hi ? -qa : qa) * dV;
        vol += dV;
    }
    out[0] = hot_sum / hot_area;
    out[1] = hot_max;
    out[2] = cold_sum / cold_area;
    out[3] = cold_max;
    out[4] = La / (s->c.chi * dTw) * vol_sum / vol;
    return 0;
}
