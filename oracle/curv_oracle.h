/*
 * curv_oracle.h -- plain FP64 CPU oracle of the RTLBFS time step on a 2D
 * body-fitted (structured curvilinear) quadrilateral mesh.
 *
 * TEST INFRASTRUCTURE ONLY, like rtlbfs_oracle.h: loaded by the test-suite
 * alone, sharing nothing with the GPU library.
 *
 * The finite-volume form of Sec. 2.2 (Eqs. 41-43) and the flux of Sec. 3.2
 * are written for arbitrary cells: each face carries its own unit normal n
 * and area dS, the local D2Q9 lattice of Fig. 1 is aligned with (n, t), and
 * the cell gradients of Eq. 55 are the discrete Gauss sums over the cell's
 * faces.  This is what Secs. 4.3 and 4.5 run on their O-type meshes.
 *
 * Mesh: ni x nj cells, cell (i, j) at index j*ni + i; vertices (ni+1) x
 * (nj+1) at index j*(ni+1) + i.  Cell (i, j) has the corners (i, j),
 * (i+1, j), (i+1, j+1), (i, j+1).  Either orientation is accepted, but every
 * cell must have the same one.  A periodic pair of sides must close the mesh
 * on itself: vertex column (or row) n coincides with column (row) 0.
 *
 * Storage: field 0 rho (deviation: r = rho - 1), 1..2 m = rho u, 3 e = rho T
 * (deviation: theta = rho (T - T0), T0 = 0.5).  Temperatures in the
 * configuration are absolute.
 */
#ifndef CURV_ORACLE_H
#define CURV_ORACLE_H

#include "rtlbfs_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_FARFIELD = 3 }; /* face against a mirrored ghost cell holding the free stream */

typedef struct {
    int ni, nj;             /* cells along i and j */
    int bc[4];              /* sides i-, i+, j-, j+: ORC_PERIODIC, ORC_WALL_ISOTHERMAL,
                               ORC_WALL_ADIABATIC or ORC_FARFIELD */
    double Tw[4];           /* absolute wall temperature of isothermal sides */
    double up[2];           /* unit vector against gravity; (0, 0): no buoyancy */
    double Tb;              /* absolute reference temperature of the buoyancy force */
    double u_inf[2];        /* far-field velocity */
    double T_inf;           /* far-field absolute temperature; rho_inf = 1 */
    double nu, chi, beta_g; /* viscosity, diffusivity, beta*g */
    double dtl, dt;         /* lattice step and time step */
    int deviation;          /* 0: (rho, m, e); 1: (r, m, theta) */
    int force_in_predictor; /* 1: buoyancy also in the predicted momentum */
    int method;             /* 0 RTLBFS, 1 TLBFS interior-face flux */
} orc_curv_cfg;

typedef struct orc_curv orc_curv;

/* x, y: vertex coordinates.  The state starts as the far-field state
 * (rho = 1, u = u_inf, T = T_inf).  Returns 0, or -1 for an invalid mesh or
 * configuration. */
int orc_curv_create(const orc_curv_cfg *cfg, const double *x, const double *y, orc_curv **out);
void orc_curv_destroy(orc_curv *s);
int orc_curv_step(orc_curv *s, long nsteps);
int orc_curv_set_prim(orc_curv *s, const double *rho, const double *u /* 2N, x then y */, const double *T);
/* f = 0 rho, 1 u_x, 2 u_y, 3 absolute T */
int orc_curv_get_prim(const orc_curv *s, int f, double *out);
int orc_curv_get_stored(const orc_curv *s, int f, double *out);
/* Cell centroids and areas. */
void orc_curv_cells(const orc_curv *s, double *cx, double *cy, double *area);
/* Eq. 65 residual of the last step: {res_u, res_T}. */
void orc_curv_residual(const orc_curv *s, double *out);
/* Wall heat of one isothermal side: out = {sum_k (T_w - T_P)/d_k dS_k, sum_k dS_k}
 * over its faces, with d_k the normal distance of the cell centroid from the
 * face.  Returns -1 if the side is not an isothermal wall. */
int orc_curv_wall_heat(const orc_curv *s, int side, double *out);
/* {sum r dV, sum rho dV, sum e dV, sum dV} with r = rho - 1, e = rho T. */
void orc_curv_integrals(const orc_curv *s, double *out);

#ifdef __cplusplus
}
#endif
#endif
