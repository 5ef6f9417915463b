/*
 * curv3_oracle.h -- plain FP64 CPU oracle of the RTLBFS time step on a 3D
 * body-fitted (structured curvilinear) hexahedral mesh, the setting of
 * Sec. 4.5 (concentric annulus, one azimuthal layer).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite alone, sharing nothing
 * with the GPU library.
 *
 * Mesh: n0 x n1 x n2 cells, cell (i, j, k) at index (k*n1 + j)*n0 + i;
 * vertices (n0+1) x (n1+1) x (n2+1) at index (k*(n1+1) + j)*(n0+1) + i.
 * A periodic pair of sides closes the mesh on itself: vertex layer n equals
 * layer 0 rotated by `rot[axis]` radians about the z axis (0 for a plain
 * closed pair).  The neighbour across such a side is the image of the cell
 * on the other side, rotated with its velocity and gradients.
 *
 * Storage: field 0 rho (deviation: r = rho - 1), 1..3 m = rho u, 4 e = rho T
 * (deviation: theta = rho (T - T0), T0 = 0.5).  Temperatures are absolute.
 */
#ifndef CURV3_ORACLE_H
#define CURV3_ORACLE_H

#include "rtlbfs_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int n[3];               /* cells along i, j, k */
    int bc[6];              /* sides i-, i+, j-, j+, k-, k+: ORC_PERIODIC, ORC_WALL_ISOTHERMAL,
                               ORC_WALL_ADIABATIC */
    double rot[3];          /* rotation about z closing a periodic axis (radians), else 0 */
    double Tw[6];           /* absolute wall temperature of isothermal sides */
    double up[3];           /* unit vector against gravity; zero: no buoyancy */
    double Tb;              /* absolute reference temperature of the buoyancy force */
    double nu, chi, beta_g; /* viscosity, diffusivity, beta*g */
    double dtl, dt;         /* lattice step and time step */
    int deviation;          /* 0: (rho, m, e); 1: (r, m, theta) */
    int force_in_predictor; /* 1: buoyancy also in the predicted momentum */
    int method;             /* 0 RTLBFS, 1 TLBFS interior-face flux */
} orc_curv3_cfg;

typedef struct orc_curv3 orc_curv3;

/* x, y, z: vertex coordinates.  The state starts at rest, rho = 1, T = T0.
 * Returns 0, or -1 for an invalid mesh or configuration. */
int orc_curv3_create(const orc_curv3_cfg *cfg, const double *x, const double *y, const double *z, orc_curv3 **out);
void orc_curv3_destroy(orc_curv3 *s);
int orc_curv3_step(orc_curv3 *s, long nsteps);
int orc_curv3_set_prim(orc_curv3 *s, const double *rho, const double *u /* 3N, x then y then z */,
                       const double *T);
/* f = 0 rho, 1..3 u_x, u_y, u_z, 4 absolute T */
int orc_curv3_get_prim(const orc_curv3 *s, int f, double *out);
/* Cell centroids and volumes. */
void orc_curv3_cells(const orc_curv3 *s, double *cx, double *cy, double *cz, double *vol);
void orc_curv3_residual(const orc_curv3 *s, double *out);
/* Wall heat of one isothermal side: {sum (T_w - T_P)/d dS, sum dS}. */
int orc_curv3_wall_heat(const orc_curv3 *s, int side, double *out);
/* {sum r dV, sum rho dV, sum e dV, sum dV}. */
void orc_curv3_integrals(const orc_curv3 *s, double *out);

#ifdef __cplusplus
}
#endif
#endif
