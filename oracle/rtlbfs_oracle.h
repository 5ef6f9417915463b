/*
 * rtlbfs_oracle.h -- plain FP64 CPU oracle of the RTLBFS time step.
 *
 * TEST INFRASTRUCTURE ONLY.  This header and rtlbfs_oracle.c define what the
 * reconstructed thermal lattice Boltzmann flux solver (RTLBFS, Lu, Dai & Yu,
 * arXiv 2202.13449, Sec. 3.2) computes, written as slow, obvious loops in
 * double precision.  Only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or constant
 * with the GPU library; the two are compared only through their outputs.
 *
 * Conventions (lattice units, c = 1, c_s^2 = 1/3, c_p = 1, reference
 * temperature T0 = 0.5 with T_low = 0, T_high = 1, rho0 = 1):
 *   field 0          rho          (deviation storage: r = rho - 1)
 *   fields 1..D      m_a = rho u_a
 *   field D+1        e = rho T    (deviation storage: theta = rho (T - T0))
 * Cells are stored x-fastest: idx = i + n0*(j + n1*k).
 */
#ifndef RTLBFS_ORACLE_H
#define RTLBFS_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_PERIODIC = 0, ORC_WALL_ISOTHERMAL = 1, ORC_WALL_ADIABATIC = 2 };
enum { ORC_INIT_REST = 0, ORC_INIT_CONDUCTION = 1 };

typedef struct {
    int dim;                /* 2 or 3 */
    int n[3];               /* cells per axis (n[2] ignored when dim == 2) */
    double stretch[3];      /* 0: unit spacing; > 0: tanh clustering, phi = stretch (Eq. 74) */
    int bc[6];              /* sides x-, x+, y-, y+, z-, z+ : ORC_* kinds */
    double Tw[6];           /* wall temperature deviation T - T0 on isothermal sides */
    int gravity_axis;       /* buoyancy along +axis (upward unit vector); -1: none */
    double nu, chi, beta_g; /* kinematic viscosity, thermal diffusivity, beta*g */
    double dtl;             /* lattice streaming step delta-t of the local lattice */
    double dt;              /* macroscopic time step Delta-t */
    int deviation;          /* 0: store (rho, m, e); 1: store (r, m, theta) */
    int force_in_predictor; /* 1: buoyancy also enters the predicted momentum */
    int init;               /* ORC_INIT_REST or ORC_INIT_CONDUCTION */
    uint64_t seed;          /* SplitMix64 seed for the initial temperature noise */
    double noise_amp;       /* T' += noise_amp * U(-1, 1) per cell */
    int method;             /* interior-face flux: 0 RTLBFS (Sec. 3.2, Eqs. 46-48, 57-59);
                               1 TLBFS (Sec. 2.2, Eqs. 29-40) */
} orc_cfg;

typedef struct orc_state orc_state;

/* Mesh node coordinates along one axis: unit spacing, or Eq. 74 scaled so that
 * the smallest cell is 1.  x must hold n+1 values.  Returns the length L. */
double orc_mesh_nodes(int n, double stretch, double *x);

/* Eq. 63 with V_c = Ma: nu = V_c L sqrt(Pr/Ra), chi = nu/Pr, beta_g = V_c^2/L
 * (Delta T = 1).  out = {nu, chi, beta_g}. */
void orc_physics_from_ra(double Ra, double Pr, double Ma, double L, double *out);

/* i-th output of a SplitMix64 generator seeded with `seed`, mapped to [-1, 1). */
double orc_splitmix_uniform(uint64_t seed, uint64_t i);

int orc_create(const orc_cfg *cfg, orc_state **out);
void orc_destroy(orc_state *s);
long orc_cells(const orc_state *s);
int orc_step(orc_state *s, long nsteps);
long orc_steps_done(const orc_state *s);

/* Stored conserved field f (0..D+1) in the storage form of the run. */
int orc_get_stored(const orc_state *s, int f, double *out);
int orc_set_stored(orc_state *s, int f, const double *in);
/* Absolute primitives: f = 0 rho, 1..D u_a, D+1 T (absolute temperature). */
int orc_get_prim(const orc_state *s, int f, double *out);
/* Set the state from absolute primitives (rho, u, T), converting to storage. */
int orc_set_prim(orc_state *s, const double *rho, const double *u /* D*N, axis-major */,
                 const double *T);

/* Axis coordinates: centres (n values) and widths (n values). */
int orc_axis(const orc_state *s, int axis, double *centres, double *widths);

/* Eq. 65 residual of the last step: out = {res_u, res_T}. */
void orc_residual(const orc_state *s, double *out);
/* Wall and volume Nusselt numbers:
 * out = {hot_avg, hot_max, cold_avg, cold_max, nu_volume}. */
int orc_nusselt(const orc_state *s, double *out);
/* Integrals: out = {sum (rho-1) dV, sum rho dV, sum e dV, sum theta dV, volume}. */
void orc_integrals(const orc_state *s, double *out);
/* Derived relaxation times: out = {tau_f, tau_g}. */
void orc_taus(const orc_state *s, double *out);

/* Single interior-face flux (RTLBFS or TLBFS by cfg->method), for pinning the
 * face arithmetic in isolation.
 * primL/primR hold D+2 primitives in the storage convention of cfg->deviation
 * (rho or r, u_a, T or T'); gradL/gradR hold their gradients [p*3 + a].
 * dL/dR: distances from the left/right cell centre to the face.  flux: D+2
 * values per unit area along +axis.  pred (optional): rho*, m*_a, e* (or
 * r*, m*, theta*) at the face centre.  With deviation storage the momentum
 * flux omits the constant pressure c_s^2 (it cancels on every cell). */
void orc_face_flux(const orc_cfg *cfg, int axis, const double *primL, const double *gradL,
                   const double *primR, const double *gradR, double dL, double dR,
                   double *flux, double *pred);

/* The same flux in a frame of its own: axis 0 is the face normal n (from the
 * left to the right cell), axes 1 (and 2) the tangents; primitives, their
 * gradients [p*3 + a], xSL = x_S - x_L, xSR = x_S - x_R and the buoyancy
 * direction fdir (unit vector against gravity, or zero) are all given in that
 * frame.  Tb is the absolute reference temperature of the buoyancy force.
 * flux: D+2 values per unit area along +n, momentum in the frame. */
void orc_face_flux_frame(const orc_cfg *cfg, const double *primL, const double *gradL, const double *primR,
                         const double *gradR, const double *xSL, const double *xSR, const double *fdir, double Tb,
                         double *flux, double *pred);

#ifdef __cplusplus
}
#endif
#endif
