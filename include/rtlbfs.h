/*
 * rtlbfs.h -- C ABI of the MI355X (gfx950) RTLBFS time-step library.
 *
 * The library advances the reconstructed thermal lattice Boltzmann flux solver
 * (RTLBFS) of Lu, Dai & Yu, arXiv 2202.13449, on structured uniform or
 * tanh-stretched (Eq. 74) meshes in 2D and 3D:
 *   predictor  Sec. 3.2(a): at every interior face a face-centred unit lattice
 *              (D2Q9 / D3Q19 offsets, Fig. 2) is filled by the one-sided linear
 *              reconstruction of Eq. 29 from Eq. 55 cell gradients (face values
 *              by Eq. 56); Eqs. 46-48 are evaluated by central differences on
 *              the lattice to give rho*, (rho u)*, (rho c_p T)*;
 *   corrector  Sec. 3.2(b): face fluxes of Eqs. 57-59 with the viscous and
 *              (tau - 1.5) dissipation terms, forward-Euler update (Eqs. 41-43)
 *              with the Boussinesq force of Eq. 64 (applied in the update and in
 *              the predicted momentum);
 *   diagnostics  Eq. 65 residual, Eq. 69 volume Nusselt number, wall Nusselt
 *              numbers (Eqs. 75-76 form), all reduced in FP64 on the GPU.
 *
 * Units: lattice units with the finest cell of size 1 and c = 1 (c_s^2 = 1/3),
 * c_p = 1, rho0 = 1, absolute temperatures T_low = 0 and T_high = 1 so the
 * reference temperature is T0 = 0.5.  Wall temperatures are given as
 * deviations T - T0.  Ra, Pr and Ma define nu, chi and beta*g through Eq. 63
 * with V_c = Ma (in units of c) and L the domain length along the axis of the
 * two isothermal walls (else along gravity, else along x).
 *
 * Conventions for every entry point:
 *   - returns RTLBFS_OK (0) or a negative RTLBFS_E* code; never aborts, never
 *     throws across the ABI, never prints;
 *   - pointers named host_* are host memory owned by the caller; the
 *     workspace and stream passed to rtlbfs_create belong to the caller and
 *     must outlive the handle;
 *   - a handle is used by one host thread at a time; work is enqueued on the
 *     handle's stream; calls documented as synchronising wait for it;
 *   - cells are stored x-fastest: index = i + nx*(j + ny*k).
 */
#ifndef RTLBFS_H
#define RTLBFS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes -- */
#define RTLBFS_OK 0
#define RTLBFS_EINVAL (-1)       /* bad argument or inconsistent problem */
#define RTLBFS_ENOMEM (-2)       /* device allocation failed or workspace too small */
#define RTLBFS_EDEVICE (-3)      /* a HIP call failed (text in rtlbfs_last_error) */
#define RTLBFS_EDIVERGED (-4)    /* NaN/Inf or local Mach >= opts.max_mach seen at a residual step */
#define RTLBFS_EUNSUPPORTED (-5) /* valid request the library does not implement */
#define RTLBFS_ESTATE (-6)       /* call order (e.g. a residual before any residual step) */

/* Boundary kinds per side (x-, x+, y-, y+, z-, z+). */
#define RTLBFS_PERIODIC 0
#define RTLBFS_WALL_ISOTHERMAL 1 /* no-slip, temperature T0 + Tdev[side] */
#define RTLBFS_WALL_ADIABATIC 2  /* no-slip, zero heat flux */

/* Storage / arithmetic of the state. */
#define RTLBFS_FP64_PLAIN 0 /* rho, rho u, rho c_p T in double */
#define RTLBFS_FP32_DEV 1   /* r = rho - 1, rho u, theta = rho c_p (T - T0) in float */
#define RTLBFS_FP64_DEV 2   /* the deviation storage in double */

/* Interior-face flux (opts.method). */
#define RTLBFS_METHOD_RTLBFS 0 /* Sec. 3.2: finite-difference predictor of Eqs. 46-48, fluxes Eqs. 57-59 */
#define RTLBFS_METHOD_TLBFS 1  /* Sec. 2.2: equilibria on the local lattice, Eqs. 29-40 */

/* Initial state. */
#define RTLBFS_INIT_REST 0       /* rho = 1, u = 0, T' = 0 (+ noise) */
#define RTLBFS_INIT_CONDUCTION 1 /* linear T' between the isothermal walls (+ noise) */

/* Field selectors for rtlbfs_get_field: absolute primitives. */
#define RTLBFS_FIELD_RHO 0
#define RTLBFS_FIELD_UX 1
#define RTLBFS_FIELD_UY 2
#define RTLBFS_FIELD_UZ 3 /* 3D only; in 2D index 3 is T */
/* The temperature is field dim + 1. */

typedef struct {
    int dim;           /* 2 or 3 */
    int n[3];          /* cells per axis; n[2] ignored in 2D; each >= 4 */
    double stretch[3]; /* 0: unit cells; > 0: Eq. 74 tanh clustering with phi = stretch,
                          scaled so the smallest cell is 1 (uniform only on periodic axes) */
} rtlbfs_mesh;

typedef struct {
    int kind[6];      /* RTLBFS_PERIODIC / _WALL_ISOTHERMAL / _WALL_ADIABATIC per side;
                         periodic sides come in pairs */
    double Tdev[6];   /* isothermal wall temperature minus T0 */
    int gravity_axis; /* buoyancy acts along +axis (the "up" unit vector); -1 none */
} rtlbfs_bc;

typedef struct {
    int precision;        /* RTLBFS_FP64_PLAIN (default), _FP32_DEV, _FP64_DEV */
    double dtl;           /* lattice streaming step delta-t; 0 -> 1 (finest cell) */
    double dt;            /* time step Delta-t; 0 -> min(0.5, 0.15 / max(nu, chi)) */
    uint64_t seed;        /* SplitMix64 seed of the initial temperature noise */
    double noise_amp;     /* T' += noise_amp * U(-1,1), U from SplitMix64(seed, cell) */
    int init;             /* RTLBFS_INIT_REST or _CONDUCTION */
    int residual_every;   /* chunk length R: the Eq. 65 residual is evaluated on the last step of
                             every R-step chunk and of every rtlbfs_step call (0 -> 100) */
    int mass_fix_every;   /* FP32_DEV: remove the total-mass drift every K steps (0 -> 1000,
                             < 0 -> never) */
    int graph_steps;      /* >= 0: every full R-step chunk is replayed from a captured HIP graph;
                             < 0: kernels are launched one by one */
    int buoyancy_update_only; /* 1: force only in the cell update (not in m*) */
    int phys_given;       /* 1: use nu, chi, beta_g below and ignore Ra, Pr, Ma */
    double nu, chi, beta_g;
    int tile;             /* 2D launch shape: 0 -> autotuned at create (every shape timed on the
                             live state); 1..5 -> one step per launch on 32x8, 16x16, 64x4, 16x8,
                             8x8 cells; 6..9 -> two steps per launch on 16x16, 32x8, 16x8, 8x8
                             (the state of the first step stays on chip; an odd last step uses
                             the one-step shape of the same tile).
                             3D launch shape: 0 or 1 -> 4x4x4 cell tiles; 2..5 -> 16x8 columns
                             marching through segments of 32, 48, 64, 96 planes along z; 6 -> 8x8
                             columns, segments of 48 planes.  The columns compute each face once
                             per segment; they agree with the tiles to rounding (FMA contraction
                             differs between the two kernels), not bit for bit. */
    int round_nearest;    /* FP32_DEV only. 0 (default): the state update u + du is rounded
                             stochastically (unbiased; random bits from a hash of cell, field and a
                             device step counter, reproducible); 1: round-to-nearest, which stalls
                             increments below half an ulp near steady state */
    int method;           /* RTLBFS_METHOD_RTLBFS (default) or RTLBFS_METHOD_TLBFS: the interior-face
                             flux; wall faces, gradients, update and diagnostics are shared */
    double max_mach;      /* divergence guard: a residual step that sees a local Mach number |u|/c_s
                             at or above this value (or a NaN/Inf) makes the next synchronising call
                             return RTLBFS_EDIVERGED; 0 -> 0.5, at most 10 */
} rtlbfs_opts;

typedef struct {
    double hot_avg, hot_max;   /* area-weighted mean and maximum over the hot wall */
    double cold_avg, cold_max; /* same over the cold wall */
    double volume;             /* Eq. 69 along the heat axis: L/(chi dT) <u_a T - chi d_a T>, absolute T */
} rtlbfs_nu;

typedef struct {
    int64_t cells;
    int64_t steps;              /* steps advanced so far */
    double L;                   /* characteristic length used in Eq. 63 */
    double nu, chi, beta_g;     /* derived or given physics */
    double tau_f, tau_g;        /* Eqs. 9-10 with dtl */
    double dtl, dt;
    double length[3];           /* domain length per axis */
    int precision;
    int tile_x, tile_y, tile_z; /* tile the step kernel runs with (3D columns: tile_z is the
                                   segment length) */
    double tune_ms[16];         /* autotuner: ms per step of each 2D launch shape, in opts.tile order
                                   (0 if not timed) */
    int steps_per_launch;       /* time steps one launch of the step kernel advances (1 or 2) */
} rtlbfs_info;

typedef struct rtlbfs_handle *rtlbfs_t;
typedef struct rtlbfs_batch_handle *rtlbfs_batch_t;

/* Static text for a status code (never NULL). */
const char *rtlbfs_strerror(int code);

/* Per-handle detail of the last failing call (never NULL; "" when none).
 * With h == NULL: detail of the last failed rtlbfs_create on this thread. */
const char *rtlbfs_last_error(rtlbfs_t h);

/* Fill *opts with the defaults described above.  EINVAL on NULL. */
int rtlbfs_opts_init(rtlbfs_opts *opts);

/* Node coordinates of one mesh axis (Eq. 74 or unit spacing), n+1 values into
 * host_x; returns the length in *L.  Host only.  EINVAL on n < 1 or NULL. */
int rtlbfs_mesh_nodes(int n, double stretch, double *host_x, double *L);

/* Device workspace needed for this mesh and precision (bytes, 256-aligned);
 * 0 when the arguments are invalid or the mesh exceeds the size limit of
 * rtlbfs_create. */
size_t rtlbfs_workspace_bytes(const rtlbfs_mesh *mesh, const rtlbfs_opts *opts);

/* Create a solver for one domain.
 *   mesh, bc: problem geometry and boundaries (see the structs);
 *   Ra, Pr, Ma: Eq. 63 inputs (ignored when opts->phys_given);
 *   opts: NULL for defaults;
 *   hip_stream: the hipStream_t to enqueue on (NULL = the null stream);
 *   workspace, ws_bytes: caller-owned device memory of at least
 *     rtlbfs_workspace_bytes(); NULL makes the library allocate (and free) it;
 *   out: receives the handle.
 * Uploads the seeded initial state (synchronising).  Errors: EINVAL
 * (validation: Ra, Pr > 0, 0 < Ma <= 0.3, n >= 4, paired periodic sides,
 * uniform mesh on periodic axes, gravity_axis < dim), ENOMEM, EDEVICE.
 * Size limit: at most 2^20 cells per axis, and every step launch within one
 * dispatch (launch-shape blocks x threads at most 2^32 - 1, about 7e8 cells
 * for a square 2D mesh); a larger mesh is EINVAL. */
int rtlbfs_create(const rtlbfs_mesh *mesh, double Ra, double Pr, double Ma, const rtlbfs_bc *bc,
                  const rtlbfs_opts *opts, void *hip_stream, void *workspace, size_t ws_bytes,
                  rtlbfs_t *out);

/* Enqueue n >= 0 time steps on the handle's stream and return.  The Eq. 65
 * residual is evaluated on every residual_every-th step and on the last step
 * of the call.  Divergence found there is reported by the next synchronising
 * call as EDIVERGED. */
int rtlbfs_step(rtlbfs_t h, int64_t n);

/* Wait for the handle's stream.  EDIVERGED if a residual step saw NaN/Inf or
 * a local Mach number at or above opts.max_mach. */
int rtlbfs_sync(rtlbfs_t h);

/* Eq. 65 ratios from the most recent residual step (synchronising):
 * sum| |u|^{n+1} - |u|^n | / sum |u|^{n+1} and sum|T^{n+1} - T^n| / sum T^{n+1}
 * with the absolute temperature.  ESTATE before any step. */
int rtlbfs_residual(rtlbfs_t h, double *res_u, double *res_T);

/* Wall and volume Nusselt numbers of the current state (synchronising).
 * EINVAL if the problem has no pair of isothermal walls on one axis. */
int rtlbfs_nusselt(rtlbfs_t h, rtlbfs_nu *out);

/* FP64 integrals of the current state (synchronising):
 * out[0] = sum (rho - 1) dV, out[1] = sum rho c_p (T - T0) dV, out[2] = volume. */
int rtlbfs_integrals(rtlbfs_t h, double out[3]);

/* Copy one absolute primitive field (0 rho, 1..dim u_a, dim+1 T) of all
 * cells into host_out (count >= cells; synchronising). */
int rtlbfs_get_field(rtlbfs_t h, int field, double *host_out, size_t count);

/* Replace the state by absolute primitives: host_rho[cells], host_u[dim*cells]
 * (axis-major), host_T[cells]; converted to the handle's storage (synchronising). */
int rtlbfs_set_state(rtlbfs_t h, const double *host_rho, const double *host_u, const double *host_T,
                     size_t cells);

/* Stored conserved field f (0..dim+1) converted to double, in the storage
 * form of the handle (for checkpoints and parity checks; synchronising). */
int rtlbfs_get_stored(rtlbfs_t h, int field, double *host_out, size_t count);

/* Eq. 65 ratios between two states held in caller device memory, with no
 * handle and no allocation.  For callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.
 *   dim: 2 or 3; precision: the storage of both states (RTLBFS_FP64_PLAIN,
 *     RTLBFS_FP32_DEV or RTLBFS_FP64_DEV), float elements for FP32_DEV,
 *     double otherwise;
 *   old_state, new_state: device pointers to dim + 2 stored fields each
 *     (rho or r, rho u_a, rho c_p T or theta), field k of a state starting
 *     at element k * fstride, cells x-fastest -- the layout of a handle's
 *     state copy; read only;
 *   dev_out: device memory for 2 doubles, receives res_u and res_T exactly
 *     as rtlbfs_residual defines them (new_state at time level n+1), with
 *     the per-cell terms formed as the step kernels form them;
 *   hip_stream: stream of the current device (NULL = null stream).
 * Enqueues two kernels and returns without synchronising.  Allocates
 * nothing: the block partial sums live in a fixed 32 KiB device array per GPU
 * (set up by the first call on each device), shared by every call on that
 * GPU, so calls that overlap on one GPU race; calls ordered on one stream do
 * not.  EINVAL for a bad dim or precision, NULL pointers, cells < 1 or
 * above RTLBFS_RESIDUAL_STATES_MAX_CELLS, or fstride < cells; EDEVICE when
 * a HIP call or launch fails. */
#define RTLBFS_RESIDUAL_STATES_MAX_CELLS ((int64_t)1 << 31)
int rtlbfs_residual_states(int dim, int precision, int64_t cells, int64_t fstride, const void *old_state,
                           const void *new_state, double *dev_out, void *hip_stream);

/* Checkpoint and bitwise resume.  A run continues bit for bit from a
 * checkpoint when the new handle has the same mesh, boundaries, physics and
 * options (seed and noise may differ: the initial state is replaced) and
 * its state is restored with:
 *   - the stored fields 0..dim+1 (rtlbfs_get_stored, field after field);
 *   - rtlbfs_checkpoint: the steps advanced so far (they key the FP32
 *     stochastic rounding), the steps since the last mass-drift correction,
 *     and the reference mass that correction restores. */
typedef struct {
    int64_t steps;     /* steps advanced so far */
    int64_t since_fix; /* steps since the last FP32 mass-drift correction */
    double mass0;      /* sum (rho - 1) dV the correction restores (FP32_DEV) */
} rtlbfs_checkpoint;

/* Fill *out for the current state (synchronising).  EINVAL on NULL. */
int rtlbfs_get_checkpoint(rtlbfs_t h, rtlbfs_checkpoint *out);

/* Replace the state by a checkpoint: host_stored holds the dim + 2 stored
 * fields in the handle's storage form, cells values each, field after field
 * (count >= (dim + 2) * cells), converted to the storage precision (values
 * read with rtlbfs_get_stored convert back exactly); ck restores the step
 * counter, the correction phase and the reference mass (synchronising).
 * EINVAL on NULL, a short buffer, or a negative step count. */
int rtlbfs_restore(rtlbfs_t h, const double *host_stored, size_t count, const rtlbfs_checkpoint *ck);

/* Handle facts (host only, no synchronisation). */
int rtlbfs_get_info(rtlbfs_t h, rtlbfs_info *out);

/* Destroy; frees only what the library allocated.  NULL is a no-op. */
int rtlbfs_destroy(rtlbfs_t h);

/* ------------------------------------------------- body-fitted 2D meshes -- */
/* The same step on a 2D structured curvilinear (body-fitted) quadrilateral
 * mesh, the setting of Secs. 4.3 and 4.5 (O-type meshes around a heated
 * cylinder and in an annulus).  Every face carries its own unit normal n and
 * area dS (edge length); the D2Q9 lattice of the predictor is aligned with
 * (n, t) on each face; cell gradients are the Gauss sums of Eq. 55 over the
 * four faces with Eq. 56 face values (inverse distances of the face midpoint
 * from the two cell centroids).  Cell centre = centroid of the quadrilateral.
 * Walls use the one-sided closure of the Cartesian meshes in the face frame,
 * with d the normal distance of the centroid from the wall face.
 *
 * A far-field side (RTLBFS_FARFIELD) is an ordinary face against a ghost
 * cell mirrored across it (same normal distance, zero gradient) that holds
 * the free stream: rho = 1, u_inf, T_inf.
 *
 * Buoyancy: beta_g rho (T - T_ref) along the unit vector `up`, in the cell
 * update and (unless opts.buoyancy_update_only) in the predicted momentum.
 * Temperatures here are absolute.  Cells are stored i-fastest: index
 * = i + ni*j, the field layout of the Cartesian 2D meshes. */
#define RTLBFS_FARFIELD 3

typedef struct {
    int n[2];        /* cells along i (n[0]) and j (n[1]); each >= 4 */
    const double *x; /* host vertex coordinates, (n[1]+1) * (n[0]+1) values, i fastest:
                        vertex (i, j) at x[j*(n[0]+1) + i]; cell (i, j) has the corners
                        (i, j), (i+1, j), (i+1, j+1), (i, j+1), all cells with the same
                        orientation and positive area.  Read during create only. */
    const double *y;
} rtlbfs_curv_mesh;

typedef struct {
    int kind[4];     /* sides i-, i+, j-, j+: RTLBFS_PERIODIC (in pairs; the mesh must close
                        on itself: vertex column n[0] (row n[1]) equals column (row) 0),
                        RTLBFS_WALL_ISOTHERMAL, RTLBFS_WALL_ADIABATIC or RTLBFS_FARFIELD */
    double Tw[4];    /* absolute temperature of isothermal walls */
    double up[2];    /* unit vector against gravity, or (0, 0) for no buoyancy */
    double T_ref;    /* absolute reference temperature of the buoyancy force */
    double u_inf[2]; /* far-field velocity (also the initial velocity) */
    double T_inf;    /* far-field absolute temperature (also the initial temperature) */
} rtlbfs_curv_bc;

/* Device workspace for a body-fitted mesh (bytes); 0 for invalid arguments
 * or a mesh beyond the size limit of rtlbfs_create. */
size_t rtlbfs_curv_workspace_bytes(const rtlbfs_curv_mesh *mesh, const rtlbfs_opts *opts);

/* Create a solver on a body-fitted mesh.  nu, chi, beta_g are given directly
 * (opts->phys_given and Ra/Pr/Ma do not apply).  The state starts at rho = 1,
 * u = u_inf, T = T_inf (+ opts->noise_amp noise on T).  Every other option,
 * the workspace and stream rules and the error codes are those of
 * rtlbfs_create, except: opts->tile 0 autotunes the launch shape among
 * 16 x 16, 16 x 8, 32 x 8 and 8 x 8 cells (every shape timed on the live
 * state at create), 1..4 fixes one of them in that order; opts->init is
 * ignored.  The handle works with rtlbfs_step, _sync,
 * _residual, _integrals, _get_field, _set_state, _get_stored, _get_info and
 * _destroy; rtlbfs_nusselt returns RTLBFS_EUNSUPPORTED (use
 * rtlbfs_wall_heat).  EINVAL also for a mesh that folds over or does not
 * close on a periodic pair. */
int rtlbfs_curv_create(const rtlbfs_curv_mesh *mesh, double nu, double chi, double beta_g,
                       const rtlbfs_curv_bc *bc, const rtlbfs_opts *opts, void *hip_stream, void *workspace,
                       size_t ws_bytes, rtlbfs_t *out);

/* Heat through one isothermal side of a body-fitted mesh (synchronising, FP64):
 * out[0] = sum_k (T_w - T_P,k) / d_k dS_k over the side's faces (the
 * one-sided wall-normal temperature gradient times the face area, heat into
 * the fluid per unit chi), out[1] = sum_k dS_k.  Nusselt numbers are formed
 * from these: Eq. 73 on a cylinder is out[0] / (pi dT), the average of
 * Eq. 78 on a cylinder of radius R and height H is R out[0] / (out[1] dT)
 * per unit height.  EINVAL if the side is not an isothermal wall,
 * EUNSUPPORTED on a Cartesian handle.  Also for 3D body-fitted handles
 * (sides 0..5). */
int rtlbfs_wall_heat(rtlbfs_t h, int side, double out[2]);

/* Geometry the library derived for a body-fitted mesh (host only): cell
 * centroids and areas, `count` >= cells values each (any pointer may be
 * NULL).  EUNSUPPORTED on a Cartesian handle. */
int rtlbfs_curv_cells(rtlbfs_t h, double *host_cx, double *host_cy, double *host_area, size_t count);

/* ------------------------------------------------- body-fitted 3D meshes -- */
/* The step on a 3D structured curvilinear hexahedral mesh, the setting of
 * Sec. 4.5 (a concentric annulus run with one azimuthal cell layer).  Each
 * face carries its unit normal n (from the diagonal cross product of its four
 * corners), a tangent t1 (its first edge without the normal part) and
 * t2 = n x t1; the D3Q19 lattice of the predictor is aligned with them; the
 * face centre is the mean of the corners; cell centroids and volumes come
 * from a tetrahedral split.  Cells are stored i-fastest: index
 * = i + n0*(j + n1*k), fields rho, u_x, u_y, u_z, T as on Cartesian 3D meshes.
 *
 * A periodic pair of sides may be closed by a rotation about the z axis
 * (rot[axis] radians): vertex layer n equals layer 0 rotated by rot, and the
 * neighbour across the pair is the cell on the other side, rotated with its
 * velocity and velocity gradient.  With one cell along that axis this is the
 * single-layer wedge of an axisymmetric problem.  Walls as on 2D body-fitted
 * meshes; no far-field sides in 3D. */
typedef struct {
    int n[3];        /* cells along i, j, k; >= 2 on walled axes, >= 1 on periodic ones */
    const double *x; /* host vertex coordinates, (n[2]+1)*(n[1]+1)*(n[0]+1) values each,
                        vertex (i, j, k) at ((k*(n[1]+1) + j)*(n[0]+1) + i); cell (i, j, k)
                        spans vertices i..i+1, j..j+1, k..k+1; one orientation for all cells.
                        Read during create only. */
    const double *y;
    const double *z;
} rtlbfs_curv3_mesh;

typedef struct {
    int kind[6];    /* sides i-, i+, j-, j+, k-, k+: RTLBFS_PERIODIC (in pairs),
                       RTLBFS_WALL_ISOTHERMAL or RTLBFS_WALL_ADIABATIC */
    double rot[3];  /* rotation about z closing each periodic axis (radians, |rot| <= 3.2), 0 otherwise */
    double Tw[6];   /* absolute temperature of isothermal walls */
    double up[3];   /* unit vector against gravity, or zero for no buoyancy */
    double T_ref;   /* absolute reference temperature of the buoyancy force; also the initial T */
} rtlbfs_curv3_bc;

/* Device workspace for a 3D body-fitted mesh (bytes); 0 for invalid sizes. */
size_t rtlbfs_curv3_workspace_bytes(const rtlbfs_curv3_mesh *mesh, const rtlbfs_opts *opts);

/* Create a solver on a 3D body-fitted mesh; nu, chi, beta_g given directly.
 * The state starts at rest with rho = 1 and T = T_ref (+ opts->noise_amp
 * noise).  Options, workspace, stream and errors as for rtlbfs_curv_create,
 * except opts->tile: 0 takes one fused launch per step (tile and halo staged
 * in LDS) when axis j is periodic with a single cell and axes i and k are
 * walled (the single-layer wedge of Sec. 4.5), three launches (per-cell
 * gradients, per-face fluxes, per-cell update) otherwise; 1 forces the three
 * launches; 2 forces the fused launch and is EINVAL on other meshes.  Both
 * compute every face with the same arithmetic.  The handle works with the single-domain entry
 * points and rtlbfs_wall_heat (sides 0..5); rtlbfs_nusselt returns
 * RTLBFS_EUNSUPPORTED. */
int rtlbfs_curv3_create(const rtlbfs_curv3_mesh *mesh, double nu, double chi, double beta_g,
                        const rtlbfs_curv3_bc *bc, const rtlbfs_opts *opts, void *hip_stream, void *workspace,
                        size_t ws_bytes, rtlbfs_t *out);

/* Centroids and volumes the library derived for a 3D body-fitted mesh (host
 * only; any pointer may be NULL).  EUNSUPPORTED on other handles. */
int rtlbfs_curv3_cells(rtlbfs_t h, double *host_cx, double *host_cy, double *host_cz, double *host_vol,
                       size_t count);

/* ----------------------------------------------------------- batched -- */
/* Many independent 2D domains advanced together: one kernel launch per step
 * covers the tiles of every member, replayed from a captured HIP graph.
 * meshes, Ra, Pr and bcs are arrays of `count`; each member has its own
 * lattice units, Eq. 63 parameters and Delta-t (the dtl/dt defaults apply per
 * member).  Precision must be the same for all (opts->precision).  The step
 * launch covers every member's tiles and must fit one dispatch (blocks x
 * threads at most 2^32 - 1, about 1.7e9 cells in total); a larger batch is
 * EINVAL (workspace bytes 0). */
size_t rtlbfs_batch_workspace_bytes(int count, const rtlbfs_mesh *meshes, const rtlbfs_opts *opts);

int rtlbfs_batch_create(int count, const rtlbfs_mesh *meshes, const double *Ra, const double *Pr, double Ma,
                        const rtlbfs_bc *bcs, const rtlbfs_opts *opts, void *hip_stream, void *workspace,
                        size_t ws_bytes, rtlbfs_batch_t *out);

/* Enqueue n steps of every member (each member takes its own Delta-t). */
int rtlbfs_batch_step(rtlbfs_batch_t h, int64_t n);

/* Per-member diagnostics and fields (synchronising). */
int rtlbfs_batch_nusselt(rtlbfs_batch_t h, int member, rtlbfs_nu *out);
int rtlbfs_batch_residual(rtlbfs_batch_t h, int member, double *res_u, double *res_T);
int rtlbfs_batch_get_field(rtlbfs_batch_t h, int member, int field, double *host_out, size_t count);
int rtlbfs_batch_get_info(rtlbfs_batch_t h, int member, rtlbfs_info *out);
int rtlbfs_batch_sync(rtlbfs_batch_t h);
/* Per-member divergence flags of the last residual step (synchronising):
 * host_flags[m] = 1 when member m held a NaN/Inf or a local Mach number at or
 * above opts.max_mach (the guard evaluated with Eq. 65), else 0.  host_flags holds `count`
 * ints owned by the caller.  A diverged member does not disturb the others,
 * so a parameter sweep keeps stepping the batch and reads the flags (the
 * stability maps of Sec. 3.3, Figs. 4-5).  Returns RTLBFS_ESTATE before the
 * first residual step, RTLBFS_OK otherwise (also when members diverged). */
int rtlbfs_batch_diverged(rtlbfs_batch_t h, int *host_flags);
int rtlbfs_batch_destroy(rtlbfs_batch_t h);

#ifdef __cplusplus
}
#endif
#endif
