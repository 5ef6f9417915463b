// rtlbfs_device.h -- device-side data structures and arithmetic of the RTLBFS
// step for gfx950 (CDNA4): domain descriptor, FP64 wave/block reductions and
// the face flux of Sec. 3.2 in 2D and 3D (Lu, Dai & Yu, arXiv 2202.13449).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rtlbfs {

constexpr double kCs2 = 1.0 / 3.0;  // c_s^2 = c^2/3 (Eq. 6)
constexpr double kT0 = 0.5;         // T_ref = (T_h + T_l)/2, T_l = 0, T_h = 1 (Eq. 64)
constexpr int kPartials = 5;        // residual partial sums per block

enum : int { kPeriodic = 0, kIsothermal = 1, kAdiabatic = 2 };

// Per-axis geometry, stored as kGeoFields arrays of n values (SoA) in the
// precision of the step kernel: the cell width, its inverse, and the Eq. 56
// inverse-distance weights of the low face (phi_S = lo_self * phi_P +
// lo_nb * phi_{P-1}) and of the high face (phi_S = hi_self * phi_P + hi_nb *
// phi_{P+1}).  Periodic axes use the wrapped neighbour; weights of wall faces
// are unused.
enum : int { kGeoW = 0, kGeoInvW, kGeoLoSelf, kGeoLoNb, kGeoHiSelf, kGeoHiNb, kGeoFields };

// Physical and lattice constants of the step: viscosity, diffusivity, lattice
// step, relaxation times (Eqs. 9-10), buoyancy beta*g, the time step Delta-t,
// and the lattice spacing h = c dt with its finite-difference factors.
// Tref_s: reference temperature of the buoyancy in the storage convention
// (absolute T, or T - T0 with deviation storage), read only by kernels that
// take it from here (face fluxes instantiated with TB); the Cartesian kernels
// use T_ref = T0.
template <typename R>
struct Phys {
    R nu, chi, dtl, tau_f, tau_g, bg, dt;
    R h, inv2h, invh2, inv4h2;
    R Tref_s;
};

// One structured domain as the kernels see it.  Lengths in lattice units;
// Tw is in the storage convention (T - T0 for deviation storage, absolute T
// for plain storage).
struct Domain {
    int dim;
    int n[3];
    int periodic[3];
    int kind[6];
    double Tw[6];
    int gaxis;        // buoyancy along +gaxis, -1 none
    int force_pred;   // 1: buoyancy also in the predicted momentum
    int sround;       // 1: stochastic rounding of the FP32 state update
    double nu, chi, bg, dtl, dt, tau_f, tau_g;
    const double *w[3];  // cell widths per axis (device, FP64; diagnostics)
    const void *geo[3];  // per-axis geometry records in the kernel precision (see kGeo*)
    int64_t cells;       // number of cells
    int64_t fstride;     // elements between consecutive fields of one state copy
    void *U[2];          // the two state copies (used by the batched kernels)
    Phys<float> phf;     // the constants above, in FP32 and in FP64
    Phys<double> phd;
    float Twf[6];        // Tw in FP32
    const double *vol;   // body-fitted meshes: cell areas (device, FP64); null on Cartesian meshes
    double guard_u2;     // divergence guard: |u|^2 at or above this (Mach max_mach) flags the run
};

// ------------------------------------------------------------ reductions --

// Sum over the 64 lanes of a wavefront (butterfly of cross-lane moves).
__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_max(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Block-wide sums of K values; the result is valid in thread 0.  `scratch`
// holds K * (blockDim/64) doubles of shared memory.  Thread k < K adds the
// wave sums of value k in wave order (the same order for every launch
// shape), so the K chains run side by side.
template <int K>
__device__ inline void block_sums(double (&v)[K], double *scratch) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
        for (int k = 0; k < K; ++k) scratch[k * nw + wave] = v[k];
    __syncthreads();
    if (threadIdx.x < K) {
        const int k = threadIdx.x;
        double s = 0.0;
        for (int w = 0; w < nw; ++w) s += scratch[k * nw + w];
        scratch[k * nw] = s;  // only this thread reads row k
    }
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = scratch[k * nw];
    __syncthreads();
}

// 1/x in the kernel precision.  FP32 kernels use the hardware reciprocal
// (v_rcp_f32, 1 ulp), which is well inside the FP32 path's own rounding
// budget and saves the correctly rounded division sequence; FP64 (and the
// host, where the face functions are also instantiated for operation
// counting) divide.
template <typename R>
__host__ __device__ inline R recip(R x) {
#if defined(__HIP_DEVICE_COMPILE__)
    if constexpr (sizeof(R) == 4) return __builtin_amdgcn_rcpf(x);
#endif
    return (R)1 / x;
}

// ------------------------------------------------------------ face flux --

// The physical and lattice constants of a step in the kernel precision; the
// host fills both precisions into the Domain once, so no kernel converts or
// divides them at run time.
template <typename R>
__device__ inline const Phys<R> &make_phys(const Domain &d) {
    if constexpr (sizeof(R) == 4) return d.phf;
    else return d.phd;
}

// Wall temperature of side s (storage convention) in the kernel precision.
template <typename R>
__device__ inline R wall_T(const Domain &d, int s) {
    if constexpr (sizeof(R) == 4) return d.Twf[s];
    else return d.Tw[s];
}

// One side of a face: cell-centre primitives (r, u_0..u_{D-1}, T) in the
// face-local frame (axis 0 = face normal n, then the tangents) and their
// gradients g[k][p] along local axis k.
template <typename R, int D>
struct Side {
    R v[D + 2];
    R g[D][D + 2];
};

// Interior-face flux per unit area along +n (Sec. 3.2), nodal form, for D = 2
// (D2Q9 node offsets) or D = 3 (D3Q19 offsets).  The kernels use face_flux
// below, which evaluates the same differences from the column polynomials;
// this form follows the paper node by node and fixes the algorithmic
// operation count (it is instantiated by the host-side operation counter and
// the host check that the two forms agree).  DEV selects the deviation storage
// (r = rho - 1, theta = rho (T - T0)); otherwise r is rho and T absolute.
// fdir: buoyancy unit vector in the local frame (added as dt * F at the face
// centre to the predicted momentum).  out = {mass, m_0..m_{D-1}, energy}.
//
// The lattice nodes X = x_S + h (a n + b t1 + c t2) take the primitives of
// Eq. 29: a < 0 from the left cell, a > 0 from the right cell, a = 0 the mean
// of both; in each column a the value is affine in (b, c).  Every node adds
// its products to the central-difference accumulators of Eqs. 46-48:
// D_k f = (f(+k) - f(-k))/2h, D_kk f = (f(+k) - 2 f(0) + f(-k))/h^2,
// D_kl f = (f(+k+l) - f(+k-l) - f(-k+l) + f(-k-l))/4h^2.
template <typename R, int D, bool DEV, bool TB = false>
__host__ __device__ inline void face_flux_nodes(const Side<R, D> &L, const Side<R, D> &Rt, R dL, R dR, const R (&fdir)[D],
                                 const Phys<R> &ph, R (&out)[D + 2]) {
    constexpr int NP = D + 2;
    const R cs2 = (R)kCs2;
    const R half = (R)0.5;
    R base[3][NP], slope[3][D][NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        base[0][p] = L.v[p] + L.g[0][p] * (dL - ph.h);       // X - x_L = (dL - h) n + ...
        base[2][p] = Rt.v[p] + Rt.g[0][p] * (ph.h - dR);     // X - x_R = (h - dR) n + ...
        base[1][p] = half * ((L.v[p] + L.g[0][p] * dL) + (Rt.v[p] - Rt.g[0][p] * dR));
#pragma unroll
        for (int k = 1; k < D; ++k) {
            slope[0][k][p] = ph.h * L.g[k][p];
            slope[2][k][p] = ph.h * Rt.g[k][p];
            slope[1][k][p] = half * (slope[0][k][p] + slope[2][k][p]);
        }
    }
    // Accumulators (local axes a, b):
    R Dn_m[D], Da_mn[D], lapm[D], gdm[D], divK[D], Dr[D];
#pragma unroll
    for (int a = 0; a < D; ++a) Dn_m[a] = Da_mn[a] = lapm[a] = gdm[a] = divK[a] = Dr[a] = (R)0;
    R divm = 0, ddK = 0, lapr = 0, divq = 0, lape = 0, Dne = 0;
    R r0 = 0, e0 = 0, T0n = 0, m0[D], K0n[D], q0n = 0;
    const R w1 = ph.inv2h, w2 = ph.invh2, w4 = ph.inv4h2;
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
            for (int c = -1; c <= 1; ++c) {
                if (D == 2 && c != 0) continue;
                if (abs(a) + abs(b) + abs(c) > 2) continue;  // D3Q19 has no corner nodes
                const int o[3] = {a, b, c};
                R v[NP];
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    R x = base[a + 1][p];
#pragma unroll
                    for (int k = 1; k < D; ++k)
                        if (o[k] != 0) x += (R)o[k] * slope[a + 1][k][p];
                    v[p] = x;
                }
                const R rv = v[0];
                const R rho = DEV ? (R)1 + rv : rv;
                R m[D];
#pragma unroll
                for (int k = 0; k < D; ++k) m[k] = rho * v[1 + k];
                const R e = rho * v[D + 1];
                const int nz = (a != 0) + (b != 0) + (c != 0);
                if (nz == 0) {
                    r0 = rv;
                    e0 = e;
                    T0n = v[D + 1];
#pragma unroll
                    for (int k = 0; k < D; ++k) {
                        m0[k] = m[k];
                        K0n[k] = m[k] * v[1];
                        lapm[k] -= (R)(2 * D) * w2 * m[k];
                        gdm[k] -= (R)2 * w2 * m[k];
                        ddK -= (R)2 * w2 * m[k] * v[1 + k];
                    }
                    q0n = e * v[1];
                    lapr -= (R)(2 * D) * w2 * rv;
                    lape -= (R)(2 * D) * w2 * e;
                } else if (nz == 1) {
                    const int k = a != 0 ? 0 : (b != 0 ? 1 : 2);
                    const R s1 = (R)o[k] * w1;
                    if (k == 0) {
#pragma unroll
                        for (int q = 0; q < D; ++q) Dn_m[q] += s1 * m[q];
                        Dne += s1 * e;
                    }
                    Da_mn[k] += s1 * m[0];
                    divm += s1 * m[k];
#pragma unroll
                    for (int q = 0; q < D; ++q) {
                        lapm[q] += w2 * m[q];
                        divK[q] += s1 * m[q] * v[1 + k];  // D_k (rho u_q u_k)
                    }
                    gdm[k] += w2 * m[k];
                    ddK += w2 * m[k] * v[1 + k];
                    Dr[k] += s1 * rv;
                    lapr += w2 * rv;
                    divq += s1 * e * v[1 + k];
                    lape += w2 * e;
                } else {
                    const int k = a != 0 ? 0 : 1;
                    const int l = c != 0 ? 2 : 1;
                    const R s4 = (R)(o[k] * o[l]) * w4;
                    gdm[k] += s4 * m[l];
                    gdm[l] += s4 * m[k];
                    ddK += (R)2 * s4 * m[k] * v[1 + l];
                }
            }
    const R dt = ph.dtl, dt2h = half * ph.dtl * ph.dtl;
    const R rho0 = DEV ? (R)1 + r0 : r0;
    // Buoyancy at the face centre (Eq. 64).
    const R Fb = ph.bg * rho0 * (TB ? T0n - ph.Tref_s : (DEV ? T0n : T0n - (R)kT0));
    // Eqs. 46-48 as increments over the face-centre values.
    const R dr = -dt * divm + dt2h * (ddK + cs2 * lapr);
    R dm[D], ms[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        dm[q] = -dt * (divK[q] + cs2 * Dr[q]) + cs2 * dt2h * (lapm[q] + (R)2 * gdm[q]) + dt * fdir[q] * Fb;
        ms[q] = m0[q] + dm[q];
    }
    const R de = -dt * divq + cs2 * dt2h * lape;
    const R rhos = rho0 + dr, es = e0 + de;
    const R inv_rhos = recip(rhos);
    // Eqs. 57-59.
    out[0] = ms[0];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        R f = K0n[q] - ph.nu * (Dn_m[q] + Da_mn[q]) - (ph.tau_f - (R)1.5) * (ms[q] * ms[0] * inv_rhos - K0n[q]);
        if (q == 0) f += cs2 * r0 - ph.nu * divm - (ph.tau_f - (R)1.5) * cs2 * dr;
        out[1 + q] = f;
    }
    R fe = q0n - ph.chi * Dne - (ph.tau_g - (R)1.5) * (ms[0] * es * inv_rhos - q0n);
    if (DEV) {
        // theta = e - T0 rho is advanced with Q - T0 P; e* = T0 rho_e* + theta*
        // with rho_e* - rho* = -dt^2/2 d_a d_b (rho u_a u_b).
        fe += (R)kT0 * (-(ph.tau_g - half) * dm[0] - ph.chi * Dr[0] + (ph.tau_g - (R)1.5) * ms[0] * dt2h * ddK * inv_rhos);
    }
    out[D + 1] = fe;
}

// Interior-face flux per unit area along +n (Sec. 3.2), column form: the
// same predictor (Eqs. 46-48) and fluxes (Eqs. 57-59) as face_flux_nodes,
// with the central differences taken from polynomial coefficients instead of
// node values.  The node X = x_S + h (a n + b t1 + c t2) lies in column a;
// along the tangents every primitive of a column is affine (Eq. 29), so a
// product of two primitives is quadratic in (b, c) and of three cubic.  A
// tangential first difference over nodes +-1 is the polynomial's odd part, a
// second difference its quadratic coefficient (zero for a single primitive),
// and a mixed difference over four corner nodes its b c coefficient (taken
// in the columns a = +-1 for the normal-tangent pairs).  Exact in exact
// arithmetic, with fewer operations than the nodal form and no rounding
// noise in differences that vanish exactly.  Arguments as for
// face_flux_nodes.
template <typename R, int D, bool DEV, bool TB = false>
__host__ __device__ inline void face_flux(const Side<R, D> &L, const Side<R, D> &Rt, R dL, R dR, const R (&fdir)[D],
                                 const Phys<R> &ph, R (&out)[D + 2]) {
    constexpr int NP = D + 2;
    const R cs2 = (R)kCs2;
    const R half = (R)0.5;
    // Column a (0: a = -1, from the left cell; 2: a = +1, from the right
    // cell; 1: a = 0, the mean of both): the primitives on the column's
    // centre line B[a][p] and their slopes per lattice step along each
    // tangent S[a][k][p] (Eq. 29).
    R B[3][NP], S[3][D][NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        B[0][p] = L.v[p] + L.g[0][p] * (dL - ph.h);
        B[2][p] = Rt.v[p] + Rt.g[0][p] * (ph.h - dR);
        B[1][p] = half * ((L.v[p] + L.g[0][p] * dL) + (Rt.v[p] - Rt.g[0][p] * dR));
#pragma unroll
        for (int k = 1; k < D; ++k) {
            S[0][k][p] = ph.h * L.g[k][p];
            S[2][k][p] = ph.h * Rt.g[k][p];
            S[1][k][p] = half * (S[0][k][p] + S[2][k][p]);
        }
    }
    const R w1 = ph.inv2h, w2 = ph.invh2, w4 = ph.inv4h2;
    const R w1x2 = w1 + w1, w2x2 = w2 + w2;
    // Centre-line conserved values of each column.
    R rho[3], m[3][D], e[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        rho[a] = DEV ? (R)1 + B[a][0] : B[a][0];
#pragma unroll
        for (int q = 0; q < D; ++q) m[a][q] = rho[a] * B[a][1 + q];
        e[a] = rho[a] * B[a][D + 1];
    }
    // Normal direction: nodes (+-1, 0, 0) and the centre.
    R Dn_m[D], lapm[D], divK[D], gdm[D], Da_mn[D], Dr[D];
    R mn_un[3], e_un[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        mn_un[a] = m[a][0] * B[a][1];
        e_un[a] = e[a] * B[a][1];
    }
#pragma unroll
    for (int q = 0; q < D; ++q) {
        Dn_m[q] = w1 * (m[2][q] - m[0][q]);
        lapm[q] = w2 * ((m[2][q] - m[1][q]) + (m[0][q] - m[1][q]));
        divK[q] = w1 * (m[2][q] * B[2][1] - m[0][q] * B[0][1]);
    }
    const R Dne = w1 * (e[2] - e[0]);
    R lape = w2 * ((e[2] - e[1]) + (e[0] - e[1]));
    Dr[0] = w1 * (B[2][0] - B[0][0]);
    const R lapr = w2 * ((B[2][0] - B[1][0]) + (B[0][0] - B[1][0]));
    R divq = w1 * (e_un[2] - e_un[0]);
    R ddK = w2 * ((mn_un[2] - mn_un[1]) + (mn_un[0] - mn_un[1]));
    Da_mn[0] = Dn_m[0];
    R divm = Dn_m[0];
    gdm[0] = lapm[0];
    // Tangent k: in column a = 0 every field is affine along the tangent, so
    // products of two fields are quadratic and of three cubic; the central
    // differences of Eqs. 46-48 are their odd and even coefficients.  The
    // mixed differences with the normal take the odd coefficients of the
    // columns a = +-1.
#pragma unroll
    for (int k = 1; k < D; ++k) {
        const R sr = S[1][k][0], sT = S[1][k][D + 1];
        const R uk = B[1][1 + k], sk = S[1][k][1 + k];
#pragma unroll
        for (int q = 0; q < D; ++q) {
            const R uq = B[1][1 + q], sq = S[1][k][1 + q];
            lapm[q] += w2x2 * (sr * sq);
            divK[q] += w1x2 * (sr * (uq * uk + sq * sk) + rho[1] * (sq * uk + uq * sk));
        }
        const R Dk_mk = w1x2 * (rho[1] * sk + sr * uk);
        Da_mn[k] = w1x2 * (rho[1] * S[1][k][1] + sr * B[1][1]);
        divm += Dk_mk;
        Dr[k] = w1x2 * sr;
        lape += w2x2 * (sr * sT);
        divq += w1x2 * (sr * (B[1][D + 1] * uk + sT * sk) + rho[1] * (sT * uk + B[1][D + 1] * sk));
        ddK += w2x2 * (sk * (rho[1] * sk + (R)2 * sr * uk));
        gdm[k] = w2x2 * (sr * sk);
        // (n, k) corners: nodes (+-1, +-1 along k).
        R om_k[2], om_n[2], omu[2];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int a = 2 * j;
            const R ar = S[a][k][0], an = S[a][k][1], ak = S[a][k][1 + k];
            const R Un = B[a][1], Uk = B[a][1 + k];
            om_k[j] = rho[a] * ak + ar * Uk;
            om_n[j] = rho[a] * an + ar * Un;
            omu[j] = ar * (Un * Uk + an * ak) + rho[a] * (an * Uk + Un * ak);
        }
        const R w4x2 = w4 + w4;
        gdm[0] += w4x2 * (om_k[1] - om_k[0]);
        gdm[k] += w4x2 * (om_n[1] - om_n[0]);
        ddK += (R)2 * w4x2 * (omu[1] - omu[0]);
    }
    if constexpr (D == 3) {
        // (t1, t2) corners: nodes (0, +-1, +-1); the sum of b c f over the four
        // is 4 times the b c coefficient of f.
        const R r1 = S[1][1][0], r2 = S[1][2][0];
        const R U1 = B[1][2], U2 = B[1][3];
        const R a1 = S[1][1][2], a2 = S[1][2][2];  // slopes of u_1 along t1, t2
        const R c1 = S[1][1][3], c2 = S[1][2][3];  // slopes of u_2 along t1, t2
        const R bc_m1 = r1 * a2 + r2 * a1;
        const R bc_m2 = r1 * c2 + r2 * c1;
        const R bc_m1u2 = r1 * (a2 * U2 + U1 * c2) + r2 * (a1 * U2 + U1 * c1) + rho[1] * (a1 * c2 + a2 * c1);
        const R w4x4 = (R)4 * w4;
        gdm[1] += w4x4 * bc_m2;
        gdm[2] += w4x4 * bc_m1;
        ddK += (R)2 * w4x4 * bc_m1u2;
    }
    const R r0 = B[1][0], e0 = e[1], T0n = B[1][D + 1];
    R m0[D], K0n[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        m0[q] = m[1][q];
        K0n[q] = m[1][q] * B[1][1];
    }
    const R q0n = e[1] * B[1][1];
    const R dt = ph.dtl, dt2h = half * ph.dtl * ph.dtl;
    const R rho0 = rho[1];
    const R Fb = ph.bg * rho0 * (TB ? T0n - ph.Tref_s : (DEV ? T0n : T0n - (R)kT0));
    const R dr = -dt * divm + dt2h * (ddK + cs2 * lapr);
    R dm[D], ms[D];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        dm[q] = -dt * (divK[q] + cs2 * Dr[q]) + cs2 * dt2h * (lapm[q] + (R)2 * gdm[q]) + dt * fdir[q] * Fb;
        ms[q] = m0[q] + dm[q];
    }
    const R de = -dt * divq + cs2 * dt2h * lape;
    const R rhos = rho0 + dr, es = e0 + de;
    const R inv_rhos = recip(rhos);
    out[0] = ms[0];
#pragma unroll
    for (int q = 0; q < D; ++q) {
        R f = K0n[q] - ph.nu * (Dn_m[q] + Da_mn[q]) - (ph.tau_f - (R)1.5) * (ms[q] * ms[0] * inv_rhos - K0n[q]);
        if (q == 0) f += cs2 * r0 - ph.nu * divm - (ph.tau_f - (R)1.5) * cs2 * dr;
        out[1 + q] = f;
    }
    R fe = q0n - ph.chi * Dne - (ph.tau_g - (R)1.5) * (ms[0] * es * inv_rhos - q0n);
    if (DEV) {
        fe += (R)kT0 * (-(ph.tau_g - half) * dm[0] - ph.chi * Dr[0] + (ph.tau_g - (R)1.5) * ms[0] * dt2h * ddK * inv_rhos);
    }
    out[D + 1] = fe;
}

// TLBFS interface flux per unit area along +n (Sec. 2.2, Eqs. 29-40), same
// arguments and frame as face_flux.  The lattice node at offset o streams
// along e_i = -o; its equilibria (Eqs. 3-4, D2Q9 / D3Q19 weights of Eq. 6)
// give the predicted moments of Eqs. 30-32 and the back-node parts of the
// fluxes of Eqs. 38-40.  The face-centre parts use the equilibrium moment
// identities (Eqs. 7-8), which hold exactly on these lattices:
// sum e_n f* = m*_n, sum e_a e_n f* = c_s^2 rho* d_an + m*_a m*_n / rho*,
// sum e_n g* = E* m*_n / rho*.
// With deviation storage every sum is carried without its O(1) part: the
// node equilibrium w rho (1 + A) enters as w phi, phi = A + r (1 + A), whose
// plain sums differ from the full ones by the lattice constants sum w = 1,
// sum w e = 0 and sum w e e = c_s^2 I; the energy is carried as theta with
// rho T = T0 rho + theta and the theta flux Q - T0 P assembled from small
// terms (A = e.u / c_s^2 + (e.u)^2 / 2c_s^4 - u^2 / 2c_s^2, B = e.u / c_s^2).
template <typename R, int D, bool DEV, bool TB = false>
__host__ __device__ inline void face_flux_tlbfs(const Side<R, D> &L, const Side<R, D> &Rt, R dL, R dR,
                                       const R (&fdir)[D], const Phys<R> &ph, R (&out)[D + 2]) {
    constexpr int NP = D + 2;
    const R cs2 = (R)kCs2;
    const R half = (R)0.5;
    R base[3][NP], slope[3][D][NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        base[0][p] = L.v[p] + L.g[0][p] * (dL - ph.h);
        base[2][p] = Rt.v[p] + Rt.g[0][p] * (ph.h - dR);
        base[1][p] = half * ((L.v[p] + L.g[0][p] * dL) + (Rt.v[p] - Rt.g[0][p] * dR));
#pragma unroll
        for (int k = 1; k < D; ++k) {
            slope[0][k][p] = ph.h * L.g[k][p];
            slope[2][k][p] = ph.h * Rt.g[k][p];
            slope[1][k][p] = half * (slope[0][k][p] + slope[2][k][p]);
        }
    }
    const R w0 = D == 2 ? (R)(4.0 / 9.0) : (R)(1.0 / 3.0);
    const R w1 = D == 2 ? (R)(1.0 / 9.0) : (R)(1.0 / 18.0);
    const R w2 = (R)(1.0 / 36.0);
    // sums over the nodes: density part rs (rho* or r*), momentum ms, back-node
    // momentum flux pb (sum e_a e_n f, or its phi part), energy es (E* or
    // theta*), back-node energy flux qb, and (deviation) sn = sum w e_n rho C
    R rs = 0, ms[D], pb[D], es = 0, qb = 0, sn = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) ms[k] = pb[k] = (R)0;
    R rho_c = 0, T_c = 0;
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
        for (int b = -1; b <= 1; ++b)
#pragma unroll
            for (int c = -1; c <= 1; ++c) {
                if (D == 2 && c != 0) continue;
                if (abs(a) + abs(b) + abs(c) > 2) continue;
                const int o[3] = {a, b, c};
                const int nz = (a != 0) + (b != 0) + (c != 0);
                const R w = nz == 0 ? w0 : (nz == 1 ? w1 : w2);
                R v[NP];
#pragma unroll
                for (int p = 0; p < NP; ++p) {
                    R x = base[a + 1][p];
#pragma unroll
                    for (int k = 1; k < D; ++k)
                        if (o[k] != 0) x += (R)o[k] * slope[a + 1][k][p];
                    v[p] = x;
                }
                // e_i = -o in the face frame
                R eu = 0, uu = 0;
#pragma unroll
                for (int k = 0; k < D; ++k) {
                    if (o[k] != 0) eu += (R)(-o[k]) * v[1 + k];
                    uu += v[1 + k] * v[1 + k];
                }
                const R A = (R)3 * eu + (R)4.5 * eu * eu - (R)1.5 * uu;
                const R B = (R)3 * eu;
                const R rho = DEV ? (R)1 + v[0] : v[0];
                if (nz == 0) {
                    rho_c = rho;
                    T_c = v[D + 1];
                }
                if (DEV) {
                    const R phi = w * (A + v[0] * ((R)1 + A));
                    const R th = rho * v[D + 1];      // theta at the node
                    const R C = (R)1.5 * uu - (R)4.5 * eu * eu;  // B - A
                    const R g = w * th * ((R)1 + B);
                    rs += phi;
                    es += g + (R)kT0 * w * rho * C;
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        if (o[k] != 0) ms[k] += (R)(-o[k]) * phi;
                    if (a != 0) {
                        const R en = (R)(-a);
#pragma unroll
                        for (int k = 0; k < D; ++k)
                            if (o[k] != 0) pb[k] += en * (R)(-o[k]) * phi;
                        qb += en * g;
                        sn += en * w * rho * C;
                    }
                } else {
                    const R f = w * rho * ((R)1 + A);
                    const R g = w * rho * v[D + 1] * ((R)1 + B);
                    rs += f;
                    es += g;
#pragma unroll
                    for (int k = 0; k < D; ++k)
                        if (o[k] != 0) ms[k] += (R)(-o[k]) * f;
                    if (a != 0) {
                        const R en = (R)(-a);
#pragma unroll
                        for (int k = 0; k < D; ++k)
                            if (o[k] != 0) pb[k] += en * (R)(-o[k]) * f;
                        qb += en * g;
                    }
                }
            }
    // buoyancy in the predicted momentum, at the face centre (Eq. 64)
    const R Fb = ph.bg * rho_c * (TB ? T_c - ph.Tref_s : (DEV ? T_c : T_c - (R)kT0));
    const R dt = ph.dtl;
#pragma unroll
    for (int k = 0; k < D; ++k) ms[k] += dt * fdir[k] * Fb;
    const R rhos = DEV ? (R)1 + rs : rs;
    const R inv_rhos = recip(rhos);
    const R cf = (R)1.5 - ph.tau_f, df = half - ph.tau_f;
    const R cg = (R)1.5 - ph.tau_g, dg = half - ph.tau_g;
    out[0] = ms[0];                                                  // Eq. 38
#pragma unroll
    for (int k = 0; k < D; ++k)                                      // Eq. 39
        out[1 + k] = cf * ((k == 0 ? cs2 * rs : (R)0) + ms[k] * ms[0] * inv_rhos) - df * pb[k];
    if (DEV)                                                         // Eq. 40, as Q - T0 P
        out[D + 1] = cg * es * ms[0] * inv_rhos - dg * ((R)kT0 * (sn - dt * fdir[0] * Fb) + qb);
    else
        out[D + 1] = cg * es * ms[0] * inv_rhos - dg * qb;
}

// Wall flux per unit area along +axis for the cell P next to a no-slip wall
// (outward normal sgn * e_axis, centre-to-wall distance d): no mass flux,
// pressure c_s^2 r on the normal, one-sided viscous stress with
// V_n = -3 m_n/d and V_t = -m_t/d, and for an isothermal wall the one-sided
// conduction -chi (rho T_w - e)/d.  m: momentum in the local frame (m[0]
// along the wall normal).
template <typename R, int D, bool DEV>
__host__ __device__ inline void wall_flux(R rP, const R (&m)[D], R eP, R sgn, R d, bool iso, R Tw, const Phys<R> &ph,
                                 R (&out)[D + 2]) {
    const R rho = DEV ? (R)1 + rP : rP;
    const R inv_d = recip(d);
    out[0] = (R)0;
    out[1] = (R)kCs2 * rP + sgn * (R)3 * ph.nu * m[0] * inv_d;
#pragma unroll
    for (int q = 1; q < D; ++q) out[1 + q] = sgn * ph.nu * m[q] * inv_d;
    out[D + 1] = iso ? -sgn * ph.chi * (rho * Tw - eP) * inv_d : (R)0;
}

// ------------------------------------------------------ stochastic rounding --

// 32-bit integer finaliser of MurmurHash3 (Appleby) applied to a combined
// (cell, field, step) key: the counter-based random source of the stochastic
// rounding below.
__device__ inline uint32_t sr_hash(uint32_t a, uint32_t b) {
    uint32_t x = a * 0x9E3779B1u ^ (b * 0x85EBCA77u + 0x27D4EB2Fu);
    x ^= x >> 16;
    x *= 0x85EBCA6Bu;
    x ^= x >> 13;
    x *= 0xC2B2AE35u;
    x ^= x >> 16;
    return x;
}

// a + b rounded stochastically to float: the exact sum s + e (TwoSum) is
// rounded to the neighbour of s on the side of e with probability |e|/gap, so
// the stored state is unbiased even when the increments are far below half an
// ulp (plain round-to-nearest would stall the slow modes near steady state).
__device__ inline float sr_add(float a, float b, uint32_t rnd) {
    const float s = a + b;
    const float bp = s - a;
    const float e = (a - (s - bp)) + (b - bp);  // s + e == a + b exactly (TwoSum)
    // neighbour of s on the side of e: one ulp up in magnitude when e has the
    // sign of s, one down otherwise (the bit pattern of a float is monotone in
    // its magnitude); s == 0 only when |a + b| is below the smallest float.
    const bool away = (e > 0.0f) == (s > 0.0f);
    const float t = __uint_as_float(__float_as_uint(s) + (away ? 1u : 0xFFFFFFFFu));
    const float u = (float)(rnd >> 8) * 5.9604644775390625e-8f;  // [0, 1), 24 random bits
    const bool up = e != 0.0f && s != 0.0f && fabsf(u * (t - s)) < fabsf(e);  // P(up) = |e| / |t - s|
    return up ? t : s;
}

__device__ inline double sr_add(double a, double b, uint32_t) { return a + b; }

__device__ inline int wrap(int i, int n) {
    i %= n;
    return i < 0 ? i + n : i;
}

// wrap(i, n) for -n <= i < 2n, by two selects instead of an integer
// remainder.  A tile kernel takes it on a periodic axis of n cells when the
// tile plus both halos is no wider than n: its halo and ragged-tile
// positions (tile start below n, halo depth h) then lie in [-h, n + tile + h).
__device__ inline int wrap_near(int i, int n) {
    return i < 0 ? i + n : (i >= n ? i - n : i);
}

// The index wrap of one periodic axis: near (a scalar, the same for the whole
// block) selects wrap_near.
__device__ inline int wrap_axis(int i, int n, bool near) {
    return near ? wrap_near(i, n) : wrap(i, n);
}

}  // namespace rtlbfs
