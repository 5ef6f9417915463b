// curv3d.h -- the RTLBFS time step on a 3D body-fitted (structured
// curvilinear) hexahedral mesh, the setting of Sec. 4.5: a concentric
// annulus run with a single azimuthal cell layer, whose two azimuthal sides
// form a periodic pair closed by a rotation about z.
//
// Each face carries its unit normal n, a tangent t1 (the face's first edge
// without its normal part) and t2 = n x t1; the D3Q19 lattice of Fig. 1 is
// aligned with (n, t1, t2).  On a general mesh a step is three launches
// over HBM buffers, one thread per item:
//   k_c3_grad    per cell: primitives and Eq. 55 gradients, sum over the six
//                faces of phi_S S_out / dV with Eq. 56 face values;
//   k_c3_flux    per face: the interior-face flux in the face frame (the
//                Eq. 29 values of a side whose centre lies off the normal are
//                shifted by the tangential gradients times the offsets) or
//                the wall closure; area-weighted, global components;
//   k_c3_update  per cell: divergence, buoyancy along `up`, forward Euler,
//                stochastic rounding of the FP32 state, Eq. 65 partials.
// On the single-layer wedge (j periodic with one cell, i and k walled) one
// fused launch, k_c3_layer, does all three in LDS per tile.
// Across a periodic side the neighbour is the image of the cell on the other
// side, rotated by -alpha (low side) or +alpha (high side) about z: its
// velocity as a vector, its velocity gradient as R G R^T.  Every face,
// including both faces of a periodic pair, computes its own flux.
//
// Face records (SoA, kernel precision), axis-a faces at index
// (k*(n1 + [a=1]) + j)*(n0 + [a=0]) + i, i.e. the vertex numbering with the
// face's own axis extended.
#pragma once

#include "rtlbfs_device.h"

namespace rtlbfs {

// n (3), t1 (3), dS, then for the low cell L and the high cell R:
// dL = (x_S - x_L).n, tL1/tL2 = (x_S - x_L).t1/t2, dR = (x_R - x_S).n,
// tR1/tR2 = (x_S - x_R).t1/t2, and the Eq. 56 weight wL of the low cell's
// value.  Images across periodic sides enter with their rotated centroids;
// a wall face stores the interior cell's normal distance in dL and dR.
enum : int {
    kC3Nx = 0, kC3Ny, kC3Nz, kC3T1x, kC3T1y, kC3T1z, kC3DS, kC3DL, kC3TL1, kC3TL2, kC3DR, kC3TR1, kC3TR2, kC3WL,
    kC3Fields
};

struct Curv3Geo {
    const void *f[3];      // face records per axis (kernel precision), kC3Fields fields each
    int64_t sf[3];         // face counts per axis (field strides)
    const void *inv_vol;   // 1 / dV per cell
    void *prim;            // scratch: 5 primitives per cell (field-major, stride = cells)
    void *grad;            // scratch: 15 gradients per cell, [p * 3 + axis]
    void *flux;            // scratch: 5 area-weighted fluxes per face, faces of the three axes concatenated
    int64_t nfaces;        // F0 + F1 + F2
    double rc[3], rs[3];   // cos, sin of the closing rotation of each periodic axis (1, 0 if none)
    double up[3];          // unit vector against gravity (0 if no buoyancy)
    float upf[3];
};

// Element a of a 3-array (6-array) held in the kernel arguments, chosen by
// selects: indexing such an array, or a private one, with a run-time index
// would copy it to scratch memory and read it back with a dependent load.
template <typename T>
__device__ inline T pick3(int a, const T (&v)[3]) {
    return a == 0 ? v[0] : (a == 1 ? v[1] : v[2]);
}

template <typename T>
__device__ inline T pick6(int s, const T (&v)[6]) {
    return s < 3 ? (s == 0 ? v[0] : (s == 1 ? v[1] : v[2])) : (s == 3 ? v[3] : (s == 4 ? v[4] : v[5]));
}

template <typename R>
__device__ inline R c3_up(const Curv3Geo &g, int a) {
    if constexpr (sizeof(R) == 4) return g.upf[a];
    else return g.up[a];
}

// Rotation about z by the angle with cosine c, sine s: v -> R v.
template <typename R>
__host__ __device__ inline void rot_z(R c, R s, R (&v)[3]) {
    const R x = c * v[0] - s * v[1], y = s * v[0] + c * v[1];
    v[0] = x;
    v[1] = y;
}

// One side of a face in the frame e[0] = n, e[1] = t1, e[2] = t2: primitives
// P = (r, u_x, u_y, u_z, T) and gradients G[p][axis] of a cell, rotated, and
// shifted by the tangential gradients times tau1, tau2.
template <typename R>
__host__ __device__ inline void side_in_frame3(const R (&P)[5], const R (&G)[5][3], const R (&e)[3][3], R tau1,
                                               R tau2, Side<R, 3> &S) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        S.g[k][0] = G[0][0] * e[k][0] + G[0][1] * e[k][1] + G[0][2] * e[k][2];
        S.g[k][4] = G[4][0] * e[k][0] + G[4][1] * e[k][1] + G[4][2] * e[k][2];
        R gu[3];  // d_k u_x, d_k u_y, d_k u_z
#pragma unroll
        for (int a = 0; a < 3; ++a) gu[a] = G[1 + a][0] * e[k][0] + G[1 + a][1] * e[k][1] + G[1 + a][2] * e[k][2];
#pragma unroll
        for (int q = 0; q < 3; ++q) S.g[k][1 + q] = e[q][0] * gu[0] + e[q][1] * gu[1] + e[q][2] * gu[2];
    }
    S.v[0] = P[0];
#pragma unroll
    for (int q = 0; q < 3; ++q) S.v[1 + q] = P[1] * e[q][0] + P[2] * e[q][1] + P[3] * e[q][2];
    S.v[4] = P[4];
#pragma unroll
    for (int p = 0; p < 5; ++p) S.v[p] += S.g[1][p] * tau1 + S.g[2][p] * tau2;
}

// Interior-face flux (RTLBFS, or TLBFS when TL) along +n times the face
// area, momentum back in global components.
template <typename R, bool DEV, bool TL>
__host__ __device__ inline void frame_flux3(const Side<R, 3> &A, const Side<R, 3> &B, R dL, R dR, const R (&e)[3][3],
                                            const R (&up)[3], bool fp, R dS, const Phys<R> &ph, R (&F)[5]) {
    R fdir[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) fdir[q] = fp ? up[0] * e[q][0] + up[1] * e[q][1] + up[2] * e[q][2] : (R)0;
    R G[5];
    if constexpr (TL) face_flux_tlbfs<R, 3, DEV, true>(A, B, dL, dR, fdir, ph, G);
    else face_flux<R, 3, DEV, true>(A, B, dL, dR, fdir, ph, G);
    F[0] = G[0] * dS;
#pragma unroll
    for (int a = 0; a < 3; ++a) F[1 + a] = (G[1] * e[0][a] + G[2] * e[1][a] + G[3] * e[2][a]) * dS;
    F[4] = G[4] * dS;
}

__device__ inline int64_t c3_cell(const Domain &d, int i, int j, int k) {
    return ((int64_t)k * d.n[1] + j) * d.n[0] + i;
}

__device__ inline int64_t c3_face(const Domain &d, int a, int i, int j, int k) {
    return ((int64_t)k * (d.n[1] + (a == 1)) + j) * (d.n[0] + (a == 0)) + i;
}

// Neighbour of cell q (index triple) across its face on `axis`, side hi:
// the mesh cell and the sine of its image rotation (cosine in *c); -1 at a
// wall.
__device__ inline int64_t c3_neighbour(const Domain &d, const Curv3Geo &g, const int (&q)[3], int axis, int hi,
                                       double &c, double &s) {
    int r[3] = {q[0], q[1], q[2]};
    r[axis] += hi ? 1 : -1;
    c = 1.0;
    s = 0.0;
    if (r[axis] < 0 || r[axis] >= d.n[axis]) {
        if (!d.periodic[axis]) return -1;
        c = g.rc[axis];
        s = hi ? g.rs[axis] : -g.rs[axis];
        r[axis] = r[axis] < 0 ? r[axis] + d.n[axis] : r[axis] - d.n[axis];
    }
    return c3_cell(d, r[0], r[1], r[2]);
}

template <typename R, bool DEV>
__device__ inline void c3_prims(const Domain &d, const R *__restrict__ U, int64_t c, R (&P)[5]) {
    const int64_t N = d.fstride;
    const R r = U[c];
    const R inv = recip<R>(DEV ? (R)1 + r : r);
    P[0] = r;
#pragma unroll
    for (int p = 1; p < 5; ++p) P[p] = U[p * N + c] * inv;
}

// Threads per block of the per-cell and per-face kernels.  The kernels are
// bound by load latency at small sizes (28,800 cells for the Sec. 4.5
// annulus); one-wavefront blocks spread the waves, and their memory
// traffic, over every CU.
constexpr int kC3Threads = 64;

template <typename R, bool DEV>
__global__ void __launch_bounds__(kC3Threads) k_c3_grad(Domain d, Curv3Geo g, const R *__restrict__ U) {
    // 32-bit index arithmetic: a body-fitted mesh holds at most 2^28 cells
    const int c = (int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
    if (c >= (int)d.cells) return;
    const int i = c % d.n[0], jk = c / d.n[0], j = jk % d.n[1], k = jk / d.n[1];
    const int q[3] = {i, j, k};
    R P[5];
    c3_prims<R, DEV>(d, U, c, P);
    R acc[5][3];
#pragma unroll
    for (int p = 0; p < 5; ++p) acc[p][0] = acc[p][1] = acc[p][2] = (R)0;
    // unrolled, so the loads of all six faces and neighbours are in flight together
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int hi = 0; hi < 2; ++hi) {
            int fq[3] = {i, j, k};
            fq[a] += hi;
            const R *rec = (const R *)g.f[a] + c3_face(d, a, fq[0], fq[1], fq[2]);
            const int64_t st = g.sf[a];
            const R so = hi ? (R)1 : (R)-1;
            const R sx = so * rec[kC3Nx * st] * rec[kC3DS * st], sy = so * rec[kC3Ny * st] * rec[kC3DS * st];
            const R sz = so * rec[kC3Nz * st] * rec[kC3DS * st];
            double cr, sr;
            const int64_t nb = c3_neighbour(d, g, q, a, hi, cr, sr);
            // The neighbour is read unconditionally (a wall face reads the
            // cell itself and discards it), so the loads of all six faces are
            // issued together instead of one wall branch after another.
            const bool wall = nb < 0;
            R Q[5];
            c3_prims<R, DEV>(d, U, wall ? (int64_t)c : nb, Q);
            R u[3] = {Q[1], Q[2], Q[3]};
            rot_z<R>((R)cr, (R)sr, u);
            Q[1] = u[0];
            Q[2] = u[1];
            Q[3] = u[2];
            const R wL = rec[kC3WL * st];
            const int side = 2 * a + hi;
            const R Tw = d.kind[side] == kIsothermal ? wall_T<R>(d, side) : P[4];
            const R pw[5] = {P[0], (R)0, (R)0, (R)0, Tw};  // wall values
            R phi[5];
#pragma unroll
            for (int p = 0; p < 5; ++p) {
                const R pin = hi ? wL * P[p] + ((R)1 - wL) * Q[p] : wL * Q[p] + ((R)1 - wL) * P[p];
                phi[p] = wall ? pw[p] : pin;
            }
#pragma unroll
            for (int p = 0; p < 5; ++p) {
                acc[p][0] += phi[p] * sx;
                acc[p][1] += phi[p] * sy;
                acc[p][2] += phi[p] * sz;
            }
        }
    const R iv = ((const R *)g.inv_vol)[c];
    R *pr = (R *)g.prim, *gr = (R *)g.grad;
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        pr[p * d.cells + c] = P[p];
#pragma unroll
        for (int a = 0; a < 3; ++a) gr[(p * 3 + a) * d.cells + c] = acc[p][a] * iv;
    }
}

// Primitives and gradients of cell c from the scratch buffers.
template <typename R>
__device__ inline void c3_load(const Domain &d, const Curv3Geo &g, int64_t c, R (&P)[5], R (&G)[5][3]) {
    const R *pr = (const R *)g.prim, *gr = (const R *)g.grad;
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        P[p] = pr[p * d.cells + c];
#pragma unroll
        for (int a = 0; a < 3; ++a) G[p][a] = gr[(p * 3 + a) * d.cells + c];
    }
}

// The loaded primitives and gradients of a cell as its image rotated by
// (cr, sr) about z.
template <typename R>
__device__ inline void c3_rotate(R cr, R sr, R (&P)[5], R (&G)[5][3]) {
    if (sr == (R)0 && cr == (R)1) return;
    R u[3] = {P[1], P[2], P[3]};
    rot_z(cr, sr, u);
    P[1] = u[0];
    P[2] = u[1];
    P[3] = u[2];
    R g0[3] = {G[0][0], G[0][1], G[0][2]}, g4[3] = {G[4][0], G[4][1], G[4][2]};
    rot_z(cr, sr, g0);
    rot_z(cr, sr, g4);
    // velocity gradient M[a][b] = d_b u_a -> R M R^T: rotate rows, then columns
    R M[3][3];
#pragma unroll
    for (int b = 0; b < 3; ++b) {
        R col[3] = {G[1][b], G[2][b], G[3][b]};
        rot_z(cr, sr, col);
#pragma unroll
        for (int a = 0; a < 3; ++a) M[a][b] = col[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        R row[3] = {M[a][0], M[a][1], M[a][2]};
        rot_z(cr, sr, row);
#pragma unroll
        for (int b = 0; b < 3; ++b) G[1 + a][b] = row[b];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        G[0][a] = g0[a];
        G[4][a] = g4[a];
    }
}

template <typename R, bool DEV, bool TL>
__global__ void __launch_bounds__(kC3Threads) k_c3_flux(Domain d, Curv3Geo g, const R *__restrict__ U) {
    // 32-bit index arithmetic: at most 2^28 cells, so fewer than 2^31 faces
    const int t = (int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x;
    if (t >= (int)g.nfaces) return;
    const int sf0 = (int)g.sf[0], sf1 = (int)g.sf[1];
    const int a = t < sf0 ? 0 : (t < sf0 + sf1 ? 1 : 2);  // face family: normal index direction
    const int f = t - (a == 0 ? 0 : (a == 1 ? sf0 : sf0 + sf1));
    const int nx = d.n[0] + (a == 0), ny = d.n[1] + (a == 1);
    const int fr = f / nx;
    const int qx = f % nx, qy = fr % ny, qz = fr / ny;
    const int qa = a == 0 ? qx : (a == 1 ? qy : qz);
    const R *rec = (const R *)pick3(a, g.f) + f;
    const int64_t st = pick3(a, g.sf);
    const int na = pick3(a, d.n);
    const bool per = pick3(a, d.periodic) != 0;
    const bool interior = per || (qa > 0 && qa < na);
    const bool low = qa == 0;  // wall faces: on the low side the fluid cell is the high one
    // The low and high cells (images rotated by -alpha at face 0 and +alpha
    // at face n of a periodic axis); at a wall both are clamped to the fluid
    // cell.  Every load below is issued for every face, before any branch,
    // so one round trip serves the face; the interior and the wall flux are
    // both evaluated and the face's own one kept.
    int la = qa - 1, ha = qa;  // index of the low and the high cell along a
    R cl = (R)1, sl = (R)0, ch = (R)1, sh = (R)0;
    const R rca = (R)pick3(a, g.rc), rsa = (R)pick3(a, g.rs);
    if (la < 0) {
        la = per ? la + na : 0;
        cl = per ? rca : (R)1;
        sl = per ? -rsa : (R)0;
    }
    if (ha >= na) {
        ha = per ? ha - na : na - 1;
        ch = per ? rca : (R)1;
        sh = per ? rsa : (R)0;
    }
    const int64_t clo = c3_cell(d, a == 0 ? la : qx, a == 1 ? la : qy, a == 2 ? la : qz);
    const int64_t chi = c3_cell(d, a == 0 ? ha : qx, a == 1 ? ha : qy, a == 2 ? ha : qz);
    R PA[5], PB[5], GA[5][3], GB[5][3];
    c3_load<R>(d, g, clo, PA, GA);
    c3_load<R>(d, g, chi, PB, GB);
    const int64_t N = d.fstride;
    const int64_t cw = low ? chi : clo;  // the fluid cell of a wall face
    const R rP = U[cw], eP = U[4 * N + cw];
    const R mw[3] = {U[N + cw], U[2 * N + cw], U[3 * N + cw]};
    R e[3][3];
    e[0][0] = rec[kC3Nx * st];
    e[0][1] = rec[kC3Ny * st];
    e[0][2] = rec[kC3Nz * st];
    e[1][0] = rec[kC3T1x * st];
    e[1][1] = rec[kC3T1y * st];
    e[1][2] = rec[kC3T1z * st];
    const R dS = rec[kC3DS * st], dL = rec[kC3DL * st], dR = rec[kC3DR * st];
    const R tl1 = rec[kC3TL1 * st], tl2 = rec[kC3TL2 * st], tr1 = rec[kC3TR1 * st], tr2 = rec[kC3TR2 * st];
    e[2][0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];  // t2 = n x t1
    e[2][1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
    e[2][2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
    const Phys<R> &ph = make_phys<R>(d);
    R F[5];
    {
        c3_rotate<R>(cl, sl, PA, GA);
        c3_rotate<R>(ch, sh, PB, GB);
        Side<R, 3> A, B;
        side_in_frame3<R>(PA, GA, e, tl1, tl2, A);
        side_in_frame3<R>(PB, GB, e, tr1, tr2, B);
        const R up[3] = {c3_up<R>(g, 0), c3_up<R>(g, 1), c3_up<R>(g, 2)};
        frame_flux3<R, DEV, TL>(A, B, dL, dR, e, up, d.force_pred != 0, dS, ph, F);
    }
    {
        const int side = 2 * a + (low ? 0 : 1);
        R ml[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) ml[k] = mw[0] * e[k][0] + mw[1] * e[k][1] + mw[2] * e[k][2];
        R G[5], Fw[5];
        const R Tw = sizeof(R) == 4 ? (R)pick6(side, d.Twf) : (R)pick6(side, d.Tw);
        wall_flux<R, 3, DEV>(rP, ml, eP, low ? (R)-1 : (R)1, low ? dR : dL, pick6(side, d.kind) == kIsothermal, Tw,
                             ph, G);
        Fw[0] = G[0] * dS;
#pragma unroll
        for (int b = 0; b < 3; ++b) Fw[1 + b] = (G[1] * e[0][b] + G[2] * e[1][b] + G[3] * e[2][b]) * dS;
        Fw[4] = G[4] * dS;
#pragma unroll
        for (int p = 0; p < 5; ++p) F[p] = interior ? F[p] : Fw[p];
    }
    R *out = (R *)g.flux;
#pragma unroll
    for (int p = 0; p < 5; ++p) out[p * g.nfaces + t] = F[p];
}

// Divergence, buoyancy along `up`, forward Euler and (FP32) stochastic
// rounding of cell c, stored to Uout; on residual steps also the cell's
// Eq. 65 terms and divergence flag in acc.  P holds the cell's primitives at
// the old time level (velocities only needed when RES), old its stored
// state, div the sum over the axes of low-face minus high-face area-weighted
// fluxes, iv = 1/dV.
template <typename R, bool DEV, bool RES>
__device__ __forceinline__ void c3_update_cell(const Domain &d, const Curv3Geo &g, int c, const R (&P)[5],
                                               const R (&old)[5], const R (&div)[5], R iv, uint32_t key,
                                               R *__restrict__ Uout, double (&acc)[kPartials]) {
    const int64_t N = d.fstride;
    const Phys<R> &ph = make_phys<R>(d);
    const R rP = P[0], TP = P[4];
    const R rhoP = DEV ? (R)1 + rP : rP;
    const R dtR = ph.dt;
    const R dt_dV = dtR * iv;
    const R Fb = dtR * ph.bg * rhoP * (TP - ph.Tref_s);
    R Un[5];
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        const R src = (p >= 1 && p <= 3) ? Fb * c3_up<R>(g, p - 1) : (R)0;
        const R inc = dt_dV * div[p] + src;
        if (sizeof(R) == 4 && d.sround) Un[p] = sr_add(old[p], inc, sr_hash((uint32_t)c, key * 5u + p));
        else Un[p] = old[p] + inc;
        Uout[p * N + c] = Un[p];
    }
    if (RES) {
        const double rn = (double)Un[0];
        const double rhon = DEV ? 1.0 + rn : rn;
        double an = 0.0, ao = 0.0;
        for (int a = 0; a < 3; ++a) {
            const double vn = (double)Un[1 + a] / rhon, vo = (double)P[1 + a];
            an += vn * vn;
            ao += vo * vo;
        }
        an = sqrt(an);
        ao = sqrt(ao);
        const double Tn = (double)Un[4] / rhon + (DEV ? kT0 : 0.0), To = (double)TP + (DEV ? kT0 : 0.0);
        acc[0] = fabs(an - ao);
        acc[1] = an;
        acc[2] = fabs(Tn - To);
        acc[3] = Tn;
        acc[4] = (an * an < d.guard_u2) && (Tn == Tn) && (fabs(Tn) < 1e30) ? 0.0 : 1.0;
    }
}

template <typename R, bool DEV, bool RES>
__global__ void __launch_bounds__(kC3Threads) k_c3_update(Domain d, Curv3Geo g, const R *__restrict__ Uin,
                                                   R *__restrict__ Uout, double *__restrict__ parts,
                                                   const uint32_t *__restrict__ ctr_in, uint32_t *__restrict__ ctr_out) {
    __shared__ double sred[kPartials * 4];
    const uint32_t key = *ctr_in;
    const int c = (int)blockIdx.x * (int)blockDim.x + (int)threadIdx.x;  // at most 2^28 cells
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (c < (int)d.cells) {
        const int i = c % d.n[0], jk = c / d.n[0], j = jk % d.n[1], k = jk / d.n[1];
        const int64_t N = d.fstride;
        const R *fl = (const R *)g.flux;
        R old[5];  // loaded with the fluxes, ahead of the per-field rounding
#pragma unroll
        for (int p = 0; p < 5; ++p) old[p] = Uin[p * N + c];
        R div[5] = {0, 0, 0, 0, 0};
        int64_t base = 0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            int hq[3] = {i, j, k};
            hq[a] += 1;
            const int64_t flo = base + c3_face(d, a, i, j, k), fhi = base + c3_face(d, a, hq[0], hq[1], hq[2]);
#pragma unroll
            for (int p = 0; p < 5; ++p) div[p] += fl[p * g.nfaces + flo] - fl[p * g.nfaces + fhi];
            base += g.sf[a];
        }
        const R *pr = (const R *)g.prim;
        R P[5] = {pr[c], (R)0, (R)0, (R)0, pr[4 * d.cells + c]};
        if (RES)
            for (int a = 1; a <= 3; ++a) P[a] = pr[a * d.cells + c];
        c3_update_cell<R, DEV, RES>(d, g, c, P, old, div, ((const R *)g.inv_vol)[c], key, Uout, acc);
    }
    if (RES) {
        block_sums<kPartials>(acc, sred);
        if (threadIdx.x == 0)
            for (int m = 0; m < kPartials; ++m) parts[(int64_t)blockIdx.x * kPartials + m] = acc[m];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) *ctr_out = key + 1u;
}

// Fused step for a single-layer wedge: axis j periodic with one cell (its
// images are the cell itself, rotated by -+alpha about z) and walls on axes
// i and k, the setting of Sec. 4.5.  A TX x TZ tile with a 2-cell halo in i
// and k then holds every value the step reads, and one launch does the work
// of the three kernels above, with their arithmetic:
//   load      every global read of the step at once: the state of the box,
//             the face records of the gradient and face phases, 1/dV;
//             primitives of the box and conserved state of the tile to LDS;
//   gradient  Eq. 55 for the tile plus a 1-cell halo (as k_c3_grad);
//   faces     the i- and k-faces of the tile and both j-faces of each of its
//             cells, each face once (as k_c3_flux);
//   update    divergence, source, forward Euler (as k_c3_update).
template <int TX, int TZ>
constexpr int c3_layer_threads() {
    constexpr int nb = (TX + 4) * (TZ + 4);
    constexpr int nf = (TX + 1) * TZ + TX * (TZ + 1) + 2 * TX * TZ;
    return ((nb > nf ? nb : nf) + 63) / 64 * 64;
}

constexpr int kC3LayerTX = 16, kC3LayerTZ = 4;  // tile of the fused kernel

template <typename R, bool DEV, bool TL, bool RES, int TX, int TZ>
__global__ void __launch_bounds__((c3_layer_threads<TX, TZ>()))
    k_c3_layer(Domain d, Curv3Geo g, const R *__restrict__ Uin, R *__restrict__ Uout, double *__restrict__ parts,
               const uint32_t *__restrict__ ctr_in, uint32_t *__restrict__ ctr_out) {
    constexpr int NT = c3_layer_threads<TX, TZ>();
    constexpr int BX = TX + 4, NB = (TX + 4) * (TZ + 4);  // box: tile + 2-cell halo in i and k
    constexpr int GX = TX + 2, NG = (TX + 2) * (TZ + 2);  // gradients: tile + 1-cell halo
    constexpr int NFI = (TX + 1) * TZ, NFK = TX * (TZ + 1), NF = NFI + NFK + 2 * TX * TZ;
    constexpr int NC = TX * TZ;
    static_assert(NB <= NT && NF <= NT && NG <= NT && NC <= NT, "every phase is one pass of the block");
    __shared__ R sp[5 * NB];   // primitives of the box
    __shared__ R su[5 * NC];   // stored state of the tile
    __shared__ R sg[15 * NG];  // gradients, [p * 3 + axis]
    __shared__ R sf[5 * NF];   // area-weighted fluxes: i-faces, k-faces, then (j = 0, j = 1) per cell
    __shared__ double sred[kPartials * (NT / 64)];
    const uint32_t key = *ctr_in;
    const int n0 = d.n[0], n2 = d.n[2];
    const int ntx = (n0 + TX - 1) / TX;
    const int i0 = ((int)blockIdx.x % ntx) * TX, k0 = ((int)blockIdx.x / ntx) * TZ;
    const int tid = threadIdx.x;
    const int64_t N = d.fstride;
    const R *__restrict__ ivp = (const R *)g.inv_vol;

    // ---- load: every global read of the step, issued before the first use
    const int bi = tid % BX, bk = tid / BX;  // box cell
    const int bgi = i0 - 2 + bi, bgk = k0 - 2 + bk;
    const bool lb = tid < NB && bgi >= 0 && bgi < n0 && bgk >= 0 && bgk < n2;  // beyond a wall: never read
    R u[5];
    if (lb) {
        const int c = bgk * n0 + bgi;
#pragma unroll
        for (int p = 0; p < 5; ++p) u[p] = Uin[p * N + c];
    }
    const int gi = tid % GX, gk = tid / GX;  // gradient cell
    const int ggi = i0 - 1 + gi, ggk = k0 - 1 + gk;
    const bool lg = tid < NG && ggi >= 0 && ggi < n0 && ggk >= 0 && ggk < n2;
    R gr[6][5];  // its six faces (a, hi): n, dS, wL
    R giv = (R)0;
    if (lg) {
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int hi = 0; hi < 2; ++hi) {
                int fq[3] = {ggi, 0, ggk};
                fq[a] += hi;
                const int64_t st = g.sf[a];
                const R *rec = (const R *)g.f[a] + c3_face(d, a, fq[0], fq[1], fq[2]);
                gr[2 * a + hi][0] = rec[kC3Nx * st];
                gr[2 * a + hi][1] = rec[kC3Ny * st];
                gr[2 * a + hi][2] = rec[kC3Nz * st];
                gr[2 * a + hi][3] = rec[kC3DS * st];
                gr[2 * a + hi][4] = rec[kC3WL * st];
            }
        giv = ivp[ggk * n0 + ggi];
    }
    // face of this thread: family fa (0: i, 1: j, 2: k), tile position, j side
    int fa, fx, fz, fj = 0;
    if (tid < NFI) {
        fa = 0;
        fx = tid % (TX + 1);
        fz = tid / (TX + 1);
    } else if (tid < NFI + NFK) {
        fa = 2;
        fx = (tid - NFI) % TX;
        fz = (tid - NFI) / TX;
    } else {
        const int q = tid - NFI - NFK;
        fa = 1;
        fx = (q >> 1) % TX;
        fz = (q >> 1) / TX;
        fj = q & 1;
    }
    const int fgi = i0 + fx, fgk = k0 + fz;
    const bool lf = tid < NF && (fa == 0 ? (fgi <= n0 && fgk < n2) : (fa == 2 ? (fgi < n0 && fgk <= n2) : (fgi < n0 && fgk < n2)));
    R fr[13];  // n, t1, dS, dL, tL1, tL2, dR, tR1, tR2
    if (lf) {
        const int fq1 = fa == 1 ? fj : 0;
        const R *rec = (const R *)pick3(fa, g.f) + c3_face(d, fa, fgi, fq1, fgk);
        const int64_t st = pick3(fa, g.sf);
#pragma unroll
        for (int m = 0; m < 13; ++m) fr[m] = rec[(kC3Nx + m) * st];
    }
    const int ux = tid % TX, uz = tid / TX;  // update cell
    const bool lu = tid < NC && i0 + ux < n0 && k0 + uz < n2;
    const R uiv = lu ? ivp[(k0 + uz) * n0 + i0 + ux] : (R)0;
    if (lb) {
        const R inv = recip<R>(DEV ? (R)1 + u[0] : u[0]);
        sp[tid] = u[0];
#pragma unroll
        for (int p = 1; p < 5; ++p) sp[p * NB + tid] = u[p] * inv;
        const int ti = bi - 2, tk = bk - 2;
        if (ti >= 0 && ti < TX && tk >= 0 && tk < TZ)
#pragma unroll
            for (int p = 0; p < 5; ++p) su[p * NC + tk * TX + ti] = u[p];
    }
    __syncthreads();

    // ---- gradients (k_c3_grad with neighbours from LDS)
    if (lg) {
        const int b = (gk + 1) * BX + gi + 1;  // this cell in the box
        R P[5];
#pragma unroll
        for (int p = 0; p < 5; ++p) P[p] = sp[p * NB + b];
        R acc[5][3];
#pragma unroll
        for (int p = 0; p < 5; ++p) acc[p][0] = acc[p][1] = acc[p][2] = (R)0;
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int hi = 0; hi < 2; ++hi) {
                const R *r5 = gr[2 * a + hi];
                const R so = hi ? (R)1 : (R)-1;
                const R sx = so * r5[0] * r5[3], sy = so * r5[1] * r5[3], sz = so * r5[2] * r5[3];
                // neighbour: along j the cell itself rotated; along i, k the box cell (a wall reads the cell)
                bool wall = false;
                int nb = b;
                R cr = (R)1, sr = (R)0;
                if (a == 1) {
                    cr = (R)g.rc[1];
                    sr = (R)(hi ? g.rs[1] : -g.rs[1]);
                } else if (a == 0) {
                    const int ni = ggi + (hi ? 1 : -1);
                    wall = ni < 0 || ni >= n0;
                    nb = wall ? b : b + (hi ? 1 : -1);
                } else {
                    const int nk = ggk + (hi ? 1 : -1);
                    wall = nk < 0 || nk >= n2;
                    nb = wall ? b : b + (hi ? BX : -BX);
                }
                R Q[5];
#pragma unroll
                for (int p = 0; p < 5; ++p) Q[p] = sp[p * NB + nb];
                R uq[3] = {Q[1], Q[2], Q[3]};
                rot_z<R>(cr, sr, uq);
                Q[1] = uq[0];
                Q[2] = uq[1];
                Q[3] = uq[2];
                const R wL = r5[4];
                const int side = 2 * a + hi;
                const R Tw = d.kind[side] == kIsothermal ? wall_T<R>(d, side) : P[4];
                const R pw[5] = {P[0], (R)0, (R)0, (R)0, Tw};
                R phi[5];
#pragma unroll
                for (int p = 0; p < 5; ++p) {
                    const R pin = hi ? wL * P[p] + ((R)1 - wL) * Q[p] : wL * Q[p] + ((R)1 - wL) * P[p];
                    phi[p] = wall ? pw[p] : pin;
                }
#pragma unroll
                for (int p = 0; p < 5; ++p) {
                    acc[p][0] += phi[p] * sx;
                    acc[p][1] += phi[p] * sy;
                    acc[p][2] += phi[p] * sz;
                }
            }
#pragma unroll
        for (int p = 0; p < 5; ++p)
#pragma unroll
            for (int a = 0; a < 3; ++a) sg[(p * 3 + a) * NG + tid] = acc[p][a] * giv;
    }
    __syncthreads();

    // ---- faces (k_c3_flux with cells from LDS)
    if (lf) {
        // low and high cells (global i, k), clamped to the fluid cell at a wall;
        // the j-faces join the cell and its image rotated by -alpha (j = 0) or +alpha (j = 1)
        int li = fgi, lk = fgk, hi_ = fgi, hk = fgk;
        R cl = (R)1, sl = (R)0, ch = (R)1, sh = (R)0;
        bool interior = true, low = false;
        if (fa == 0) {
            interior = fgi > 0 && fgi < n0;
            low = fgi == 0;
            li = fgi > 0 ? fgi - 1 : 0;
            hi_ = fgi < n0 ? fgi : n0 - 1;
        } else if (fa == 2) {
            interior = fgk > 0 && fgk < n2;
            low = fgk == 0;
            lk = fgk > 0 ? fgk - 1 : 0;
            hk = fgk < n2 ? fgk : n2 - 1;
        } else {
            low = fj == 0;
            const R rc = (R)g.rc[1], rs = (R)g.rs[1];
            cl = fj == 0 ? rc : (R)1;
            sl = fj == 0 ? -rs : (R)0;
            ch = fj == 0 ? (R)1 : rc;
            sh = fj == 0 ? (R)0 : rs;
        }
        const int bl = (lk - k0 + 2) * BX + li - i0 + 2, bh = (hk - k0 + 2) * BX + hi_ - i0 + 2;
        const int gl = (lk - k0 + 1) * GX + li - i0 + 1, gh = (hk - k0 + 1) * GX + hi_ - i0 + 1;
        R PA[5], PB[5], GA[5][3], GB[5][3];
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            PA[p] = sp[p * NB + bl];
            PB[p] = sp[p * NB + bh];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                GA[p][a] = sg[(p * 3 + a) * NG + gl];
                GB[p][a] = sg[(p * 3 + a) * NG + gh];
            }
        }
        // the fluid cell of a wall face is a cell of this tile; other faces
        // read their own cell's slot, unused
        const int wi = low ? hi_ : li, wk = low ? hk : lk;
        const int wt = interior ? (fa == 1 ? fz * TX + fx : 0) : (wk - k0) * TX + (wi - i0);
        const R rP = su[wt], eP = su[4 * NC + wt];
        const R mw[3] = {su[NC + wt], su[2 * NC + wt], su[3 * NC + wt]};
        R e[3][3];
        e[0][0] = fr[kC3Nx - kC3Nx];
        e[0][1] = fr[kC3Ny - kC3Nx];
        e[0][2] = fr[kC3Nz - kC3Nx];
        e[1][0] = fr[kC3T1x - kC3Nx];
        e[1][1] = fr[kC3T1y - kC3Nx];
        e[1][2] = fr[kC3T1z - kC3Nx];
        const R dS = fr[kC3DS - kC3Nx], dL = fr[kC3DL - kC3Nx], dR = fr[kC3DR - kC3Nx];
        const R tl1 = fr[kC3TL1 - kC3Nx], tl2 = fr[kC3TL2 - kC3Nx], tr1 = fr[kC3TR1 - kC3Nx];
        const R tr2 = fr[kC3TR2 - kC3Nx];
        e[2][0] = e[0][1] * e[1][2] - e[0][2] * e[1][1];  // t2 = n x t1
        e[2][1] = e[0][2] * e[1][0] - e[0][0] * e[1][2];
        e[2][2] = e[0][0] * e[1][1] - e[0][1] * e[1][0];
        const Phys<R> &ph = make_phys<R>(d);
        R F[5];
        {
            c3_rotate<R>(cl, sl, PA, GA);
            c3_rotate<R>(ch, sh, PB, GB);
            Side<R, 3> A, B;
            side_in_frame3<R>(PA, GA, e, tl1, tl2, A);
            side_in_frame3<R>(PB, GB, e, tr1, tr2, B);
            const R up[3] = {c3_up<R>(g, 0), c3_up<R>(g, 1), c3_up<R>(g, 2)};
            frame_flux3<R, DEV, TL>(A, B, dL, dR, e, up, d.force_pred != 0, dS, ph, F);
        }
        {
            const int side = 2 * fa + (low ? 0 : 1);
            R ml[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) ml[k] = mw[0] * e[k][0] + mw[1] * e[k][1] + mw[2] * e[k][2];
            R G[5], Fw[5];
            const R Tw = sizeof(R) == 4 ? (R)pick6(side, d.Twf) : (R)pick6(side, d.Tw);
            wall_flux<R, 3, DEV>(rP, ml, eP, low ? (R)-1 : (R)1, low ? dR : dL, pick6(side, d.kind) == kIsothermal,
                                 Tw, ph, G);
            Fw[0] = G[0] * dS;
#pragma unroll
            for (int b = 0; b < 3; ++b) Fw[1 + b] = (G[1] * e[0][b] + G[2] * e[1][b] + G[3] * e[2][b]) * dS;
            Fw[4] = G[4] * dS;
#pragma unroll
            for (int p = 0; p < 5; ++p) F[p] = interior ? F[p] : Fw[p];
        }
#pragma unroll
        for (int p = 0; p < 5; ++p) sf[p * NF + tid] = F[p];
    }
    __syncthreads();

    // ---- update (k_c3_update with fluxes from LDS)
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (lu) {
        const int c = (k0 + uz) * n0 + i0 + ux;
        const int b = (uz + 2) * BX + ux + 2;
        R P[5], old[5], div[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int p = 0; p < 5; ++p) {
            P[p] = sp[p * NB + b];
            old[p] = su[p * NC + tid];
        }
        const int fi = uz * (TX + 1) + ux, fk = NFI + uz * TX + ux, fjl = NFI + NFK + 2 * tid;
#pragma unroll
        for (int p = 0; p < 5; ++p) div[p] += sf[p * NF + fi] - sf[p * NF + fi + 1];
#pragma unroll
        for (int p = 0; p < 5; ++p) div[p] += sf[p * NF + fjl] - sf[p * NF + fjl + 1];
#pragma unroll
        for (int p = 0; p < 5; ++p) div[p] += sf[p * NF + fk] - sf[p * NF + fk + TX];
        c3_update_cell<R, DEV, RES>(d, g, c, P, old, div, uiv, key, Uout, acc);
    }
    if (RES) {
        block_sums<kPartials>(acc, sred);
        if (tid == 0)
            for (int m = 0; m < kPartials; ++m) parts[(int64_t)blockIdx.x * kPartials + m] = acc[m];
    }
    if (blockIdx.x == 0 && tid == 0) *ctr_out = key + 1u;
}

// Wall heat of one side: {sum (T_w - T_P)/d dS, sum dS} (single block, FP64
// records).
template <typename R, bool DEV>
__global__ void __launch_bounds__(256) k_c3_wall_heat(Domain d, const double *__restrict__ rec64, int64_t st,
                                                      const R *__restrict__ U, int side, double Tw_abs,
                                                      double *__restrict__ out) {
    __shared__ double sred[2 * 4];
    const int a = side / 2, hi = side & 1;
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    const int n1 = d.n[b1], n2 = d.n[b2];
    const int64_t N = d.fstride;
    double acc[2] = {0.0, 0.0};
    for (int64_t m = threadIdx.x; m < (int64_t)n1 * n2; m += blockDim.x) {
        int q[3];
        q[a] = hi ? d.n[a] : 0;
        q[b1] = (int)(m % n1);
        q[b2] = (int)(m / n1);
        const double *r = rec64 + c3_face(d, a, q[0], q[1], q[2]);
        int w[3] = {q[0], q[1], q[2]};
        if (hi) w[a] -= 1;
        const int64_t c = c3_cell(d, w[0], w[1], w[2]);
        const double dS = r[kC3DS * st], dist = hi ? r[kC3DL * st] : r[kC3DR * st];
        const double rr = (double)U[c];
        const double rho = DEV ? 1.0 + rr : rr;
        const double TP = (double)U[4 * N + c] / rho + (DEV ? kT0 : 0.0);
        acc[0] += (Tw_abs - TP) / dist * dS;
        acc[1] += dS;
    }
    block_sums<2>(acc, sred);
    if (threadIdx.x == 0) {
        out[0] = acc[0];
        out[1] = acc[1];
    }
}

}  // namespace rtlbfs
