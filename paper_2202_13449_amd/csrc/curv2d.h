// curv2d.h -- the RTLBFS time step on a 2D body-fitted (structured
// curvilinear) quadrilateral mesh, as run by Secs. 4.3 and 4.5 on O-type
// meshes.  Each face has its own unit normal n and area dS; the D2Q9 lattice
// of Fig. 1 sits on the face aligned with (n, t), t = n rotated by +90 deg.
//
// One launch advances a TX x TY tile of cells by one step, in four phases
// separated by workgroup barriers, all through LDS (one thread per face of
// the tile, so each phase is one pass of the block; the faces in the hybrid
// layout of the Cartesian step, whole wavefronts of i-faces and of j-faces
// around one wavefront holding both tails):
//   load       conserved state of the tile plus a 2-cell halo, primitives;
//   gradients  Eq. 55 for the tile plus a 1-cell halo: (1/dV) sum over the
//              cell's four faces of phi_S n_out dS, with Eq. 56 face values on
//              interior faces, wall values on walls and the mean of cell and
//              ghost on far-field faces;
//   faces      every face of the tile once: interior faces by the lattice
//              predictor-corrector in the face frame (the Eq. 29 node values
//              of a side whose centre lies off the face normal are shifted by
//              the tangential gradient times that offset, which is exact for
//              the linear reconstruction), walls by the one-sided closure,
//              far-field faces as interior faces against a mirrored ghost
//              cell; area-weighted fluxes along +n in global components;
//   update     divergence, Boussinesq source along the given upward unit
//              vector, forward Euler (Eqs. 41-43, 64); FP64 partial sums of
//              Eq. 65 on residual steps.
//
// Face geometry is precomputed on the host in FP64 and stored in the kernel
// precision as kCf* records (SoA): i-faces (i, j), i = 0..ni, at index
// j*(ni+1) + i, between cells (i-1, j) and (i, j); j-faces (i, j),
// j = 0..nj, at index j*ni + i, between (i, j-1) and (i, j).  On a periodic
// axis face n equals face 0.
#pragma once

#include "rtlbfs_device.h"
#include "step2d.h"

namespace rtlbfs {

// n_x, n_y (unit normal from the low to the high cell), dS, then for the low
// cell L and high cell R: dL = (x_S - x_L).n, tL = (x_S - x_L).t,
// dR = (x_R - x_S).n, tR = (x_S - x_R).t, and the Eq. 56 weight wL of the
// low cell's value.  A boundary face stores the interior cell's normal
// distance in both dL and dR (the far-field ghost is its mirror image) and
// its tangential offset in both tL and tR.
enum : int { kCfNx = 0, kCfNy, kCfDS, kCfDL, kCfTL, kCfDR, kCfTR, kCfWL, kCurvFaceFields };
enum : int { kFarfield = 3 };

// Body-fitted geometry and far-field data as the kernels see them.
struct CurvGeo {
    const void *fi, *fj;       // face records in the kernel precision, kCurvFaceFields fields each
    const void *inv_area;      // 1 / dV per cell, kernel precision
    int64_t sfi, sfj;          // field strides of the records
    double up[2];              // unit vector against gravity (0 if no buoyancy)
    double uinf[2], Tinf_s;    // far-field velocity, temperature (storage convention)
    float upf[2], uinff[2], Tinff_s;
};

template <typename R>
__device__ inline R cg_up(const CurvGeo &g, int a) {
    if constexpr (sizeof(R) == 4) return g.upf[a];
    else return g.up[a];
}
template <typename R>
__device__ inline R cg_uinf(const CurvGeo &g, int a) {
    if constexpr (sizeof(R) == 4) return g.uinff[a];
    else return g.uinf[a];
}
template <typename R>
__device__ inline R cg_Tinf(const CurvGeo &g) {
    if constexpr (sizeof(R) == 4) return g.Tinff_s;
    else return g.Tinf_s;
}

// One side of a face in the face frame (n, t), t = (-n_y, n_x): primitives
// P = (r, u_x, u_y, T) and their gradients G[p][axis] of a cell, rotated, and
// shifted by the tangential gradient times tau = (x_S - x_C).t (the Eq. 29
// values of a centre that lies off the face normal).
template <typename R>
__host__ __device__ inline void side_in_frame(const R (&P)[4], const R (&G)[4][2], R nx, R ny, R tau,
                                              Side<R, 2> &S) {
    const R tx = -ny, ty = nx;
    const R e[2][2] = {{nx, ny}, {tx, ty}};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        S.g[k][0] = G[0][0] * e[k][0] + G[0][1] * e[k][1];
        S.g[k][3] = G[3][0] * e[k][0] + G[3][1] * e[k][1];
        const R gux = G[1][0] * e[k][0] + G[1][1] * e[k][1];  // d_k u_x, d_k u_y
        const R guy = G[2][0] * e[k][0] + G[2][1] * e[k][1];
#pragma unroll
        for (int q = 0; q < 2; ++q) S.g[k][1 + q] = e[q][0] * gux + e[q][1] * guy;  // d_k u_q = e_q . (grad u) e_k
    }
    S.v[0] = P[0] + S.g[1][0] * tau;
    S.v[1] = P[1] * nx + P[2] * ny + S.g[1][1] * tau;
    S.v[2] = P[1] * tx + P[2] * ty + S.g[1][2] * tau;
    S.v[3] = P[3] + S.g[1][3] * tau;
}

// Interior-face flux (RTLBFS, or TLBFS when TL) along +n times the face area,
// momentum back in global components; the buoyancy direction `up` enters
// the predictor in the face frame when fp.
template <typename R, bool DEV, bool TL>
__host__ __device__ inline void frame_flux(const Side<R, 2> &A, const Side<R, 2> &B, R dL, R dR, R nx, R ny, R upx,
                                           R upy, bool fp, R dS, const Phys<R> &ph, R (&Fg)[4]) {
    const R tx = -ny, ty = nx;
    const R fdir[2] = {fp ? upx * nx + upy * ny : (R)0, fp ? upx * tx + upy * ty : (R)0};
    R G[4];
    if constexpr (TL) face_flux_tlbfs<R, 2, DEV, true>(A, B, dL, dR, fdir, ph, G);
    else face_flux<R, 2, DEV, true>(A, B, dL, dR, fdir, ph, G);
    Fg[0] = G[0] * dS;
    Fg[1] = (G[1] * nx + G[2] * tx) * dS;
    Fg[2] = (G[1] * ny + G[2] * ty) * dS;
    Fg[3] = G[3] * dS;
}

template <int TX, int TY>
constexpr int curv_threads() {
    return (region_faces<TX, TY>() + 63) / 64 * 64;
}

// Ghost primitives (r, u_x, u_y, T in storage convention) of a far-field
// face: the free stream (rho = 1, u_inf, T_inf).
template <typename R, bool DEV>
__device__ inline void ghost_prims(const CurvGeo &g, R (&G)[4]) {
    G[0] = DEV ? (R)0 : (R)1;
    G[1] = cg_uinf<R>(g, 0);
    G[2] = cg_uinf<R>(g, 1);
    G[3] = cg_Tinf<R>(g);
}

template <typename R, bool DEV, bool TL, int TX, int TY, bool RES>
__device__ __forceinline__ void tile_step_curv(const Domain &d, const CurvGeo &g, int i0, int j0,
                                               const R *__restrict__ Uin, R *__restrict__ Uout,
                                               double *__restrict__ part, uint32_t step_key) {
    constexpr int PX = TX + 4, PY = TY + 4, PF = PX * PY;  // primitives with a 2-cell halo
    constexpr int GX = TX + 2, GY = TY + 2, GF = GX * GY;  // gradients with a 1-cell halo
    constexpr int NFX = (TX + 1) * TY;
    constexpr int NF = region_faces<TX, TY>();
    constexpr int NT = curv_threads<TX, TY>();
    constexpr int SCF = TX * TY;
    static_assert(PF <= NT && GF <= NT && NF <= NT, "every phase is one pass of the block");
    __shared__ R sp[4 * PF];
    __shared__ R sg[4 * 2 * GF];  // d/dx, d/dy of (r, u_x, u_y, T)
    __shared__ R sf[4 * NF];
    __shared__ R sc[4 * SCF];
    __shared__ double sred[kPartials * 16];
    __shared__ R swT[4];
    __shared__ int swKind[4];

    const int nx = d.n[0], ny = d.n[1];
    const int64_t N = d.fstride;
    const bool px = d.periodic[0], py = d.periodic[1];
    // a periodic axis at least as long as the tile plus both 2-cell halos wraps by selects
    const bool nearx = nx >= TX + 4, neary = ny >= TY + 4;
    const Phys<R> &ph = make_phys<R>(d);
    const R *__restrict__ fi = (const R *)g.fi;
    const R *__restrict__ fj = (const R *)g.fj;
    const R *__restrict__ iA = (const R *)g.inv_area;
    const int tid = threadIdx.x;
    auto SP = [&](int p, int y, int x) -> R { return sp[p * PF + y * PX + x]; };
    auto FI = [&](int k, int i, int j) -> R { return fi[k * g.sfi + (int64_t)j * (nx + 1) + i]; };
    auto FJ = [&](int k, int i, int j) -> R { return fj[k * g.sfj + (int64_t)j * nx + i]; };

    // ---- load
    if (tid < PF) {
        const int li = tid % PX, lj = tid / PX;
        int gi = i0 - 2 + li, gj = j0 - 2 + lj;
        if (px) gi = wrap_axis(gi, nx, nearx);
        if (py) gj = wrap_axis(gj, ny, neary);
        if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) {
            const int64_t c = (int64_t)gj * nx + gi;
            const R r = Uin[c], mx = Uin[N + c], my = Uin[2 * N + c], e = Uin[3 * N + c];
            const R inv_rho = recip<R>(DEV ? (R)1 + r : r);
            sp[0 * PF + tid] = r;
            sp[1 * PF + tid] = mx * inv_rho;
            sp[2 * PF + tid] = my * inv_rho;
            sp[3 * PF + tid] = e * inv_rho;
            const int ti = li - 2, tj = lj - 2;
            if (ti >= 0 && ti < TX && tj >= 0 && tj < TY) {
                const int o = tj * TX + ti;
                sc[0 * SCF + o] = r;
                sc[1 * SCF + o] = mx;
                sc[2 * SCF + o] = my;
                sc[3 * SCF + o] = e;
            }
        }
    }
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            swT[k] = wall_T<R>(d, k);
            swKind[k] = d.kind[k];
        }
    }
    __syncthreads();

    // ---- gradients (Eq. 55)
    if (tid < GF) {
        const int li = tid % GX, lj = tid / GX;
        int gi = i0 - 1 + li, gj = j0 - 1 + lj;
        if (px) gi = wrap_axis(gi, nx, nearx);
        if (py) gj = wrap_axis(gj, ny, neary);
        if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) {
            const int ci = li + 1, cj = lj + 1;  // position in sp
            R P[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) P[p] = SP(p, cj, ci);
            R gx[4] = {0, 0, 0, 0}, gy[4] = {0, 0, 0, 0};
            // faces: 0 west (i-face gi), 1 east (gi + 1), 2 south (j-face gj), 3 north (gj + 1)
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const bool isi = f < 2, hi = f & 1;
                const int fi_ = isi ? gi + hi : gi, fj_ = isi ? gj : gj + hi;
                const R nxf = isi ? FI(kCfNx, fi_, fj_) : FJ(kCfNx, fi_, fj_);
                const R nyf = isi ? FI(kCfNy, fi_, fj_) : FJ(kCfNy, fi_, fj_);
                const R dS = isi ? FI(kCfDS, fi_, fj_) : FJ(kCfDS, fi_, fj_);
                const R wL = isi ? FI(kCfWL, fi_, fj_) : FJ(kCfWL, fi_, fj_);
                const R so = hi ? (R)1 : (R)-1;  // outward normal = so * n
                const bool per = isi ? px : py;
                const int gk = isi ? gi : gj, nk = isi ? nx : ny;
                const bool bnd = !per && (hi ? gk == nk - 1 : gk == 0);
                const int side = isi ? (hi ? 1 : 0) : (hi ? 3 : 2);
                R phi[4];
                if (!bnd) {
                    const int qx = isi ? ci + (hi ? 1 : -1) : ci, qy = isi ? cj : cj + (hi ? 1 : -1);
                    // Eq. 56: wL weighs the low cell
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        const R Q = SP(p, qy, qx);
                        phi[p] = hi ? wL * P[p] + ((R)1 - wL) * Q : wL * Q + ((R)1 - wL) * P[p];
                    }
                } else if (swKind[side] == kFarfield) {
                    R G[4];
                    ghost_prims<R, DEV>(g, G);
#pragma unroll
                    for (int p = 0; p < 4; ++p) phi[p] = (R)0.5 * (P[p] + G[p]);
                } else {
                    phi[0] = P[0];
                    phi[1] = phi[2] = (R)0;
                    phi[3] = swKind[side] == kIsothermal ? swT[side] : P[3];
                }
                const R ax = so * nxf * dS, ay = so * nyf * dS;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    gx[p] += phi[p] * ax;
                    gy[p] += phi[p] * ay;
                }
            }
            const R ia = iA[(int64_t)gj * nx + gi];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                sg[(p * 2 + 0) * GF + tid] = gx[p] * ia;
                sg[(p * 2 + 1) * GF + tid] = gy[p] * ia;
            }
        }
    }
    __syncthreads();

    // ---- faces.  face(isi, q) handles face q of its family (i-faces, then
    // j-faces in sf); it is inlined at each call, so a literal isi folds every
    // choice between the families.  Hybrid layout (as in the Cartesian step):
    // whole wavefronts of i-faces, one wavefront with the i tail and the
    // j tail, then whole wavefronts of j-faces; shared layout where the tails
    // do not fit in one wavefront.
    auto face = [&](bool isi, int q) __attribute__((always_inline)) {
        if (q >= (isi ? NFX : NF - NFX)) return;
        const int lx = isi ? q % (TX + 1) : q % TX;
        const int ly = isi ? q / (TX + 1) : q / TX;
        const int gx_ = i0 + lx, gy_ = j0 + ly;  // face index (i, j); the tile's cells need faces up to n
        const bool ok = isi ? (gx_ <= nx && gy_ < ny) : (gx_ < nx && gy_ <= ny);
        if (ok) {
            // record index: on a periodic axis face n is face 0
            const int ri = isi && px && gx_ == nx ? 0 : gx_, rj = !isi && py && gy_ == ny ? 0 : gy_;
            auto REC = [&](int k) -> R { return isi ? FI(k, ri, rj) : FJ(k, ri, rj); };
            const R nxf = REC(kCfNx), nyf = REC(kCfNy), dS = REC(kCfDS);
            const R txf = -nyf, tyf = nxf;
            const int hx = lx + 2, hy = ly + 2;                              // high cell in sp
            const int lox = isi ? hx - 1 : hx, loy = isi ? hy : hy - 1;      // low cell in sp
            const int gk = isi ? gx_ : gy_, nk = isi ? nx : ny;
            const bool per = isi ? px : py;
            const bool low_b = !per && gk == 0, high_b = !per && gk == nk;
            R Fg[4];  // flux along +n times dS, momentum in global components
            if (!low_b && !high_b) {
                Side<R, 2> A, B;
                const int gL = (loy - 1) * GX + (lox - 1), gR = (hy - 1) * GX + (hx - 1);
                R PA[4], PB[4], GA[4][2], GB[4][2];
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    PA[p] = SP(p, loy, lox);
                    PB[p] = SP(p, hy, hx);
                    GA[p][0] = sg[(p * 2 + 0) * GF + gL];
                    GA[p][1] = sg[(p * 2 + 1) * GF + gL];
                    GB[p][0] = sg[(p * 2 + 0) * GF + gR];
                    GB[p][1] = sg[(p * 2 + 1) * GF + gR];
                }
                side_in_frame(PA, GA, nxf, nyf, REC(kCfTL), A);
                side_in_frame(PB, GB, nxf, nyf, REC(kCfTR), B);
                frame_flux<R, DEV, TL>(A, B, REC(kCfDL), REC(kCfDR), nxf, nyf, cg_up<R>(g, 0), cg_up<R>(g, 1),
                                       d.force_pred != 0, dS, ph, Fg);
            } else {
                const int side = isi ? (low_b ? 0 : 1) : (low_b ? 2 : 3);
                const int wx = low_b ? hx : lox, wy = low_b ? hy : loy;  // the fluid cell
                const R so = low_b ? (R)-1 : (R)1;                      // outward normal = so * n
                const R dist = low_b ? REC(kCfDR) : REC(kCfDL);
                const R rP = SP(0, wy, wx), uxP = SP(1, wy, wx), uyP = SP(2, wy, wx), TP = SP(3, wy, wx);
                const R rho = DEV ? (R)1 + rP : rP;
                if (swKind[side] != kFarfield) {
                    const R mloc[2] = {rho * (uxP * nxf + uyP * nyf), rho * (uxP * txf + uyP * tyf)};
                    R G[4];
                    wall_flux<R, 2, DEV>(rP, mloc, rho * TP, so, dist, swKind[side] == kIsothermal, swT[side], ph, G);
                    Fg[0] = G[0] * dS;
                    Fg[1] = (G[1] * nxf + G[2] * txf) * dS;
                    Fg[2] = (G[1] * nyf + G[2] * tyf) * dS;
                    Fg[3] = G[3] * dS;
                } else {
                    // interior-face flux against the mirrored ghost, in the
                    // frame of the outward normal so n with the fluid cell on
                    // the low side; the flux along +n is so times that one
                    const int gidx = (wy - 1) * GX + (wx - 1);
                    const R nox = so * nxf, noy = so * nyf;
                    const R tau = so * (low_b ? REC(kCfTR) : REC(kCfTL));
                    const R Pv[4] = {rP, uxP, uyP, TP};
                    R Gd[4][2];
#pragma unroll
                    for (int p = 0; p < 4; ++p) {
                        Gd[p][0] = sg[(p * 2 + 0) * GF + gidx];
                        Gd[p][1] = sg[(p * 2 + 1) * GF + gidx];
                    }
                    Side<R, 2> A, B;
                    side_in_frame(Pv, Gd, nox, noy, tau, A);
                    R Gh[4];
                    ghost_prims<R, DEV>(g, Gh);
                    B.v[0] = Gh[0];
                    B.v[1] = Gh[1] * nox + Gh[2] * noy;
                    B.v[2] = -Gh[1] * noy + Gh[2] * nox;
                    B.v[3] = Gh[3];
#pragma unroll
                    for (int k = 0; k < 2; ++k)
#pragma unroll
                        for (int p = 0; p < 4; ++p) B.g[k][p] = (R)0;
                    R Fo[4];
                    frame_flux<R, DEV, TL>(A, B, dist, dist, nox, noy, cg_up<R>(g, 0), cg_up<R>(g, 1),
                                           d.force_pred != 0, dS, ph, Fo);
#pragma unroll
                    for (int p = 0; p < 4; ++p) Fg[p] = so * Fo[p];
                }
            }
            const int fo = isi ? q : NFX + q;
#pragma unroll
            for (int p = 0; p < 4; ++p) sf[p * NF + fo] = Fg[p];
        }
    };
    constexpr int XW = NFX / 64, TXT = NFX % 64, TYT = (NF - NFX) % 64;
    if constexpr (TXT + TYT > 0 && TXT + TYT <= 64) {
        const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // a scalar: uniform branches
        const int lane = tid - 64 * XW;
        if (wave < XW) face(true, tid);
        else if (wave > XW) face(false, TYT + tid - 64 * (XW + 1));
        else if (lane < TXT + TYT) face(lane < TXT, lane < TXT ? 64 * XW + lane : lane - TXT);
    } else {
        if (tid < NF) face(tid < NFX, tid < NFX ? tid : tid - NFX);
    }
    __syncthreads();

    // ---- update
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (tid < TX * TY) {
        const int lc = tid % TX, lr = tid / TX;
        const int gi = i0 + lc, gj = j0 + lr;
        if (gi < nx && gj < ny) {
            const int64_t c = (int64_t)gj * nx + gi;
            const int fw = lr * (TX + 1) + lc, fs = NFX + lr * TX + lc;
            const R dtR = ph.dt;
            const R dt_dV = dtR * iA[c];
            const R rP = SP(0, lr + 2, lc + 2);
            const R rhoP = DEV ? (R)1 + rP : rP;
            const R TP = SP(3, lr + 2, lc + 2);
            const R Fb = dtR * ph.bg * rhoP * (TP - ph.Tref_s);
            const R src[4] = {(R)0, Fb * cg_up<R>(g, 0), Fb * cg_up<R>(g, 1), (R)0};
            R Un[4];
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const R inc = dt_dV * ((sf[f * NF + fw] - sf[f * NF + fw + 1]) + (sf[f * NF + fs] - sf[f * NF + fs + TX])) +
                              src[f];
                const R old = sc[f * SCF + tid];
                if (sizeof(R) == 4 && d.sround) Un[f] = sr_add(old, inc, sr_hash((uint32_t)c, step_key * 4u + f));
                else Un[f] = old + inc;
            }
#pragma unroll
            for (int f = 0; f < 4; ++f) Uout[f * N + c] = Un[f];
            if (RES) {
                const double rn = (double)Un[0];
                const double rhon = DEV ? 1.0 + rn : rn;
                const double un = (double)Un[1] / rhon, vn = (double)Un[2] / rhon;
                const double Tn = (double)Un[3] / rhon + (DEV ? kT0 : 0.0);
                const double uo = (double)SP(1, lr + 2, lc + 2), vo = (double)SP(2, lr + 2, lc + 2);
                const double To = (double)TP + (DEV ? kT0 : 0.0);
                const double an = sqrt(un * un + vn * vn), ao = sqrt(uo * uo + vo * vo);
                acc[0] += fabs(an - ao);
                acc[1] += an;
                acc[2] += fabs(Tn - To);
                acc[3] += Tn;
                const bool okm = (an * an < d.guard_u2) && (Tn == Tn) && (fabs(Tn) < 1e30);
                acc[4] += okm ? 0.0 : 1.0;
            }
        }
    }
    if (RES) {
        block_sums<kPartials>(acc, sred);
        if (tid == 0)
            for (int k = 0; k < kPartials; ++k) part[k] = acc[k];
    }
}

// Wall heat of one side: {sum (T_w - T_P)/d dS, sum dS} over its faces, in
// FP64 from the FP64 face records (single block, fixed order).
template <typename R, bool DEV>
__global__ void __launch_bounds__(256) k_curv_wall_heat(Domain d, const double *__restrict__ fi64,
                                                        const double *__restrict__ fj64, int64_t sfi, int64_t sfj,
                                                        const R *__restrict__ U, int side, double Tw_abs,
                                                        double *__restrict__ out) {
    __shared__ double sred[2 * 4];
    const int nx = d.n[0], ny = d.n[1];
    const int64_t N = d.fstride;
    const bool isi = side < 2, hi = side & 1;
    const int nf = isi ? ny : nx;
    double acc[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < nf; k += blockDim.x) {
        const int i = isi ? (hi ? nx : 0) : k, j = isi ? k : (hi ? ny : 0);
        const int ci = isi ? (hi ? nx - 1 : 0) : k, cj = isi ? k : (hi ? ny - 1 : 0);
        const double *rec = isi ? fi64 + (int64_t)j * (nx + 1) + i : fj64 + (int64_t)j * nx + i;
        const int64_t st = isi ? sfi : sfj;
        const double dS = rec[kCfDS * st];
        const double dist = hi ? rec[kCfDL * st] : rec[kCfDR * st];
        const int64_t c = (int64_t)cj * nx + ci;
        const double r = (double)U[c];
        const double rho = DEV ? 1.0 + r : r;
        const double TP = (double)U[3 * N + c] / rho + (DEV ? kT0 : 0.0);
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
