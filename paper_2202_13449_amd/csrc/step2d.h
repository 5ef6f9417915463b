// step2d.h -- fused RTLBFS time steps over a TX x TY tile of a 2D domain.
//
// One launch advances the tile by NSUB (1 or 2) time steps.  The state of the
// tile plus a 2*NSUB-cell halo is loaded once; sub-step s then updates the
// region "tile grown by 2*(NSUB-1-s) cells", so that the last sub-step has
// the 2-cell halo it needs, and only the last one writes to HBM.  With
// NSUB = 2 the intermediate state stays in LDS: one global load, one global
// store, one launch and one dispatch per two steps, at the price of
// recomputing the halo ring of the first sub-step.  A ring cell is computed
// from the same inputs, by the same code and with the same stochastic-rounding
// key as in the tile that owns it, so two sub-steps equal two launches.
//
// Phases of a sub-step, each separated by a workgroup barrier, all in LDS:
//   a. Eq. 55 gradients (Eq. 56 face values, wall values on walls) for the
//      update region plus a 1-cell halo;
//   b. every face of the update region once: interior / periodic faces by the
//      lattice predictor-corrector (RTLBFS, or TLBFS when TL), wall faces by
//      the wall closure; area-weighted fluxes go to LDS and are shared by the
//      two cells of the face;
//   c. divergence, Boussinesq source, forward-Euler update (Eqs. 57-59, 64):
//      into LDS (new conserved state and primitives) for an intermediate
//      sub-step; to HBM, with the FP64 partial sums of Eq. 65 on residual
//      steps, for the last one.
// The block has one thread per face of the largest update region, so every
// phase is a single straight pass.  The face pass comes in three layouts:
//   - shared: x- and y-faces side by side, rounded up to whole wavefronts
//     once; all interior faces run one code path with the face frame chosen
//     per lane (LDS addresses and selects);
//   - split: the x-faces and the y-faces each in whole wavefronts, so the
//     axis is wave-uniform and each side runs code with its frame fixed
//     (compile-time offsets, no per-lane selects between x and y);
//   - hybrid: whole wavefronts of x-faces, one wavefront holding the x tail
//     and the y tail (shared code), then whole wavefronts of y-faces.  It
//     uses the shared layout's wavefront count when the two tails fit in
//     one wavefront, with every other wavefront running axis-fixed code.
// One-step launches take the hybrid layout where the tails fit, the split
// one where there are no tails, and the shared one otherwise: large domains keep many blocks per CU, where the
// total instruction count sets the time and idle lanes cost.  Two-step
// launches take the split layout: they serve small domains, one tile per
// CU, where the wavefronts on the busiest SIMD set the time; for the 20 x 20
// first region of a 16 x 16 tile (420 + 420 faces) the split adds no
// wavefront.
// Within a wavefront the phases avoid divergence: neighbour values are read
// unconditionally and chosen by selects rather than by branches around single
// LDS reads.
#pragma once

#include "rtlbfs_device.h"

namespace rtlbfs {

// Faces of a UX x UY update region: x-faces (UX + 1) x UY, then y-faces.
template <int UX, int UY>
constexpr int region_faces() {
    return (UX + 1) * UY + UX * (UY + 1);
}

// Face-pass layouts: shared, split, hybrid (described at the top of this file).
enum : int { kFacesShared = 0, kFacesSplit = 1, kFacesHybrid = 2 };

// Layout of the face pass of a UX x UY update region in a launch of NSUB
// steps.  Without tails (both face counts multiples of 64) the split layout
// has no idle lane and is taken.
template <int UX, int UY, int NSUB>
constexpr int face_layout() {
    constexpr int tails = ((UX + 1) * UY) % 64 + (UX * (UY + 1)) % 64;
    return NSUB == 2 || tails == 0 ? kFacesSplit : (tails <= 64 ? kFacesHybrid : kFacesShared);
}

// Threads of a UX x UY update region's face pass in the given layout.
template <int UX, int UY, int LAYOUT>
constexpr int region_face_threads() {
    return LAYOUT == kFacesSplit ? ((UX + 1) * UY + 63) / 64 * 64 + (UX * (UY + 1) + 63) / 64 * 64
                                 : (region_faces<UX, UY>() + 63) / 64 * 64;
}

template <int TX, int TY, int NSUB = 1>
constexpr int tile2_threads() {
    constexpr int UX = TX + 4 * (NSUB - 1), UY = TY + 4 * (NSUB - 1);  // largest update region
    return region_face_threads<UX, UY, face_layout<UX, UY, NSUB>()>();
}

// Block -> tile order that keeps each XCD on a contiguous band of tiles.
// Workgroups are dispatched round-robin over the 8 XCDs (block b runs on XCD
// b % 8); giving XCD k the tiles [k*nb/8, (k+1)*nb/8) makes the halo of most
// tiles, and the state written by the previous step, local to that XCD's L2.
__device__ inline int xcd_tile(int b, int nb) {
    constexpr int kXcd = 8;
    const int full = nb / kXcd * kXcd;
    if (b >= full) return b;
    return (b % kXcd) * (full / kXcd) + b / kXcd;
}

// Shared-memory views of one sub-step over a UX x UY update region:
//   sp  primitives of the region plus a 2-cell halo, (UX + 4) x (UY + 4)
//       row-major per field;
//   sg  gradients of the region plus a 1-cell halo, (UX + 2) x (UY + 2) per
//       (field, axis);
//   sf  area-weighted face fluxes, region_faces per field;
//   sc  old conserved state: cell (c, r) of the region at sc[sc0 + r*scs + c]
//       of each field, fields scf apart;
//   sgx/sgy geometry records (field stride gsx / gsy), the sp column / row 0
//       of the region at record gx0 / gy0.
template <typename R>
struct SubView {
    const R *sp;
    R *sg;
    R *sf;
    R *sc;
    int sc0, scs, scf;
    const R *sgx, *sgy;
    int gsx, gsy, gx0, gy0;
};

template <typename R, bool DEV, bool TL, int UX, int UY, bool LAST, bool RES, int NT, int LAYOUT>
__device__ __forceinline__ void substep_2d(const Domain &d, int ux0, int uy0, const SubView<R> &v, R *sp_next,
                                           const R *swT, const int *swIso, R *__restrict__ Uout,
                                           double *__restrict__ part, double *sred, uint32_t step_key, bool nearx,
                                           bool neary) {
    constexpr int PX = UX + 4, PY = UY + 4;  // primitives with a 2-cell halo
    constexpr int GX = UX + 2, GY = UY + 2;  // gradients with a 1-cell halo
    constexpr int NFX = (UX + 1) * UY;
    constexpr int NF = region_faces<UX, UY>();
    constexpr int PF = PX * PY, GF = GX * GY;  // field strides in sp and sg
    static_assert(GX * GY <= NT && region_face_threads<UX, UY, LAYOUT>() <= NT && UX * UY <= NT,
                  "every phase is one pass of the block");
    const int nx = d.n[0], ny = d.n[1];
    const int64_t N = d.fstride;
    const bool px = d.periodic[0], py = d.periodic[1];
    const Phys<R> &ph = make_phys<R>(d);
    const int tid = threadIdx.x;
    const R *sp = v.sp;
    auto SP = [&](int p, int y, int x) -> R { return sp[p * PF + y * PX + x]; };
    auto GEOX = [&](int k, int l) -> R { return v.sgx[k * v.gsx + v.gx0 + l]; };
    auto GEOY = [&](int k, int l) -> R { return v.sgy[k * v.gsy + v.gy0 + l]; };

    // (a) gradients, (phi_hi - phi_lo) / width with Eq. 56 face values.
    // Halo entries beyond a wall hold no data; they are read but never used.
    if (tid < GX * GY) {
        const int li = tid % GX, lj = tid / GX;
        int gi = ux0 - 1 + li, gj = uy0 - 1 + lj;
        if (px) gi = wrap_axis(gi, nx, nearx);
        if (py) gj = wrap_axis(gj, ny, neary);
        if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) {
            const int ci = li + 1, cj = lj + 1;  // position in sp
            const bool wall_w = !px && gi == 0, wall_e = !px && gi == nx - 1;
            const bool wall_s = !py && gj == 0, wall_n = !py && gj == ny - 1;
            const R xls = GEOX(kGeoLoSelf, ci), xln = GEOX(kGeoLoNb, ci), xhs = GEOX(kGeoHiSelf, ci);
            const R xhn = GEOX(kGeoHiNb, ci);
            const R yls = GEOY(kGeoLoSelf, cj), yln = GEOY(kGeoLoNb, cj), yhs = GEOY(kGeoHiSelf, cj);
            const R yhn = GEOY(kGeoHiNb, cj);
            const R ixP = GEOX(kGeoInvW, ci), iyP = GEOY(kGeoInvW, cj);
            R vP[4], vW[4], vE[4], vS[4], vN[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                vP[p] = SP(p, cj, ci);
                vW[p] = SP(p, cj, ci - 1);
                vE[p] = SP(p, cj, ci + 1);
                vS[p] = SP(p, cj - 1, ci);
                vN[p] = SP(p, cj + 1, ci);
            }
            const R TwW = swIso[0] ? swT[0] : vP[3];
            const R TwE = swIso[1] ? swT[1] : vP[3];
            const R TwS = swIso[2] ? swT[2] : vP[3];
            const R TwN = swIso[3] ? swT[3] : vP[3];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                const R fw0 = vP[p] * xls + vW[p] * xln, fe0 = vP[p] * xhs + vE[p] * xhn;
                const R fs0 = vP[p] * yls + vS[p] * yln, fn0 = vP[p] * yhs + vN[p] * yhn;
                const R zw = p == 0 ? vP[0] : p == 3 ? TwW : (R)0;
                const R ze = p == 0 ? vP[0] : p == 3 ? TwE : (R)0;
                const R zs = p == 0 ? vP[0] : p == 3 ? TwS : (R)0;
                const R zn = p == 0 ? vP[0] : p == 3 ? TwN : (R)0;
                const R fw = wall_w ? zw : fw0, fe = wall_e ? ze : fe0;
                const R fs = wall_s ? zs : fs0, fnn = wall_n ? zn : fn0;
                v.sg[(p * 2 + 0) * GF + tid] = (fe - fw) * ixP;
                v.sg[(p * 2 + 1) * GF + tid] = (fnn - fs) * iyP;
            }
        }
    }
    __syncthreads();

    // (b) every face once.  x-face (lx, ly): between cells (lx - 1, ly) and
    // (lx, ly) of the region; y-face (lx, ly): between (lx, ly - 1) and
    // (lx, ly).  On a periodic axis every face is real (the halo wraps); on a
    // walled axis the faces run from the low wall to the high wall.  The
    // fluxes go to sf with the x-faces first.  face(isx, q) handles face q of
    // its axis; it is inlined at each call, so a literal isx folds every
    // choice between x and y.
    auto face = [&](bool isx, int q) __attribute__((always_inline)) {
        const int FW = isx ? UX + 1 : UX;  // faces per row
        const int NFA = isx ? NFX : NF - NFX;
        if (q >= NFA) return;
        const int lx = q % FW, ly = q / FW;
        const int gx = ux0 + lx, gy = uy0 + ly;
        const bool okx = px || (isx ? (gx >= 0 && gx <= nx) : (gx >= 0 && gx < nx));
        const bool oky = py || (isx ? (gy >= 0 && gy < ny) : (gy >= 0 && gy <= ny));
        if (!(okx && oky)) return;
        const int ax = isx ? 1 : 0, ay = isx ? 0 : 1;  // step from the low to the high cell
        const int hx = lx + 2, hy = ly + 2;                 // high cell in sp
        const int lox = hx - ax, loy = hy - ay;             // low cell in sp
        const int gface = isx ? gx : gy, nn = isx ? nx : ny;
        const bool wall = !(isx ? px : py) && (gface == 0 || gface == nn);
        const R area = isx ? GEOY(kGeoW, hy) : GEOX(kGeoW, hx);
        // components in the face frame: (r, u_n, u_t, T); y-faces swap u, v
        const int pn = isx ? 1 : 2, pt = isx ? 2 : 1;
        R G[4];
        if (wall) {
            const bool low = gface == 0;  // wall on the low side: the fluid cell is the high one
            const int side = isx ? (low ? 0 : 1) : (low ? 2 : 3);
            const int wx = low ? hx : lox, wy = low ? hy : loy;
            const R sgn = low ? (R)-1 : (R)1;
            const R rP = SP(0, wy, wx);
            const R rho = DEV ? (R)1 + rP : rP;
            const R wcell = isx ? GEOX(kGeoW, wx) : GEOY(kGeoW, wy);
            const R d_w = (R)0.5 * wcell;
            const R mloc[2] = {rho * SP(pn, wy, wx), rho * SP(pt, wy, wx)};
            wall_flux<R, 2, DEV>(rP, mloc, rho * SP(3, wy, wx), sgn, d_w, swIso[side] != 0, swT[side], ph, G);
        } else {
            Side<R, 2> A, B;
            const int gn = isx ? 0 : 1, gt = isx ? 1 : 0;  // gradient components along n and t
            const int pp[4] = {0, pn, pt, 3};
            const int gL = (loy - 1) * GX + (lox - 1), gR = (hy - 1) * GX + (hx - 1);
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                A.v[p] = SP(pp[p], loy, lox);
                B.v[p] = SP(pp[p], hy, hx);
                A.g[0][p] = v.sg[(pp[p] * 2 + gn) * GF + gL];
                A.g[1][p] = v.sg[(pp[p] * 2 + gt) * GF + gL];
                B.g[0][p] = v.sg[(pp[p] * 2 + gn) * GF + gR];
                B.g[1][p] = v.sg[(pp[p] * 2 + gt) * GF + gR];
            }
            const R wL = isx ? GEOX(kGeoW, lox) : GEOY(kGeoW, loy);
            const R wR = isx ? GEOX(kGeoW, hx) : GEOY(kGeoW, hy);
            const int na = isx ? 0 : 1, ta = isx ? 1 : 0;
            const R fdir[2] = {(d.force_pred && d.gaxis == na) ? (R)1 : (R)0,
                               (d.force_pred && d.gaxis == ta) ? (R)1 : (R)0};
            if constexpr (TL) face_flux_tlbfs<R, 2, DEV>(A, B, (R)0.5 * wL, (R)0.5 * wR, fdir, ph, G);
            else face_flux<R, 2, DEV>(A, B, (R)0.5 * wL, (R)0.5 * wR, fdir, ph, G);
        }
        // back to global components (mass, m_x, m_y, energy)
        const int fo = isx ? q : NFX + q;
        v.sf[0 * NF + fo] = G[0] * area;
        v.sf[1 * NF + fo] = (isx ? G[1] : G[2]) * area;
        v.sf[2 * NF + fo] = (isx ? G[2] : G[1]) * area;
        v.sf[3 * NF + fo] = G[3] * area;
    };
    // The wavefront index, read as a scalar, makes the layout's branches
    // uniform.
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    if constexpr (LAYOUT == kFacesSplit) {
        // threads [0, WX) take the x-faces, [WX, WX + NF - NFX) the y-faces
        constexpr int WX = (NFX + 63) / 64 * 64;
        if (wave < WX / 64) face(true, tid);
        else face(false, tid - WX);
    } else if constexpr (LAYOUT == kFacesHybrid) {
        // wavefronts [0, XW): x-faces [0, 64 XW); wavefront XW: lanes [0, TXT)
        // the x-faces from 64 XW, lanes [TXT, TXT + TYT) the y-faces [0, TYT);
        // the wavefronts after it: y-faces from TYT
        constexpr int XW = NFX / 64, TXT = NFX % 64, TYT = (NF - NFX) % 64;
        static_assert(TXT + TYT > 0 && TXT + TYT <= 64, "both tails fit in one wavefront");
        const int lane = tid - 64 * XW;
        if (wave < XW) face(true, tid);
        else if (wave > XW) face(false, TYT + tid - 64 * (XW + 1));
        else if (lane < TXT + TYT) face(lane < TXT, lane < TXT ? 64 * XW + lane : lane - TXT);
    } else {
        // threads [0, NFX) take the x-faces, [NFX, NF) the y-faces
        if (tid < NF) face(tid < NFX, tid < NFX ? tid : tid - NFX);
    }
    __syncthreads();

    // (c) divergence, Boussinesq source and update.  The last sub-step updates
    // the cells of the tile that exist; an intermediate one every real cell of
    // its region (periodic ring cells by their wrapped index, which also keys
    // the stochastic rounding, so a ring cell gets exactly the value its owner
    // tile computes).
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const R dtR = ph.dt;
    if (tid < UX * UY) {
        const int lc = tid % UX, lr = tid / UX;
        int gi = ux0 + lc, gj = uy0 + lr;
        bool ok;
        if (LAST) {
            ok = gi < nx && gj < ny;
        } else {
            if (px) gi = wrap_axis(gi, nx, nearx);
            if (py) gj = wrap_axis(gj, ny, neary);
            ok = gi >= 0 && gi < nx && gj >= 0 && gj < ny;
        }
        if (ok) {
            const int64_t c = (int64_t)gj * nx + gi;
            const int fw = lr * (UX + 1) + lc, fs = NFX + lr * UX + lc;  // west and south faces
            const R dt_dV = dtR * GEOX(kGeoInvW, lc + 2) * GEOY(kGeoInvW, lr + 2);
            const R rP = SP(0, lr + 2, lc + 2);
            const R rhoP = DEV ? (R)1 + rP : rP;
            const R TP = SP(3, lr + 2, lc + 2);
            R *sc = v.sc + v.sc0 + lr * v.scs + lc;  // this cell's old conserved state
            R Un[4];
            if (sizeof(R) == 4 && d.sround) {
                // increments first, then one stochastically rounded addition per field
                R inc[4];
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    inc[f] = dt_dV * ((v.sf[f * NF + fw] - v.sf[f * NF + fw + 1]) +
                                      (v.sf[f * NF + fs] - v.sf[f * NF + fs + UX]));
                if (d.gaxis >= 0) inc[1 + d.gaxis] += dtR * ph.bg * rhoP * (DEV ? TP : TP - (R)kT0);
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    Un[f] = sr_add(sc[f * v.scf], inc[f], sr_hash((uint32_t)c, step_key * 4u + f));
            } else {
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const R div = (v.sf[f * NF + fw] - v.sf[f * NF + fw + 1]) +
                                  (v.sf[f * NF + fs] - v.sf[f * NF + fs + UX]);
                    Un[f] = sc[f * v.scf] + dt_dV * div;
                }
                if (d.gaxis >= 0) Un[1 + d.gaxis] += dtR * ph.bg * rhoP * (DEV ? TP : TP - (R)kT0);
            }
            if (LAST) {
#pragma unroll
                for (int f = 0; f < 4; ++f) Uout[f * N + c] = Un[f];
            } else {
                // new conserved state in place; new primitives for the next
                // sub-step, whose 2-cell-halo box is exactly this region
#pragma unroll
                for (int f = 0; f < 4; ++f) sc[f * v.scf] = Un[f];
                const R inv_rho = recip<R>(DEV ? (R)1 + Un[0] : Un[0]);
                const int o = lr * UX + lc;
                sp_next[0 * UX * UY + o] = Un[0];
                sp_next[1 * UX * UY + o] = Un[1] * inv_rho;
                sp_next[2 * UX * UY + o] = Un[2] * inv_rho;
                sp_next[3 * UX * UY + o] = Un[3] * inv_rho;
            }
            if (LAST && RES) {
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
                // divergence guard: NaN/Inf or local Mach |u|/c_s > 0.5
                const bool okm = (an * an < d.guard_u2) && (Tn == Tn) && (fabs(Tn) < 1e30);
                acc[4] += okm ? 0.0 : 1.0;
            }
        }
    }
    if (LAST && RES) {
        block_sums<kPartials>(acc, sred);
        if (tid == 0)
            for (int k = 0; k < kPartials; ++k) part[k] = acc[k];
    }
}

template <typename R, bool DEV, int TX, int TY, bool RES, bool TL, int NSUB = 1>
__device__ __forceinline__ void tile_step_2d(const Domain &d, int i0, int j0, const R *__restrict__ Uin,
                                             R *__restrict__ Uout, double *__restrict__ part, uint32_t step_key) {
    static_assert(NSUB == 1 || NSUB == 2, "one or two sub-steps per launch");
    constexpr int H = 2 * NSUB;                                          // loaded halo
    constexpr int U0X = TX + 4 * (NSUB - 1), U0Y = TY + 4 * (NSUB - 1);  // first update region
    constexpr int LX = TX + 2 * H, LY = TY + 2 * H;                      // first region + 2-cell halo
    constexpr int NT = tile2_threads<TX, TY, NSUB>();
    constexpr int SCF = U0X * U0Y;
    static_assert(LX * LY <= NT && LX + LY <= NT, "the load is one pass of the block");
    __shared__ R spA[4 * LX * LY];
    __shared__ R spB[NSUB == 2 ? 4 * SCF : 1];
    __shared__ R sg[4 * 2 * (U0X + 2) * (U0Y + 2)];
    __shared__ R sf[4 * region_faces<U0X, U0Y>()];
    __shared__ R sc[4 * SCF];  // old conserved state of the first update region
    __shared__ R sgx[kGeoFields * LX];
    __shared__ R sgy[kGeoFields * LY];
    __shared__ double sred[kPartials * 16];
    __shared__ R swT[4];     // wall value of T per side (T_w if isothermal, else unused)
    __shared__ int swIso[4]; // side is an isothermal wall

    const int nx = d.n[0], ny = d.n[1];
    const int64_t N = d.fstride;
    const bool px = d.periodic[0], py = d.periodic[1];
    // a periodic axis at least as long as the tile plus both halos wraps by selects
    const bool nearx = nx >= TX + 2 * H, neary = ny >= TY + 2 * H;
    const R *__restrict__ geox = (const R *)d.geo[0];
    const R *__restrict__ geoy = (const R *)d.geo[1];
    const int tid = threadIdx.x;

    // Load: state of the tile and its halo, then the geometry of the halo
    // columns and rows; all global loads are issued before the first use.
    {
        const int li = tid % LX, lj = tid / LX;
        int gi = i0 - H + li, gj = j0 - H + lj;
        if (px) gi = wrap_axis(gi, nx, nearx);
        if (py) gj = wrap_axis(gj, ny, neary);
        const bool ld = tid < LX * LY && gi >= 0 && gi < nx && gj >= 0 && gj < ny;  // outside a wall: never read
        R r = 0, mx = 0, my = 0, e = 0;
        if (ld) {
            const int64_t c = (int64_t)gj * nx + gi;
            r = Uin[c];
            mx = Uin[N + c];
            my = Uin[2 * N + c];
            e = Uin[3 * N + c];
        }
        const bool isx = tid < LX;
        const int gl = isx ? tid : tid - LX;
        const int gn = isx ? nx : ny;
        int g = (isx ? i0 : j0) - H + gl;
        if (isx ? px : py) g = wrap_axis(g, gn, nearx && neary);  // one choice for the block
        const bool lg = tid < LX + LY && g >= 0 && g < gn;
        R gv[kGeoFields];
        if (lg) {
            const R *src = isx ? geox : geoy;
#pragma unroll
            for (int k = 0; k < kGeoFields; ++k) gv[k] = src[k * gn + g];
        }
        if (ld) {
            const R inv_rho = recip<R>(DEV ? (R)1 + r : r);
            const int ti = li - 2, tj = lj - 2;  // position in the first update region
            if (ti >= 0 && ti < U0X && tj >= 0 && tj < U0Y) {
                const int o = tj * U0X + ti;
                sc[0 * SCF + o] = r;
                sc[1 * SCF + o] = mx;
                sc[2 * SCF + o] = my;
                sc[3 * SCF + o] = e;
            }
            const int o = lj * LX + li;
            spA[0 * LX * LY + o] = r;
            spA[1 * LX * LY + o] = mx * inv_rho;
            spA[2 * LX * LY + o] = my * inv_rho;
            spA[3 * LX * LY + o] = e * inv_rho;
        }
        if (lg) {
#pragma unroll
            for (int k = 0; k < kGeoFields; ++k) {
                if (isx) sgx[k * LX + gl] = gv[k];
                else sgy[k * LY + gl] = gv[k];
            }
        }
        // per-side wall data through LDS, so a lane can pick its side by
        // index without a per-lane load from the kernel arguments
        if (tid == 0) {  // compile-time side indices: scalar loads of the arguments
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                swT[k] = wall_T<R>(d, k);
                swIso[k] = d.kind[k] == kIsothermal;
            }
        }
    }
    __syncthreads();

    constexpr int LA = face_layout<U0X, U0Y, NSUB>(), LB = face_layout<TX, TY, NSUB>();
    if constexpr (NSUB == 1) {
        const SubView<R> v{spA, sg, sf, sc, 0, TX, SCF, sgx, sgy, LX, LY, 0, 0};
        substep_2d<R, DEV, TL, TX, TY, true, RES, NT, LB>(d, i0, j0, v, nullptr, swT, swIso, Uout, part, sred,
                                                          step_key, nearx, neary);
    } else {
        const SubView<R> va{spA, sg, sf, sc, 0, U0X, SCF, sgx, sgy, LX, LY, 0, 0};
        substep_2d<R, DEV, TL, U0X, U0Y, false, false, NT, LA>(d, i0 - 2, j0 - 2, va, spB, swT, swIso, nullptr,
                                                               nullptr, sred, step_key, nearx, neary);
        __syncthreads();
        // second sub-step: primitives from spB, old state inside sc at (2, 2),
        // geometry shifted by the two cells the region shrank by
        const SubView<R> vb{spB, sg, sf, sc, 2 * U0X + 2, U0X, SCF, sgx, sgy, LX, LY, 2, 2};
        substep_2d<R, DEV, TL, TX, TY, true, RES, NT, LB>(d, i0, j0, vb, nullptr, swT, swIso, Uout, part, sred,
                                                          step_key + 1u, nearx, neary);
    }
}

}  // namespace rtlbfs
