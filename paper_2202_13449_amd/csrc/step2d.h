// step2d.h -- one fused RTLBFS step over a TX x TY tile of a 2D domain.
//
// Phases, each separated by a workgroup barrier, all through LDS:
//   1. load the state of the tile plus a 2-cell halo and convert it to
//      primitives (r or rho, u, v, T or T');
//   2. Eq. 55 gradients (Eq. 56 face values, wall values on walls) for the
//      tile plus a 1-cell halo;
//   3. every face of the tile once: interior / periodic faces by the lattice
//      predictor-corrector (RTLBFS, or TLBFS when TL), wall faces by the wall
//      closure; area-weighted
//      fluxes go to LDS and are shared by the two cells of the face;
//   4. divergence, Boussinesq source, forward-Euler update (Eqs. 57-59, 64),
//      and on residual steps the FP64 partial sums of Eq. 65.
// The block has one thread per face of the tile (rounded up to whole
// wavefronts), so every phase is a single straight pass.  Latency, not issue
// rate, decides the time of a small domain (one tile per CU), so the phases
// avoid divergence: all interior faces, x and y alike, run one code path
// with per-lane LDS addresses, and neighbour values are read unconditionally
// and chosen by selects rather than by branches around single LDS reads.
#pragma once

#include "rtlbfs_device.h"

namespace rtlbfs {

template <int TX, int TY>
constexpr int tile2_threads() {
    return (((TX + 1) * TY + TX * (TY + 1)) + 63) / 64 * 64;
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

template <typename R, bool DEV, int TX, int TY, bool RES, bool TL>
__device__ __forceinline__ void tile_step_2d(const Domain &d, int i0, int j0, const R *__restrict__ Uin,
                                             R *__restrict__ Uout, double *__restrict__ part, uint32_t step_key) {
    constexpr int PX = TX + 4, PY = TY + 4;  // primitives with a 2-cell halo
    constexpr int GX = TX + 2, GY = TY + 2;  // gradients with a 1-cell halo
    constexpr int NFX = (TX + 1) * TY;       // x-faces, row-major (TX + 1) per row
    constexpr int NF = NFX + TX * (TY + 1);  // then the y-faces, row-major TX per row
    constexpr int NT = tile2_threads<TX, TY>();
    static_assert(PX * PY <= NT && GX * GY <= NT && NF <= NT && PX + PY <= NT,
                  "every phase is one pass of the block");
    __shared__ R sp[4][PY][PX];
    __shared__ R sg[4][2][GY][GX];
    __shared__ R sf[4][NF];            // area-weighted face fluxes
    __shared__ R sc[4][TY][TX];        // old conserved state of the tile cells
    __shared__ R sgx[kGeoFields][PX];  // geometry of the tile columns (with halo)
    __shared__ R sgy[kGeoFields][PY];  // geometry of the tile rows (with halo)
    __shared__ double sred[kPartials * 16];
    __shared__ R swT[4];     // wall value of T per side (T_w if isothermal, else unused)
    __shared__ int swIso[4]; // side is an isothermal wall

    const int nx = d.n[0], ny = d.n[1];
    const int64_t N = d.fstride;
    const bool px = d.periodic[0], py = d.periodic[1];
    const R *__restrict__ geox = (const R *)d.geo[0];
    const R *__restrict__ geoy = (const R *)d.geo[1];
    const Phys<R> &ph = make_phys<R>(d);
    const int tid = threadIdx.x;

    // Phase 1: state of the tile and halo, then the geometry of the halo
    // columns and rows; all global loads are issued before the first use.
    {
        const int li = tid % PX, lj = tid / PX;
        int gi = i0 - 2 + li, gj = j0 - 2 + lj;
        if (px) gi = wrap(gi, nx);
        if (py) gj = wrap(gj, ny);
        const bool ld = tid < PX * PY && gi >= 0 && gi < nx && gj >= 0 && gj < ny;  // outside a wall: never read
        R r = 0, mx = 0, my = 0, e = 0;
        if (ld) {
            const int64_t c = (int64_t)gj * nx + gi;
            r = Uin[c];
            mx = Uin[N + c];
            my = Uin[2 * N + c];
            e = Uin[3 * N + c];
        }
        const bool isx = tid < PX;
        const int gl = isx ? tid : tid - PX;
        const int gn = isx ? nx : ny;
        int g = (isx ? i0 : j0) - 2 + gl;
        if (isx ? px : py) g = wrap(g, gn);
        const bool lg = tid < PX + PY && g >= 0 && g < gn;
        R gv[kGeoFields];
        if (lg) {
            const R *src = isx ? geox : geoy;
#pragma unroll
            for (int k = 0; k < kGeoFields; ++k) gv[k] = src[k * gn + g];
        }
        if (ld) {
            const R inv_rho = recip<R>(DEV ? (R)1 + r : r);
            const int ti = li - 2, tj = lj - 2;
            if (ti >= 0 && ti < TX && tj >= 0 && tj < TY) {
                sc[0][tj][ti] = r;
                sc[1][tj][ti] = mx;
                sc[2][tj][ti] = my;
                sc[3][tj][ti] = e;
            }
            sp[0][lj][li] = r;
            sp[1][lj][li] = mx * inv_rho;
            sp[2][lj][li] = my * inv_rho;
            sp[3][lj][li] = e * inv_rho;
        }
        if (lg) {
#pragma unroll
            for (int k = 0; k < kGeoFields; ++k) {
                if (isx) sgx[k][gl] = gv[k];
                else sgy[k][gl] = gv[k];
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

    // Phase 2: gradients, (phi_hi - phi_lo) / width with Eq. 56 face values
    // (wall faces: r_S = r_P, u_S = 0, T_S = T_w if isothermal else T_P).
    // Halo entries beyond a wall hold no data; they are read but never used.
    if (tid < GX * GY) {
        const int li = tid % GX, lj = tid / GX;
        int gi = i0 - 1 + li, gj = j0 - 1 + lj;
        if (px) gi = wrap(gi, nx);
        if (py) gj = wrap(gj, ny);
        if (gi >= 0 && gi < nx && gj >= 0 && gj < ny) {
            const int ci = li + 1, cj = lj + 1;  // position in sp
            const bool wall_w = !px && gi == 0, wall_e = !px && gi == nx - 1;
            const bool wall_s = !py && gj == 0, wall_n = !py && gj == ny - 1;
            const R xls = sgx[kGeoLoSelf][ci], xln = sgx[kGeoLoNb][ci], xhs = sgx[kGeoHiSelf][ci];
            const R xhn = sgx[kGeoHiNb][ci];
            const R yls = sgy[kGeoLoSelf][cj], yln = sgy[kGeoLoNb][cj], yhs = sgy[kGeoHiSelf][cj];
            const R yhn = sgy[kGeoHiNb][cj];
            const R ixP = sgx[kGeoInvW][ci], iyP = sgy[kGeoInvW][cj];
            R vP[4], vW[4], vE[4], vS[4], vN[4];
#pragma unroll
            for (int p = 0; p < 4; ++p) {
                vP[p] = sp[p][cj][ci];
                vW[p] = sp[p][cj][ci - 1];
                vE[p] = sp[p][cj][ci + 1];
                vS[p] = sp[p][cj - 1][ci];
                vN[p] = sp[p][cj + 1][ci];
            }
            const R TwW = d.kind[0] == kIsothermal ? wall_T<R>(d, 0) : vP[3];
            const R TwE = d.kind[1] == kIsothermal ? wall_T<R>(d, 1) : vP[3];
            const R TwS = d.kind[2] == kIsothermal ? wall_T<R>(d, 2) : vP[3];
            const R TwN = d.kind[3] == kIsothermal ? wall_T<R>(d, 3) : vP[3];
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
                sg[p][0][lj][li] = (fe - fw) * ixP;
                sg[p][1][lj][li] = (fnn - fs) * iyP;
            }
        }
    }
    __syncthreads();

    // Phase 3: every face once.  Face frame: normal axis a (0 for x-faces),
    // tangent axis b; (tl, tr) are the tile coordinates of the cell on the
    // low side, one step along a gives the cell on the high side.
    if (tid < NF) {
        const bool isx = tid < NFX;
        const int qy = tid - NFX;
        // x-face (lf, lr): between cells (lf - 1, lr) and (lf, lr);
        // y-face (lc, lf): between cells (lc, lf - 1) and (lc, lf).
        const int lx = isx ? tid % (TX + 1) : qy % TX;  // x of the face (x-faces) / of the cells (y-faces)
        const int ly = isx ? tid / (TX + 1) : qy / TX;
        const int gx = i0 + lx, gy = j0 + ly;
        const bool valid = isx ? (gy < ny && gx <= nx) : (gx < nx && gy <= ny);
        if (valid) {
            const int ax = isx ? 1 : 0, ay = isx ? 0 : 1;  // step from the low to the high cell
            const int hx = lx + 2, hy = ly + 2;               // high cell in sp
            const int lox = hx - ax, loy = hy - ay;           // low cell in sp
            const int gface = isx ? gx : gy, nn = isx ? nx : ny;
            const bool wall = !(isx ? px : py) && (gface == 0 || gface == nn);
            const R area = isx ? sgy[kGeoW][hy] : sgx[kGeoW][hx];
            // components in the face frame: (r, u_n, u_t, T); y-faces swap u, v
            const int pn = isx ? 1 : 2, pt = isx ? 2 : 1;
            R G[4];
            if (wall) {
                const bool low = gface == 0;  // wall on the low side: the fluid cell is the high one
                const int side = isx ? (low ? 0 : 1) : (low ? 2 : 3);
                const int wx = low ? hx : lox, wy = low ? hy : loy;
                const R sgn = low ? (R)-1 : (R)1;
                const R rP = sp[0][wy][wx];
                const R rho = DEV ? (R)1 + rP : rP;
                const R wcell = isx ? sgx[kGeoW][wx] : sgy[kGeoW][wy];
                const R d_w = (R)0.5 * wcell;
                const R mloc[2] = {rho * sp[pn][wy][wx], rho * sp[pt][wy][wx]};
                wall_flux<R, 2, DEV>(rP, mloc, rho * sp[3][wy][wx], sgn, d_w, swIso[side] != 0, swT[side], ph, G);
            } else {
                Side<R, 2> A, B;
                const int gn = isx ? 0 : 1, gt = isx ? 1 : 0;  // gradient components along n and t
                const int pp[4] = {0, pn, pt, 3};
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    A.v[p] = sp[pp[p]][loy][lox];
                    B.v[p] = sp[pp[p]][hy][hx];
                    A.g[0][p] = sg[pp[p]][gn][loy - 1][lox - 1];
                    A.g[1][p] = sg[pp[p]][gt][loy - 1][lox - 1];
                    B.g[0][p] = sg[pp[p]][gn][hy - 1][hx - 1];
                    B.g[1][p] = sg[pp[p]][gt][hy - 1][hx - 1];
                }
                const R wL = isx ? sgx[kGeoW][lox] : sgy[kGeoW][loy];
                const R wR = isx ? sgx[kGeoW][hx] : sgy[kGeoW][hy];
                const int na = isx ? 0 : 1, ta = isx ? 1 : 0;
                const R fdir[2] = {(d.force_pred && d.gaxis == na) ? (R)1 : (R)0,
                                   (d.force_pred && d.gaxis == ta) ? (R)1 : (R)0};
                if constexpr (TL) face_flux_tlbfs<R, 2, DEV>(A, B, (R)0.5 * wL, (R)0.5 * wR, fdir, ph, G);
                else face_flux<R, 2, DEV>(A, B, (R)0.5 * wL, (R)0.5 * wR, fdir, ph, G);
            }
            // back to global components (mass, m_x, m_y, energy)
            sf[0][tid] = G[0] * area;
            sf[1][tid] = (isx ? G[1] : G[2]) * area;
            sf[2][tid] = (isx ? G[2] : G[1]) * area;
            sf[3][tid] = G[3] * area;
        }
    }
    __syncthreads();

    // Phase 4: divergence, Boussinesq source and update.
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const R dtR = ph.dt;
    if (tid < TX * TY) {
        const int lc = tid % TX, lr = tid / TX;
        const int gi = i0 + lc, gj = j0 + lr;
        if (gi < nx && gj < ny) {
            const int64_t c = (int64_t)gj * nx + gi;
            const int fw = lr * (TX + 1) + lc, fs = NFX + lr * TX + lc;  // west and south faces
            const R dt_dV = dtR * sgx[kGeoInvW][lc + 2] * sgy[kGeoInvW][lr + 2];
            const R rP = sp[0][lr + 2][lc + 2];
            const R rhoP = DEV ? (R)1 + rP : rP;
            const R TP = sp[3][lr + 2][lc + 2];
            R Un[4];
            if (sizeof(R) == 4 && d.sround) {
                // increments first, then one stochastically rounded addition per field
                R inc[4];
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    inc[f] = dt_dV * ((sf[f][fw] - sf[f][fw + 1]) + (sf[f][fs] - sf[f][fs + TX]));
                if (d.gaxis >= 0) inc[1 + d.gaxis] += dtR * ph.bg * rhoP * (DEV ? TP : TP - (R)kT0);
#pragma unroll
                for (int f = 0; f < 4; ++f)
                    Un[f] = sr_add(sc[f][lr][lc], inc[f], sr_hash((uint32_t)c, step_key * 4u + f));
            } else {
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    const R div = (sf[f][fw] - sf[f][fw + 1]) + (sf[f][fs] - sf[f][fs + TX]);
                    Un[f] = sc[f][lr][lc] + dt_dV * div;
                }
                if (d.gaxis >= 0) Un[1 + d.gaxis] += dtR * ph.bg * rhoP * (DEV ? TP : TP - (R)kT0);
            }
#pragma unroll
            for (int f = 0; f < 4; ++f) Uout[f * N + c] = Un[f];
            if (RES) {
                const double rn = (double)Un[0];
                const double rhon = DEV ? 1.0 + rn : rn;
                const double un = (double)Un[1] / rhon, vn = (double)Un[2] / rhon;
                const double Tn = (double)Un[3] / rhon + (DEV ? kT0 : 0.0);
                const double uo = (double)sp[1][lr + 2][lc + 2], vo = (double)sp[2][lr + 2][lc + 2];
                const double To = (double)TP + (DEV ? kT0 : 0.0);
                const double an = sqrt(un * un + vn * vn), ao = sqrt(uo * uo + vo * vo);
                acc[0] += fabs(an - ao);
                acc[1] += an;
                acc[2] += fabs(Tn - To);
                acc[3] += Tn;
                // divergence guard: NaN/Inf or local Mach |u|/c_s > 0.5
                const bool ok = (an * an < 0.25 * kCs2) && (Tn == Tn) && (fabs(Tn) < 1e30);
                acc[4] += ok ? 0.0 : 1.0;
            }
        }
    }
    if (RES) {
        block_sums<kPartials>(acc, sred);
        if (tid == 0)
            for (int k = 0; k < kPartials; ++k) part[k] = acc[k];
    }
}

}  // namespace rtlbfs
