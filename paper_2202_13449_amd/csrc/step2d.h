// step2d.h -- one fused RTLBFS step over a TX x TY tile of a 2D domain.
//
// Phases, each separated by a workgroup barrier, all through LDS:
//   1. load the state of the tile plus a 2-cell halo and convert it to
//      primitives (r or rho, u, v, T or T');
//   2. Eq. 55 gradients (Eq. 56 face values, wall values on walls) for the
//      tile plus a 1-cell halo;
//   3. every face of the tile once: interior / periodic faces by the lattice
//      predictor-corrector, wall faces by the wall closure; area-weighted
//      fluxes go to LDS and are shared by the two cells of the face;
//   4. divergence, Boussinesq source, forward-Euler update (Eqs. 57-59, 64),
//      and on residual steps the FP64 partial sums of Eq. 65.
// The block has one thread per face of the tile (rounded up to whole
// wavefronts), so every phase is a single pass and each CU keeps several
// wavefronts per SIMD in flight.
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

template <typename R, bool DEV, int TX, int TY, bool RES>
__device__ __forceinline__ void tile_step_2d(const Domain &d, int i0, int j0, const R *__restrict__ Uin,
                                             R *__restrict__ Uout, double *__restrict__ part, uint32_t step_key) {
    constexpr int PX = TX + 4, PY = TY + 4;  // primitives with a 2-cell halo
    constexpr int GX = TX + 2, GY = TY + 2;  // gradients with a 1-cell halo
    __shared__ R sp[4][PY][PX];
    __shared__ R sg[4][2][GY][GX];
    __shared__ R sfx[4][TY][TX + 1];
    __shared__ R sfy[4][TY + 1][TX];
    __shared__ R sc[4][TY][TX];  // old conserved state of the tile cells
    __shared__ R sgx[kGeoFields][PX];  // geometry of the tile columns (with halo)
    __shared__ R sgy[kGeoFields][PY];  // geometry of the tile rows (with halo)
    __shared__ double sred[kPartials * 16];

    const int nx = d.n[0], ny = d.n[1];
    const int64_t N = d.fstride;
    const bool px = d.periodic[0], py = d.periodic[1];
    const R *__restrict__ geox = (const R *)d.geo[0];
    const R *__restrict__ geoy = (const R *)d.geo[1];
    const Phys<R> ph = make_phys<R>(d);
    const int tid = threadIdx.x, nthr = blockDim.x;

    // Phase 1a: geometry of the halo columns and rows.
    for (int q = tid; q < PX + PY; q += nthr) {
        const bool isx = q < PX;
        const int l = isx ? q : q - PX;
        const int n = isx ? nx : ny;
        int g = (isx ? i0 : j0) - 2 + l;
        if (isx ? px : py) g = wrap(g, n);
        if (g < 0 || g >= n) continue;
        const R *src = isx ? geox : geoy;
#pragma unroll
        for (int k = 0; k < kGeoFields; ++k) {
            if (isx) sgx[k][l] = src[k * n + g];
            else sgy[k][l] = src[k * n + g];
        }
    }

    // Phase 1: load + primitives.
    for (int q = tid; q < PX * PY; q += nthr) {
        const int li = q % PX, lj = q / PX;
        int gi = i0 - 2 + li, gj = j0 - 2 + lj;
        if (px) gi = wrap(gi, nx);
        if (py) gj = wrap(gj, ny);
        if (gi < 0 || gi >= nx || gj < 0 || gj >= ny) continue;  // outside a wall: never read
        const int64_t c = (int64_t)gj * nx + gi;
        const R r = Uin[c], mx = Uin[N + c], my = Uin[2 * N + c], e = Uin[3 * N + c];
        const R inv_rho = (R)1 / (DEV ? (R)1 + r : r);
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
    __syncthreads();

    // Phase 2: gradients, (phi_hi - phi_lo) / width with Eq. 56 face values.
    for (int q = tid; q < GX * GY; q += nthr) {
        const int li = q % GX, lj = q / GX;
        int gi = i0 - 1 + li, gj = j0 - 1 + lj;
        if (px) gi = wrap(gi, nx);
        if (py) gj = wrap(gj, ny);
        if (gi < 0 || gi >= nx || gj < 0 || gj >= ny) continue;
        const int ci = li + 1, cj = lj + 1;  // position in sp
        const bool wall_w = !px && gi == 0, wall_e = !px && gi == nx - 1;
        const bool wall_s = !py && gj == 0, wall_n = !py && gj == ny - 1;
        const R xls = sgx[kGeoLoSelf][ci], xln = sgx[kGeoLoNb][ci], xhs = sgx[kGeoHiSelf][ci], xhn = sgx[kGeoHiNb][ci];
        const R yls = sgy[kGeoLoSelf][cj], yln = sgy[kGeoLoNb][cj], yhs = sgy[kGeoHiSelf][cj], yhn = sgy[kGeoHiNb][cj];
        const R ixP = sgx[kGeoInvW][ci], iyP = sgy[kGeoInvW][cj];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            const R vP = sp[p][cj][ci];
            // wall face values: r_S = r_P, u_S = 0, T_S = T_w (isothermal) or T_P
            auto wallv = [&](int side) -> R {
                if (p == 0) return vP;
                if (p < 3) return (R)0;
                return d.kind[side] == kIsothermal ? (R)d.Tw[side] : vP;
            };
            // Eq. 56 face values with precomputed inverse-distance weights
            const R fw = wall_w ? wallv(0) : vP * xls + sp[p][cj][ci - 1] * xln;
            const R fe = wall_e ? wallv(1) : vP * xhs + sp[p][cj][ci + 1] * xhn;
            const R fs = wall_s ? wallv(2) : vP * yls + sp[p][cj - 1][ci] * yln;
            const R fnn = wall_n ? wallv(3) : vP * yhs + sp[p][cj + 1][ci] * yhn;
            sg[p][0][lj][li] = (fe - fw) * ixP;
            sg[p][1][lj][li] = (fnn - fs) * iyP;
        }
    }
    __syncthreads();

    // Phase 3: faces.  x-faces: (TX+1) x TY; y-faces: TX x (TY+1).
    constexpr int NFX = (TX + 1) * TY, NFY = TX * (TY + 1);
    for (int q = tid; q < NFX + NFY; q += nthr) {
        R F[4];
        if (q < NFX) {
            const int lf = q % (TX + 1), lr = q / (TX + 1);
            const int gf = i0 + lf, gj = j0 + lr;
            if (gj >= ny || gf > nx) continue;
            const R area = sgy[kGeoW][lr + 2];
            if (!px && (gf == 0 || gf == nx)) {
                const int side = gf == 0 ? 0 : 1;
                const int ci = gf == 0 ? lf + 2 : lf + 1;  // the wall cell in sp
                const R sgn = gf == 0 ? (R)-1 : (R)1;
                const R rP = sp[0][lr + 2][ci];
                const R rho = DEV ? (R)1 + rP : rP;
                const R d_w = (R)0.5 * sgx[kGeoW][ci];
                const R mloc[2] = {rho * sp[1][lr + 2][ci], rho * sp[2][lr + 2][ci]};
                wall_flux<R, 2, DEV>(rP, mloc, rho * sp[3][lr + 2][ci], sgn, d_w, d.kind[side] == kIsothermal,
                                     (R)d.Tw[side], ph, F);
            } else {
                Side<R, 2> A, B;
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    // normal = x, tangent = y: (r, u_n = u, u_t = v, T)
                    A.v[p] = sp[p][lr + 2][lf + 1];
                    B.v[p] = sp[p][lr + 2][lf + 2];
                    A.g[0][p] = sg[p][0][lr + 1][lf];
                    A.g[1][p] = sg[p][1][lr + 1][lf];
                    B.g[0][p] = sg[p][0][lr + 1][lf + 1];
                    B.g[1][p] = sg[p][1][lr + 1][lf + 1];
                }
                const R dL = (R)0.5 * sgx[kGeoW][lf + 1];
                const R dR = (R)0.5 * sgx[kGeoW][lf + 2];
                const R fdir[2] = {(d.force_pred && d.gaxis == 0) ? (R)1 : (R)0,
                                   (d.force_pred && d.gaxis == 1) ? (R)1 : (R)0};
                face_flux<R, 2, DEV>(A, B, dL, dR, fdir, ph, F);
            }
            sfx[0][lr][lf] = F[0] * area;
            sfx[1][lr][lf] = F[1] * area;
            sfx[2][lr][lf] = F[2] * area;
            sfx[3][lr][lf] = F[3] * area;
        } else {
            const int qq = q - NFX;
            const int lc = qq % TX, lf = qq / TX;
            const int gi = i0 + lc, gf = j0 + lf;
            if (gi >= nx || gf > ny) continue;
            const R area = sgx[kGeoW][lc + 2];
            R G[4];
            if (!py && (gf == 0 || gf == ny)) {
                const int side = gf == 0 ? 2 : 3;
                const int cj = gf == 0 ? lf + 2 : lf + 1;
                const R sgn = gf == 0 ? (R)-1 : (R)1;
                const R rP = sp[0][cj][lc + 2];
                const R rho = DEV ? (R)1 + rP : rP;
                const R d_w = (R)0.5 * sgy[kGeoW][cj];
                // normal = y: m_a = m_y, m_b = m_x
                const R mloc[2] = {rho * sp[2][cj][lc + 2], rho * sp[1][cj][lc + 2]};
                wall_flux<R, 2, DEV>(rP, mloc, rho * sp[3][cj][lc + 2], sgn, d_w, d.kind[side] == kIsothermal,
                                     (R)d.Tw[side], ph, G);
            } else {
                Side<R, 2> A, B;
                // normal = y, tangent = x: (r, u_n = v, u_t = u, T)
                const int perm[4] = {0, 2, 1, 3};
#pragma unroll
                for (int p = 0; p < 4; ++p) {
                    const int pp = perm[p];
                    A.v[p] = sp[pp][lf + 1][lc + 2];
                    B.v[p] = sp[pp][lf + 2][lc + 2];
                    A.g[0][p] = sg[pp][1][lf][lc + 1];
                    A.g[1][p] = sg[pp][0][lf][lc + 1];
                    B.g[0][p] = sg[pp][1][lf + 1][lc + 1];
                    B.g[1][p] = sg[pp][0][lf + 1][lc + 1];
                }
                const R dL = (R)0.5 * sgy[kGeoW][lf + 1];
                const R dR = (R)0.5 * sgy[kGeoW][lf + 2];
                const R fdir[2] = {(d.force_pred && d.gaxis == 1) ? (R)1 : (R)0,
                                   (d.force_pred && d.gaxis == 0) ? (R)1 : (R)0};
                face_flux<R, 2, DEV>(A, B, dL, dR, fdir, ph, G);
            }
            // back to global components: (mass, m_x = m_t, m_y = m_n, energy)
            F[0] = G[0];
            F[1] = G[2];
            F[2] = G[1];
            F[3] = G[3];
            sfy[0][lf][lc] = F[0] * area;
            sfy[1][lf][lc] = F[1] * area;
            sfy[2][lf][lc] = F[2] * area;
            sfy[3][lf][lc] = F[3] * area;
        }
    }
    __syncthreads();

    // Phase 4: update.
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const R dtR = (R)d.dt;
    for (int q = tid; q < TX * TY; q += nthr) {
        const int lc = q % TX, lr = q / TX;
        const int gi = i0 + lc, gj = j0 + lr;
        if (gi >= nx || gj >= ny) continue;
        const int64_t c = (int64_t)gj * nx + gi;
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
                inc[f] = dt_dV * ((sfx[f][lr][lc] - sfx[f][lr][lc + 1]) + (sfy[f][lr][lc] - sfy[f][lr + 1][lc]));
            if (d.gaxis >= 0) inc[1 + d.gaxis] += dtR * (R)d.bg * rhoP * (DEV ? TP : TP - (R)kT0);
#pragma unroll
            for (int f = 0; f < 4; ++f) Un[f] = sr_add(sc[f][lr][lc], inc[f], sr_hash((uint32_t)c, step_key * 4u + f));
        } else {
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const R div = (sfx[f][lr][lc] - sfx[f][lr][lc + 1]) + (sfy[f][lr][lc] - sfy[f][lr + 1][lc]);
                Un[f] = sc[f][lr][lc] + dt_dV * div;
            }
            if (d.gaxis >= 0) Un[1 + d.gaxis] += dtR * (R)d.bg * rhoP * (DEV ? TP : TP - (R)kT0);
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
    if (RES) {
        block_sums<kPartials>(acc, sred);
        if (tid == 0)
            for (int k = 0; k < kPartials; ++k) part[k] = acc[k];
    }
}

}  // namespace rtlbfs
