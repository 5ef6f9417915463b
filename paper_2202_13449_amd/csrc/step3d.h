// step3d.h -- one fused RTLBFS step over a TX x TY x TZ tile of a 3D domain
// (D3Q19 face lattice).  Same phases as the 2D tile: LDS-staged primitives
// with a 2-cell halo, Eq. 55 gradients with a 1-cell halo, every face of the
// tile once (lattice predictor-corrector or wall closure) into LDS, then the
// divergence, buoyancy and forward-Euler update with optional FP64 Eq. 65
// partial sums.
#pragma once

#include <type_traits>

#include "rtlbfs_device.h"

namespace rtlbfs {

template <int TX, int TY, int TZ>
struct Tile3 {
    static constexpr int PX = TX + 4, PY = TY + 4, PZ = TZ + 4;
    static constexpr int GX = TX + 2, GY = TY + 2, GZ = TZ + 2;
    static constexpr int NP = PX * PY * PZ;
    static constexpr int NG = GX * GY * GZ;
    // faces normal to axis a: (T[a] + 1) along a, T elsewhere
    static constexpr int NF0 = (TX + 1) * TY * TZ, NF1 = TX * (TY + 1) * TZ, NF2 = TX * TY * (TZ + 1);
    __device__ static int pidx(int x, int y, int z) { return (z * PY + y) * PX + x; }  // cell at tile coords - 2
    __device__ static int gidx(int x, int y, int z) { return (z * GY + y) * GX + x; }  // cell at tile coords - 1
};

// One thread per face of the tile, rounded up to whole wavefronts.
template <int TX, int TY, int TZ>
constexpr int tile3_threads() {
    return (((TX + 1) * TY * TZ + TX * (TY + 1) * TZ + TX * TY * (TZ + 1)) + 63) / 64 * 64;
}

template <typename R, bool DEV, int TX, int TY, int TZ, bool RES>
__device__ __forceinline__ void tile_step_3d(const Domain &d, int i0, int j0, int k0, const R *__restrict__ Uin,
                                             R *__restrict__ Uout, double *__restrict__ part, uint32_t step_key) {
    using TL = Tile3<TX, TY, TZ>;
    constexpr int NPRIM = 5;
    __shared__ R sp[NPRIM][TL::NP];
    __shared__ R sg[NPRIM][3][TL::NG];
    __shared__ R sf0[NPRIM][TL::NF0];
    __shared__ R sf1[NPRIM][TL::NF1];
    __shared__ R sf2[NPRIM][TL::NF2];
    __shared__ double sred[kPartials * 16];
    __shared__ R sgeo0[kGeoFields][TL::PX];
    __shared__ R sgeo1[kGeoFields][TL::PY];
    __shared__ R sgeo2[kGeoFields][TL::PZ];

    const int n[3] = {d.n[0], d.n[1], d.n[2]};
    const int org[3] = {i0, j0, k0};
    const int64_t N = d.fstride;
    const Phys<R> ph = make_phys<R>(d);
    const int tid = threadIdx.x, nthr = blockDim.x;
    auto gcell = [&](int c, int a, bool &inside) -> int {  // global index along a, wrapped if periodic
        if (d.periodic[a]) c = wrap(c, n[a]);
        inside = c >= 0 && c < n[a];
        return c;
    };

    // geometry of axis a, halo position l (l = global index - origin + 2)
    auto geo = [&](int a, int k, int l) -> R {
        return a == 0 ? sgeo0[k][l] : (a == 1 ? sgeo1[k][l] : sgeo2[k][l]);
    };
    // Phase 1a: geometry of the halo lines of the three axes.
    for (int q = tid; q < TL::PX + TL::PY + TL::PZ; q += nthr) {
        const int a = q < TL::PX ? 0 : (q < TL::PX + TL::PY ? 1 : 2);
        const int l = a == 0 ? q : (a == 1 ? q - TL::PX : q - TL::PX - TL::PY);
        bool inside;
        const int g = gcell(org[a] - 2 + l, a, inside);
        if (!inside) continue;
        const R *src = (const R *)d.geo[a];
#pragma unroll
        for (int k = 0; k < kGeoFields; ++k) {
            const R v = src[k * n[a] + g];
            if (a == 0) sgeo0[k][l] = v;
            else if (a == 1) sgeo1[k][l] = v;
            else sgeo2[k][l] = v;
        }
    }

    // Phase 1: load + primitives.
    for (int q = tid; q < TL::NP; q += nthr) {
        const int lx = q % TL::PX, ly = (q / TL::PX) % TL::PY, lz = q / (TL::PX * TL::PY);
        bool in0, in1, in2;
        const int gx = gcell(i0 - 2 + lx, 0, in0), gy = gcell(j0 - 2 + ly, 1, in1), gz = gcell(k0 - 2 + lz, 2, in2);
        if (!(in0 && in1 && in2)) continue;
        const int64_t c = ((int64_t)gz * n[1] + gy) * n[0] + gx;
        const R r = Uin[c];
        const R inv_rho = (R)1 / (DEV ? (R)1 + r : r);
        sp[0][q] = r;
        sp[1][q] = Uin[N + c] * inv_rho;
        sp[2][q] = Uin[2 * N + c] * inv_rho;
        sp[3][q] = Uin[3 * N + c] * inv_rho;
        sp[4][q] = Uin[4 * N + c] * inv_rho;
    }
    __syncthreads();

    // Phase 2: gradients.
    for (int q = tid; q < TL::NG; q += nthr) {
        const int lx = q % TL::GX, ly = (q / TL::GX) % TL::GY, lz = q / (TL::GX * TL::GY);
        int g[3];
        bool in[3];
        g[0] = gcell(i0 - 1 + lx, 0, in[0]);
        g[1] = gcell(j0 - 1 + ly, 1, in[1]);
        g[2] = gcell(k0 - 1 + lz, 2, in[2]);
        if (!(in[0] && in[1] && in[2])) continue;
        const int pc = TL::pidx(lx + 1, ly + 1, lz + 1);
        const int lpos[3] = {lx + 1, ly + 1, lz + 1};  // positions in the halo lines
        for (int a = 0; a < 3; ++a) {
            const int step = a == 0 ? 1 : (a == 1 ? TL::PX : TL::PX * TL::PY);
            const R iwP = geo(a, kGeoInvW, lpos[a]);
            const bool wlo = !d.periodic[a] && g[a] == 0, whi = !d.periodic[a] && g[a] == n[a] - 1;
            const R ls = geo(a, kGeoLoSelf, lpos[a]), ln = geo(a, kGeoLoNb, lpos[a]);
            const R hs = geo(a, kGeoHiSelf, lpos[a]), hn = geo(a, kGeoHiNb, lpos[a]);
#pragma unroll
            for (int p = 0; p < NPRIM; ++p) {
                const R vP = sp[p][pc];
                auto wallv = [&](int side) -> R {
                    if (p == 0) return vP;
                    if (p < 4) return (R)0;
                    return d.kind[side] == kIsothermal ? (R)d.Tw[side] : vP;
                };
                // Eq. 56 face values with precomputed inverse-distance weights
                const R flo = wlo ? wallv(2 * a) : vP * ls + sp[p][pc - step] * ln;
                const R fhi = whi ? wallv(2 * a + 1) : vP * hs + sp[p][pc + step] * hn;
                sg[p][a][q] = (fhi - flo) * iwP;
            }
        }
    }
    __syncthreads();

    // Phase 3: faces of the three axes (one thread per face; the axis is a
    // compile-time constant inside face_axis, so no private array is indexed
    // at run time).
    auto face_axis = [&](auto AXC, int qq) {
        constexpr int AX = decltype(AXC)::value;
        constexpr int T1 = AX == 0 ? 1 : 0, T2 = AX == 2 ? 1 : 2;  // tangents in increasing order
        constexpr int FX = AX == 0 ? TX + 1 : TX, FY = AX == 1 ? TY + 1 : TY;
        int f[3];
        f[0] = qq % FX;
        f[1] = (qq / FX) % FY;
        f[2] = qq / (FX * FY);
        if (org[0] + f[0] > n[0] - (AX == 0 ? 0 : 1)) return;
        if (org[1] + f[1] > n[1] - (AX == 1 ? 0 : 1)) return;
        if (org[2] + f[2] > n[2] - (AX == 2 ? 0 : 1)) return;
        const int gf = org[AX] + f[AX];
        const R area = geo(T1, kGeoW, f[T1] + 2) * geo(T2, kGeoW, f[T2] + 2);
        int cL[3] = {f[0], f[1], f[2]};
        cL[AX] -= 1;
        R F[5];
        if (!d.periodic[AX] && (gf == 0 || gf == n[AX])) {
            const int side = 2 * AX + (gf == 0 ? 0 : 1);
            const int wx = gf == 0 ? f[0] : cL[0], wy = gf == 0 ? f[1] : cL[1], wz = gf == 0 ? f[2] : cL[2];
            const int wa = AX == 0 ? wx : (AX == 1 ? wy : wz);
            const int pc = TL::pidx(wx + 2, wy + 2, wz + 2);
            const R sgn = gf == 0 ? (R)-1 : (R)1;
            const R rP = sp[0][pc];
            const R rho = DEV ? (R)1 + rP : rP;
            const R d_w = (R)0.5 * geo(AX, kGeoW, wa + 2);
            const R mloc[3] = {rho * sp[1 + AX][pc], rho * sp[1 + T1][pc], rho * sp[1 + T2][pc]};
            R G[5];
            wall_flux<R, 3, DEV>(rP, mloc, rho * sp[4][pc], sgn, d_w, d.kind[side] == kIsothermal, (R)d.Tw[side],
                                 ph, G);
            F[0] = G[0];
            F[1 + AX] = G[1];
            F[1 + T1] = G[2];
            F[1 + T2] = G[3];
            F[4] = G[4];
        } else {
            Side<R, 3> A, B;
            const int pL = TL::pidx(cL[0] + 2, cL[1] + 2, cL[2] + 2), pR = TL::pidx(f[0] + 2, f[1] + 2, f[2] + 2);
            const int gL = TL::gidx(cL[0] + 1, cL[1] + 1, cL[2] + 1), gR = TL::gidx(f[0] + 1, f[1] + 1, f[2] + 1);
            // local primitive order: r, u_n, u_t1, u_t2, T; local axes n, t1, t2
            constexpr int pmap[5] = {0, 1 + AX, 1 + T1, 1 + T2, 4};
            constexpr int amap[3] = {AX, T1, T2};
#pragma unroll
            for (int p = 0; p < 5; ++p) {
                A.v[p] = sp[pmap[p]][pL];
                B.v[p] = sp[pmap[p]][pR];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    A.g[k][p] = sg[pmap[p]][amap[k]][gL];
                    B.g[k][p] = sg[pmap[p]][amap[k]][gR];
                }
            }
            const R dL = (R)0.5 * geo(AX, kGeoW, cL[AX] + 2);
            const R dR = (R)0.5 * geo(AX, kGeoW, f[AX] + 2);
            R fdir[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) fdir[k] = (d.force_pred && d.gaxis == amap[k]) ? (R)1 : (R)0;
            R G[5];
            face_flux<R, 3, DEV>(A, B, dL, dR, fdir, ph, G);
            F[0] = G[0];
            F[1 + AX] = G[1];
            F[1 + T1] = G[2];
            F[1 + T2] = G[3];
            F[4] = G[4];
        }
        if (AX == 0) {
            const int o = (f[2] * TY + f[1]) * (TX + 1) + f[0];
#pragma unroll
            for (int k = 0; k < 5; ++k) sf0[k][o] = F[k] * area;
        } else if (AX == 1) {
            const int o = (f[2] * (TY + 1) + f[1]) * TX + f[0];
#pragma unroll
            for (int k = 0; k < 5; ++k) sf1[k][o] = F[k] * area;
        } else {
            const int o = (f[2] * TY + f[1]) * TX + f[0];
#pragma unroll
            for (int k = 0; k < 5; ++k) sf2[k][o] = F[k] * area;
        }
    };
    for (int q = tid; q < TL::NF0 + TL::NF1 + TL::NF2; q += nthr) {
        if (q < TL::NF0) face_axis(std::integral_constant<int, 0>{}, q);
        else if (q < TL::NF0 + TL::NF1) face_axis(std::integral_constant<int, 1>{}, q - TL::NF0);
        else face_axis(std::integral_constant<int, 2>{}, q - TL::NF0 - TL::NF1);
    }
    __syncthreads();

    // Phase 4: update.
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const R dtR = (R)d.dt;
    for (int q = tid; q < TX * TY * TZ; q += nthr) {
        const int x = q % TX, y = (q / TX) % TY, z = q / (TX * TY);
        const int gx = i0 + x, gy = j0 + y, gz = k0 + z;
        if (gx >= n[0] || gy >= n[1] || gz >= n[2]) continue;
        const int64_t c = ((int64_t)gz * n[1] + gy) * n[0] + gx;
        const R dt_dV = dtR * sgeo0[kGeoInvW][x + 2] * sgeo1[kGeoInvW][y + 2] * sgeo2[kGeoInvW][z + 2];
        const int o0 = (z * TY + y) * (TX + 1) + x;
        const int o1 = (z * (TY + 1) + y) * TX + x;
        const int o2 = (z * TY + y) * TX + x;
        const int pc = TL::pidx(x + 2, y + 2, z + 2);
        const R rP = sp[0][pc];
        const R rhoP = DEV ? (R)1 + rP : rP;
        const R TP = sp[4][pc];
        R Un[5];
        if (sizeof(R) == 4 && d.sround) {
            R inc[5];
#pragma unroll
            for (int k = 0; k < 5; ++k)
                inc[k] = dt_dV * ((sf0[k][o0] - sf0[k][o0 + 1]) + (sf1[k][o1] - sf1[k][o1 + TX]) +
                                  (sf2[k][o2] - sf2[k][o2 + TX * TY]));
            if (d.gaxis >= 0) inc[1 + d.gaxis] += dtR * (R)d.bg * rhoP * (DEV ? TP : TP - (R)kT0);
#pragma unroll
            for (int k = 0; k < 5; ++k) Un[k] = sr_add(Uin[k * N + c], inc[k], sr_hash((uint32_t)c, step_key * 5u + k));
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const R div = (sf0[k][o0] - sf0[k][o0 + 1]) + (sf1[k][o1] - sf1[k][o1 + TX]) +
                              (sf2[k][o2] - sf2[k][o2 + TX * TY]);
                Un[k] = Uin[k * N + c] + dt_dV * div;
            }
            if (d.gaxis >= 0) Un[1 + d.gaxis] += dtR * (R)d.bg * rhoP * (DEV ? TP : TP - (R)kT0);
        }
#pragma unroll
        for (int k = 0; k < 5; ++k) Uout[k * N + c] = Un[k];
        if (RES) {
            const double rn = (double)Un[0];
            const double rhon = DEV ? 1.0 + rn : rn;
            double an = 0.0, ao = 0.0;
            for (int a = 0; a < 3; ++a) {
                const double un = (double)Un[1 + a] / rhon, uo = (double)sp[1 + a][pc];
                an += un * un;
                ao += uo * uo;
            }
            const double Tn = (double)Un[4] / rhon + (DEV ? kT0 : 0.0);
            const double To = (double)TP + (DEV ? kT0 : 0.0);
            const bool ok = (an < 0.25 * kCs2) && (Tn == Tn) && (fabs(Tn) < 1e30);
            an = sqrt(an);
            ao = sqrt(ao);
            acc[0] += fabs(an - ao);
            acc[1] += an;
            acc[2] += fabs(Tn - To);
            acc[3] += Tn;
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
