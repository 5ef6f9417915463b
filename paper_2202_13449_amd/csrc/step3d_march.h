// step3d_march.h -- one fused RTLBFS step of a 3D domain by columns: a block
// owns a TX x TY column of cells and marches along z through a segment of
// planes (2.5-D blocking), so each face of the segment is computed once.
//
// Per plane z the block keeps in LDS the primitives of planes z, z+1 and
// z+2 (a ring of three, each with a 2-cell halo in x and y), the Eq. 55
// gradients of planes z and z+1 (a ring of two, 1-cell halo) and the flux
// of the z-faces below plane z (carried from the previous plane).  One
// plane costs three barriers:
//   A  stage plane z+2 (fetched during the previous plane) and fetch z+3;
//   G  gradients of plane z+1;
//   F  x- and y-faces of plane z and the z-faces between z and z+1;
//   U  divergence, buoyancy and update of plane z, store.
// The conserved state of a tile cell waits in LDS, written and read only by
// the thread that loads and updates that cell, so U reads no primitive of
// another thread and needs no barrier before the next A.
//
// The per-face and per-cell arithmetic is that of the 4x4x4 tile kernel
// (face_flux / face_flux_tlbfs / wall_flux with the same inputs,
// grad_axis3, update_cell3): both give the same bits.  A segment of SZ
// planes computes SZ + 1 planes of z-faces; x and y faces on the column's
// sides are computed by both neighbouring columns.
#pragma once

#include "rtlbfs_device.h"
#include "step3d.h"

namespace rtlbfs {

template <int TX, int TY>
struct Col3 {
    static constexpr int PX = TX + 4, PY = TY + 4;  // primitives plane, 2-cell halo
    static constexpr int GX = TX + 2, GY = TY + 2;  // gradients plane, 1-cell halo
    static constexpr int NP = PX * PY, NG = GX * GY, NC = TX * TY;
    static constexpr int NF0 = (TX + 1) * TY, NF1 = TX * (TY + 1);  // x- and y-faces of a plane
    static constexpr int NFXY = NF0 + NF1;
    static constexpr int NFACE = NFXY + NC;  // and the z-faces above the plane
    static constexpr int NT = (NFACE + 63) / 64 * 64;
    static constexpr int GEO = PX + PY;
};

template <int TX, int TY>
constexpr int col3_threads() {
    return Col3<TX, TY>::NT;
}

// Position (lx, ly) in the primitives plane of load slot q: the tile cells
// first (q < TX*TY, so the loading thread of a tile cell is the thread that
// updates it), then the 2-cell halo ring: two full rows below, two above,
// then two cells on each side of every tile row.
template <int TX, int TY>
__device__ __forceinline__ void col3_load_pos(int q, int &lx, int &ly) {
    using C = Col3<TX, TY>;
    if (q < C::NC) {
        lx = 2 + q % TX;
        ly = 2 + q / TX;
        return;
    }
    const int r = q - C::NC;
    if (r < 2 * C::PX) {
        lx = r % C::PX;
        ly = r / C::PX;
    } else if (r < 4 * C::PX) {
        const int r2 = r - 2 * C::PX;
        lx = r2 % C::PX;
        ly = C::PY - 2 + r2 / C::PX;
    } else {
        const int r3 = r - 4 * C::PX;
        const int k = r3 & 3;
        ly = 2 + (r3 >> 2);
        lx = k < 2 ? k : C::PX - 4 + k;
    }
}

template <typename R, bool DEV, int TX, int TY, bool RES, bool TL>
__device__ __forceinline__ void column_step_3d(const Domain &d, int i0, int j0, int z0, int z1,
                                               const R *__restrict__ Uin, R *__restrict__ Uout,
                                               double *__restrict__ part, uint32_t step_key) {
    using C = Col3<TX, TY>;
    constexpr int NT = C::NT;
    static_assert(C::NP <= NT && C::NG <= NT && C::GEO <= NT, "load, gradient and geometry phases are one pass");
    __shared__ R sp[3][5][C::NP];      // primitives r, u_x, u_y, u_z, T of three planes
    __shared__ R sg[2][5][3][C::NG];   // their gradients along x, y, z, two planes
    __shared__ R sfz[2][5][C::NC];     // area-weighted z-face fluxes below and above the plane
    __shared__ R sfxy[5][C::NFXY];     // area-weighted x- and y-face fluxes of the plane
    // Conserved state of the tile cells, planes z, z + 1, z + 2 (ring), and
    // the Eq. 65 partial sums of each tile cell's thread.  Each entry is
    // written and read only by the thread that loads and updates that cell.
    __shared__ R scons[3][5][C::NC];
    __shared__ double sacc[RES ? kPartials : 1][RES ? C::NC : 1];
    __shared__ R sgeo[kGeoFields][C::GEO];
    __shared__ double sred[kPartials * (NT / 64)];
    __shared__ R swT[6];
    __shared__ int swIso[6];
    constexpr int offy = C::PX;  // start of the y halo line in sgeo

    const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const bool px = d.periodic[0], py = d.periodic[1], pz = d.periodic[2];
    const int64_t N = d.fstride;
    const int64_t nxy = (int64_t)nx * ny;
    const Phys<R> &ph = make_phys<R>(d);
    const R *__restrict__ geoz = (const R *)d.geo[2];
    const int tid = threadIdx.x;
    const bool nearx = nx >= TX + 4, neary = ny >= TY + 4;

    // plane index after the periodic wrap, or -1 beyond a z wall
    auto zplane = [&](int p) { return pz ? wrap(p, nz) : ((p >= 0 && p < nz) ? p : -1); };
    // z geometry record k of plane p (uniform over the block)
    auto zgeo = [&](int k, int p) { return geoz[(int64_t)k * nz + p]; };

    // Loader role: one position of the primitives plane per thread.
    int lx = 0, ly = 0;
    const bool loader = tid < C::NP;
    if (loader) col3_load_pos<TX, TY>(tid, lx, ly);
    int gxl = i0 - 2 + lx, gyl = j0 - 2 + ly;
    if (px) gxl = wrap_axis(gxl, nx, nearx);
    if (py) gyl = wrap_axis(gyl, ny, neary);
    const bool lin = loader && gxl >= 0 && gxl < nx && gyl >= 0 && gyl < ny;
    const int64_t cxy = (int64_t)gyl * nx + gxl;
    const int lpos = ly * C::PX + lx;

    R st[5];
    auto fetch = [&](int p) {
        const int q = zplane(p);
        if (lin && q >= 0) {
            const int64_t c = (int64_t)q * nxy + cxy;
#pragma unroll
            for (int k = 0; k < 5; ++k) st[k] = Uin[k * N + c];
        }
    };
    auto stage = [&](int slot, int p) {
        if (lin && zplane(p) >= 0) {
            const R r = st[0];
            const R inv_rho = recip<R>(DEV ? (R)1 + r : r);
            sp[slot][0][lpos] = r;
#pragma unroll
            for (int k = 1; k < 5; ++k) sp[slot][k][lpos] = st[k] * inv_rho;
        }
    };
    // rings: primitives slot of plane p, gradients slot of plane p, z-flux
    // slot of the face above plane p
    auto pslot = [&](int p) { return (p - z0 + 2) % 3; };
    auto gslot = [&](int p) { return (p - z0 + 1) & 1; };

    // Gradients of plane p (1-cell halo) from the primitives of planes p-1,
    // p and p+1; t is the thread index.
    auto gradients = [&](int p, int t) {
        const int q = zplane(p);
        if (t >= C::NG || q < 0) return;
        const int gx_ = t % C::GX, gy_ = t / C::GX;
        int gx = i0 - 1 + gx_, gy = j0 - 1 + gy_;
        if (px) gx = wrap_axis(gx, nx, nearx);
        if (py) gy = wrap_axis(gy, ny, neary);
        if (gx < 0 || gx >= nx || gy < 0 || gy >= ny) return;
        const int pc = (gy_ + 1) * C::PX + gx_ + 1;
        const int s0 = pslot(p), smm = (s0 + 2) % 3, spp = (s0 + 1) % 3;  // planes p, p - 1, p + 1
        const int gs = gslot(p);
        R vP[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) vP[k] = sp[s0][k][pc];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            R iwP, ls, ln, hs, hn;
            bool wlo, whi;
            R vlo[5], vhi[5], g[5];
            if (a < 2) {
                const int lp = a == 0 ? gx_ + 1 : offy + gy_ + 1;  // geometry line position of the cell
                iwP = sgeo[kGeoInvW][lp];
                ls = sgeo[kGeoLoSelf][lp];
                ln = sgeo[kGeoLoNb][lp];
                hs = sgeo[kGeoHiSelf][lp];
                hn = sgeo[kGeoHiNb][lp];
                const int gq = a == 0 ? gx : gy, nq = a == 0 ? nx : ny;
                const bool pq = a == 0 ? px : py;
                wlo = !pq && gq == 0;
                whi = !pq && gq == nq - 1;
                const int st_ = a == 0 ? 1 : C::PX;
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    vlo[k] = sp[s0][k][pc - st_];
                    vhi[k] = sp[s0][k][pc + st_];
                }
            } else {
                iwP = zgeo(kGeoInvW, q);
                ls = zgeo(kGeoLoSelf, q);
                ln = zgeo(kGeoLoNb, q);
                hs = zgeo(kGeoHiSelf, q);
                hn = zgeo(kGeoHiNb, q);
                wlo = !pz && q == 0;
                whi = !pz && q == nz - 1;
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    vlo[k] = sp[smm][k][pc];
                    vhi[k] = sp[spp][k][pc];
                }
            }
            const R Tlo = d.kind[2 * a] == kIsothermal ? wall_T<R>(d, 2 * a) : vP[4];
            const R Thi = d.kind[2 * a + 1] == kIsothermal ? wall_T<R>(d, 2 * a + 1) : vP[4];
            grad_axis3<R>(vP, vlo, vhi, ls, ln, hs, hn, iwP, wlo, whi, Tlo, Thi, g);
#pragma unroll
            for (int k = 0; k < 5; ++k) sg[gs][k][a][t] = g[k];
        }
    };

    // ---------------------------------------------------------- set-up --
    if (tid < C::GEO) {
        const bool isx = tid < C::PX;
        const int gl = isx ? tid : tid - C::PX;
        const int gn = isx ? nx : ny;
        int g = (isx ? i0 : j0) - 2 + gl;
        if (isx ? px : py) g = wrap_axis(g, gn, nearx && neary);
        if (g >= 0 && g < gn) {
            const R *src = (const R *)(isx ? d.geo[0] : d.geo[1]);
#pragma unroll
            for (int k = 0; k < kGeoFields; ++k) sgeo[k][tid] = src[k * gn + g];
        }
    }
    if (tid == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            swT[k] = wall_T<R>(d, k);
            swIso[k] = d.kind[k] == kIsothermal;
        }
    }
    if (RES && tid < C::NC)
#pragma unroll
        for (int k = 0; k < kPartials; ++k) sacc[k][tid] = 0.0;
    fetch(z0 - 2);
    stage(pslot(z0 - 2), z0 - 2);
    fetch(z0 - 1);
    stage(pslot(z0 - 1), z0 - 1);
    fetch(z0);

    // ---------------------------------------------------------- march --
    // Iteration z stages plane z + 2, computes the gradients of plane z + 1,
    // the faces of plane z and the z-faces above it, and updates plane z.
    // The loop starts two planes early: z0 - 2 only stages and computes the
    // gradients of z0 - 1, z0 - 1 adds the z-faces below the segment.
    const R dtR = ph.dt;
    for (int z = z0 - 2; z < z1; ++z) {
        // The thread index, made opaque each plane: the index arithmetic and
        // the x / y geometry reads below do not depend on z, and hoisting them
        // out of the loop would keep them live through the face arithmetic.
        int lt = tid;
        asm volatile("" : "+v"(lt));
        // A: plane z + 2 (fetched during the previous plane) into the ring
        stage(pslot(z + 2), z + 2);
        if (lt < C::NC)
#pragma unroll
            for (int k = 0; k < 5; ++k) scons[pslot(z + 2)][k][lt] = st[k];
        fetch(z + 3);
        __syncthreads();
        // G
        gradients(z + 1, lt);
        __syncthreads();
        // F: one face per thread: x- and y-faces of plane z (when z is in the
        // segment), then the z-face above tile cell lt - NFXY.
        if (z >= z0 - 1 && lt < C::NFACE && (z >= z0 || lt >= C::NFXY)) {
            const bool isz = lt >= C::NFXY;
            const bool isx = lt < C::NF0;
            const int ax = isz ? 2 : (isx ? 0 : 1);
            const int qq = isz ? lt - C::NFXY : (isx ? lt : lt - C::NF0);
            const int fx = isx ? qq % (TX + 1) : qq % TX;
            const int fy = isx ? qq / (TX + 1) : qq / TX;
            const int gfx = i0 + fx, gfy = j0 + fy;
            const bool valid = isz ? (gfx < nx && gfy < ny)
                                   : (isx ? (gfx <= nx && gfy < ny) : (gfx < nx && gfy <= ny));
            if (valid) {
                const int pR = (fy + 2) * C::PX + fx + 2, pL = isz ? pR : pR - (isx ? 1 : C::PX);
                const int gR = (fy + 1) * C::GX + fx + 1, gL = isz ? gR : gR - (isx ? 1 : C::GX);
                const int sL = pslot(z), sR = isz ? pslot(z + 1) : sL;
                const int gLs = gslot(z), gRs = isz ? gslot(z + 1) : gLs;
                const int q = zplane(z), q1 = zplane(z + 1);
                bool wall, low;
                R area, dL, dR;
                if (isz) {
                    wall = q < 0 || q1 < 0;  // below the first plane or above the last
                    low = q < 0;
                    area = sgeo[kGeoW][fx + 2] * sgeo[kGeoW][offy + fy + 2];
                    dL = q >= 0 ? (R)0.5 * zgeo(kGeoW, q) : (R)0;
                    dR = q1 >= 0 ? (R)0.5 * zgeo(kGeoW, q1) : (R)0;
                } else {
                    const int gf = isx ? gfx : gfy, na = isx ? nx : ny;
                    const bool pa = isx ? px : py;
                    wall = !pa && (gf == 0 || gf == na);
                    low = gf == 0;
                    const int fa = isx ? fx : fy, oa = isx ? 0 : offy;
                    // the two tangential widths in (t1, t2) order
                    area = (isx ? sgeo[kGeoW][offy + fy + 2] : sgeo[kGeoW][fx + 2]) * zgeo(kGeoW, q);
                    dL = (R)0.5 * sgeo[kGeoW][oa + fa + 1];
                    dR = (R)0.5 * sgeo[kGeoW][oa + fa + 2];
                }
                const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
                const int pm[5] = {0, 1 + ax, 1 + t1, 1 + t2, 4};
                R G[5];
                if (wall) {
                    const int side = 2 * ax + (low ? 0 : 1);
                    const int sc_ = low ? sR : sL, pc = low ? pR : pL;
                    const R sgn = low ? (R)-1 : (R)1;
                    const R rP = sp[sc_][0][pc];
                    const R rho = DEV ? (R)1 + rP : rP;
                    const R d_w = low ? dR : dL;
                    const R mloc[3] = {rho * sp[sc_][pm[1]][pc], rho * sp[sc_][pm[2]][pc], rho * sp[sc_][pm[3]][pc]};
                    wall_flux<R, 3, DEV>(rP, mloc, rho * sp[sc_][4][pc], sgn, d_w, swIso[side] != 0, swT[side], ph,
                                         G);
                } else {
                    Side<R, 3> A, B;
                    const int am[3] = {ax, t1, t2};
#pragma unroll
                    for (int p = 0; p < 5; ++p) {
                        A.v[p] = sp[sL][pm[p]][pL];
                        B.v[p] = sp[sR][pm[p]][pR];
#pragma unroll
                        for (int k = 0; k < 3; ++k) {
                            A.g[k][p] = sg[gLs][pm[p]][am[k]][gL];
                            B.g[k][p] = sg[gRs][pm[p]][am[k]][gR];
                        }
                    }
                    R fdir[3];
#pragma unroll
                    for (int k = 0; k < 3; ++k) fdir[k] = (d.force_pred && d.gaxis == am[k]) ? (R)1 : (R)0;
                    if constexpr (TL) face_flux_tlbfs<R, 3, DEV>(A, B, dL, dR, fdir, ph, G);
                    else face_flux<R, 3, DEV>(A, B, dL, dR, fdir, ph, G);
                }
                // back to global components (mass, m_x, m_y, m_z, energy), area-weighted
                R Fg[5];
                Fg[0] = G[0] * area;
                Fg[1] = (ax == 0 ? G[1] : G[2]) * area;
                Fg[2] = (ax == 0 ? G[2] : (ax == 1 ? G[1] : G[3])) * area;
                Fg[3] = (ax == 2 ? G[1] : G[3]) * area;
                Fg[4] = G[4] * area;
                if (isz) {
#pragma unroll
                    for (int k = 0; k < 5; ++k) sfz[gslot(z)][k][qq] = Fg[k];
                } else {
#pragma unroll
                    for (int k = 0; k < 5; ++k) sfxy[k][lt] = Fg[k];
                }
            }
        }
        __syncthreads();
        // U: tile cell lt of plane z
        if (z >= z0 && lt < C::NC) {
            const int x = lt % TX, y = lt / TX;
            const int gx = i0 + x, gy = j0 + y;
            if (gx < nx && gy < ny) {
                const int64_t c = (int64_t)z * nxy + (int64_t)gy * nx + gx;
                const R dt_dV = dtR * sgeo[kGeoInvW][x + 2] * sgeo[kGeoInvW][offy + y + 2] * zgeo(kGeoInvW, z);
                const int o0 = y * (TX + 1) + x;
                const int o1 = C::NF0 + y * TX + x;
                R U0[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) U0[k] = scons[pslot(z)][k][lt];
                const R rP = U0[0];
                const R rhoP = DEV ? (R)1 + rP : rP;
                const R inv_rho = recip<R>(rhoP);
                const R TP = U0[4] * inv_rho;
                R Un[5], fw[5], fe[5], fs[5], fn[5], fb[5], ft[5];
#pragma unroll
                for (int k = 0; k < 5; ++k) {
                    fw[k] = sfxy[k][o0];
                    fe[k] = sfxy[k][o0 + 1];
                    fs[k] = sfxy[k][o1];
                    fn[k] = sfxy[k][o1 + TX];
                    fb[k] = sfz[gslot(z - 1)][k][lt];
                    ft[k] = sfz[gslot(z)][k][lt];
                }
                update_cell3<R, DEV>(d, ph, U0, fw, fe, fs, fn, fb, ft, dt_dV, rhoP, TP, c, step_key, Un);
#pragma unroll
                for (int k = 0; k < 5; ++k) Uout[k * N + c] = Un[k];
                if (RES) {
                    const double rn = (double)Un[0];
                    const double rhon = DEV ? 1.0 + rn : rn;
                    double an = 0.0, ao = 0.0;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const double un = (double)Un[1 + a] / rhon, uo = (double)(U0[1 + a] * inv_rho);
                        an += un * un;
                        ao += uo * uo;
                    }
                    const double Tn = (double)Un[4] / rhon + (DEV ? kT0 : 0.0);
                    const double To = (double)TP + (DEV ? kT0 : 0.0);
                    const bool ok = (an < d.guard_u2) && (Tn == Tn) && (fabs(Tn) < 1e30);
                    an = sqrt(an);
                    ao = sqrt(ao);
                    sacc[0][lt] += fabs(an - ao);
                    sacc[1][lt] += an;
                    sacc[2][lt] += fabs(Tn - To);
                    sacc[3][lt] += Tn;
                    sacc[4][lt] += ok ? 0.0 : 1.0;
                }
            }
        }
    }
    if (RES) {
        double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
        if (tid < C::NC)
#pragma unroll
            for (int k = 0; k < kPartials; ++k) acc[k] = sacc[k][tid];
        block_sums<kPartials>(acc, sred);
        if (tid == 0)
            for (int k = 0; k < kPartials; ++k) part[k] = acc[k];
    }
}

}  // namespace rtlbfs
