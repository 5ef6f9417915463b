// step3d.h -- one fused RTLBFS step over a TX x TY x TZ tile of a 3D domain
// (D3Q19 face lattice).  Same phases as the 2D tile: LDS-staged primitives
// with a 2-cell halo, Eq. 55 gradients with a 1-cell halo, every face of the
// tile once (RTLBFS or, when TL, TLBFS lattice flux, or the wall closure)
// into LDS, then the divergence, buoyancy and forward-Euler update with
// optional FP64 Eq. 65 partial sums.  As in 2D, the faces of all three axes
// run one code path (the face frame is chosen per lane through LDS addresses
// and selects, never by indexing a private array at run time), and neighbour
// values are read without branches.
#pragma once

#include "rtlbfs_device.h"

namespace rtlbfs {

template <int TX, int TY, int TZ>
struct Tile3 {
    static constexpr int PX = TX + 4, PY = TY + 4, PZ = TZ + 4;
    static constexpr int GX = TX + 2, GY = TY + 2, GZ = TZ + 2;
    static constexpr int NP = PX * PY * PZ;
    static constexpr int NG = GX * GY * GZ;
    static constexpr int NC = TX * TY * TZ;
    // faces normal to axis a: (T[a] + 1) along a, T elsewhere; stored in
    // this order, each block x-fastest
    static constexpr int NF0 = (TX + 1) * TY * TZ, NF1 = TX * (TY + 1) * TZ, NF2 = TX * TY * (TZ + 1);
    static constexpr int NF = NF0 + NF1 + NF2;
    static constexpr int GEO = PX + PY + PZ;  // halo lines of the three axes, concatenated
    __device__ static int pidx(int x, int y, int z) { return (z * PY + y) * PX + x; }  // cell at tile coords - 2
    __device__ static int gidx(int x, int y, int z) { return (z * GY + y) * GX + x; }  // cell at tile coords - 1
};

// One thread per face of the tile, rounded up to whole wavefronts.
template <int TX, int TY, int TZ>
constexpr int tile3_threads() {
    return (((TX + 1) * TY * TZ + TX * (TY + 1) * TZ + TX * TY * (TZ + 1)) + 63) / 64 * 64;
}

// Eq. 55 gradient of the five primitives (r, u_x, u_y, u_z, T) along one
// axis: (phi_hi - phi_lo) / width with the Eq. 56 face values
// phi_lo = ls phi_P + ln phi_{P-1} and phi_hi = hs phi_P + hn phi_{P+1}; a
// wall face takes r_S = r_P, u_S = 0 and T_S = Tw (Tlo / Thi: the wall
// temperature if isothermal, else T_P).  Shared by the 3D step kernels so
// they produce the same bits.
template <typename R>
__device__ __forceinline__ void grad_axis3(const R (&vP)[5], const R (&vlo)[5], const R (&vhi)[5], R ls, R ln, R hs,
                                           R hn, R iwP, bool wlo, bool whi, R Tlo, R Thi, R (&g)[5]) {
#pragma unroll
    for (int p = 0; p < 5; ++p) {
        const R flo0 = vP[p] * ls + vlo[p] * ln, fhi0 = vP[p] * hs + vhi[p] * hn;
        const R zlo = p == 0 ? vP[0] : (p == 4 ? Tlo : (R)0);
        const R zhi = p == 0 ? vP[0] : (p == 4 ? Thi : (R)0);
        const R flo = wlo ? zlo : flo0, fhi = whi ? zhi : fhi0;
        g[p] = (fhi - flo) * iwP;
    }
}

// Flux divergence, Boussinesq source and forward-Euler update of one cell
// (Eqs. 57-59, 64): U^{n+1} = U^n + dt/dV [(F_w - F_e) + (F_s - F_n) +
// (F_b - F_t)] + dt beta_g rho (T - T_ref) along gravity, where F_w ... F_t
// are the area-weighted fluxes of its west, east, south, north, bottom and
// top faces.  FP32 with stochastic rounding adds the increment in one
// rounding keyed by (cell, step, field).  Shared by the 3D step kernels.
template <typename R, bool DEV>
__device__ __forceinline__ void update_cell3(const Domain &d, const Phys<R> &ph, const R (&sc)[5], const R (&fw)[5],
                                             const R (&fe)[5], const R (&fs)[5], const R (&fn)[5], const R (&fb)[5],
                                             const R (&ft)[5], R dt_dV, R rhoP, R TP, int64_t c, uint32_t step_key,
                                             R (&Un)[5]) {
    const R dtR = ph.dt;
    if (sizeof(R) == 4 && d.sround) {
        R inc[5];
#pragma unroll
        for (int k = 0; k < 5; ++k) inc[k] = dt_dV * ((fw[k] - fe[k]) + (fs[k] - fn[k]) + (fb[k] - ft[k]));
        if (d.gaxis >= 0) inc[1 + d.gaxis] += dtR * ph.bg * rhoP * (DEV ? TP : TP - (R)kT0);
#pragma unroll
        for (int k = 0; k < 5; ++k) Un[k] = sr_add(sc[k], inc[k], sr_hash((uint32_t)c, step_key * 5u + k));
    } else {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const R div = (fw[k] - fe[k]) + (fs[k] - fn[k]) + (fb[k] - ft[k]);
            Un[k] = sc[k] + dt_dV * div;
        }
        if (d.gaxis >= 0) Un[1 + d.gaxis] += dtR * ph.bg * rhoP * (DEV ? TP : TP - (R)kT0);
    }
}

template <typename R, bool DEV, int TX, int TY, int TZ, bool RES, bool TL>
__device__ __forceinline__ void tile_step_3d(const Domain &d, int i0, int j0, int k0, const R *__restrict__ Uin,
                                             R *__restrict__ Uout, double *__restrict__ part, uint32_t step_key) {
    using TT = Tile3<TX, TY, TZ>;
    constexpr int NPRIM = 5;
    constexpr int NT = tile3_threads<TX, TY, TZ>();
    constexpr int NIT = (TT::NP + NT - 1) / NT;  // passes of the load phase
    static_assert(TT::NG <= NT && TT::NF <= NT && TT::NC <= NT && TT::GEO <= NT,
                  "gradient, face and update phases are one pass of the block");
    __shared__ R sp[NPRIM][TT::NP];
    __shared__ R sg[NPRIM][3][TT::NG];
    // The face fluxes reuse the gradients' LDS: every face has read its
    // gradients before the barrier that precedes the first flux store.  The
    // saving lets a third FP64 4 x 4 x 4 block onto a CU.
    static_assert(TT::NF <= 3 * TT::NG, "the fluxes fit in the gradients' space");
    R(*const sf)[TT::NF] = reinterpret_cast<R(*)[TT::NF]>(&sg[0][0][0]);
    __shared__ R sc[NPRIM][TT::NC];  // old conserved state of the tile cells
    __shared__ R sgeo[kGeoFields][TT::GEO];
    __shared__ double sred[kPartials * 16];
    __shared__ R swT[6];     // wall value of T per side (T_w if isothermal, else unused)
    __shared__ int swIso[6]; // side is an isothermal wall
    constexpr int off1 = TT::PX, off2 = TT::PX + TT::PY;  // start of the y and z halo lines in sgeo

    const int nx = d.n[0], ny = d.n[1], nz = d.n[2];
    const bool px = d.periodic[0], py = d.periodic[1], pz = d.periodic[2];
    const int64_t N = d.fstride;
    const Phys<R> &ph = make_phys<R>(d);
    const int tid = threadIdx.x;
    // a periodic axis at least as long as the tile plus both 2-cell halos wraps by selects
    const bool nearx = nx >= TX + 4, neary = ny >= TY + 4, nearz = nz >= TZ + 4;

    // Phase 1: state of the tile and halo (NIT passes, all loads issued
    // before the first use), then the geometry of the three halo lines.
    {
        R st[NIT][NPRIM];
        bool ld[NIT];
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            const int q = tid + it * NT;
            const int lx = q % TT::PX, ly = (q / TT::PX) % TT::PY, lz = q / (TT::PX * TT::PY);
            int gx = i0 - 2 + lx, gy = j0 - 2 + ly, gz = k0 - 2 + lz;
            if (px) gx = wrap_axis(gx, nx, nearx);
            if (py) gy = wrap_axis(gy, ny, neary);
            if (pz) gz = wrap_axis(gz, nz, nearz);
            ld[it] = q < TT::NP && gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz;
            if (ld[it]) {
                const int64_t c = ((int64_t)gz * ny + gy) * nx + gx;
#pragma unroll
                for (int k = 0; k < NPRIM; ++k) st[it][k] = Uin[k * N + c];
            }
        }
        const int ga = tid < TT::PX ? 0 : (tid < off2 ? 1 : 2);
        const int gl = tid - (ga == 0 ? 0 : (ga == 1 ? off1 : off2));
        const int gn = ga == 0 ? nx : (ga == 1 ? ny : nz);
        int g = (ga == 0 ? i0 : (ga == 1 ? j0 : k0)) - 2 + gl;
        if (ga == 0 ? px : (ga == 1 ? py : pz)) g = wrap_axis(g, gn, nearx && neary && nearz);  // one choice
        const bool lg = tid < TT::GEO && g >= 0 && g < gn;
        R gv[kGeoFields];
        if (lg) {
            const R *src = (const R *)(ga == 0 ? d.geo[0] : (ga == 1 ? d.geo[1] : d.geo[2]));
#pragma unroll
            for (int k = 0; k < kGeoFields; ++k) gv[k] = src[k * gn + g];
        }
#pragma unroll
        for (int it = 0; it < NIT; ++it) {
            if (!ld[it]) continue;
            const int q = tid + it * NT;
            const int lx = q % TT::PX, ly = (q / TT::PX) % TT::PY, lz = q / (TT::PX * TT::PY);
            const R r = st[it][0];
            const R inv_rho = recip<R>(DEV ? (R)1 + r : r);
            sp[0][q] = r;
#pragma unroll
            for (int k = 1; k < NPRIM; ++k) sp[k][q] = st[it][k] * inv_rho;
            const int tx = lx - 2, ty = ly - 2, tz = lz - 2;
            if (tx >= 0 && tx < TX && ty >= 0 && ty < TY && tz >= 0 && tz < TZ) {
                const int o = (tz * TY + ty) * TX + tx;
#pragma unroll
                for (int k = 0; k < NPRIM; ++k) sc[k][o] = st[it][k];
            }
        }
        if (lg) {
#pragma unroll
            for (int k = 0; k < kGeoFields; ++k) sgeo[k][tid] = gv[k];
        }
        // per-side wall data through LDS, so a lane can pick its side by
        // index without a per-lane load from the kernel arguments
        if (tid == 0) {  // compile-time side indices: scalar loads of the arguments
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                swT[k] = wall_T<R>(d, k);
                swIso[k] = d.kind[k] == kIsothermal;
            }
        }
    }
    __syncthreads();

    // Phase 2: gradients, (phi_hi - phi_lo) / width per axis with Eq. 56 face
    // values (wall faces: r_S = r_P, u_S = 0, T_S = T_w if isothermal else
    // T_P).  Halo entries beyond a wall hold no data; they are read but never
    // used.
    if (tid < TT::NG) {
        const int lx = tid % TT::GX, ly = (tid / TT::GX) % TT::GY, lz = tid / (TT::GX * TT::GY);
        int gx = i0 - 1 + lx, gy = j0 - 1 + ly, gz = k0 - 1 + lz;
        if (px) gx = wrap_axis(gx, nx, nearx);
        if (py) gy = wrap_axis(gy, ny, neary);
        if (pz) gz = wrap_axis(gz, nz, nearz);
        if (gx >= 0 && gx < nx && gy >= 0 && gy < ny && gz >= 0 && gz < nz) {
            const int pc = TT::pidx(lx + 1, ly + 1, lz + 1);
            const int gq[3] = {gx, gy, gz};
            const int nq[3] = {nx, ny, nz};
            const bool pq[3] = {px, py, pz};
            const int lpos[3] = {lx + 1, ly + 1 + off1, lz + 1 + off2};  // positions in sgeo
            constexpr int step[3] = {1, TT::PX, TT::PX * TT::PY};
            R vP[NPRIM];
#pragma unroll
            for (int p = 0; p < NPRIM; ++p) vP[p] = sp[p][pc];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const R iwP = sgeo[kGeoInvW][lpos[a]];
                const R ls = sgeo[kGeoLoSelf][lpos[a]], ln = sgeo[kGeoLoNb][lpos[a]];
                const R hs = sgeo[kGeoHiSelf][lpos[a]], hn = sgeo[kGeoHiNb][lpos[a]];
                const bool wlo = !pq[a] && gq[a] == 0, whi = !pq[a] && gq[a] == nq[a] - 1;
                const R Tlo = d.kind[2 * a] == kIsothermal ? wall_T<R>(d, 2 * a) : vP[4];
                const R Thi = d.kind[2 * a + 1] == kIsothermal ? wall_T<R>(d, 2 * a + 1) : vP[4];
                R vlo[NPRIM], vhi[NPRIM], g[NPRIM];
#pragma unroll
                for (int p = 0; p < NPRIM; ++p) {
                    vlo[p] = sp[p][pc - step[a]];
                    vhi[p] = sp[p][pc + step[a]];
                }
                grad_axis3<R>(vP, vlo, vhi, ls, ln, hs, hn, iwP, wlo, whi, Tlo, Thi, g);
#pragma unroll
                for (int p = 0; p < NPRIM; ++p) sg[p][a][tid] = g[p];
            }
        }
    }
    __syncthreads();

    // Phase 3: every face once.  Per lane: normal axis ax with tangents
    // (t1, t2) in increasing order, face coordinates f (the high cell's tile
    // coordinates), and the LDS strides of one step along ax.  The
    // area-weighted flux in global components waits in Fg until every face
    // has read the gradients.
    R Fg[5];
    bool fvalid = false;
    if (tid < TT::NF) {
        const int ax = tid < TT::NF0 ? 0 : (tid < TT::NF0 + TT::NF1 ? 1 : 2);
        const int qq = tid - (ax == 0 ? 0 : (ax == 1 ? TT::NF0 : TT::NF0 + TT::NF1));
        // decompositions with compile-time divisors, then a select
        const int fx = ax == 0 ? qq % (TX + 1) : qq % TX;
        const int fy = ax == 0 ? (qq / (TX + 1)) % TY : (ax == 1 ? (qq / TX) % (TY + 1) : (qq / TX) % TY);
        const int fz = ax == 0 ? qq / ((TX + 1) * TY) : (ax == 1 ? qq / (TX * (TY + 1)) : qq / (TX * TY));
        const int gfx = i0 + fx, gfy = j0 + fy, gfz = k0 + fz;
        const bool valid = gfx <= nx - (ax == 0 ? 0 : 1) && gfy <= ny - (ax == 1 ? 0 : 1) &&
                           gfz <= nz - (ax == 2 ? 0 : 1);
        if (valid) {
            const int gf = ax == 0 ? gfx : (ax == 1 ? gfy : gfz);
            const int fa = ax == 0 ? fx : (ax == 1 ? fy : fz);          // face coordinate along ax
            const int na = ax == 0 ? nx : (ax == 1 ? ny : nz);
            const bool pa = ax == 0 ? px : (ax == 1 ? py : pz);
            const int sP = ax == 0 ? 1 : (ax == 1 ? TT::PX : TT::PX * TT::PY);
            const int sG = ax == 0 ? 1 : (ax == 1 ? TT::GX : TT::GX * TT::GY);
            const int oa = ax == 0 ? 0 : (ax == 1 ? off1 : off2);        // sgeo line of ax
            // tangents: ax 0 -> (y, z), 1 -> (x, z), 2 -> (x, y)
            const int t1 = ax == 0 ? 1 : 0, t2 = ax == 2 ? 1 : 2;
            const int lt1 = ax == 0 ? fy + 2 + off1 : fx + 2;              // sgeo positions of the tangents
            const int lt2 = ax == 2 ? fy + 2 + off1 : fz + 2 + off2;
            const R area = sgeo[kGeoW][lt1] * sgeo[kGeoW][lt2];
            const int pR = TT::pidx(fx + 2, fy + 2, fz + 2), pL = pR - sP;
            // local primitive order: r, u_n, u_t1, u_t2, T
            const int pm[5] = {0, 1 + ax, 1 + t1, 1 + t2, 4};
            R G[5];
            if (!pa && (gf == 0 || gf == na)) {
                const bool low = gf == 0;  // wall on the low side: the fluid cell is the high one
                const int side = 2 * ax + (low ? 0 : 1);
                const int pc = low ? pR : pL;
                const R sgn = low ? (R)-1 : (R)1;
                const R rP = sp[0][pc];
                const R rho = DEV ? (R)1 + rP : rP;
                const R d_w = (R)0.5 * sgeo[kGeoW][oa + (low ? fa + 2 : fa + 1)];
                const R mloc[3] = {rho * sp[pm[1]][pc], rho * sp[pm[2]][pc], rho * sp[pm[3]][pc]};
                wall_flux<R, 3, DEV>(rP, mloc, rho * sp[4][pc], sgn, d_w, swIso[side] != 0, swT[side], ph, G);
            } else {
                Side<R, 3> A, B;
                const int gR = TT::gidx(fx + 1, fy + 1, fz + 1), gL = gR - sG;
                const int am[3] = {ax, t1, t2};
#pragma unroll
                for (int p = 0; p < 5; ++p) {
                    A.v[p] = sp[pm[p]][pL];
                    B.v[p] = sp[pm[p]][pR];
#pragma unroll
                    for (int k = 0; k < 3; ++k) {
                        A.g[k][p] = sg[pm[p]][am[k]][gL];
                        B.g[k][p] = sg[pm[p]][am[k]][gR];
                    }
                }
                const R dL = (R)0.5 * sgeo[kGeoW][oa + fa + 1];
                const R dR = (R)0.5 * sgeo[kGeoW][oa + fa + 2];
                R fdir[3];
#pragma unroll
                for (int k = 0; k < 3; ++k) fdir[k] = (d.force_pred && d.gaxis == am[k]) ? (R)1 : (R)0;
                if constexpr (TL) face_flux_tlbfs<R, 3, DEV>(A, B, dL, dR, fdir, ph, G);
                else face_flux<R, 3, DEV>(A, B, dL, dR, fdir, ph, G);
            }
            // back to global components (mass, m_x, m_y, m_z, energy)
            Fg[0] = G[0] * area;
            Fg[1] = (ax == 0 ? G[1] : G[2]) * area;
            Fg[2] = (ax == 0 ? G[2] : (ax == 1 ? G[1] : G[3])) * area;
            Fg[3] = (ax == 2 ? G[1] : G[3]) * area;
            Fg[4] = G[4] * area;
            fvalid = true;
        }
    }
    __syncthreads();  // gradients read: their space now takes the fluxes
    if (fvalid)
#pragma unroll
        for (int p = 0; p < 5; ++p) sf[p][tid] = Fg[p];
    __syncthreads();

    // Phase 4: divergence, Boussinesq source and update.
    double acc[kPartials] = {0.0, 0.0, 0.0, 0.0, 0.0};
    const R dtR = ph.dt;
    if (tid < TT::NC) {
        const int x = tid % TX, y = (tid / TX) % TY, z = tid / (TX * TY);
        const int gx = i0 + x, gy = j0 + y, gz = k0 + z;
        if (gx < nx && gy < ny && gz < nz) {
            const int64_t c = ((int64_t)gz * ny + gy) * nx + gx;
            const R dt_dV = dtR * sgeo[kGeoInvW][x + 2] * sgeo[kGeoInvW][off1 + y + 2] * sgeo[kGeoInvW][off2 + z + 2];
            const int o0 = (z * TY + y) * (TX + 1) + x;                  // west face
            const int o1 = TT::NF0 + (z * (TY + 1) + y) * TX + x;        // south face
            const int o2 = TT::NF0 + TT::NF1 + (z * TY + y) * TX + x;    // bottom face
            const int pc = TT::pidx(x + 2, y + 2, z + 2);
            const R rP = sp[0][pc];
            const R rhoP = DEV ? (R)1 + rP : rP;
            const R TP = sp[4][pc];
            R Un[5], sc0[5], fw[5], fe[5], fs[5], fn[5], fb[5], ft[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                sc0[k] = sc[k][tid];
                fw[k] = sf[k][o0];
                fe[k] = sf[k][o0 + 1];
                fs[k] = sf[k][o1];
                fn[k] = sf[k][o1 + TX];
                fb[k] = sf[k][o2];
                ft[k] = sf[k][o2 + TX * TY];
            }
            update_cell3<R, DEV>(d, ph, sc0, fw, fe, fs, fn, fb, ft, dt_dV, rhoP, TP, c, step_key, Un);
#pragma unroll
            for (int k = 0; k < 5; ++k) Uout[k * N + c] = Un[k];
            if (RES) {
                const double rn = (double)Un[0];
                const double rhon = DEV ? 1.0 + rn : rn;
                double an = 0.0, ao = 0.0;
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const double un = (double)Un[1 + a] / rhon, uo = (double)sp[1 + a][pc];
                    an += un * un;
                    ao += uo * uo;
                }
                const double Tn = (double)Un[4] / rhon + (DEV ? kT0 : 0.0);
                const double To = (double)TP + (DEV ? kT0 : 0.0);
                const bool ok = (an < d.guard_u2) && (Tn == Tn) && (fabs(Tn) < 1e30);
                an = sqrt(an);
                ao = sqrt(ao);
                acc[0] += fabs(an - ao);
                acc[1] += an;
                acc[2] += fabs(Tn - To);
                acc[3] += Tn;
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
