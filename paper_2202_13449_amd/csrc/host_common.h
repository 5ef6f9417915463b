// host_common.h -- host-side helpers shared by the single-domain and batched
// runtimes: SplitMix64 noise, Eq. 74 mesh, storage sizes.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstddef>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rtlbfs.h"
#include "rtlbfs_device.h"

namespace rtlbfs {
namespace host {

inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

inline double splitmix_uniform(uint64_t seed, uint64_t i) {
    // SplitMix64 (Steele, Lea & Flood 2014): i-th output of the generator
    // seeded with `seed`, top 53 bits to [0, 1), then to [-1, 1).
    uint64_t z = seed + (i + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z ^= z >> 31;
    return 2.0 * ((double)(z >> 11) * 0x1.0p-53) - 1.0;
}

inline int mesh_nodes(int n, double stretch, double *x, double *L) {
    if (n < 1 || !x) return RTLBFS_EINVAL;
    if (!(stretch > 0.0)) {
        for (int i = 0; i <= n; ++i) x[i] = i;
        if (L) *L = n;
        return RTLBFS_OK;
    }
    // Eq. 74 on the unit interval, rescaled so the finest cell has size 1.
    const double th = std::tanh(stretch);
    for (int i = 0; i <= n; ++i) x[i] = 0.5 * (th + std::tanh(2.0 * stretch * ((double)i / n - 0.5))) / th;
    double hmin = 1e300;
    for (int i = 0; i < n; ++i) hmin = std::min(hmin, x[i + 1] - x[i]);
    const double len = 1.0 / hmin;
    for (int i = 0; i <= n; ++i) x[i] *= len;
    if (L) *L = len;
    return RTLBFS_OK;
}


inline int elem_size(int precision) { return precision == RTLBFS_FP32_DEV ? 4 : 8; }

// Elements between consecutive stored fields: the cell count rounded up to 64
// so that every field starts 256-byte aligned.
inline int64_t field_stride(int64_t cells) { return (cells + 63) / 64 * 64; }

inline int heat_axis(const rtlbfs_mesh &m, const rtlbfs_bc &bc) {
    for (int a = 0; a < m.dim; ++a)
        if (bc.kind[2 * a] == RTLBFS_WALL_ISOTHERMAL && bc.kind[2 * a + 1] == RTLBFS_WALL_ISOTHERMAL) return a;
    return -1;
}

inline int validate(const rtlbfs_mesh *m, const rtlbfs_bc *bc, const rtlbfs_opts &o, double Ra, double Pr, double Ma,
             std::string &why) {
    if (!m || !bc) return why = "mesh or bc is NULL", RTLBFS_EINVAL;
    if (m->dim != 2 && m->dim != 3) return why = "dim must be 2 or 3", RTLBFS_EINVAL;
    for (int a = 0; a < m->dim; ++a) {
        if (m->n[a] < 4) return why = "each axis needs >= 4 cells", RTLBFS_EINVAL;
        if (m->n[a] > (1 << 20)) return why = "axis too long", RTLBFS_EINVAL;
        const int k0 = bc->kind[2 * a], k1 = bc->kind[2 * a + 1];
        for (int k : {k0, k1})
            if (k != RTLBFS_PERIODIC && k != RTLBFS_WALL_ISOTHERMAL && k != RTLBFS_WALL_ADIABATIC)
                return why = "unknown boundary kind", RTLBFS_EINVAL;
        if ((k0 == RTLBFS_PERIODIC) != (k1 == RTLBFS_PERIODIC))
            return why = "periodic sides must come in pairs", RTLBFS_EINVAL;
        if (k0 == RTLBFS_PERIODIC && m->stretch[a] > 0.0)
            return why = "periodic axes must be uniform", RTLBFS_EINVAL;
        if (!(m->stretch[a] >= 0.0) || m->stretch[a] > 10.0) return why = "stretch out of range", RTLBFS_EINVAL;
    }
    if (bc->gravity_axis < -1 || bc->gravity_axis >= m->dim) return why = "gravity_axis out of range", RTLBFS_EINVAL;
    if (o.precision != RTLBFS_FP64_PLAIN && o.precision != RTLBFS_FP32_DEV && o.precision != RTLBFS_FP64_DEV)
        return why = "unknown precision", RTLBFS_EINVAL;
    if (o.phys_given) {
        if (!(o.nu > 0.0) || !(o.chi > 0.0) || !(o.beta_g >= 0.0)) return why = "nu, chi > 0, beta_g >= 0", RTLBFS_EINVAL;
    } else {
        if (!(Ra > 0.0) || !(Pr > 0.0)) return why = "Ra and Pr must be > 0", RTLBFS_EINVAL;
        if (!(Ma > 0.0) || Ma > 0.3) return why = "Ma must be in (0, 0.3]", RTLBFS_EINVAL;
    }
    if (!(o.dtl >= 0.0) || !(o.dt >= 0.0)) return why = "dtl and dt must be >= 0", RTLBFS_EINVAL;
    if (o.init != RTLBFS_INIT_REST && o.init != RTLBFS_INIT_CONDUCTION) return why = "unknown init", RTLBFS_EINVAL;
    if (o.tile < 0 || o.tile > 9) return why = "opts.tile out of range", RTLBFS_EINVAL;
    if (!(o.max_mach >= 0.0) || o.max_mach > 10.0) return why = "opts.max_mach out of range", RTLBFS_EINVAL;
    if (o.method != RTLBFS_METHOD_RTLBFS && o.method != RTLBFS_METHOD_TLBFS)
        return why = "unknown opts.method", RTLBFS_EINVAL;
    return RTLBFS_OK;
}


// Host view of one domain: geometry, Eq. 63 physics, time steps.
struct Problem {
    rtlbfs_mesh mesh;
    rtlbfs_bc bc;
    int D = 2;
    int64_t cells = 0;
    double length[3] = {1, 1, 1};
    double L = 0;        // characteristic length of Eq. 63
    int haxis = -1;      // axis of the two isothermal walls, -1 none
    std::vector<double> widths;   // per-axis cell widths, concatenated
    std::vector<double> centres;  // cell centres of the heat axis
    double nu = 0, chi = 0, bg = 0, dtl = 1, dt = 0.5;
};

// Validate and derive everything the kernels need for one domain.
inline int setup_problem(const rtlbfs_mesh *mesh, const rtlbfs_bc *bc, const rtlbfs_opts &o, double Ra, double Pr,
                         double Ma, Problem &p, std::string &why) {
    int rc = validate(mesh, bc, o, Ra, Pr, Ma, why);
    if (rc != RTLBFS_OK) return rc;
    p.mesh = *mesh;
    p.bc = *bc;
    p.D = mesh->dim;
    if (p.D == 2) {
        p.mesh.n[2] = 1;
        p.mesh.stretch[2] = 0.0;
    }
    p.cells = (int64_t)p.mesh.n[0] * p.mesh.n[1] * p.mesh.n[2];
    p.widths.clear();
    for (int a = 0; a < p.D; ++a) {
        std::vector<double> x(p.mesh.n[a] + 1);
        mesh_nodes(p.mesh.n[a], p.mesh.stretch[a], x.data(), &p.length[a]);
        for (int i = 0; i < p.mesh.n[a]; ++i) p.widths.push_back(x[i + 1] - x[i]);
    }
    p.haxis = heat_axis(p.mesh, *bc);
    p.centres.clear();
    if (p.haxis >= 0) {
        std::vector<double> x(p.mesh.n[p.haxis] + 1);
        mesh_nodes(p.mesh.n[p.haxis], p.mesh.stretch[p.haxis], x.data(), nullptr);
        for (int i = 0; i < p.mesh.n[p.haxis]; ++i) p.centres.push_back(0.5 * (x[i] + x[i + 1]));
    }
    const int la = p.haxis >= 0 ? p.haxis : (bc->gravity_axis >= 0 ? bc->gravity_axis : 0);
    p.L = p.length[la];
    if (o.phys_given) {
        p.nu = o.nu;
        p.chi = o.chi;
        p.bg = o.beta_g;
    } else {
        // Eq. 63 with V_c = Ma and dT = 1.
        p.nu = Ma * p.L * std::sqrt(Pr / Ra);
        p.chi = p.nu / Pr;
        p.bg = Ma * Ma / p.L;
    }
    p.dtl = o.dtl > 0.0 ? o.dtl : 1.0;
    p.dt = o.dt > 0.0 ? o.dt : std::min(0.5, 0.15 / std::max(p.nu, p.chi));
    return RTLBFS_OK;
}

// Initial T - T0 per cell: 0 (rest) or the linear conduction profile between
// the isothermal walls, plus seeded SplitMix64 noise.
inline void initial_Tdev(const Problem &p, const rtlbfs_opts &o, std::vector<double> &Tdev) {
    Tdev.assign((size_t)p.cells, 0.0);
    const int ha = p.haxis;
    const int64_t stride = ha <= 0 ? 1 : (ha == 1 ? p.mesh.n[0] : (int64_t)p.mesh.n[0] * p.mesh.n[1]);
    for (int64_t c = 0; c < p.cells; ++c) {
        double Tp = 0.0;
        if (o.init == RTLBFS_INIT_CONDUCTION && ha >= 0) {
            const int i = (int)((c / stride) % p.mesh.n[ha]);
            const double xi = p.centres[i] / p.length[ha];
            Tp = p.bc.Tdev[2 * ha] + (p.bc.Tdev[2 * ha + 1] - p.bc.Tdev[2 * ha]) * xi;
        }
        Tdev[c] = Tp + o.noise_amp * splitmix_uniform(o.seed, (uint64_t)c);
    }
}

// Geometry records of every axis (layout of kGeo*), in double; the caller
// converts to the kernel precision.  geo[a] holds kGeoFields * n[a] values.
inline void build_geometry(const Problem &p, std::vector<double> geo[3]) {
    size_t off = 0;
    for (int a = 0; a < p.D; ++a) {
        const int n = p.mesh.n[a];
        const bool per = p.bc.kind[2 * a] == RTLBFS_PERIODIC;
        const double *w = p.widths.data() + off;
        off += n;
        geo[a].assign((size_t)kGeoFields * n, 0.0);
        for (int i = 0; i < n; ++i) {
            const double wp = w[i];
            geo[a][kGeoW * n + i] = wp;
            geo[a][kGeoInvW * n + i] = 1.0 / wp;
            const bool has_lo = per || i > 0, has_hi = per || i < n - 1;
            if (has_lo) {
                const double wn = w[(i - 1 + n) % n];
                geo[a][kGeoLoSelf * n + i] = wn / (wp + wn);  // Eq. 56: weight |x_N - x_S| of phi_P
                geo[a][kGeoLoNb * n + i] = wp / (wp + wn);
            }
            if (has_hi) {
                const double wn = w[(i + 1) % n];
                geo[a][kGeoHiSelf * n + i] = wn / (wp + wn);
                geo[a][kGeoHiNb * n + i] = wp / (wp + wn);
            }
        }
    }
}

// Bytes of the geometry records of all axes in the kernel precision.
inline size_t geometry_bytes(const rtlbfs_mesh &m, int precision) {
    size_t b = 0;
    for (int a = 0; a < m.dim; ++a) b += align256((size_t)kGeoFields * m.n[a] * elem_size(precision));
    return b;
}

// Convert the geometry to the kernel precision into `bytes` (per-axis blocks
// 256-aligned); offsets[a] receives each axis block's byte offset.
inline void pack_geometry(const Problem &p, int precision, std::vector<char> &bytes, size_t offsets[3]) {
    std::vector<double> geo[3];
    build_geometry(p, geo);
    bytes.assign(geometry_bytes(p.mesh, precision), 0);
    size_t off = 0;
    for (int a = 0; a < p.D; ++a) {
        offsets[a] = off;
        for (size_t k = 0; k < geo[a].size(); ++k) {
            if (precision == RTLBFS_FP32_DEV) ((float *)(bytes.data() + off))[k] = (float)geo[a][k];
            else ((double *)(bytes.data() + off))[k] = geo[a][k];
        }
        off += align256(geo[a].size() * elem_size(precision));
    }
}

// Everything of the kernel-side Domain except the device pointers.
inline void fill_domain(const Problem &p, int precision, int force_pred, int round_nearest, double max_mach,
                        Domain &d) {
    std::memset(&d, 0, sizeof(d));
    const double mm = max_mach > 0.0 ? max_mach : 0.5;
    d.guard_u2 = mm * mm * kCs2;  // (Mach * c_s)^2
    d.dim = p.D;
    for (int a = 0; a < 3; ++a) {
        d.n[a] = a < p.D ? p.mesh.n[a] : 1;
        d.periodic[a] = a < p.D ? p.bc.kind[2 * a] == RTLBFS_PERIODIC : 1;
    }
    const bool dev = precision != RTLBFS_FP64_PLAIN;
    for (int s = 0; s < 6; ++s) {
        d.kind[s] = s < 2 * p.D ? p.bc.kind[s] : RTLBFS_PERIODIC;
        d.Tw[s] = dev ? p.bc.Tdev[s] : kT0 + p.bc.Tdev[s];
    }
    d.gaxis = p.bc.gravity_axis;
    d.force_pred = force_pred;
    d.sround = (precision == RTLBFS_FP32_DEV && !round_nearest) ? 1 : 0;
    d.nu = p.nu;
    d.chi = p.chi;
    d.bg = p.bg;
    d.dtl = p.dtl;
    d.dt = p.dt;
    d.tau_f = 0.5 + p.nu / (kCs2 * p.dtl);  // Eq. 9
    d.tau_g = 0.5 + p.chi / (kCs2 * p.dtl); // Eq. 10
    d.cells = p.cells;
    d.fstride = field_stride(p.cells);
    Phys<double> ph;
    ph.nu = d.nu;
    ph.chi = d.chi;
    ph.dtl = d.dtl;
    ph.tau_f = d.tau_f;
    ph.tau_g = d.tau_g;
    ph.bg = d.bg;
    ph.dt = d.dt;
    ph.h = d.dtl;  // lattice spacing c * delta-t with c = 1
    ph.inv2h = 1.0 / (2.0 * d.dtl);
    ph.invh2 = 1.0 / (d.dtl * d.dtl);
    ph.inv4h2 = 1.0 / (4.0 * d.dtl * d.dtl);
    ph.Tref_s = dev ? 0.0 : kT0;  // T_ref = T0 on the Cartesian meshes
    d.phd = ph;
    d.phf = {(float)ph.nu, (float)ph.chi, (float)ph.dtl, (float)ph.tau_f, (float)ph.tau_g, (float)ph.bg,
             (float)ph.dt, (float)ph.h, (float)ph.inv2h, (float)ph.invh2, (float)ph.inv4h2, (float)ph.Tref_s};
    for (int s = 0; s < 6; ++s) d.Twf[s] = (float)d.Tw[s];
}

}  // namespace host
}  // namespace rtlbfs
