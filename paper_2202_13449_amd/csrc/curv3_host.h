// curv3_host.h -- host-side set-up of a 3D body-fitted hexahedral mesh:
// validation, FP64 cell volumes and centroids, and the per-face records of
// curv3d.h (kC3*), with the rotated images across periodic sides.
#pragma once

#include <array>
#include <cmath>
#include <string>
#include <vector>

#include "../../include/rtlbfs.h"
#include "curv3d.h"
#include "host_common.h"

namespace rtlbfs {
namespace host {

struct Curv3Problem {
    int n[3] = {0, 0, 0};
    int64_t cells = 0;
    int64_t nf[3] = {0, 0, 0};
    std::vector<double> cx, cy, cz, vol;
    std::vector<double> rec[3];  // kC3Fields * nf[a] values per axis, field-major
};

using V3 = std::array<double, 3>;

inline V3 v3sub(const V3 &a, const V3 &b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
inline double v3dot(const V3 &a, const V3 &b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline V3 v3cross(const V3 &a, const V3 &b) {
    return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
inline V3 v3rotz(const V3 &v, double ang) {
    const double c = std::cos(ang), s = std::sin(ang);
    return {c * v[0] - s * v[1], s * v[0] + c * v[1], v[2]};
}

inline int curv3_setup(const rtlbfs_curv3_mesh *m, const rtlbfs_curv3_bc *bc, Curv3Problem &p, std::string &why) {
    if (!m || !bc || !m->x || !m->y || !m->z) return why = "mesh, bc or vertex arrays are NULL", RTLBFS_EINVAL;
    for (int a = 0; a < 3; ++a) {
        const int k0 = bc->kind[2 * a], k1 = bc->kind[2 * a + 1];
        for (int k : {k0, k1})
            if (k != RTLBFS_PERIODIC && k != RTLBFS_WALL_ISOTHERMAL && k != RTLBFS_WALL_ADIABATIC)
                return why = "unknown boundary kind (3D body-fitted meshes take periodic and wall sides)", RTLBFS_EINVAL;
        if ((k0 == RTLBFS_PERIODIC) != (k1 == RTLBFS_PERIODIC)) return why = "periodic sides must come in pairs", RTLBFS_EINVAL;
        const int lo = k0 == RTLBFS_PERIODIC ? 1 : 2;
        if (m->n[a] < lo || m->n[a] > (1 << 16)) return why = "cells per axis out of range", RTLBFS_EINVAL;
        if (k0 != RTLBFS_PERIODIC && bc->rot[a] != 0.0) return why = "rot applies to periodic axes only", RTLBFS_EINVAL;
        if (!std::isfinite(bc->rot[a]) || std::fabs(bc->rot[a]) > 3.2) return why = "rot out of range", RTLBFS_EINVAL;
    }
    const double upn = bc->up[0] * bc->up[0] + bc->up[1] * bc->up[1] + bc->up[2] * bc->up[2];
    if (!(upn == 0.0 || std::fabs(upn - 1.0) <= 1e-12)) return why = "up must be a unit vector or zero", RTLBFS_EINVAL;
    for (int a = 0; a < 3; ++a) p.n[a] = m->n[a];
    const int n0 = p.n[0], n1 = p.n[1], n2 = p.n[2];
    p.cells = (int64_t)n0 * n1 * n2;
    if (p.cells > (int64_t)1 << 28) return why = "mesh too large", RTLBFS_EINVAL;
    auto VI = [&](int i, int j, int k) { return ((int64_t)k * (n1 + 1) + j) * (n0 + 1) + i; };
    auto V = [&](int i, int j, int k) -> V3 {
        const int64_t v = VI(i, j, k);
        return {m->x[v], m->y[v], m->z[v]};
    };
    const int64_t NV = (int64_t)(n0 + 1) * (n1 + 1) * (n2 + 1);
    double scale = 1.0;
    for (int64_t v = 0; v < NV; ++v) {
        if (!std::isfinite(m->x[v]) || !std::isfinite(m->y[v]) || !std::isfinite(m->z[v]))
            return why = "non-finite vertex", RTLBFS_EINVAL;
        scale = std::max(scale, std::max(std::fabs(m->x[v]), std::max(std::fabs(m->y[v]), std::fabs(m->z[v]))));
    }
    // a periodic pair closes the mesh up to its rotation about z
    for (int a = 0; a < 3; ++a) {
        if (bc->kind[2 * a] != RTLBFS_PERIODIC) continue;
        int lim[3] = {n0, n1, n2};
        lim[a] = 0;
        for (int k = 0; k <= lim[2]; ++k)
            for (int j = 0; j <= lim[1]; ++j)
                for (int i = 0; i <= lim[0]; ++i) {
                    int q[3] = {i, j, k};
                    q[a] = p.n[a];
                    const V3 r0 = v3rotz(V(i, j, k), bc->rot[a]), r1 = V(q[0], q[1], q[2]);
                    for (int b = 0; b < 3; ++b)
                        if (std::fabs(r0[b] - r1[b]) > 1e-9 * scale)
                            return why = "a periodic pair does not close the mesh (with rot about z)", RTLBFS_EINVAL;
                }
    }
    // face corners in the cyclic order of the spanning axes
    auto corners = [&](int a, int i, int j, int k, V3 (&q)[4]) {
        const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
        int r[4][3];
        for (int t = 0; t < 4; ++t) {
            r[t][0] = i;
            r[t][1] = j;
            r[t][2] = k;
        }
        r[1][b1] += 1;
        r[2][b1] += 1;
        r[2][b2] += 1;
        r[3][b2] += 1;
        for (int t = 0; t < 4; ++t) q[t] = V(r[t][0], r[t][1], r[t][2]);
    };
    // cells: 24 tetrahedra from the cell's first corner to the face-centre fans
    p.cx.assign(p.cells, 0.0);
    p.cy.assign(p.cells, 0.0);
    p.cz.assign(p.cells, 0.0);
    p.vol.assign(p.cells, 0.0);
    int sign = 0;
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                const V3 apex = V(i, j, k);
                double Vs = 0.0;
                V3 Ms = {0, 0, 0};
                for (int a = 0; a < 3; ++a)
                    for (int hi = 0; hi < 2; ++hi) {
                        int f[3] = {i, j, k};
                        f[a] += hi;
                        V3 q[4];
                        corners(a, f[0], f[1], f[2], q);
                        V3 cf;
                        for (int b = 0; b < 3; ++b) cf[b] = 0.25 * (q[0][b] + q[1][b] + q[2][b] + q[3][b]);
                        for (int t = 0; t < 4; ++t) {
                            const V3 &qa = q[t], &qb = q[(t + 1) % 4];
                            // tetrahedron (apex, cf, qa, qb), oriented by the face's +axis side
                            const double vt =
                                (hi ? 1.0 : -1.0) * v3dot(v3sub(cf, apex), v3cross(v3sub(qa, cf), v3sub(qb, cf))) / 6.0;
                            Vs += vt;
                            for (int b = 0; b < 3; ++b) Ms[b] += vt * 0.25 * (apex[b] + cf[b] + qa[b] + qb[b]);
                        }
                    }
                const int sg = Vs > 0.0 ? 1 : (Vs < 0.0 ? -1 : 0);
                if (sg == 0 || (sign != 0 && sg != sign)) return why = "cells fold over or are degenerate", RTLBFS_EINVAL;
                sign = sg;
                const int64_t c = ((int64_t)k * n1 + j) * n0 + i;
                p.cx[c] = Ms[0] / Vs;
                p.cy[c] = Ms[1] / Vs;
                p.cz[c] = Ms[2] / Vs;
                p.vol[c] = std::fabs(Vs);
            }
    // faces
    for (int a = 0; a < 3; ++a) {
        const int fx = n0 + (a == 0), fy = n1 + (a == 1), fz = n2 + (a == 2);
        p.nf[a] = (int64_t)fx * fy * fz;
        p.rec[a].assign((size_t)kC3Fields * p.nf[a], 0.0);
        const bool per = bc->kind[2 * a] == RTLBFS_PERIODIC;
        for (int k = 0; k < fz; ++k)
            for (int j = 0; j < fy; ++j)
                for (int i = 0; i < fx; ++i) {
                    V3 q[4];
                    corners(a, i, j, k, q);
                    V3 xs, d1 = v3sub(q[2], q[0]), d2 = v3sub(q[3], q[1]), ed = v3sub(q[1], q[0]);
                    for (int b = 0; b < 3; ++b) xs[b] = 0.25 * (q[0][b] + q[1][b] + q[2][b] + q[3][b]);
                    V3 S = v3cross(d1, d2);
                    for (int b = 0; b < 3; ++b) S[b] *= 0.5 * sign;
                    const double dS = std::sqrt(v3dot(S, S));
                    if (!(dS > 0.0)) return why = "zero-area face", RTLBFS_EINVAL;
                    V3 n = {S[0] / dS, S[1] / dS, S[2] / dS};
                    const double en = v3dot(ed, n);
                    V3 t1 = {ed[0] - en * n[0], ed[1] - en * n[1], ed[2] - en * n[2]};
                    const double lt = std::sqrt(v3dot(t1, t1));
                    if (!(lt > 0.0)) return why = "degenerate face edge", RTLBFS_EINVAL;
                    for (int b = 0; b < 3; ++b) t1[b] /= lt;
                    const V3 t2 = v3cross(n, t1);
                    int qq[3] = {i, j, k};
                    const int idx = qq[a];
                    const bool hasL = idx > 0 || per, hasR = idx < p.n[a] || per;
                    auto centroid = [&](int off) -> V3 {  // centroid of the cell (or image) at index idx + off
                        int r[3] = {i, j, k};
                        r[a] = idx + off;
                        double ang = 0.0;
                        if (r[a] < 0) {
                            r[a] += p.n[a];
                            ang = -bc->rot[a];
                        } else if (r[a] >= p.n[a]) {
                            r[a] -= p.n[a];
                            ang = bc->rot[a];
                        }
                        const int64_t c = ((int64_t)r[2] * n1 + r[1]) * n0 + r[0];
                        return v3rotz(V3{p.cx[c], p.cy[c], p.cz[c]}, ang);
                    };
                    double dL = 0, tL1 = 0, tL2 = 0, dR = 0, tR1 = 0, tR2 = 0, wL = 0.5;
                    V3 xL{}, xR{};
                    if (hasL) {
                        xL = centroid(-1);
                        const V3 r = v3sub(xs, xL);
                        dL = v3dot(r, n);
                        tL1 = v3dot(r, t1);
                        tL2 = v3dot(r, t2);
                    }
                    if (hasR) {
                        xR = centroid(0);
                        const V3 r = v3sub(xs, xR);
                        dR = -v3dot(r, n);
                        tR1 = v3dot(r, t1);
                        tR2 = v3dot(r, t2);
                    }
                    if (hasL && hasR) {
                        const double lL = std::sqrt(v3dot(v3sub(xL, xs), v3sub(xL, xs)));
                        const double lR = std::sqrt(v3dot(v3sub(xR, xs), v3sub(xR, xs)));
                        wL = lR / (lL + lR);  // Eq. 56: the far cell's distance weighs the near value
                    } else if (hasL) {
                        dR = dL;
                        tR1 = tL1;
                        tR2 = tL2;
                    } else {
                        dL = dR;
                        tL1 = tR1;
                        tL2 = tR2;
                    }
                    if (!(dL > 0.0) || !(dR > 0.0)) return why = "a cell centroid lies on the wrong side of a face", RTLBFS_EINVAL;
                    const double vals[kC3Fields] = {n[0], n[1], n[2], t1[0], t1[1], t1[2], dS,
                                                    dL,   tL1,  tL2,  dR,    tR1,   tR2,   wL};
                    const int64_t f = ((int64_t)k * fy + j) * fx + i;
                    for (int t = 0; t < kC3Fields; ++t) p.rec[a][(size_t)t * p.nf[a] + f] = vals[t];
                }
    }
    return RTLBFS_OK;
}

}  // namespace host
}  // namespace rtlbfs
