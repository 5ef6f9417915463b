// curv_host.h -- host-side set-up of a body-fitted 2D mesh: validation, FP64
// cell areas and centroids, and the per-face records the curvilinear step
// kernel reads (layout of kCf* in curv2d.h).
#pragma once

#include <cmath>
#include <string>
#include <vector>

#include "../../include/rtlbfs.h"
#include "curv2d.h"
#include "host_common.h"

namespace rtlbfs {
namespace host {

struct CurvProblem {
    int ni = 0, nj = 0;
    int64_t cells = 0;
    int64_t nfi = 0, nfj = 0;             // face counts: (ni+1)*nj and ni*(nj+1)
    std::vector<double> cx, cy, area;     // per cell
    std::vector<double> fi, fj;           // kCurvFaceFields * nfi (nfj) values, field-major
};

// Cell (i, j) with corners p0..p3 = (i, j), (i+1, j), (i+1, j+1), (i, j+1):
// signed area from the cross product of the diagonals, centroid as the
// area-weighted mean of the centroids of the triangles (p0, p1, p2) and
// (p0, p2, p3).
inline double quad_shape(const double *px, const double *py, double &cx, double &cy) {
    const double A = 0.5 * ((px[2] - px[0]) * (py[3] - py[1]) - (py[2] - py[0]) * (px[3] - px[1]));
    // triangle areas relative to p0 keep the products small
    const double ax = px[1] - px[0], ay = py[1] - py[0], bx = px[2] - px[0], by = py[2] - py[0];
    const double qx = px[3] - px[0], qy = py[3] - py[0];
    const double A1 = 0.5 * (ax * by - ay * bx), A2 = 0.5 * (bx * qy - by * qx);
    const double c1x = (ax + bx) / 3.0, c1y = (ay + by) / 3.0;
    const double c2x = (bx + qx) / 3.0, c2y = (by + qy) / 3.0;
    cx = px[0] + (A1 * c1x + A2 * c2x) / (A1 + A2);
    cy = py[0] + (A1 * c1y + A2 * c2y) / (A1 + A2);
    return A;
}

inline int curv_setup(const rtlbfs_curv_mesh *m, const rtlbfs_curv_bc *bc, CurvProblem &p, std::string &why) {
    if (!m || !bc || !m->x || !m->y) return why = "mesh, bc or vertex arrays are NULL", RTLBFS_EINVAL;
    const int ni = m->n[0], nj = m->n[1];
    if (ni < 4 || nj < 4) return why = "each axis needs >= 4 cells", RTLBFS_EINVAL;
    if (ni > (1 << 20) || nj > (1 << 20)) return why = "axis too long", RTLBFS_EINVAL;
    for (int s = 0; s < 4; ++s)
        if (bc->kind[s] < RTLBFS_PERIODIC || bc->kind[s] > RTLBFS_FARFIELD) return why = "unknown boundary kind", RTLBFS_EINVAL;
    for (int a = 0; a < 2; ++a)
        if ((bc->kind[2 * a] == RTLBFS_PERIODIC) != (bc->kind[2 * a + 1] == RTLBFS_PERIODIC))
            return why = "periodic sides must come in pairs", RTLBFS_EINVAL;
    const double upn = bc->up[0] * bc->up[0] + bc->up[1] * bc->up[1];
    if (!(upn == 0.0 || std::fabs(upn - 1.0) <= 1e-12)) return why = "up must be a unit vector or zero", RTLBFS_EINVAL;
    p.ni = ni;
    p.nj = nj;
    p.cells = (int64_t)ni * nj;
    const int VX = ni + 1;
    const double *X = m->x, *Y = m->y;
    auto V = [&](int i, int j) { return (int64_t)j * VX + i; };
    double scale = 0.0;
    for (int64_t v = 0; v < (int64_t)VX * (nj + 1); ++v) {
        if (!std::isfinite(X[v]) || !std::isfinite(Y[v])) return why = "non-finite vertex", RTLBFS_EINVAL;
        scale = std::max(scale, std::max(std::fabs(X[v]), std::fabs(Y[v])));
    }
    const double tol = 1e-9 * std::max(scale, 1.0);
    if (bc->kind[0] == RTLBFS_PERIODIC)
        for (int j = 0; j <= nj; ++j)
            if (std::fabs(X[V(0, j)] - X[V(ni, j)]) > tol || std::fabs(Y[V(0, j)] - Y[V(ni, j)]) > tol)
                return why = "periodic i sides: vertex column n[0] must equal column 0", RTLBFS_EINVAL;
    if (bc->kind[2] == RTLBFS_PERIODIC)
        for (int i = 0; i <= ni; ++i)
            if (std::fabs(X[V(i, 0)] - X[V(i, nj)]) > tol || std::fabs(Y[V(i, 0)] - Y[V(i, nj)]) > tol)
                return why = "periodic j sides: vertex row n[1] must equal row 0", RTLBFS_EINVAL;

    // cells
    p.cx.assign(p.cells, 0.0);
    p.cy.assign(p.cells, 0.0);
    p.area.assign(p.cells, 0.0);
    int sign = 0;
    for (int j = 0; j < nj; ++j)
        for (int i = 0; i < ni; ++i) {
            const int64_t v[4] = {V(i, j), V(i + 1, j), V(i + 1, j + 1), V(i, j + 1)};
            double qx[4], qy[4];
            for (int k = 0; k < 4; ++k) {
                qx[k] = X[v[k]];
                qy[k] = Y[v[k]];
            }
            const int64_t c = (int64_t)j * ni + i;
            const double A = quad_shape(qx, qy, p.cx[c], p.cy[c]);
            const int sg = A > 0.0 ? 1 : (A < 0.0 ? -1 : 0);
            if (sg == 0 || (sign != 0 && sg != sign)) return why = "cells fold over or are degenerate", RTLBFS_EINVAL;
            sign = sg;
            p.area[c] = std::fabs(A);
        }

    // faces
    p.nfi = (int64_t)(ni + 1) * nj;
    p.nfj = (int64_t)ni * (nj + 1);
    p.fi.assign((size_t)kCurvFaceFields * p.nfi, 0.0);
    p.fj.assign((size_t)kCurvFaceFields * p.nfj, 0.0);
    const bool per[2] = {bc->kind[0] == RTLBFS_PERIODIC, bc->kind[2] == RTLBFS_PERIODIC};
    for (int axis = 0; axis < 2; ++axis) {
        const int na = axis == 0 ? ni + 1 : nj + 1;  // faces along the axis
        const int nc = axis == 0 ? nj : ni;          // across
        const int nk = axis == 0 ? ni : nj;          // cells along the axis
        std::vector<double> &rec = axis == 0 ? p.fi : p.fj;
        const int64_t stride = axis == 0 ? p.nfi : p.nfj;
        for (int a = 0; a < na; ++a)
            for (int b = 0; b < nc; ++b) {
                const int i = axis == 0 ? a : b, j = axis == 0 ? b : a;
                const int64_t va = V(i, j), vb = axis == 0 ? V(i, j + 1) : V(i + 1, j);
                const double ex = X[vb] - X[va], ey = Y[vb] - Y[va];
                const double len = std::sqrt(ex * ex + ey * ey);
                if (!(len > 0.0)) return why = "zero-length face", RTLBFS_EINVAL;
                // normal toward +i (+j): the edge turned by -90 deg (+90 deg) on a
                // counter-clockwise mesh, the opposite on a clockwise one
                const double nx = sign * (axis == 0 ? ey : -ey) / len, ny = sign * (axis == 0 ? -ex : ex) / len;
                const double tx = -ny, ty = nx;
                const double sx = 0.5 * (X[va] + X[vb]), sy = 0.5 * (Y[va] + Y[vb]);
                const bool hasL = a > 0 || per[axis], hasR = a < nk || per[axis];
                const int la = (a - 1 + nk) % nk, ra = a % nk;
                auto cell = [&](int k) { return axis == 0 ? (int64_t)j * ni + k : (int64_t)k * ni + i; };
                const int64_t f = (int64_t)j * (axis == 0 ? ni + 1 : ni) + i;
                double dL = 0, tL = 0, dR = 0, tR = 0, wL = 0.5;
                if (hasL) {
                    const int64_t L = cell(la);
                    dL = (sx - p.cx[L]) * nx + (sy - p.cy[L]) * ny;
                    tL = (sx - p.cx[L]) * tx + (sy - p.cy[L]) * ty;
                }
                if (hasR) {
                    const int64_t R = cell(ra);
                    dR = (p.cx[R] - sx) * nx + (p.cy[R] - sy) * ny;
                    tR = (sx - p.cx[R]) * tx + (sy - p.cy[R]) * ty;
                }
                if (hasL && hasR) {
                    const int64_t L = cell(la), R = cell(ra);
                    const double rl = std::hypot(p.cx[L] - sx, p.cy[L] - sy), rr = std::hypot(p.cx[R] - sx, p.cy[R] - sy);
                    wL = rr / (rl + rr);  // Eq. 56: the far cell's distance weighs the near value
                } else if (hasL) {
                    dR = dL;
                    tR = tL;
                } else {
                    dL = dR;
                    tL = tR;
                }
                if (!(dL > 0.0) || !(dR > 0.0)) return why = "a cell centroid lies on the wrong side of a face", RTLBFS_EINVAL;
                const double vals[kCurvFaceFields] = {nx, ny, len, dL, tL, dR, tR, wL};
                for (int k = 0; k < kCurvFaceFields; ++k) rec[(size_t)k * stride + f] = vals[k];
            }
        // on a periodic axis the last face is the first one
        if (per[axis])
            for (int b = 0; b < nc; ++b) {
                const int64_t f0 = axis == 0 ? (int64_t)b * (ni + 1) : b;
                const int64_t fn = axis == 0 ? (int64_t)b * (ni + 1) + ni : (int64_t)nj * ni + b;
                for (int k = 0; k < kCurvFaceFields; ++k) rec[(size_t)k * stride + fn] = rec[(size_t)k * stride + f0];
            }
    }
    return RTLBFS_OK;
}

}  // namespace host
}  // namespace rtlbfs
