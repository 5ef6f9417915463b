"""The TLBFS route to the interface flux (Sec. 2.2), used to pin the oracle.

The oracle implements the macroscopic form (MEs-TLBFS, Eqs. 46-51 / 57-59).
Sec. 3.1 derives that form from the lattice Boltzmann route of Sec. 2.2 by a
second-order Taylor expansion (Eqs. 44-45).  For fields whose equilibria are
quadratic in space the expansion has no remainder, so the two routes must
agree exactly, up to the one term the paper drops in Eqs. 50-51 (the
(tau - 0.5) * 0.5 dt^2 second derivative of the fourth / third equilibrium
moment).  This module evaluates the lattice Boltzmann route directly from the
equilibria (Eqs. 3-4), the velocity sets and weights (Eqs. 5-6), the
predicted moments (Eqs. 30-32) and the fluxes (Eqs. 38-40).
"""
from __future__ import annotations

import itertools

import numpy as np

CS2 = 1.0 / 3.0


def velocity_set(dim: int):
    """Eqs. 5-6: D2Q9 / D3Q19 velocities (c = 1) and weights."""
    if dim == 2:
        e = [(0, 0), (1, 0), (0, 1), (-1, 0), (0, -1), (1, 1), (-1, 1), (-1, -1), (1, -1)]
        w = [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4
    else:
        e = [(0, 0, 0)]
        e += [v for v in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, v)) == 1]
        e += [v for v in itertools.product((-1, 0, 1), repeat=3) if sum(map(abs, v)) == 2]
        w = [1 / 3] + [1 / 18] * 6 + [1 / 36] * 12
    return np.array(e, dtype=np.float64), np.array(w)


def feq(w, e, rho, u):
    """Eq. 3."""
    eu = e @ u
    return w * rho * (1.0 + eu / CS2 + eu * eu / (2 * CS2 * CS2) - (u @ u) / (2 * CS2))


def geq(w, e, rho, u, T):
    """Eq. 4 with c_p = 1."""
    return w * rho * T * (1.0 + (e @ u) / CS2)


def tlbfs_face(dim, fields, xs, normal_axis, dtl, nu, chi):
    """Interface flux along +normal_axis at xs by the lattice Boltzmann route.

    fields(x) -> (rho, u[dim], T) gives the time-n primitives at any point
    (for a field linear on each side of the face this is what Eq. 29
    reconstructs).  Returns (predicted (rho*, m*, e*), flux, correction) where
    correction is the dropped O(dt^2) term of Eqs. 50-51, evaluated exactly
    for quadratic equilibria by central differences of the equilibrium
    moments on the same lattice.
    """
    e, w = velocity_set(dim)
    tau_f = 0.5 + nu / (CS2 * dtl)
    tau_g = 0.5 + chi / (CS2 * dtl)
    Q = len(w)
    f_back = np.zeros(Q)
    g_back = np.zeros(Q)
    for i in range(Q):
        rho, u, T = fields(xs - e[i] * dtl)          # x_S - e_i dt
        f_back[i] = feq(w, e, rho, u)[i]
        g_back[i] = geq(w, e, rho, u, T)[i]
    rho_s = f_back.sum()                              # Eq. 30
    m_s = e.T @ f_back                                # Eq. 31
    E_s = g_back.sum()                                # Eq. 32
    u_s = m_s / rho_s
    T_s = E_s / rho_s
    f_star = feq(w, e, rho_s, u_s)                    # f^eq(x_S, t + dt)
    g_star = geq(w, e, rho_s, u_s, T_s)
    n = normal_axis
    P = (e[:, n] * f_star).sum()                      # Eq. 38
    Pi = np.array([(e[:, a] * e[:, n] * (f_star + (0.5 - tau_f) * (f_star - f_back))).sum()
                   for a in range(dim)])              # Eq. 39
    Qn = (e[:, n] * (g_star + (0.5 - tau_g) * (g_star - g_back))).sum()  # Eq. 40

    # The O(dt^2) term dropped between Eq. 39 and Eq. 50 (and Eq. 40 / 51):
    # (tau - 0.5) * 0.5 dt^2 * d_c d_d M, where M is the fourth moment of f^eq
    # (third of g^eq) at time n.  Exact second derivatives of a quadratic field
    # by central differences on a lattice of spacing dtl.
    def moments_at(x):
        rho, u, T = fields(x)
        f = feq(w, e, rho, u)
        g = geq(w, e, rho, u, T)
        M4 = np.einsum("q,qa,qb,qc,qd->abcd", f, e, e, e, e)
        M3 = np.einsum("q,qa,qb,qc->abc", g, e, e, e)
        return M4, M3

    hgt = dtl
    corr_m = np.zeros(dim)
    corr_e = 0.0
    for c in range(dim):
        for d in range(dim):
            ec = np.eye(dim)[c] * hgt
            ed = np.eye(dim)[d] * hgt
            if c == d:
                Mp4, Mp3 = moments_at(xs + ec)
                M04, M03 = moments_at(xs)
                Mm4, Mm3 = moments_at(xs - ec)
                d4 = (Mp4 - 2 * M04 + Mm4) / hgt**2
                d3 = (Mp3 - 2 * M03 + Mm3) / hgt**2
            else:
                pp4, pp3 = moments_at(xs + ec + ed)
                pm4, pm3 = moments_at(xs + ec - ed)
                mp4, mp3 = moments_at(xs - ec + ed)
                mm4, mm3 = moments_at(xs - ec - ed)
                d4 = (pp4 - pm4 - mp4 + mm4) / (4 * hgt**2)
                d3 = (pp3 - pm3 - mp3 + mm3) / (4 * hgt**2)
            corr_m += (tau_f - 0.5) * 0.5 * dtl**2 * d4[:, n, c, d]
            corr_e += (tau_g - 0.5) * 0.5 * dtl**2 * d3[n, c, d]
    pred = np.concatenate([[rho_s], m_s, [E_s]])
    flux = np.concatenate([[P], Pi, [Qn]])
    corr = np.concatenate([[0.0], corr_m, [corr_e]])
    return pred, flux, corr
