"""Seeded synthetic inputs shared by the oracle pins and the GPU parity tests.

This module holds no arithmetic of the method: only problem set-ups (mesh
sizes, boundary kinds, Eq. 63 parameters derived by the caller), analytic
initial fields and seeded random numbers.
"""
from __future__ import annotations

import numpy as np

PERIODIC, WALL_ISOTHERMAL, WALL_ADIABATIC = 0, 1, 2


def rng(seed: int) -> np.random.Generator:
    return np.random.default_rng(seed)


def dhc_bc(dim: int = 2, hot_low: bool = True):
    """Differentially heated cavity: isothermal walls on x (hot at x = 0 when
    hot_low), adiabatic elsewhere, gravity along +y (2D) / +z (3D) upward."""
    hot, cold = (0.5, -0.5) if hot_low else (-0.5, 0.5)
    if dim == 2:
        bc = (WALL_ISOTHERMAL, WALL_ISOTHERMAL, WALL_ADIABATIC, WALL_ADIABATIC, PERIODIC, PERIODIC)
        return bc, (hot, cold, 0.0, 0.0, 0.0, 0.0), 1
    bc = (WALL_ISOTHERMAL, WALL_ISOTHERMAL, WALL_ADIABATIC, WALL_ADIABATIC, WALL_ADIABATIC, WALL_ADIABATIC)
    return bc, (hot, cold, 0.0, 0.0, 0.0, 0.0), 2


def rb_bc():
    """Rayleigh-Benard box: periodic in x, hot bottom / cold top, gravity +y."""
    bc = (PERIODIC, PERIODIC, WALL_ISOTHERMAL, WALL_ISOTHERMAL, PERIODIC, PERIODIC)
    return bc, (0.0, 0.0, 0.5, -0.5, 0.0, 0.0), 1


def gaussian_hill(xc: np.ndarray, yc: np.ndarray, L: float, t: float, chi: float, u0: float) -> np.ndarray:
    """Eq. 67 on the periodic box [0, 2L]^2 with x0 = (0.5 L, 0), sigma = 0.05 L,
    T0 = 2 pi sigma^2 (so the initial peak is 1); minimum-image distances."""
    sig = 0.05 * L
    s2 = 2.0 * chi * t + sig * sig
    X, Y = np.meshgrid(xc, yc)
    dx = (X - 0.5 * L - u0 * t + L) % (2.0 * L) - L
    dy = (Y + L) % (2.0 * L) - L
    return sig * sig / s2 * np.exp(-(dx * dx + dy * dy) / (2.0 * s2))


def random_state(N: int, dim: int, seed: int, amp_rho=1e-3, amp_u=0.02, amp_T=0.2):
    """Seeded smooth-ish random absolute primitives (rho, u[dim, N], T) used for
    short-horizon parity runs."""
    g = rng(seed)
    rho = 1.0 + amp_rho * g.uniform(-1, 1, N)
    u = amp_u * g.uniform(-1, 1, (dim, N))
    T = 0.5 + amp_T * g.uniform(-1, 1, N)
    return rho, u, T


# ------------------------------------------------------ curvilinear meshes --

FARFIELD = 3


def cartesian_vertices(xn, yn):
    """Vertex arrays (nj + 1, ni + 1) of the Cartesian mesh with node
    coordinates xn along i and yn along j."""
    X, Y = np.meshgrid(np.asarray(xn, dtype=np.float64), np.asarray(yn, dtype=np.float64))
    return X.copy(), Y.copy()


def rotated(x, y, angle):
    c, s = np.cos(angle), np.sin(angle)
    return c * x - s * y, s * x + c * y


def wavy_vertices(xn, yn, amp):
    """A Cartesian mesh bent by smooth sine displacements of relative size
    `amp`; the outer boundary stays rectangular."""
    X, Y = cartesian_vertices(xn, yn)
    Lx, Ly = X.max() - X.min(), Y.max() - Y.min()
    sx = np.sin(np.pi * (X - X.min()) / Lx)
    sy = np.sin(np.pi * (Y - Y.min()) / Ly)
    return X + amp * Lx * sx * sy * np.sin(2 * np.pi * (Y - Y.min()) / Ly), \
        Y + amp * Ly * sx * sy * np.cos(2 * np.pi * (X - X.min()) / Lx)


def o_mesh(ni, nj, r_in, r_out, first, theta0=0.0):
    from paper_2202_13449_amd.workloads import o_mesh as _o

    x, y = _o(ni, nj, r_in, r_out, first, theta0)
    return np.array(x), np.array(y)


def cartesian_vertices3(xn, yn, zn):
    """Vertex arrays (nk + 1, nj + 1, ni + 1) of a 3D Cartesian mesh."""
    Z, Y, X = np.meshgrid(np.asarray(zn, float), np.asarray(yn, float), np.asarray(xn, float), indexing="ij")
    return X.copy(), Y.copy(), Z.copy()


def wavy_vertices3(xn, yn, zn, amp):
    """A 3D Cartesian mesh bent by smooth displacements that vanish on the
    box faces' normal components (the outer boundary stays a box)."""
    X, Y, Z = cartesian_vertices3(xn, yn, zn)
    L = [X.max() - X.min(), Y.max() - Y.min(), Z.max() - Z.min()]
    sx = np.sin(np.pi * (X - X.min()) / L[0])
    sy = np.sin(np.pi * (Y - Y.min()) / L[1])
    sz = np.sin(np.pi * (Z - Z.min()) / L[2])
    b = sx * sy * sz
    return (X + amp * L[0] * b * np.cos(2 * np.pi * (Y - Y.min()) / L[1]),
            Y + amp * L[1] * b * np.sin(2 * np.pi * (Z - Z.min()) / L[2]),
            Z + amp * L[2] * b * np.cos(2 * np.pi * (X - X.min()) / L[0]))


def annulus_wedge(nr, nth, nz, r_in, r_out, height, dtheta):
    from paper_2202_13449_amd.workloads import annulus_wedge as _w

    return tuple(np.array(v) for v in _w(nr, nth, nz, r_in, r_out, height, dtheta))
