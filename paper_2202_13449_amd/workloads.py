"""Seeded synthetic workloads shaped like the paper's benchmark problems.

Pure problem descriptions (mesh sizes, boundary kinds, Ra, Pr): no arithmetic
of the method.  Random choices use SplitMix64 (Steele, Lea & Flood 2014) so
the draws are reproducible across machines.
"""
from __future__ import annotations

import math

MASK = (1 << 64) - 1


def splitmix_u01(seed: int, i: int) -> float:
    """i-th SplitMix64 output for `seed`, top 53 bits as a float in [0, 1)."""
    z = (seed + (i + 1) * 0x9E3779B97F4A7C15) & MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK
    z ^= z >> 31
    return (z >> 11) * 2.0 ** -53


CAVITY_KIND = (1, 1, 2, 2)           # isothermal x walls, adiabatic y walls
CAVITY_TDEV = (0.5, -0.5, 0.0, 0.0)  # hot at x = 0, cold at x = L
CAVITY_GRAVITY = 1


def batch_cavities(count: int = 256, seed: int = 4):
    """Differentially heated cavities with side N in {64, 128, 256, 512},
    Ra log-uniform in [1e3, 1e7], Pr in {0.71, 7.0}, uniform or tanh
    (phi = 1.5) mesh with probability 1/2 each.  Returns a list of dicts
    (n, stretch, Ra, Pr)."""
    out = []
    for m in range(count):
        u = [splitmix_u01(seed, 4 * m + k) for k in range(4)]
        N = (64, 128, 256, 512)[min(3, int(u[0] * 4))]
        Ra = 10.0 ** (3.0 + 4.0 * u[1])
        Pr = 0.71 if u[2] < 0.5 else 7.0
        stretch = 1.5 if u[3] < 0.5 else 0.0
        out.append(dict(n=N, stretch=stretch, Ra=Ra, Pr=Pr))
    return out


def total_cells(members) -> int:
    return sum(m["n"] * m["n"] for m in members)


# ---------------------------------------------------------------- curvilinear

def geometric_radii(n: int, r0: float, r1: float, first: float):
    """n + 1 radii from r0 to r1 whose spacing starts at `first` and grows by
    a constant ratio (found by bisection); uniform if first * n equals r1 - r0."""
    L = r1 - r0
    if abs(first * n - L) <= 1e-12 * L:
        return [r0 + L * k / n for k in range(n + 1)]

    def span(q):
        return first * (q ** n - 1.0) / (q - 1.0)

    lo, hi = (1.0 + 1e-12, 2.0) if first * n < L else (1e-3, 1.0 - 1e-12)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if span(mid) < L:
            lo = mid
        else:
            hi = mid
    q = 0.5 * (lo + hi)
    r = [r0 + first * (q ** k - 1.0) / (q - 1.0) for k in range(n + 1)]
    r[-1] = r1
    return r


def o_mesh(ni: int, nj: int, r_in: float, r_out: float, first: float, theta0: float = 0.0):
    """Vertices of an O-type mesh between circles of radii r_in and r_out:
    i runs counter-clockwise around (vertex column ni is column 0 again, so
    the i sides are periodic), j runs outward with geometric radial spacing
    that starts at `first`.  Returns x, y as nested lists (nj + 1) x (ni + 1)."""
    r = geometric_radii(nj, r_in, r_out, first)
    th = [theta0 + 2.0 * math.pi * (i % ni) / ni for i in range(ni + 1)]
    x = [[rj * math.cos(t) for t in th] for rj in r]
    y = [[rj * math.sin(t) for t in th] for rj in r]
    return x, y


# Sec. 4.3: mixed convection from a heated circular cylinder.  O-type mesh of
# 300 x 450 cells (read here as 450 around the cylinder and 300 outward), far
# field 52.5 D from the centre, first cell 0.003 D; free stream 0.1 c_s along
# +y (against gravity: buoyancy aids the flow), T_inf = 0, T_wall = 1,
# Re = 20, Pr = 0.7, Gr in {0, 100, 800, 1600}.  Lengths in units of the
# first cell, so D = 1 / 0.003.
CYLINDER = dict(ni=450, nj=300, far=52.5, first=0.003, Re=20.0, Pr=0.7, Gr=(0.0, 100.0, 800.0, 1600.0),
                u_inf_cs=0.1, T_wall=1.0, T_inf=0.0)


def cylinder_mesh(ni: int = 450, nj: int = 300, far: float = 52.5, first: float = 0.003):
    """O-mesh of the cylinder of diameter D = 1/first (first cell of unit
    size) with the far field at `far` * D from the centre.  Returns (x, y, D)."""
    D = 1.0 / first
    x, y = o_mesh(ni, nj, 0.5 * D, far * D, 1.0, theta0=-0.5 * math.pi)
    return x, y, D


def annulus_wedge(nr: int, nth: int, nz: int, r_in: float, r_out: float, height: float, dtheta: float):
    """Vertices of a wedge of a concentric annulus: i runs outward (uniform
    in r), j around z over nth cells of angle dtheta (symmetric about the x
    axis), k up (uniform in z).  Vertex layer j = nth is layer 0 rotated by
    nth * dtheta about z.  Returns x, y, z as nested lists
    (nz + 1) x (nth + 1) x (nr + 1)."""
    r = [r_in + (r_out - r_in) * i / nr for i in range(nr + 1)]
    th = [(j - 0.5 * nth) * dtheta for j in range(nth + 1)]
    zz = [height * k / nz for k in range(nz + 1)]
    x = [[[ri * math.cos(t) for ri in r] for t in th] for _ in zz]
    y = [[[ri * math.sin(t) for ri in r] for t in th] for _ in zz]
    z = [[[zk for _ in r] for _ in th] for zk in zz]
    return x, y, z


# Sec. 4.5: natural convection in a concentric annulus, Ar = R_o/R_i = 2,
# eta = H/(R_o - R_i) = 2, Pr = 0.71, V_c = 0.1, Ra in {1e4, 1e5}, inner
# wall T_i = 1, outer T_o = 0, top and bottom adiabatic; 120 x 1 x 240
# cells (r, theta, z), one azimuthal layer closed by rotational periodicity.
# Lengths in units of the radial cell: R_i = 120, R_o = 240, H = 240; the
# wedge angle (not given) is taken as 1/120 rad, so the cells at the inner
# wall are cubes.
ANNULUS = dict(nr=120, nth=1, nz=240, Ar=2.0, eta=2.0, Pr=0.71, Vc=0.1, Ra=(1e4, 1e5))


def annulus_mesh(nr: int = 120, nz: int = 240, Ar: float = 2.0, eta: float = 2.0, nth: int = 1):
    """The Sec. 4.5 wedge: radial gap of nr unit cells, R_i = nr / (Ar - 1),
    height eta * nr, wedge angle 1/R_i per azimuthal cell.  Returns
    (x, y, z, R_i, R_o, H, dtheta)."""
    gap = float(nr)
    r_in = gap / (Ar - 1.0)
    H = eta * gap
    dth = 1.0 / r_in
    x, y, z = annulus_wedge(nr, nth, nz, r_in, r_in + gap, H, dth)
    return x, y, z, r_in, r_in + gap, H, dth
