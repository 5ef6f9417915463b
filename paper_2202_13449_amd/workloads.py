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
