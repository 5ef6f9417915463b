"""ctypes wrapper of the curvilinear-mesh oracle (test infrastructure only).

The RTLBFS step of Sec. 3.2 on a 2D body-fitted quadrilateral mesh, the
setting of Secs. 4.3 (heated cylinder, O-type mesh) and 4.5: per-face
normals and areas, Eq. 55 Gauss gradients, the local D2Q9 lattice aligned
with each face.  See curv_oracle.h for the conventions.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
from typing import Sequence

import numpy as np

from .oracle import RTLBFS, _load, _ptr

FARFIELD = 3


class _CurvCfg(C.Structure):
    _fields_ = [
        ("ni", C.c_int),
        ("nj", C.c_int),
        ("bc", C.c_int * 4),
        ("Tw", C.c_double * 4),
        ("up", C.c_double * 2),
        ("Tb", C.c_double),
        ("u_inf", C.c_double * 2),
        ("T_inf", C.c_double),
        ("nu", C.c_double),
        ("chi", C.c_double),
        ("beta_g", C.c_double),
        ("dtl", C.c_double),
        ("dt", C.c_double),
        ("deviation", C.c_int),
        ("force_in_predictor", C.c_int),
        ("method", C.c_int),
    ]


_bound = False


def _lib():
    global _bound
    lib = _load()
    if not _bound:
        P, I, L, VP = C.POINTER(C.c_double), C.c_int, C.c_long, C.c_void_p
        lib.orc_curv_create.argtypes = [C.POINTER(_CurvCfg), P, P, C.POINTER(VP)]
        lib.orc_curv_create.restype = I
        lib.orc_curv_destroy.argtypes = [VP]
        lib.orc_curv_step.argtypes = [VP, L]
        lib.orc_curv_set_prim.argtypes = [VP, P, P, P]
        lib.orc_curv_get_prim.argtypes = [VP, I, P]
        lib.orc_curv_get_prim.restype = I
        lib.orc_curv_get_stored.argtypes = [VP, I, P]
        lib.orc_curv_get_stored.restype = I
        lib.orc_curv_cells.argtypes = [VP, P, P, P]
        lib.orc_curv_residual.argtypes = [VP, P]
        lib.orc_curv_wall_heat.argtypes = [VP, I, P]
        lib.orc_curv_wall_heat.restype = I
        lib.orc_curv_integrals.argtypes = [VP, P]
        _bound = True
    return lib


@dataclasses.dataclass
class CurvConfig:
    """Sides (i-, i+, j-, j+) take PERIODIC, WALL_ISOTHERMAL, WALL_ADIABATIC
    or FARFIELD; temperatures are absolute."""
    bc: Sequence[int] = (0, 0, 1, FARFIELD)
    Tw: Sequence[float] = (0.0, 0.0, 1.0, 0.0)
    up: Sequence[float] = (0.0, 0.0)
    Tb: float = 0.0
    u_inf: Sequence[float] = (0.0, 0.0)
    T_inf: float = 0.0
    nu: float = 0.1
    chi: float = 0.1
    beta_g: float = 0.0
    dtl: float = 1.0
    dt: float = 0.5
    deviation: int = 0
    force_in_predictor: int = 1
    method: int = RTLBFS


class CurvOracle:
    """One oracle run on the mesh with vertex coordinates x, y of shape
    (nj + 1, ni + 1)."""

    def __init__(self, cfg: CurvConfig, x: np.ndarray, y: np.ndarray):
        self._lib = _lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        assert x.shape == y.shape and x.ndim == 2
        self.nj, self.ni = x.shape[0] - 1, x.shape[1] - 1
        self.N = self.ni * self.nj
        c = _CurvCfg()
        c.ni, c.nj = self.ni, self.nj
        c.bc[:] = [int(v) for v in cfg.bc]
        c.Tw[:] = [float(v) for v in cfg.Tw]
        c.up[:] = [float(v) for v in cfg.up]
        c.Tb = cfg.Tb
        c.u_inf[:] = [float(v) for v in cfg.u_inf]
        c.T_inf = cfg.T_inf
        c.nu, c.chi, c.beta_g, c.dtl, c.dt = cfg.nu, cfg.chi, cfg.beta_g, cfg.dtl, cfg.dt
        c.deviation, c.force_in_predictor, c.method = cfg.deviation, cfg.force_in_predictor, cfg.method
        self.cfg, self._c = cfg, c
        h = C.c_void_p()
        if self._lib.orc_curv_create(C.byref(c), _ptr(x), _ptr(y), C.byref(h)) != 0:
            raise ValueError("oracle rejected the mesh or configuration")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_curv_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, n: int = 1):
        self._lib.orc_curv_step(self._h, n)

    def prim(self, f: int) -> np.ndarray:
        """0 rho, 1 u_x, 2 u_y, 3 absolute T."""
        out = np.zeros(self.N)
        if self._lib.orc_curv_get_prim(self._h, f, _ptr(out)) != 0:
            raise IndexError(f)
        return out

    def stored(self, f: int) -> np.ndarray:
        out = np.zeros(self.N)
        if self._lib.orc_curv_get_stored(self._h, f, _ptr(out)) != 0:
            raise IndexError(f)
        return out

    def set_prim(self, rho, u, T):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        assert rho.size == self.N and T.size == self.N and u.size == 2 * self.N
        self._lib.orc_curv_set_prim(self._h, _ptr(rho), _ptr(u), _ptr(T))

    def cells(self):
        """Centroids (x, y) and areas of the cells."""
        cx, cy, a = np.zeros(self.N), np.zeros(self.N), np.zeros(self.N)
        self._lib.orc_curv_cells(self._h, _ptr(cx), _ptr(cy), _ptr(a))
        return cx, cy, a

    def residual(self) -> tuple[float, float]:
        out = np.zeros(2)
        self._lib.orc_curv_residual(self._h, _ptr(out))
        return float(out[0]), float(out[1])

    def wall_heat(self, side: int) -> tuple[float, float]:
        """(sum (T_w - T_P)/d dS, sum dS) over the faces of an isothermal side."""
        out = np.zeros(2)
        if self._lib.orc_curv_wall_heat(self._h, side, _ptr(out)) != 0:
            raise ValueError("side is not an isothermal wall")
        return float(out[0]), float(out[1])

    def integrals(self) -> dict:
        out = np.zeros(4)
        self._lib.orc_curv_integrals(self._h, _ptr(out))
        return dict(mass_dev=out[0], mass=out[1], energy=out[2], volume=out[3])


# ------------------------------------------------------------------ 3D --

class _Curv3Cfg(C.Structure):
    _fields_ = [
        ("n", C.c_int * 3),
        ("bc", C.c_int * 6),
        ("rot", C.c_double * 3),
        ("Tw", C.c_double * 6),
        ("up", C.c_double * 3),
        ("Tb", C.c_double),
        ("nu", C.c_double),
        ("chi", C.c_double),
        ("beta_g", C.c_double),
        ("dtl", C.c_double),
        ("dt", C.c_double),
        ("deviation", C.c_int),
        ("force_in_predictor", C.c_int),
        ("method", C.c_int),
    ]


_bound3 = False


def _lib3():
    global _bound3
    lib = _load()
    if not _bound3:
        P, I, L, VP = C.POINTER(C.c_double), C.c_int, C.c_long, C.c_void_p
        lib.orc_curv3_create.argtypes = [C.POINTER(_Curv3Cfg), P, P, P, C.POINTER(VP)]
        lib.orc_curv3_create.restype = I
        lib.orc_curv3_destroy.argtypes = [VP]
        lib.orc_curv3_step.argtypes = [VP, L]
        lib.orc_curv3_set_prim.argtypes = [VP, P, P, P]
        lib.orc_curv3_get_prim.argtypes = [VP, I, P]
        lib.orc_curv3_get_prim.restype = I
        lib.orc_curv3_cells.argtypes = [VP, P, P, P, P]
        lib.orc_curv3_residual.argtypes = [VP, P]
        lib.orc_curv3_wall_heat.argtypes = [VP, I, P]
        lib.orc_curv3_wall_heat.restype = I
        lib.orc_curv3_integrals.argtypes = [VP, P]
        _bound3 = True
    return lib


@dataclasses.dataclass
class Curv3Config:
    """Sides (i-, i+, j-, j+, k-, k+) take PERIODIC, WALL_ISOTHERMAL or
    WALL_ADIABATIC; rot[a] closes a periodic axis by a rotation about z;
    temperatures are absolute."""
    bc: Sequence[int] = (1, 1, 0, 0, 2, 2)
    rot: Sequence[float] = (0.0, 0.0, 0.0)
    Tw: Sequence[float] = (1.0, 0.0, 0.0, 0.0, 0.0, 0.0)
    up: Sequence[float] = (0.0, 0.0, 0.0)
    Tb: float = 0.5
    nu: float = 0.1
    chi: float = 0.1
    beta_g: float = 0.0
    dtl: float = 1.0
    dt: float = 0.5
    deviation: int = 0
    force_in_predictor: int = 1
    method: int = RTLBFS


class Curv3Oracle:
    """One oracle run on the hexahedral mesh with vertex arrays x, y, z of
    shape (nk + 1, nj + 1, ni + 1)."""

    def __init__(self, cfg: Curv3Config, x, y, z):
        self._lib = _lib3()
        x, y, z = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, z))
        assert x.shape == y.shape == z.shape and x.ndim == 3
        self.n = (x.shape[2] - 1, x.shape[1] - 1, x.shape[0] - 1)
        self.N = self.n[0] * self.n[1] * self.n[2]
        c = _Curv3Cfg()
        c.n[:] = list(self.n)
        c.bc[:] = [int(v) for v in cfg.bc]
        c.rot[:] = [float(v) for v in cfg.rot]
        c.Tw[:] = [float(v) for v in cfg.Tw]
        c.up[:] = [float(v) for v in cfg.up]
        c.Tb = cfg.Tb
        c.nu, c.chi, c.beta_g, c.dtl, c.dt = cfg.nu, cfg.chi, cfg.beta_g, cfg.dtl, cfg.dt
        c.deviation, c.force_in_predictor, c.method = cfg.deviation, cfg.force_in_predictor, cfg.method
        self.cfg, self._c = cfg, c
        h = C.c_void_p()
        if self._lib.orc_curv3_create(C.byref(c), _ptr(x), _ptr(y), _ptr(z), C.byref(h)) != 0:
            raise ValueError("oracle rejected the mesh or configuration")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_curv3_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, n: int = 1):
        self._lib.orc_curv3_step(self._h, n)

    def prim(self, f: int) -> np.ndarray:
        """0 rho, 1..3 u, 4 absolute T."""
        out = np.zeros(self.N)
        if self._lib.orc_curv3_get_prim(self._h, f, _ptr(out)) != 0:
            raise IndexError(f)
        return out

    def set_prim(self, rho, u, T):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        assert rho.size == self.N and T.size == self.N and u.size == 3 * self.N
        self._lib.orc_curv3_set_prim(self._h, _ptr(rho), _ptr(u), _ptr(T))

    def cells(self):
        out = [np.zeros(self.N) for _ in range(4)]
        self._lib.orc_curv3_cells(self._h, *(_ptr(v) for v in out))
        return tuple(out)

    def residual(self) -> tuple[float, float]:
        out = np.zeros(2)
        self._lib.orc_curv3_residual(self._h, _ptr(out))
        return float(out[0]), float(out[1])

    def wall_heat(self, side: int) -> tuple[float, float]:
        out = np.zeros(2)
        if self._lib.orc_curv3_wall_heat(self._h, side, _ptr(out)) != 0:
            raise ValueError("side is not an isothermal wall")
        return float(out[0]), float(out[1])

    def integrals(self) -> dict:
        out = np.zeros(4)
        self._lib.orc_curv3_integrals(self._h, _ptr(out))
        return dict(mass_dev=out[0], mass=out[1], energy=out[2], volume=out[3])
