"""ctypes wrapper of the plain C oracle (test infrastructure only).

The oracle follows Sec. 3.2 of Lu, Dai & Yu (arXiv 2202.13449): predictor by
finite differences of Eqs. 46-48 on a face-centred unit lattice filled by
Eq. 29, corrector Eqs. 57-59, body force Eq. 64, residual Eq. 65.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
from typing import Sequence

import numpy as np

from .build import LIB, SRCS, build

PERIODIC, WALL_ISOTHERMAL, WALL_ADIABATIC = 0, 1, 2
INIT_REST, INIT_CONDUCTION = 0, 1
RTLBFS, TLBFS = 0, 1  # interior-face flux: Sec. 3.2 (Eqs. 46-48, 57-59) or Sec. 2.2 (Eqs. 29-40)


class _Cfg(C.Structure):
    _fields_ = [
        ("dim", C.c_int),
        ("n", C.c_int * 3),
        ("stretch", C.c_double * 3),
        ("bc", C.c_int * 6),
        ("Tw", C.c_double * 6),
        ("gravity_axis", C.c_int),
        ("nu", C.c_double),
        ("chi", C.c_double),
        ("beta_g", C.c_double),
        ("dtl", C.c_double),
        ("dt", C.c_double),
        ("deviation", C.c_int),
        ("force_in_predictor", C.c_int),
        ("init", C.c_int),
        ("seed", C.c_uint64),
        ("noise_amp", C.c_double),
        ("method", C.c_int),
    ]


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    newest = max(os.path.getmtime(f) for f in SRCS + [f[:-2] + ".h" for f in SRCS])
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < newest:
        build()
    lib = C.CDLL(LIB)
    D, P, I, L = C.c_double, C.POINTER(C.c_double), C.c_int, C.c_long
    VP = C.c_void_p
    lib.orc_mesh_nodes.argtypes = [I, D, P]
    lib.orc_mesh_nodes.restype = D
    lib.orc_physics_from_ra.argtypes = [D, D, D, D, P]
    lib.orc_splitmix_uniform.argtypes = [C.c_uint64, C.c_uint64]
    lib.orc_splitmix_uniform.restype = D
    lib.orc_create.argtypes = [C.POINTER(_Cfg), C.POINTER(VP)]
    lib.orc_create.restype = I
    lib.orc_destroy.argtypes = [VP]
    lib.orc_cells.argtypes = [VP]
    lib.orc_cells.restype = L
    lib.orc_step.argtypes = [VP, L]
    lib.orc_step.restype = I
    lib.orc_steps_done.argtypes = [VP]
    lib.orc_steps_done.restype = L
    for fn in (lib.orc_get_stored, lib.orc_set_stored, lib.orc_get_prim):
        fn.argtypes = [VP, I, P]
        fn.restype = I
    lib.orc_set_prim.argtypes = [VP, P, P, P]
    lib.orc_axis.argtypes = [VP, I, P, P]
    lib.orc_residual.argtypes = [VP, P]
    lib.orc_nusselt.argtypes = [VP, P]
    lib.orc_nusselt.restype = I
    lib.orc_integrals.argtypes = [VP, P]
    lib.orc_taus.argtypes = [VP, P]
    lib.orc_face_flux.argtypes = [C.POINTER(_Cfg), I, P, P, P, P, D, D, P, P]
    lib.orc_face_flux_frame.argtypes = [C.POINTER(_Cfg), P, P, P, P, P, P, P, D, P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclasses.dataclass
class OracleConfig:
    """Problem definition in lattice units (finest cell = 1, c = 1)."""
    dim: int = 2
    n: Sequence[int] = (64, 64, 1)
    stretch: Sequence[float] = (0.0, 0.0, 0.0)
    bc: Sequence[int] = (WALL_ISOTHERMAL, WALL_ISOTHERMAL, WALL_ADIABATIC, WALL_ADIABATIC, PERIODIC, PERIODIC)
    Tw: Sequence[float] = (0.5, -0.5, 0.0, 0.0, 0.0, 0.0)
    gravity_axis: int = 1
    nu: float = 0.1
    chi: float = 0.1
    beta_g: float = 0.0
    dtl: float = 1.0
    dt: float = 0.5
    deviation: int = 0
    force_in_predictor: int = 1
    init: int = INIT_REST
    seed: int = 0
    noise_amp: float = 0.0
    method: int = RTLBFS

    def to_c(self) -> _Cfg:
        c = _Cfg()
        c.dim = self.dim
        n = list(self.n) + [1] * (3 - len(self.n))
        c.n[:] = [int(v) for v in n[:3]]
        st = list(self.stretch) + [0.0] * (3 - len(self.stretch))
        c.stretch[:] = [float(v) for v in st[:3]]
        c.bc[:] = [int(v) for v in self.bc]
        c.Tw[:] = [float(v) for v in self.Tw]
        c.gravity_axis = self.gravity_axis
        c.nu, c.chi, c.beta_g = self.nu, self.chi, self.beta_g
        c.dtl, c.dt = self.dtl, self.dt
        c.deviation = self.deviation
        c.force_in_predictor = self.force_in_predictor
        c.init = self.init
        c.seed = self.seed
        c.noise_amp = self.noise_amp
        c.method = self.method
        return c


def mesh_nodes(n: int, stretch: float) -> tuple[np.ndarray, float]:
    lib = _load()
    x = np.zeros(n + 1)
    L = lib.orc_mesh_nodes(n, stretch, _ptr(x))
    return x, L


def physics_from_ra(Ra: float, Pr: float, Ma: float, L: float) -> tuple[float, float, float]:
    lib = _load()
    out = np.zeros(3)
    lib.orc_physics_from_ra(Ra, Pr, Ma, L, _ptr(out))
    return float(out[0]), float(out[1]), float(out[2])


def splitmix_uniform(seed: int, i: int) -> float:
    return _load().orc_splitmix_uniform(seed, i)


def face_flux(cfg: OracleConfig, axis: int, primL, gradL, primR, gradR, dL: float, dR: float):
    """One interior-face flux; grad arrays are (D+2, 3).  Returns (flux, pred)."""
    lib = _load()
    c = cfg.to_c()
    D = cfg.dim
    pL = np.ascontiguousarray(primL, dtype=np.float64)
    pR = np.ascontiguousarray(primR, dtype=np.float64)
    gL = np.zeros((D + 2, 3))
    gR = np.zeros((D + 2, 3))
    aL = np.asarray(gradL, dtype=np.float64).reshape(D + 2, -1)
    aR = np.asarray(gradR, dtype=np.float64).reshape(D + 2, -1)
    gL[:, :aL.shape[1]] = aL
    gR[:, :aR.shape[1]] = aR
    flux = np.zeros(D + 2)
    pred = np.zeros(D + 2)
    lib.orc_face_flux(C.byref(c), axis, _ptr(pL), _ptr(gL), _ptr(pR), _ptr(gR), dL, dR, _ptr(flux), _ptr(pred))
    return flux, pred


def face_flux_frame(cfg: OracleConfig, primL, gradL, primR, gradR, xSL, xSR, fdir, Tb: float):
    """The interior-face flux in its own frame (axis 0 = face normal): grad
    arrays (D+2, D), offsets xSL = x_S - x_L and xSR = x_S - x_R, buoyancy
    direction fdir, absolute buoyancy reference Tb.  Returns (flux, pred)."""
    lib = _load()
    c = cfg.to_c()
    D = cfg.dim
    vec = lambda v: np.concatenate([np.asarray(v, dtype=np.float64).reshape(-1), np.zeros(3)])[:3].copy()
    pL = np.ascontiguousarray(primL, dtype=np.float64)
    pR = np.ascontiguousarray(primR, dtype=np.float64)
    gL = np.zeros((D + 2, 3))
    gR = np.zeros((D + 2, 3))
    aL = np.asarray(gradL, dtype=np.float64).reshape(D + 2, -1)
    aR = np.asarray(gradR, dtype=np.float64).reshape(D + 2, -1)
    gL[:, :aL.shape[1]] = aL
    gR[:, :aR.shape[1]] = aR
    flux = np.zeros(D + 2)
    pred = np.zeros(D + 2)
    lib.orc_face_flux_frame(C.byref(c), _ptr(pL), _ptr(gL), _ptr(pR), _ptr(gR), _ptr(vec(xSL)), _ptr(vec(xSR)),
                            _ptr(vec(fdir)), Tb, _ptr(flux), _ptr(pred))
    return flux, pred


class Oracle:
    """One oracle run: create, step, read fields and diagnostics."""

    def __init__(self, cfg: OracleConfig):
        self.cfg = cfg
        self._lib = _load()
        self._c = cfg.to_c()
        h = C.c_void_p()
        rc = self._lib.orc_create(C.byref(self._c), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle rejected the configuration (rc={rc})")
        self._h = h
        self.D = cfg.dim
        self.N = self._lib.orc_cells(h)
        n = list(cfg.n) + [1, 1]
        self.shape = tuple(int(v) for v in (n[:3] if cfg.dim == 3 else n[:2]))

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def step(self, n: int = 1):
        self._lib.orc_step(self._h, n)

    @property
    def steps(self) -> int:
        return self._lib.orc_steps_done(self._h)

    def _field(self, fn, f: int) -> np.ndarray:
        out = np.zeros(self.N)
        if fn(self._h, f, _ptr(out)) != 0:
            raise IndexError(f)
        return out

    def stored(self, f: int) -> np.ndarray:
        return self._field(self._lib.orc_get_stored, f)

    def set_stored(self, f: int, v: np.ndarray):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1)
        assert v.size == self.N
        self._lib.orc_set_stored(self._h, f, _ptr(v))

    def prim(self, f: int) -> np.ndarray:
        """Absolute primitive: 0 rho, 1..D u_a, D+1 T."""
        return self._field(self._lib.orc_get_prim, f)

    def grid(self, f_values: np.ndarray) -> np.ndarray:
        """Reshape a flat field to (nz, ny, nx) / (ny, nx) with x fastest."""
        return f_values.reshape(tuple(reversed(self.shape)))

    def set_prim(self, rho: np.ndarray, u: np.ndarray, T: np.ndarray):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        assert rho.size == self.N and T.size == self.N and u.size == self.D * self.N
        self._lib.orc_set_prim(self._h, _ptr(rho), _ptr(u), _ptr(T))

    def axis(self, a: int) -> tuple[np.ndarray, np.ndarray]:
        n = self.shape[a]
        c, w = np.zeros(n), np.zeros(n)
        self._lib.orc_axis(self._h, a, _ptr(c), _ptr(w))
        return c, w

    def residual(self) -> tuple[float, float]:
        out = np.zeros(2)
        self._lib.orc_residual(self._h, _ptr(out))
        return float(out[0]), float(out[1])

    def nusselt(self) -> dict:
        out = np.zeros(5)
        if self._lib.orc_nusselt(self._h, _ptr(out)) != 0:
            raise ValueError("no pair of isothermal walls")
        return dict(hot_avg=out[0], hot_max=out[1], cold_avg=out[2], cold_max=out[3], volume=out[4])

    def integrals(self) -> dict:
        out = np.zeros(5)
        self._lib.orc_integrals(self._h, _ptr(out))
        return dict(mass_dev=out[0], mass=out[1], energy=out[2], theta=out[3], volume=out[4])

    def taus(self) -> tuple[float, float]:
        out = np.zeros(2)
        self._lib.orc_taus(self._h, _ptr(out))
        return float(out[0]), float(out[1])
