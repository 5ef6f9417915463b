"""Python binding of the gfx950 RTLBFS library (ctypes argument marshalling).

Every step of the method runs in the HIP kernels of librtlbfs.so; this module
only converts arguments, owns the torch-allocated device workspace and passes
torch's current HIP stream.  It fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librtlbfs.so")

OK, EINVAL, ENOMEM, EDEVICE, EDIVERGED, EUNSUPPORTED, ESTATE = 0, -1, -2, -3, -4, -5, -6
PERIODIC, WALL_ISOTHERMAL, WALL_ADIABATIC, FARFIELD = 0, 1, 2, 3
FP64_PLAIN, FP32_DEV, FP64_DEV = 0, 1, 2
INIT_REST, INIT_CONDUCTION = 0, 1
METHOD_RTLBFS, METHOD_TLBFS = 0, 1


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("n", C.c_int * 3), ("stretch", C.c_double * 3)]


class BC(C.Structure):
    _fields_ = [("kind", C.c_int * 6), ("Tdev", C.c_double * 6), ("gravity_axis", C.c_int)]


class Opts(C.Structure):
    _fields_ = [
        ("precision", C.c_int),
        ("dtl", C.c_double),
        ("dt", C.c_double),
        ("seed", C.c_uint64),
        ("noise_amp", C.c_double),
        ("init", C.c_int),
        ("residual_every", C.c_int),
        ("mass_fix_every", C.c_int),
        ("graph_steps", C.c_int),
        ("buoyancy_update_only", C.c_int),
        ("phys_given", C.c_int),
        ("nu", C.c_double),
        ("chi", C.c_double),
        ("beta_g", C.c_double),
        ("tile", C.c_int),
        ("round_nearest", C.c_int),
        ("method", C.c_int),
        ("max_mach", C.c_double),
    ]


class CurvMesh(C.Structure):
    _fields_ = [("n", C.c_int * 2), ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double))]


class CurvBC(C.Structure):
    _fields_ = [("kind", C.c_int * 4), ("Tw", C.c_double * 4), ("up", C.c_double * 2), ("T_ref", C.c_double),
                ("u_inf", C.c_double * 2), ("T_inf", C.c_double)]


class Curv3Mesh(C.Structure):
    _fields_ = [("n", C.c_int * 3), ("x", C.POINTER(C.c_double)), ("y", C.POINTER(C.c_double)),
                ("z", C.POINTER(C.c_double))]


class Curv3BC(C.Structure):
    _fields_ = [("kind", C.c_int * 6), ("rot", C.c_double * 3), ("Tw", C.c_double * 6), ("up", C.c_double * 3),
                ("T_ref", C.c_double)]


class NuOut(C.Structure):
    _fields_ = [("hot_avg", C.c_double), ("hot_max", C.c_double), ("cold_avg", C.c_double),
                ("cold_max", C.c_double), ("volume", C.c_double)]


class Info(C.Structure):
    _fields_ = [
        ("cells", C.c_int64),
        ("steps", C.c_int64),
        ("L", C.c_double),
        ("nu", C.c_double),
        ("chi", C.c_double),
        ("beta_g", C.c_double),
        ("tau_f", C.c_double),
        ("tau_g", C.c_double),
        ("dtl", C.c_double),
        ("dt", C.c_double),
        ("length", C.c_double * 3),
        ("precision", C.c_int),
        ("tile_x", C.c_int),
        ("tile_y", C.c_int),
        ("tile_z", C.c_int),
        ("tune_ms", C.c_double * 16),
        ("steps_per_launch", C.c_int),
    ]


class Checkpoint(C.Structure):
    _fields_ = [("steps", C.c_int64), ("since_fix", C.c_int64), ("mass0", C.c_double)]


class RtlbfsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (code {code})")
        self.code = code


_lib = None


def load_library() -> C.CDLL:
    """Load librtlbfs.so (built in-tree by build.py); raise if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_2202_13449_amd/build.py`")
    # torch must load its HIP runtime first: the library then binds to that
    # same runtime (same SONAME), so device pointers and streams are shared.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    I, D, VP, SZ, I64 = C.c_int, C.c_double, C.c_void_p, C.c_size_t, C.c_int64
    PD = C.POINTER(C.c_double)
    lib.rtlbfs_strerror.argtypes = [I]
    lib.rtlbfs_strerror.restype = C.c_char_p
    lib.rtlbfs_last_error.argtypes = [VP]
    lib.rtlbfs_last_error.restype = C.c_char_p
    lib.rtlbfs_opts_init.argtypes = [C.POINTER(Opts)]
    lib.rtlbfs_mesh_nodes.argtypes = [I, D, PD, PD]
    lib.rtlbfs_workspace_bytes.argtypes = [C.POINTER(Mesh), C.POINTER(Opts)]
    lib.rtlbfs_workspace_bytes.restype = SZ
    lib.rtlbfs_create.argtypes = [C.POINTER(Mesh), D, D, D, C.POINTER(BC), C.POINTER(Opts), VP, VP, SZ,
                                  C.POINTER(VP)]
    lib.rtlbfs_step.argtypes = [VP, I64]
    lib.rtlbfs_sync.argtypes = [VP]
    lib.rtlbfs_residual.argtypes = [VP, PD, PD]
    lib.rtlbfs_nusselt.argtypes = [VP, C.POINTER(NuOut)]
    lib.rtlbfs_integrals.argtypes = [VP, PD]
    lib.rtlbfs_get_field.argtypes = [VP, I, PD, SZ]
    lib.rtlbfs_get_stored.argtypes = [VP, I, PD, SZ]
    lib.rtlbfs_set_state.argtypes = [VP, PD, PD, PD, SZ]
    lib.rtlbfs_get_info.argtypes = [VP, C.POINTER(Info)]
    lib.rtlbfs_destroy.argtypes = [VP]
    lib.rtlbfs_curv_workspace_bytes.argtypes = [C.POINTER(CurvMesh), C.POINTER(Opts)]
    lib.rtlbfs_curv_workspace_bytes.restype = SZ
    lib.rtlbfs_curv_create.argtypes = [C.POINTER(CurvMesh), D, D, D, C.POINTER(CurvBC), C.POINTER(Opts), VP, VP, SZ,
                                       C.POINTER(VP)]
    lib.rtlbfs_wall_heat.argtypes = [VP, I, PD]
    lib.rtlbfs_curv_cells.argtypes = [VP, PD, PD, PD, SZ]
    lib.rtlbfs_curv3_workspace_bytes.argtypes = [C.POINTER(Curv3Mesh), C.POINTER(Opts)]
    lib.rtlbfs_curv3_workspace_bytes.restype = SZ
    lib.rtlbfs_curv3_create.argtypes = [C.POINTER(Curv3Mesh), D, D, D, C.POINTER(Curv3BC), C.POINTER(Opts), VP, VP,
                                        SZ, C.POINTER(VP)]
    lib.rtlbfs_curv3_cells.argtypes = [VP, PD, PD, PD, PD, SZ]
    lib.rtlbfs_batch_workspace_bytes.argtypes = [I, C.POINTER(Mesh), C.POINTER(Opts)]
    lib.rtlbfs_batch_workspace_bytes.restype = SZ
    lib.rtlbfs_batch_create.argtypes = [I, C.POINTER(Mesh), PD, PD, D, C.POINTER(BC), C.POINTER(Opts), VP, VP, SZ,
                                        C.POINTER(VP)]
    lib.rtlbfs_batch_step.argtypes = [VP, I64]
    lib.rtlbfs_batch_nusselt.argtypes = [VP, I, C.POINTER(NuOut)]
    lib.rtlbfs_batch_residual.argtypes = [VP, I, PD, PD]
    lib.rtlbfs_batch_get_field.argtypes = [VP, I, I, PD, SZ]
    lib.rtlbfs_batch_get_info.argtypes = [VP, I, C.POINTER(Info)]
    lib.rtlbfs_batch_sync.argtypes = [VP]
    lib.rtlbfs_batch_diverged.argtypes = [VP, C.POINTER(C.c_int)]
    lib.rtlbfs_batch_destroy.argtypes = [VP]
    lib.rtlbfs_residual_states.argtypes = [I, I, I64, I64, VP, VP, VP, VP]
    lib.rtlbfs_get_checkpoint.argtypes = [VP, C.POINTER(Checkpoint)]
    lib.rtlbfs_restore.argtypes = [VP, PD, SZ, C.POINTER(Checkpoint)]
    for name in ("rtlbfs_opts_init", "rtlbfs_mesh_nodes", "rtlbfs_create", "rtlbfs_step", "rtlbfs_sync",
                 "rtlbfs_residual", "rtlbfs_nusselt", "rtlbfs_integrals", "rtlbfs_get_field", "rtlbfs_get_stored",
                 "rtlbfs_set_state", "rtlbfs_get_info", "rtlbfs_destroy", "rtlbfs_curv_create", "rtlbfs_wall_heat",
                 "rtlbfs_curv_cells", "rtlbfs_curv3_create", "rtlbfs_curv3_cells", "rtlbfs_batch_create",
                 "rtlbfs_batch_step",
                 "rtlbfs_batch_nusselt", "rtlbfs_batch_residual", "rtlbfs_batch_get_field", "rtlbfs_batch_get_info",
                 "rtlbfs_batch_sync", "rtlbfs_batch_diverged", "rtlbfs_batch_destroy", "rtlbfs_residual_states",
                 "rtlbfs_get_checkpoint", "rtlbfs_restore"):
        getattr(lib, name).restype = I
    _lib = lib
    return lib


def _pd(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def strerror(code: int) -> str:
    return load_library().rtlbfs_strerror(code).decode()


def make_mesh(dim: int, n: Sequence[int], stretch: Sequence[float] = (0.0, 0.0, 0.0)) -> Mesh:
    m = Mesh()
    m.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    m.n[:] = [int(v) for v in nn[:3]]
    st = list(stretch) + [0.0] * (3 - len(stretch))
    m.stretch[:] = [float(v) for v in st[:3]]
    return m


def make_bc(kind: Sequence[int], Tdev: Sequence[float], gravity_axis: int) -> BC:
    b = BC()
    k = list(kind) + [PERIODIC] * (6 - len(kind))
    t = list(Tdev) + [0.0] * (6 - len(Tdev))
    b.kind[:] = [int(v) for v in k[:6]]
    b.Tdev[:] = [float(v) for v in t[:6]]
    b.gravity_axis = gravity_axis
    return b


def make_opts(**kw) -> Opts:
    o = Opts()
    load_library().rtlbfs_opts_init(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise AttributeError(k)
        setattr(o, k, v)
    return o


def mesh_nodes(n: int, stretch: float) -> tuple[np.ndarray, float]:
    x = np.zeros(n + 1)
    L = C.c_double()
    rc = load_library().rtlbfs_mesh_nodes(n, stretch, _pd(x), C.byref(L))
    if rc != OK:
        raise RtlbfsError(rc, strerror(rc))
    return x, L.value


def _torch_stream_and_alloc(nbytes: int):
    import torch

    if not torch.cuda.is_available():
        raise RuntimeError("the RTLBFS library needs a HIP GPU (torch.cuda.is_available() is False)")
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    return ws, stream


def residual_states(dim: int, precision: int, cells: int, fstride: int, old_state, new_state, out) -> None:
    """Eq. 65 ratios between two stored states in device memory (torch
    tensors in the handle's SoA layout: dim + 2 fields, `fstride` elements
    apart) into `out` (a float64 device tensor of 2), through
    rtlbfs_residual_states on torch's current stream.  Allocates nothing."""
    import torch

    for t in (old_state, new_state, out):
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
            raise ValueError("device tensors expected")
    want = torch.float32 if precision == FP32_DEV else torch.float64
    if old_state.dtype != want or new_state.dtype != want or out.dtype != torch.float64 or out.numel() < 2:
        raise ValueError("dtype or size mismatch")
    if old_state.numel() < (dim + 2) * fstride or new_state.numel() < (dim + 2) * fstride:
        raise ValueError("state tensors shorter than (dim + 2) * fstride")
    rc = load_library().rtlbfs_residual_states(dim, precision, int(cells), int(fstride),
                                                C.c_void_p(old_state.data_ptr()), C.c_void_p(new_state.data_ptr()),
                                                C.c_void_p(out.data_ptr()),
                                                C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if rc != OK:
        raise RtlbfsError(rc, "rtlbfs_residual_states: " + strerror(rc))


class Solver:
    """One domain advanced by the gfx950 kernels.

    Device memory is a torch uint8 tensor owned by this object; work goes on
    torch's current HIP stream at construction time.
    """

    def __init__(self, dim: int, n: Sequence[int], stretch: Sequence[float], kind: Sequence[int],
                 Tdev: Sequence[float], gravity_axis: int, Ra: float = 1e3, Pr: float = 0.71, Ma: float = 0.1,
                 **opts):
        self._lib = load_library()
        self.dim = dim
        self.mesh = make_mesh(dim, n, stretch)
        self.bc = make_bc(kind, Tdev, gravity_axis)
        self.opts = make_opts(**opts)
        nbytes = self._lib.rtlbfs_workspace_bytes(C.byref(self.mesh), C.byref(self.opts))
        if nbytes == 0:
            raise RtlbfsError(EINVAL, "invalid mesh")
        self.workspace, self.stream = _torch_stream_and_alloc(nbytes)
        h = C.c_void_p()
        rc = self._lib.rtlbfs_create(C.byref(self.mesh), Ra, Pr, Ma, C.byref(self.bc), C.byref(self.opts),
                                     C.c_void_p(self.stream), C.c_void_p(self.workspace.data_ptr()),
                                     self.workspace.numel(), C.byref(h))
        if rc != OK:
            detail = self._lib.rtlbfs_last_error(None).decode()
            raise RtlbfsError(rc, f"rtlbfs_create: {strerror(rc)}: {detail}")
        self._h = h
        self.info = self.get_info()
        self.cells = int(self.info.cells)
        nn = [int(v) for v in self.mesh.n]
        self.shape = tuple(nn[:dim])

    # -- lifetime --
    def close(self):
        if getattr(self, "_h", None):
            self._lib.rtlbfs_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc != OK:
            detail = self._lib.rtlbfs_last_error(self._h).decode() if self._h else ""
            raise RtlbfsError(rc, f"{what}: {strerror(rc)} {detail}".strip())

    # -- stepping and diagnostics --
    def step(self, n: int = 1):
        self._check(self._lib.rtlbfs_step(self._h, int(n)), "rtlbfs_step")

    def sync(self):
        self._check(self._lib.rtlbfs_sync(self._h), "rtlbfs_sync")

    def residual(self) -> tuple[float, float]:
        a, b = C.c_double(), C.c_double()
        self._check(self._lib.rtlbfs_residual(self._h, C.byref(a), C.byref(b)), "rtlbfs_residual")
        return a.value, b.value

    def nusselt(self) -> dict:
        o = NuOut()
        self._check(self._lib.rtlbfs_nusselt(self._h, C.byref(o)), "rtlbfs_nusselt")
        return dict(hot_avg=o.hot_avg, hot_max=o.hot_max, cold_avg=o.cold_avg, cold_max=o.cold_max,
                    volume=o.volume)

    def integrals(self) -> dict:
        out = np.zeros(3)
        self._check(self._lib.rtlbfs_integrals(self._h, _pd(out)), "rtlbfs_integrals")
        return dict(mass_dev=out[0], theta=out[1], volume=out[2])

    def get_info(self) -> Info:
        i = Info()
        self._check(self._lib.rtlbfs_get_info(self._h, C.byref(i)), "rtlbfs_get_info")
        return i

    # -- fields --
    def field(self, f: int) -> np.ndarray:
        out = np.zeros(self.cells)
        self._check(self._lib.rtlbfs_get_field(self._h, f, _pd(out), out.size), "rtlbfs_get_field")
        return out

    def stored(self, f: int) -> np.ndarray:
        out = np.zeros(self.cells)
        self._check(self._lib.rtlbfs_get_stored(self._h, f, _pd(out), out.size), "rtlbfs_get_stored")
        return out

    def checkpoint(self) -> tuple[np.ndarray, Checkpoint]:
        """The stored fields (dim + 2, cells) and the step counters of the
        current state."""
        ck = Checkpoint()
        self._check(self._lib.rtlbfs_get_checkpoint(self._h, C.byref(ck)), "rtlbfs_get_checkpoint")
        return np.stack([self.stored(f) for f in range(self.dim + 2)]), ck

    def restore(self, stored: np.ndarray, ck: Checkpoint):
        """Continue from a checkpoint taken with checkpoint()."""
        buf = np.ascontiguousarray(stored, dtype=np.float64).reshape(-1)
        self._check(self._lib.rtlbfs_restore(self._h, _pd(buf), buf.size, C.byref(ck)), "rtlbfs_restore")

    def set_state(self, rho: np.ndarray, u: np.ndarray, T: np.ndarray):
        rho = np.ascontiguousarray(rho, dtype=np.float64).reshape(-1)
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
        T = np.ascontiguousarray(T, dtype=np.float64).reshape(-1)
        if rho.size != self.cells or T.size != self.cells or u.size != self.dim * self.cells:
            raise ValueError("state arrays do not match the mesh")
        self._check(self._lib.rtlbfs_set_state(self._h, _pd(rho), _pd(u), _pd(T), self.cells), "rtlbfs_set_state")

    def grid(self, values: np.ndarray) -> np.ndarray:
        return values.reshape(tuple(reversed(self.shape)))


class CurvSolver(Solver):
    """One 2D body-fitted (structured curvilinear) mesh advanced by the gfx950
    kernels: vertex arrays x, y of shape (nj + 1, ni + 1), sides (i-, i+, j-,
    j+) of kinds PERIODIC / WALL_ISOTHERMAL / WALL_ADIABATIC / FARFIELD,
    absolute temperatures, buoyancy beta_g (T - T_ref) along the unit vector
    `up`, far-field state (u_inf, T_inf, rho = 1) that is also the initial
    state."""

    def __init__(self, x: np.ndarray, y: np.ndarray, kind: Sequence[int], Tw: Sequence[float] = (0.0,) * 4,
                 up: Sequence[float] = (0.0, 0.0), T_ref: float = 0.0, u_inf: Sequence[float] = (0.0, 0.0),
                 T_inf: float = 0.0, nu: float = 0.1, chi: float = 0.1, beta_g: float = 0.0, **opts):
        self._h = None
        self._lib = load_library()
        x = np.ascontiguousarray(x, dtype=np.float64)
        y = np.ascontiguousarray(y, dtype=np.float64)
        if x.ndim != 2 or x.shape != y.shape:
            raise ValueError("x and y must be (nj + 1, ni + 1) arrays")
        self.dim = 2
        self.cmesh = CurvMesh()
        self.cmesh.n[:] = [x.shape[1] - 1, x.shape[0] - 1]
        self.cmesh.x, self.cmesh.y = _pd(x), _pd(y)
        self._xy = (x, y)  # keep the vertex arrays alive for the create call
        self.cbc = CurvBC()
        self.cbc.kind[:] = [int(v) for v in kind]
        self.cbc.Tw[:] = [float(v) for v in Tw]
        self.cbc.up[:] = [float(v) for v in up]
        self.cbc.T_ref = float(T_ref)
        self.cbc.u_inf[:] = [float(v) for v in u_inf]
        self.cbc.T_inf = float(T_inf)
        self.opts = make_opts(**opts)
        nbytes = self._lib.rtlbfs_curv_workspace_bytes(C.byref(self.cmesh), C.byref(self.opts))
        if nbytes == 0:
            raise RtlbfsError(EINVAL, "invalid mesh")
        self.workspace, self.stream = _torch_stream_and_alloc(nbytes)
        h = C.c_void_p()
        rc = self._lib.rtlbfs_curv_create(C.byref(self.cmesh), nu, chi, beta_g, C.byref(self.cbc),
                                          C.byref(self.opts), C.c_void_p(self.stream),
                                          C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(), C.byref(h))
        if rc != OK:
            detail = self._lib.rtlbfs_last_error(None).decode()
            raise RtlbfsError(rc, f"rtlbfs_curv_create: {strerror(rc)}: {detail}")
        self._h = h
        self.info = self.get_info()
        self.cells = int(self.info.cells)
        self.shape = (int(self.cmesh.n[0]), int(self.cmesh.n[1]))

    def wall_heat(self, side: int) -> tuple[float, float]:
        """(sum (T_w - T_P)/d dS, sum dS) over the faces of an isothermal side."""
        out = np.zeros(2)
        self._check(self._lib.rtlbfs_wall_heat(self._h, side, _pd(out)), "rtlbfs_wall_heat")
        return float(out[0]), float(out[1])

    def geometry(self) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
        """Cell centroids (x, y) and areas the library derived."""
        cx, cy, a = np.zeros(self.cells), np.zeros(self.cells), np.zeros(self.cells)
        self._check(self._lib.rtlbfs_curv_cells(self._h, _pd(cx), _pd(cy), _pd(a), self.cells), "rtlbfs_curv_cells")
        return cx, cy, a


class Curv3Solver(Solver):
    """One 3D body-fitted (structured curvilinear) hexahedral mesh advanced by
    the gfx950 kernels: vertex arrays x, y, z of shape (nk + 1, nj + 1, ni + 1),
    sides (i-, i+, j-, j+, k-, k+) PERIODIC / WALL_ISOTHERMAL / WALL_ADIABATIC,
    `rot` closing periodic axes by a rotation about z, absolute temperatures,
    buoyancy beta_g (T - T_ref) along the unit vector `up`; starts at rest at
    T = T_ref."""

    def __init__(self, x, y, z, kind: Sequence[int], rot: Sequence[float] = (0.0, 0.0, 0.0),
                 Tw: Sequence[float] = (0.0,) * 6, up: Sequence[float] = (0.0, 0.0, 0.0), T_ref: float = 0.5,
                 nu: float = 0.1, chi: float = 0.1, beta_g: float = 0.0, **opts):
        self._h = None
        self._lib = load_library()
        x, y, z = (np.ascontiguousarray(v, dtype=np.float64) for v in (x, y, z))
        if x.ndim != 3 or not (x.shape == y.shape == z.shape):
            raise ValueError("x, y, z must be (nk + 1, nj + 1, ni + 1) arrays")
        self.dim = 3
        self.cmesh = Curv3Mesh()
        self.cmesh.n[:] = [x.shape[2] - 1, x.shape[1] - 1, x.shape[0] - 1]
        self.cmesh.x, self.cmesh.y, self.cmesh.z = _pd(x), _pd(y), _pd(z)
        self._xyz = (x, y, z)
        self.cbc = Curv3BC()
        self.cbc.kind[:] = [int(v) for v in kind]
        self.cbc.rot[:] = [float(v) for v in rot]
        self.cbc.Tw[:] = [float(v) for v in Tw]
        self.cbc.up[:] = [float(v) for v in up]
        self.cbc.T_ref = float(T_ref)
        self.opts = make_opts(**opts)
        nbytes = self._lib.rtlbfs_curv3_workspace_bytes(C.byref(self.cmesh), C.byref(self.opts))
        if nbytes == 0:
            raise RtlbfsError(EINVAL, "invalid mesh")
        self.workspace, self.stream = _torch_stream_and_alloc(nbytes)
        h = C.c_void_p()
        rc = self._lib.rtlbfs_curv3_create(C.byref(self.cmesh), nu, chi, beta_g, C.byref(self.cbc),
                                           C.byref(self.opts), C.c_void_p(self.stream),
                                           C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(), C.byref(h))
        if rc != OK:
            detail = self._lib.rtlbfs_last_error(None).decode()
            raise RtlbfsError(rc, f"rtlbfs_curv3_create: {strerror(rc)}: {detail}")
        self._h = h
        self.info = self.get_info()
        self.cells = int(self.info.cells)
        self.shape = tuple(int(v) for v in self.cmesh.n)

    def wall_heat(self, side: int) -> tuple[float, float]:
        """(sum (T_w - T_P)/d dS, sum dS) over the faces of an isothermal side."""
        out = np.zeros(2)
        self._check(self._lib.rtlbfs_wall_heat(self._h, side, _pd(out)), "rtlbfs_wall_heat")
        return float(out[0]), float(out[1])

    def geometry(self):
        """Cell centroids (x, y, z) and volumes the library derived."""
        out = [np.zeros(self.cells) for _ in range(4)]
        self._check(self._lib.rtlbfs_curv3_cells(self._h, *(_pd(v) for v in out), self.cells), "rtlbfs_curv3_cells")
        return tuple(out)


class Batch:
    """Many independent 2D domains stepped by one kernel launch per step."""

    def __init__(self, meshes: Sequence[Mesh], Ra: Sequence[float], Pr: Sequence[float], bcs: Sequence[BC],
                 Ma: float = 0.1, **opts):
        self._lib = load_library()
        self.count = len(meshes)
        self.meshes = (Mesh * self.count)(*meshes)
        self.bcs = (BC * self.count)(*bcs)
        self.Ra = np.ascontiguousarray(Ra, dtype=np.float64)
        self.Pr = np.ascontiguousarray(Pr, dtype=np.float64)
        self.opts = make_opts(**opts)
        nbytes = self._lib.rtlbfs_batch_workspace_bytes(self.count, self.meshes, C.byref(self.opts))
        if nbytes == 0:
            raise RtlbfsError(EINVAL, "invalid batch")
        self.workspace, self.stream = _torch_stream_and_alloc(nbytes)
        h = C.c_void_p()
        rc = self._lib.rtlbfs_batch_create(self.count, self.meshes, _pd(self.Ra), _pd(self.Pr), Ma, self.bcs,
                                           C.byref(self.opts), C.c_void_p(self.stream),
                                           C.c_void_p(self.workspace.data_ptr()), self.workspace.numel(),
                                           C.byref(h))
        if rc != OK:
            raise RtlbfsError(rc, "rtlbfs_batch_create: " + strerror(rc))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.rtlbfs_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc != OK:
            raise RtlbfsError(rc, f"{what}: {strerror(rc)}")

    def step(self, n: int = 1):
        self._check(self._lib.rtlbfs_batch_step(self._h, int(n)), "rtlbfs_batch_step")

    def sync(self):
        self._check(self._lib.rtlbfs_batch_sync(self._h), "rtlbfs_batch_sync")

    def diverged(self) -> np.ndarray:
        """Per-member divergence flags of the last residual step."""
        flags = (C.c_int * self.count)()
        self._check(self._lib.rtlbfs_batch_diverged(self._h, flags), "rtlbfs_batch_diverged")
        return np.array(list(flags), dtype=bool)

    def info(self, k: int) -> Info:
        i = Info()
        self._check(self._lib.rtlbfs_batch_get_info(self._h, k, C.byref(i)), "rtlbfs_batch_get_info")
        return i

    def nusselt(self, k: int) -> dict:
        o = NuOut()
        self._check(self._lib.rtlbfs_batch_nusselt(self._h, k, C.byref(o)), "rtlbfs_batch_nusselt")
        return dict(hot_avg=o.hot_avg, hot_max=o.hot_max, cold_avg=o.cold_avg, cold_max=o.cold_max,
                    volume=o.volume)

    def residual(self, k: int) -> tuple[float, float]:
        a, b = C.c_double(), C.c_double()
        self._check(self._lib.rtlbfs_batch_residual(self._h, k, C.byref(a), C.byref(b)), "rtlbfs_batch_residual")
        return a.value, b.value

    def residuals(self) -> np.ndarray:
        """Eq. 65 residuals (count x 2) of every member, also when some
        members diverged (theirs are NaN or meaningless; see diverged())."""
        out = np.zeros((self.count, 2))
        for k in range(self.count):
            a, b = C.c_double(), C.c_double()
            rc = self._lib.rtlbfs_batch_residual(self._h, k, C.byref(a), C.byref(b))
            if rc not in (OK, EDIVERGED):
                self._check(rc, "rtlbfs_batch_residual")
            out[k] = a.value, b.value
        return out

    def field(self, k: int, f: int) -> np.ndarray:
        cells = int(self.info(k).cells)
        out = np.zeros(cells)
        self._check(self._lib.rtlbfs_batch_get_field(self._h, k, f, _pd(out), cells), "rtlbfs_batch_get_field")
        return out
