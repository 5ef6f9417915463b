"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol the header declares, and its host-only entry points and
argument validation behave as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2202_13449_amd as rt
from paper_2202_13449_amd import rtlbfs as rtb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "rtlbfs.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rtlbfs_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = rt.load_library()
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_strerror_covers_all_codes():
    for code in (0, -1, -2, -3, -4, -5, -6):
        assert rt.strerror(code) and rt.strerror(code) != "unknown status"
    assert rt.strerror(-99) == "unknown status"


def test_opts_defaults():
    o = rt.make_opts()
    assert o.precision == rt.FP64_PLAIN and o.residual_every == 100 and o.mass_fix_every == 1000
    assert o.graph_steps == 0 and o.phys_given == 0 and o.dtl == 0.0 and o.dt == 0.0


def test_mesh_nodes_match_oracle_mesh():
    """The library's Eq. 74 mesh equals the oracle's (both from the equation)."""
    from oracle import mesh_nodes as orc_mesh
    for n, phi in [(64, 0.0), (256, 1.5), (192, 1.8), (7, 2.0)]:
        x, L = rt.mesh_nodes(n, phi)
        y, M = orc_mesh(n, phi)
        assert abs(L - M) <= 1e-12 * M
        assert np.abs(x - y).max() <= 1e-12 * M


def test_workspace_bytes():
    lib = rt.load_library()
    m = rt.make_mesh(2, (64, 64))
    o = rt.make_opts()
    b64 = lib.rtlbfs_workspace_bytes(C.byref(m), C.byref(o))
    o32 = rt.make_opts(precision=rt.FP32_DEV)
    b32 = lib.rtlbfs_workspace_bytes(C.byref(m), C.byref(o32))
    assert b64 >= 2 * 4 * 4096 * 8 and b32 >= 2 * 4 * 4096 * 4 and b64 > b32
    assert b64 % 256 == 0
    bad = rt.make_mesh(2, (3, 64))
    assert lib.rtlbfs_workspace_bytes(C.byref(bad), C.byref(o)) == 0
    assert lib.rtlbfs_workspace_bytes(None, C.byref(o)) == 0


def _create(mesh, bc, Ra=1e3, Pr=0.71, Ma=0.1, opts=None):
    lib = rt.load_library()
    h = C.c_void_p()
    o = opts or rt.make_opts()
    rc = lib.rtlbfs_create(C.byref(mesh), Ra, Pr, Ma, C.byref(bc), C.byref(o), None, None, 0, C.byref(h))
    return rc, h


@pytest.mark.parametrize("case", ["dim", "small", "periodic_pair", "periodic_stretch", "Ra", "Pr", "Ma", "gravity",
                                  "precision", "kind", "method", "tile", "max_mach"])
def test_create_rejects_invalid_problems_before_touching_the_device(case):
    mesh = rt.make_mesh(2, (16, 16))
    bc = rt.make_bc((1, 1, 2, 2), (0.5, -0.5, 0, 0), 1)
    Ra, Pr, Ma, opts = 1e3, 0.71, 0.1, None
    if case == "dim":
        mesh.dim = 4
    elif case == "small":
        mesh.n[0] = 3
    elif case == "periodic_pair":
        bc.kind[0] = rt.PERIODIC
    elif case == "periodic_stretch":
        bc.kind[0] = bc.kind[1] = rt.PERIODIC
        mesh.stretch[0] = 1.5
    elif case == "Ra":
        Ra = -1.0
    elif case == "Pr":
        Pr = 0.0
    elif case == "Ma":
        Ma = 0.5
    elif case == "gravity":
        bc.gravity_axis = 2
    elif case == "precision":
        opts = rt.make_opts(precision=7)
    elif case == "kind":
        bc.kind[2] = 9
    elif case == "method":
        opts = rt.make_opts(method=2)
    elif case == "tile":
        opts = rt.make_opts(tile=10)
    elif case == "max_mach":
        opts = rt.make_opts(max_mach=-0.1)
    rc, h = _create(mesh, bc, Ra, Pr, Ma, opts)
    assert rc == rt.EINVAL and not h.value


def test_null_arguments():
    lib = rt.load_library()
    assert lib.rtlbfs_step(None, 1) == rt.EINVAL
    assert lib.rtlbfs_destroy(None) == rt.OK
    assert lib.rtlbfs_opts_init(None) == rt.EINVAL
    assert lib.rtlbfs_mesh_nodes(0, 0.0, None, None) == rt.EINVAL
    ck = rtb.Checkpoint()
    assert lib.rtlbfs_get_checkpoint(None, C.byref(ck)) == rt.EINVAL
    assert lib.rtlbfs_restore(None, None, 0, C.byref(ck)) == rt.EINVAL
    assert isinstance(lib.rtlbfs_last_error(None), bytes)  # last failed create on this thread
    mesh = rt.make_mesh(2, (16, 16))
    bc = rt.make_bc((1, 1, 2, 2), (0.5, -0.5, 0, 0), 1)
    o = rt.make_opts()
    assert lib.rtlbfs_create(C.byref(mesh), 1e3, 0.71, 0.1, C.byref(bc), C.byref(o), None, None, 0, None) \
        == rt.EINVAL


def test_binding_refuses_to_run_without_a_gpu(monkeypatch):
    """The product path has no CPU fallback: without a GPU it raises."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError, match="needs a HIP GPU"):
        rt.Solver(2, (16, 16), (0, 0), (1, 1, 2, 2), (0.5, -0.5, 0, 0), 1)


def test_binding_fails_loudly_without_the_library(monkeypatch, tmp_path):
    monkeypatch.setattr(rtb, "_lib", None)
    monkeypatch.setattr(rtb, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError, match="missing"):
        rtb.load_library()


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2202_13449_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "rtlbfs_oracle" not in text and "orc_" not in text, f


# ------------------------------------------------------ body-fitted meshes --

def _curv_mesh(ni=12, nj=8, periodic=True):
    import inputs
    x, y = inputs.o_mesh(ni, nj, 10.0, 30.0, 1.5)
    return x, y


def _curv_create(x, y, bc, nu=0.1, chi=0.1, beta_g=0.0, opts=None):
    lib = rt.load_library()
    m = rtb.CurvMesh()
    m.n[:] = [x.shape[1] - 1, x.shape[0] - 1]
    x = np.ascontiguousarray(x)
    y = np.ascontiguousarray(y)
    m.x, m.y = rtb._pd(x), rtb._pd(y)
    o = opts or rt.make_opts()
    h = C.c_void_p()
    rc = lib.rtlbfs_curv_create(C.byref(m), nu, chi, beta_g, C.byref(bc), C.byref(o), None, None, 0, C.byref(h))
    return rc, h


def _curv_bc(kind=(0, 0, 1, 3), up=(0.0, 1.0)):
    b = rtb.CurvBC()
    b.kind[:] = list(kind)
    b.Tw[:] = [0.0, 0.0, 1.0, 0.0]
    b.up[:] = list(up)
    b.u_inf[:] = [0.05, 0.0]
    return b


@pytest.mark.parametrize("case", ["small", "kind", "pair", "not_closed", "folded", "up", "tile", "nu", "beta_g",
                                  "precision", "method", "nan"])
def test_curv_create_rejects_invalid_problems_before_touching_the_device(case):
    x, y = _curv_mesh()
    bc = _curv_bc()
    kw = {}
    if case == "small":
        x, y = x[:, :4], y[:, :4]
        bc.kind[0] = bc.kind[1] = rt.WALL_ADIABATIC
    elif case == "kind":
        bc.kind[3] = 4
    elif case == "pair":
        bc.kind[1] = rt.WALL_ADIABATIC
    elif case == "not_closed":
        x = x.copy()
        x[:, -1] += 0.5  # the last vertex column no longer meets the first
    elif case == "folded":
        x, y = x.copy(), y.copy()
        x[3, 4], x[4, 4] = x[4, 4], x[3, 4]  # two radial vertices swapped
        y[3, 4], y[4, 4] = y[4, 4], y[3, 4]
    elif case == "up":
        bc.up[:] = [0.5, 0.5]
    elif case == "tile":
        kw["opts"] = rt.make_opts(tile=5)
    elif case == "nu":
        kw["nu"] = 0.0
    elif case == "beta_g":
        kw["beta_g"] = -1.0
    elif case == "precision":
        kw["opts"] = rt.make_opts(precision=5)
    elif case == "method":
        kw["opts"] = rt.make_opts(method=3)
    elif case == "nan":
        x = x.copy()
        x[2, 2] = np.nan
    rc, h = _curv_create(x, y, bc, **kw)
    assert rc == rt.EINVAL and not h.value, rt.load_library().rtlbfs_last_error(None)


def test_curv_workspace_bytes_and_cartesian_only_calls():
    lib = rt.load_library()
    m = rtb.CurvMesh()
    m.n[:] = [450, 300]
    o64, o32 = rt.make_opts(), rt.make_opts(precision=rt.FP32_DEV)
    b64 = lib.rtlbfs_curv_workspace_bytes(C.byref(m), C.byref(o64))
    b32 = lib.rtlbfs_curv_workspace_bytes(C.byref(m), C.byref(o32))
    cells = 450 * 300
    assert b64 >= 2 * 4 * cells * 8 + 8 * 2 * cells * 8 and b64 % 256 == 0
    assert b32 >= 2 * 4 * cells * 4 + 8 * 2 * cells * (4 + 8)  # FP32 records plus the FP64 copy
    m.n[:] = [3, 300]
    assert lib.rtlbfs_curv_workspace_bytes(C.byref(m), C.byref(o64)) == 0
    out = np.zeros(2)
    assert lib.rtlbfs_wall_heat(None, 2, rtb._pd(out)) == rt.EINVAL
    assert lib.rtlbfs_curv_cells(None, None, None, None, 0) == rt.EINVAL


def _c3_create(X, Y, Z, bc, nu=0.1, opts=None):
    lib = rt.load_library()
    m = rtb.Curv3Mesh()
    m.n[:] = [X.shape[2] - 1, X.shape[1] - 1, X.shape[0] - 1]
    X, Y, Z = (np.ascontiguousarray(v) for v in (X, Y, Z))
    m.x, m.y, m.z = rtb._pd(X), rtb._pd(Y), rtb._pd(Z)
    o = opts or rt.make_opts()
    h = C.c_void_p()
    rc = lib.rtlbfs_curv3_create(C.byref(m), nu, 0.1, 0.0, C.byref(bc), C.byref(o), None, None, 0, C.byref(h))
    return rc, h


@pytest.mark.parametrize("case", ["farfield", "pair", "rot_walled", "not_closed", "folded", "up", "tile",
                                  "tile_not_layer", "nu", "small"])
def test_curv3_create_rejects_invalid_problems_before_touching_the_device(case):
    import inputs
    X, Y, Z = inputs.annulus_wedge(5, 1, 4, 10.0, 15.0, 4.0, 0.1)
    b = rtb.Curv3BC()
    b.kind[:] = [1, 1, 0, 0, 2, 2]
    b.rot[:] = [0.0, 0.1, 0.0]
    b.up[:] = [0.0, 0.0, 1.0]
    kw = {}
    if case == "farfield":
        b.kind[1] = 3
    elif case == "pair":
        b.kind[3] = 2
    elif case == "rot_walled":
        b.rot[0] = 0.1
    elif case == "not_closed":
        b.rot[1] = 0.12
    elif case == "folded":
        X, Y, Z = X.copy(), Y.copy(), Z.copy()
        X[:, :, 2], X[:, :, 3] = X[:, :, 3].copy(), X[:, :, 2].copy()
        Y[:, :, 2], Y[:, :, 3] = Y[:, :, 3].copy(), Y[:, :, 2].copy()
    elif case == "up":
        b.up[:] = [0.0, 0.5, 0.5]
    elif case == "tile":
        kw["opts"] = rt.make_opts(tile=3)
    elif case == "tile_not_layer":
        # the fused kernel (tile 2) needs a single periodic cell layer: two cells of 0.05 rad here
        X, Y, Z = inputs.annulus_wedge(5, 2, 4, 10.0, 15.0, 4.0, 0.05)
        kw["opts"] = rt.make_opts(tile=2)
    elif case == "nu":
        kw["nu"] = -1.0
    elif case == "small":
        X, Y, Z = X[:, :, :2], Y[:, :, :2], Z[:, :, :2]  # one radial cell between two walls
    rc, h = _c3_create(X, Y, Z, b, **kw)
    assert rc == rt.EINVAL and not h.value, rt.load_library().rtlbfs_last_error(None)


def test_meshes_beyond_one_dispatch_are_rejected_before_touching_the_device():
    """Maximum sizes.  Every axis may hold 2^20 cells, but a step launch must
    fit one dispatch: blocks x threads of every launch shape at most
    2^32 - 1.  A mesh past that has no workspace size and is EINVAL at
    create, for the single-domain, batched and body-fitted entry points;
    meshes just inside are accepted."""
    lib = rt.load_library()
    o = rt.make_opts(precision=rt.FP32_DEV)
    big2 = rt.make_mesh(2, (1 << 20, 8192))        # 8.6e9 cells: the 8 x 8 two-step shape needs 5e10 work-items
    assert lib.rtlbfs_workspace_bytes(C.byref(big2), C.byref(o)) == 0
    bc = rt.make_bc((1, 1, 2, 2), (0.5, -0.5, 0, 0), 1)
    rc, h = _create(big2, bc, opts=o)
    assert rc == rt.EINVAL and not h.value
    assert b"too large" in lib.rtlbfs_last_error(None)
    ok2 = rt.make_mesh(2, (4096, 4096))
    assert lib.rtlbfs_workspace_bytes(C.byref(ok2), C.byref(o)) > 0
    big3 = rt.make_mesh(3, (1024, 1024, 1024))     # 2^24 tiles of 256 threads: 2^32 work-items
    ok3 = rt.make_mesh(3, (1000, 1000, 1000))      # 1.6e7 tiles: 4.0e9
    assert lib.rtlbfs_workspace_bytes(C.byref(big3), C.byref(o)) == 0
    assert lib.rtlbfs_workspace_bytes(C.byref(ok3), C.byref(o)) > 0
    too_long = rt.make_mesh(2, ((1 << 20) + 1, 4))
    assert lib.rtlbfs_workspace_bytes(C.byref(too_long), C.byref(o)) == 0
    # batch: two members of 2^20 x 4096 need 2.1e10 work-items together
    meshes = (rtb.Mesh * 2)(rt.make_mesh(2, (1 << 20, 4096)), rt.make_mesh(2, (1 << 20, 4096)))
    assert lib.rtlbfs_batch_workspace_bytes(2, meshes, C.byref(o)) == 0
    bcs = (rtb.BC * 2)(bc, bc)
    Ra, Pr = (C.c_double * 2)(1e3, 1e3), (C.c_double * 2)(0.71, 0.71)
    hb = C.c_void_p()
    assert lib.rtlbfs_batch_create(2, meshes, Ra, Pr, 0.1, bcs, C.byref(o), None, None, 0, C.byref(hb)) == rt.EINVAL
    assert not hb.value
    small = (rtb.Mesh * 2)(rt.make_mesh(2, (64, 64)), rt.make_mesh(2, (128, 96)))
    assert lib.rtlbfs_batch_workspace_bytes(2, small, C.byref(o)) > 0
    # body-fitted 2D
    cm = rtb.CurvMesh()
    cm.n[:] = [1 << 20, 8192]
    assert lib.rtlbfs_curv_workspace_bytes(C.byref(cm), C.byref(o)) == 0


def test_residual_states_validates_before_touching_the_device():
    """The allocation-free Eq. 65 entry point rejects bad arguments (dim,
    precision, NULL pointers, sizes beyond its documented maximum, a field
    stride below the cell count) with EINVAL before any HIP call."""
    lib = rt.load_library()
    p = C.c_void_p(0x1000)  # never dereferenced: validation fails first
    f = lib.rtlbfs_residual_states
    assert f(1, rt.FP64_PLAIN, 64, 64, p, p, p, None) == rt.EINVAL
    assert f(4, rt.FP64_PLAIN, 64, 64, p, p, p, None) == rt.EINVAL
    assert f(2, 7, 64, 64, p, p, p, None) == rt.EINVAL
    assert f(2, rt.FP32_DEV, 64, 64, None, p, p, None) == rt.EINVAL
    assert f(2, rt.FP32_DEV, 64, 64, p, None, p, None) == rt.EINVAL
    assert f(2, rt.FP32_DEV, 64, 64, p, p, None, None) == rt.EINVAL
    assert f(2, rt.FP64_DEV, 0, 64, p, p, p, None) == rt.EINVAL
    assert f(3, rt.FP64_DEV, 100, 99, p, p, p, None) == rt.EINVAL
    big = (1 << 31) + 1
    assert f(3, rt.FP64_PLAIN, big, big, p, p, p, None) == rt.EINVAL
