"""3D body-fitted meshes on the GPU against the 3D curvilinear oracle (the
setting of Sec. 4.5: a concentric annulus with one azimuthal cell layer whose
azimuthal sides are a periodic pair closed by a rotation about z).

The library derives its own geometry (a different tetrahedral split, its own
face records and rotated images) from the vertex arrays.
"""
import numpy as np
import pytest

import inputs
import paper_2202_13449_amd as rt
from oracle import RTLBFS, TLBFS, Curv3Config, Curv3Oracle

pytestmark = pytest.mark.gpu

ISO, ADI, PER = rt.WALL_ISOTHERMAL, rt.WALL_ADIABATIC, rt.PERIODIC
FP64_TOL = 1e-12


def make_pair(X, Y, Z, precision=rt.FP64_PLAIN, method=rt.METHOD_RTLBFS, **bc):
    kind = bc.pop("kind")
    rot = tuple(bc.pop("rot", (0.0, 0.0, 0.0)))
    Tw = tuple(bc.pop("Tw", (0.0,) * 6))
    up = tuple(bc.pop("up", (0.0, 0.0, 0.0)))
    T_ref = bc.pop("T_ref", 0.5)
    phys = dict(nu=bc.pop("nu", 0.06), chi=bc.pop("chi", 0.08), beta_g=bc.pop("beta_g", 3e-4))
    s = rt.Curv3Solver(X, Y, Z, kind, rot=rot, Tw=Tw, up=up, T_ref=T_ref, precision=precision, method=method,
                       dt=0.5, residual_every=20, **phys)
    cfg = Curv3Config(bc=tuple(kind), rot=rot, Tw=Tw, up=up, Tb=T_ref, dt=0.5,
                      deviation=0 if precision == rt.FP64_PLAIN else 1,
                      method=RTLBFS if method == rt.METHOD_RTLBFS else TLBFS, **phys)
    o = Curv3Oracle(cfg, X, Y, Z)
    o.set_prim(np.ones(o.N), np.zeros(3 * o.N), np.full(o.N, T_ref))
    return s, o


def rel_errors(s, o, Vc=0.02):
    out = []
    for f in range(5):
        a, b = s.field(f), o.prim(f)
        if f == 0:
            a, b = a - 1.0, b - 1.0
            scale = max(np.abs(b).max(), 1e-300)
        elif f < 4:
            scale = max(np.abs(b).max(), Vc)
        else:
            scale = np.abs(b).max()
        out.append(float(np.abs(a - b).max() / scale))
    return out


def wavy_box():
    return inputs.wavy_vertices3(np.linspace(0, 11, 12), np.linspace(0, 9, 10), np.linspace(0, 8, 9), 0.04)


def wedge(nth=1, nr=13, nz=20, dth=0.08):
    return inputs.annulus_wedge(nr, nth, nz, 13.0, 26.0, 20.0, dth)


BOX = dict(kind=(ISO, ISO, ADI, ADI, ADI, ADI), Tw=(1.0, 0.0, 0, 0, 0, 0), up=(0.0, 0.0, 1.0))


def wedge_bc(nth, dth=0.08):
    return dict(kind=(ISO, ISO, PER, PER, ADI, ADI), rot=(0.0, nth * dth, 0.0), Tw=(1.0, 0.0, 0, 0, 0, 0),
                up=(0.0, 0.0, 1.0), beta_g=5e-4)


def test_geometry_matches_the_oracle():
    for (X, Y, Z), bc in ((wavy_box(), BOX), (wedge(), wedge_bc(1)), (wedge(nth=4, dth=0.2), wedge_bc(4, 0.2))):
        s, o = make_pair(X, Y, Z, **dict(bc))
        a, b = s.geometry(), o.cells()
        xscale = max(np.abs(b[k]).max() for k in range(3))  # coordinates against the mesh extent
        for k in range(4):
            scale = xscale if k < 3 else np.abs(b[3]).max()
            assert np.abs(a[k] - b[k]).max() <= 1e-12 * scale, k


@pytest.mark.parametrize("precision", [rt.FP64_PLAIN, rt.FP64_DEV])
@pytest.mark.parametrize("method", [rt.METHOD_RTLBFS, rt.METHOD_TLBFS])
def test_wavy_box_parity(precision, method):
    X, Y, Z = wavy_box()
    s, o = make_pair(X, Y, Z, precision, method, **dict(BOX))
    rho, u, T = inputs.random_state(s.cells, 3, seed=89)
    s.set_state(rho, u, T)
    o.set_prim(rho, u, T)
    s.step(40)
    o.step(40)
    rel = rel_errors(s, o)
    assert max(rel) <= FP64_TOL, rel
    assert np.allclose(s.residual(), o.residual(), rtol=1e-9)
    for side in (0, 1):
        ha, hb = s.wall_heat(side), o.wall_heat(side)
        assert abs(ha[0] - hb[0]) <= 1e-11 * abs(hb[0]) and abs(ha[1] - hb[1]) <= 1e-12 * hb[1]


@pytest.mark.parametrize("precision", [rt.FP64_PLAIN, rt.FP64_DEV])
@pytest.mark.parametrize("method", [rt.METHOD_RTLBFS, rt.METHOD_TLBFS])
def test_annulus_wedge_parity(precision, method):
    """One azimuthal cell (its neighbours are its own rotated images): heated
    inner wall, buoyancy along z, 300 steps from rest."""
    X, Y, Z = wedge()
    s, o = make_pair(X, Y, Z, precision, method, **wedge_bc(1))
    s.step(300)
    o.step(300)
    rel = rel_errors(s, o)
    assert max(rel) <= FP64_TOL, rel
    for side in (0, 1):
        ha, hb = s.wall_heat(side), o.wall_heat(side)
        assert abs(ha[0] - hb[0]) <= 1e-11 * abs(hb[0])


def test_four_cell_wedge_random_state_parity():
    """Four azimuthal cells from a random (not axisymmetric) state: ordinary
    azimuthal faces and the rotated seam together."""
    X, Y, Z = wedge(nth=4, nr=9, nz=11, dth=0.2)
    s, o = make_pair(X, Y, Z, **wedge_bc(4, 0.2))
    rho, u, T = inputs.random_state(s.cells, 3, seed=97)
    s.set_state(rho, u, T)
    o.set_prim(rho, u, T)
    s.step(60)
    o.step(60)
    rel = rel_errors(s, o)
    assert max(rel) <= FP64_TOL, rel


def test_annulus_wedge_fp32_deviation():
    """FP32 deviation storage on the single-layer wedge, which runs the fused
    one-launch kernel by default, against the FP64 oracle.  (A single-cell
    periodic layer needs a rotation: with rot = 0 its two periodic vertex
    layers would coincide, which create rejects.)"""
    X, Y, Z = wedge()
    s, o = make_pair(X, Y, Z, rt.FP32_DEV, **wedge_bc(1))
    assert (s.info.tile_x, s.info.tile_z) == (16, 4)  # the fused kernel's tile
    s.step(300)
    o.step(300)
    rel = rel_errors(s, o)
    assert max(rel[1:]) <= 1e-5 and rel[0] <= 1e-4, rel


def test_graph_replay_equals_eager_launches_3d():
    X, Y, Z = wedge()
    bc = wedge_bc(1)
    kw = dict(rot=bc["rot"], Tw=bc["Tw"], up=bc["up"], T_ref=0.5, nu=0.06, chi=0.08, beta_g=bc["beta_g"],
              precision=rt.FP32_DEV, dt=0.5, residual_every=40)
    a = rt.Curv3Solver(X, Y, Z, bc["kind"], **kw)
    b = rt.Curv3Solver(X, Y, Z, bc["kind"], graph_steps=-1, **kw)
    for s in (a, b):
        s.step(250)
    for f in range(5):
        assert np.array_equal(a.stored(f), b.stored(f)), f
    with pytest.raises(rt.RtlbfsError) as e:
        a.wall_heat(4)  # adiabatic
    assert e.value.code == rt.EINVAL


@pytest.mark.parametrize("precision", [rt.FP64_PLAIN, rt.FP32_DEV])
def test_fused_layer_kernel_equals_three_kernels(precision):
    """A single-layer wedge (j periodic with one cell, walls along i and k)
    runs one fused launch per step by default; opts.tile 1 forces the
    three-launch path.  From a random, non-axisymmetric state on a
    21 x 1 x 27 wedge (ragged 16 x 4 tiles in i and k), both give the same
    fields; the fused path also matches the oracle."""
    X, Y, Z = wedge(nr=21, nz=27, dth=0.1)
    bc = wedge_bc(1, 0.1)
    kw = dict(rot=bc["rot"], Tw=bc["Tw"], up=bc["up"], T_ref=0.5, nu=0.06, chi=0.08, beta_g=bc["beta_g"],
              precision=precision, dt=0.5, residual_every=20)
    runs = {t: rt.Curv3Solver(X, Y, Z, bc["kind"], tile=t, **kw) for t in (0, 1)}
    assert (runs[0].info.tile_x, runs[0].info.tile_z) == (16, 4)  # the default is the fused kernel
    assert runs[1].info.tile_x == 64 and runs[1].info.tile_z == 1
    rho, u, T = inputs.random_state(runs[0].cells, 3, seed=31)
    for s in runs.values():
        s.set_state(rho, u, T)
        s.step(150)
    tol = FP64_TOL if precision == rt.FP64_PLAIN else 2e-6  # FP64: the oracle parity bar
    for f in range(5):
        a, b = runs[0].field(f), runs[1].field(f)
        scale = max(np.abs(b - (1.0 if f == 0 else 0.0)).max(), 1e-3)
        assert np.abs(a - b).max() <= tol * scale, (f, np.abs(a - b).max() / scale)
    if precision == rt.FP64_PLAIN:
        ra, rb = runs[0].residual(), runs[1].residual()
        assert abs(ra[0] - rb[0]) <= 1e-9 * abs(rb[0]) and abs(ra[1] - rb[1]) <= 1e-9 * abs(rb[1])
        s, o = make_pair(X, Y, Z, precision, **wedge_bc(1, 0.1))
        s.set_state(rho, u, T)
        o.set_prim(rho, u, T)
        s.step(60)
        o.step(60)
        assert max(rel_errors(s, o)) <= FP64_TOL
