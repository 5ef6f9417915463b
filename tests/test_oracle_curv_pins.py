"""Pins of the curvilinear-mesh oracle (Secs. 4.3 and 4.5 run RTLBFS on
body-fitted O-type meshes; Sec. 2.2's finite-volume form with per-face
normals and areas, the Fig. 1 lattice aligned with each face).

What fixes the oracle here, without retyping it:
  - on a Cartesian mesh given as vertices it must reproduce the Cartesian
    oracle (a different code path: axis-aligned faces, separable widths);
  - the step is covariant: a rotated mesh with rotated velocities and gravity
    gives the rotated fields, and the numbering direction of the cells does
    not matter;
  - a uniform far-field state on a closed curvilinear mesh is preserved (the
    face normals of every cell sum to zero), and a closed annulus conserves
    mass and energy;
  - steady conduction between concentric cylinders approaches the closed
    form, the heat rate 2 pi chi dT / ln(R_o / R_i), at second order.
"""
import numpy as np
import pytest

import inputs
from oracle import (PERIODIC, RTLBFS, TLBFS, WALL_ADIABATIC, WALL_ISOTHERMAL, CurvConfig, CurvOracle, FARFIELD,
                    Oracle, OracleConfig, face_flux, face_flux_frame, mesh_nodes)

ISO, ADI = WALL_ISOTHERMAL, WALL_ADIABATIC


def _cavity_cfgs(method, dev, n=(14, 11)):
    xn, _ = mesh_nodes(n[0], 1.5)
    yn, _ = mesh_nodes(n[1], 1.5)
    kw = dict(nu=0.07, chi=0.09, beta_g=2e-4, dtl=1.0, dt=0.5, deviation=dev, method=method)
    cart = OracleConfig(n=n, stretch=(1.5, 1.5), bc=(ISO, ISO, ADI, ADI, PERIODIC, PERIODIC),
                        Tw=(0.5, -0.5, 0, 0, 0, 0), gravity_axis=1, **kw)
    curv = CurvConfig(bc=(ISO, ISO, ADI, ADI), Tw=(1.0, 0.0, 0.0, 0.0), up=(0.0, 1.0), Tb=0.5, **kw)
    return cart, curv, xn, yn


@pytest.mark.parametrize("method", [RTLBFS, TLBFS])
@pytest.mark.parametrize("dev", [0, 1])
def test_cartesian_mesh_reproduces_the_cartesian_oracle(method, dev):
    cart, curv, xn, yn = _cavity_cfgs(method, dev)
    X, Y = inputs.cartesian_vertices(xn, yn)
    a = Oracle(cart)
    b = CurvOracle(curv, X, Y)
    N = a.N
    rho, u, T = inputs.random_state(N, 2, seed=31 + dev)
    a.set_prim(rho, u, T)
    b.set_prim(rho, u, T)
    cx, cy, area = b.cells()
    xc, wx = a.axis(0)
    yc, wy = a.axis(1)
    assert np.allclose(cx.reshape(11, 14), xc[None, :], rtol=0, atol=1e-12 * xc.max())
    assert np.allclose(cy.reshape(11, 14), yc[:, None], rtol=0, atol=1e-12 * yc.max())
    assert np.allclose(area.reshape(11, 14), wy[:, None] * wx[None, :], rtol=1e-13)
    a.step(60)
    b.step(60)
    for f in range(4):
        ref = a.prim(f)
        scale = np.abs(ref).max() if f != 0 else 1.0
        assert np.abs(b.prim(f) - ref).max() <= 1e-12 * scale, f
    assert np.allclose(a.residual(), b.residual(), rtol=1e-9)


def _wavy_box(n=(13, 10), amp=0.04):
    xn = np.linspace(0.0, 13.0, n[0] + 1)
    yn = np.linspace(0.0, 11.0, n[1] + 1)
    return inputs.wavy_vertices(xn, yn, amp)


@pytest.mark.parametrize("method", [RTLBFS, TLBFS])
def test_rotated_mesh_gives_rotated_fields(method):
    X, Y = _wavy_box()
    ang = 0.6435
    Xr, Yr = inputs.rotated(X, Y, ang)
    up = np.array([0.0, 1.0])
    upr = np.array(inputs.rotated(up[0], up[1], ang))
    kw = dict(bc=(ISO, ISO, ADI, ADI), Tw=(1.0, 0.0, 0, 0), Tb=0.5, nu=0.06, chi=0.08, beta_g=3e-4, deviation=1,
              method=method)
    a = CurvOracle(CurvConfig(up=tuple(up), **kw), X, Y)
    b = CurvOracle(CurvConfig(up=tuple(upr), **kw), Xr, Yr)
    rho, u, T = inputs.random_state(a.N, 2, seed=41)
    ur = np.vstack(inputs.rotated(u[0], u[1], ang))
    a.set_prim(rho, u, T)
    b.set_prim(rho, ur, T)
    a.step(50)
    b.step(50)
    ua = np.vstack(inputs.rotated(a.prim(1), a.prim(2), ang))
    vs = np.abs(ua).max()
    assert np.abs(b.prim(1) - ua[0]).max() <= 1e-11 * vs
    assert np.abs(b.prim(2) - ua[1]).max() <= 1e-11 * vs
    assert np.abs(b.prim(0) - a.prim(0)).max() <= 1e-13
    assert np.abs(b.prim(3) - a.prim(3)).max() <= 1e-12
    ha, hb = a.wall_heat(0), b.wall_heat(0)
    assert abs(ha[0] - hb[0]) <= 1e-11 * abs(ha[0]) and abs(ha[1] - hb[1]) <= 1e-12 * ha[1]


def test_cell_numbering_direction_does_not_matter():
    """Swap the roles of i and j (the corners then run clockwise): the same
    cells carry the same values."""
    X, Y = _wavy_box()
    kw = dict(Tb=0.5, up=(0.0, 1.0), nu=0.06, chi=0.08, beta_g=3e-4, deviation=0)
    a = CurvOracle(CurvConfig(bc=(ISO, ADI, ADI, ISO), Tw=(1.0, 0, 0, 0.2), **kw), X, Y)
    b = CurvOracle(CurvConfig(bc=(ADI, ISO, ISO, ADI), Tw=(0, 0.2, 1.0, 0), **kw), X.T.copy(), Y.T.copy())
    rho, u, T = inputs.random_state(a.N, 2, seed=43)
    a.set_prim(rho, u, T)
    perm = lambda f: f.reshape(a.nj, a.ni).T.reshape(-1)
    b.set_prim(perm(rho), np.vstack([perm(u[0]), perm(u[1])]), perm(T))
    a.step(40)
    b.step(40)
    for f in range(4):
        ref = perm(a.prim(f))
        assert np.abs(b.prim(f) - ref).max() <= 1e-12 * max(np.abs(ref).max(), 1e-3), f


def _annulus(ni, nj, r_in, r_out, first=None):
    first = (r_out - r_in) / nj if first is None else first
    return inputs.o_mesh(ni, nj, r_in, r_out, first, theta0=0.3)


@pytest.mark.parametrize("method", [RTLBFS, TLBFS])
@pytest.mark.parametrize("dev", [0, 1])
def test_uniform_far_field_state_is_preserved(method, dev):
    X, Y = _annulus(24, 10, 20.0, 90.0, first=2.0)
    cfg = CurvConfig(bc=(PERIODIC, PERIODIC, FARFIELD, FARFIELD), u_inf=(0.03, -0.012), T_inf=0.3, Tb=0.3,
                     up=(0.0, 1.0), beta_g=1e-4, nu=0.05, chi=0.07, deviation=dev, method=method)
    o = CurvOracle(cfg, X, Y)
    o.step(200)
    assert np.abs(o.prim(0) - 1.0).max() <= 1e-14
    assert np.abs(o.prim(1) - 0.03).max() <= 1e-15
    assert np.abs(o.prim(2) + 0.012).max() <= 1e-15
    assert np.abs(o.prim(3) - 0.3).max() <= 1e-14


@pytest.mark.parametrize("dev", [0, 1])
def test_closed_annulus_conserves_mass_and_energy(dev):
    X, Y = _annulus(20, 8, 10.0, 22.0, first=1.0)
    cfg = CurvConfig(bc=(PERIODIC, PERIODIC, ADI, ADI), up=(0.0, 1.0), Tb=0.5, beta_g=5e-4, nu=0.05, chi=0.07,
                     deviation=dev)
    o = CurvOracle(cfg, X, Y)
    rho, u, T = inputs.random_state(o.N, 2, seed=47)
    o.set_prim(rho, u, T)
    I0 = o.integrals()
    o.step(400)
    I1 = o.integrals()
    assert abs(I1["mass"] - I0["mass"]) <= 1e-13 * I0["mass"]
    assert abs(I1["energy"] - I0["energy"]) <= 1e-13 * I0["energy"]


def _conduction_heat(k):
    """Steady conduction, T = 1 on r = 8k, T = 0 on r = 16k, k^2 times the
    cells of the coarse mesh; returns (inner heat, outer heat, exact) per
    unit chi, from sum (T_w - T_P)/d dS."""
    ni, nj = 32 * k, 8 * k
    ri, ro = 8.0 * k, 16.0 * k
    X, Y = _annulus(ni, nj, ri, ro)
    chi = 0.2
    cfg = CurvConfig(bc=(PERIODIC, PERIODIC, ISO, ISO), Tw=(0, 0, 1.0, 0.0), nu=0.1, chi=chi, dt=0.5)
    o = CurvOracle(cfg, X, Y)
    cx, cy, _ = o.cells()
    r = np.hypot(cx, cy)
    o.set_prim(np.ones(o.N), np.zeros(2 * o.N), np.log(r / ro) / np.log(ri / ro))
    for _ in range(60):
        o.step(500)
        if max(o.residual()) < 1e-13:
            break
    qi = o.wall_heat(2)[0]
    qo = -o.wall_heat(3)[0]
    return qi, qo, 2.0 * np.pi / np.log(ro / ri)


def test_concentric_cylinder_conduction_converges_to_the_closed_form():
    e = []
    for k in (1, 2):
        qi, qo, exact = _conduction_heat(k)
        assert abs(qi - qo) <= 1e-6 * exact, (qi, qo)  # steady: what enters leaves
        e.append(abs(qi - exact) / exact)
    order = np.log2(e[0] / e[1])
    assert e[0] < 0.05 and 1.7 <= order <= 2.3, (e, order)


@pytest.mark.parametrize("method", [RTLBFS, TLBFS])
def test_tangential_offset_is_a_shift_of_the_cell_values(method):
    """Eq. 29 is linear: a face centre displaced tangentially by tau from a
    cell centre adds g_t * tau to every node value of that side."""
    g = inputs.rng(53 + method)
    cfg = OracleConfig(dim=2, nu=0.08, chi=0.11, beta_g=2e-4, gravity_axis=-1, deviation=1, method=method)
    for _ in range(5):
        pL, pR = g.uniform(-0.05, 0.05, 4), g.uniform(-0.05, 0.05, 4)
        gL, gR = g.uniform(-0.01, 0.01, (4, 2)), g.uniform(-0.01, 0.01, (4, 2))
        dL, dR, tL, tR = g.uniform(0.4, 2.0), g.uniform(0.4, 2.0), g.uniform(-1, 1), g.uniform(-1, 1)
        fdir = g.uniform(-1, 1, 2)
        fdir /= np.linalg.norm(fdir)
        f1, p1 = face_flux_frame(cfg, pL, gL, pR, gR, (dL, tL), (-dR, tR), fdir, 0.5)
        cfg_g = OracleConfig(dim=2, nu=0.08, chi=0.11, beta_g=2e-4, gravity_axis=-1, deviation=1, method=method)
        f2, p2 = face_flux_frame(cfg_g, pL + gL[:, 1] * tL, gL, pR + gR[:, 1] * tR, gR, (dL, 0.0), (-dR, 0.0), fdir,
                                 0.5)
        assert np.abs(f1 - f2).max() <= 1e-14 * (np.abs(f2).max() + 1e-3)
        # and with no offset and buoyancy along +x it is the Cartesian face flux
        cfg_c = OracleConfig(dim=2, nu=0.08, chi=0.11, beta_g=2e-4, gravity_axis=0, deviation=1, method=method)
        f3, _ = face_flux_frame(cfg_c, pL, gL, pR, gR, (dL, 0.0), (-dR, 0.0), (1.0, 0.0), 0.5)
        f4, _ = face_flux(cfg_c, 0, pL, gL, pR, gR, dL, dR)
        assert np.array_equal(f3, f4)
