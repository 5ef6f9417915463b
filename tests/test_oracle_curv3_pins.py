"""Pins of the 3D body-fitted oracle (Sec. 4.5 runs RTLBFS on a concentric
annulus with a single azimuthal cell layer, so the mesh is a thin wedge whose
two azimuthal faces are a periodic pair closed by a rotation).

What fixes the oracle, without retyping it:
  - a Cartesian mesh given as vertices reproduces the Cartesian 3D oracle;
  - a rotated mesh with rotated velocities and gravity gives the rotated
    fields (any rotation: the face frames are attached to the mesh);
  - a wedge of one cell, whose azimuthal neighbours are its own rotated
    images, equals every cell of a wedge of four such cells at rest
    (axisymmetric data), whose inner azimuthal faces are ordinary faces;
  - a closed annulus wedge conserves mass and energy;
  - steady conduction between concentric cylinders approaches the closed
    form 1 / ln(R_o / R_i) for R (dT/dr) / dT at second order.
"""
import numpy as np
import pytest

import inputs
from oracle import (PERIODIC, RTLBFS, TLBFS, WALL_ADIABATIC, WALL_ISOTHERMAL, Curv3Config, Curv3Oracle, Oracle,
                    OracleConfig, mesh_nodes)

ISO, ADI, PER = WALL_ISOTHERMAL, WALL_ADIABATIC, PERIODIC


@pytest.mark.parametrize("method", [RTLBFS, TLBFS])
@pytest.mark.parametrize("dev", [0, 1])
def test_cartesian_mesh_reproduces_the_cartesian_oracle(method, dev):
    n = (7, 6, 5)
    nodes = [mesh_nodes(k, 1.5)[0] for k in n]
    kw = dict(nu=0.07, chi=0.09, beta_g=3e-4, dtl=1.0, dt=0.5, deviation=dev, method=method)
    a = Oracle(OracleConfig(dim=3, n=n, stretch=(1.5,) * 3, bc=(ISO, ISO, ADI, ADI, ADI, ADI),
                            Tw=(-0.5, 0.5, 0, 0, 0, 0), gravity_axis=2, **kw))
    X, Y, Z = inputs.cartesian_vertices3(*nodes)
    b = Curv3Oracle(Curv3Config(bc=(ISO, ISO, ADI, ADI, ADI, ADI), Tw=(0.0, 1.0, 0, 0, 0, 0), up=(0, 0, 1),
                                Tb=0.5, **kw), X, Y, Z)
    rho, u, T = inputs.random_state(a.N, 3, seed=71 + dev)
    a.set_prim(rho, u, T)
    b.set_prim(rho, u, T)
    cx, cy, cz, vol = b.cells()
    xc = [a.axis(k) for k in range(3)]
    assert np.allclose(cx.reshape(5, 6, 7), xc[0][0][None, None, :], rtol=0, atol=1e-12 * xc[0][0].max())
    assert np.allclose(vol.reshape(5, 6, 7), xc[2][1][:, None, None] * xc[1][1][None, :, None]
                       * xc[0][1][None, None, :], rtol=1e-13)
    a.step(30)
    b.step(30)
    for f in range(5):
        ref = a.prim(f)
        scale = np.abs(ref).max() if f else 1.0
        assert np.abs(b.prim(f) - ref).max() <= 1e-12 * scale, f


def _rotation(ax, ang):
    ax = np.asarray(ax, float) / np.linalg.norm(ax)
    K = np.array([[0, -ax[2], ax[1]], [ax[2], 0, -ax[0]], [-ax[1], ax[0], 0]])
    return np.eye(3) + np.sin(ang) * K + (1 - np.cos(ang)) * K @ K


@pytest.mark.parametrize("method", [RTLBFS, TLBFS])
def test_rotated_mesh_gives_rotated_fields(method):
    X, Y, Z = inputs.wavy_vertices3(np.linspace(0, 9, 8), np.linspace(0, 8, 7), np.linspace(0, 7, 6), 0.04)
    Q = _rotation((0.3, -0.5, 0.8), 0.9)
    P = np.stack([X, Y, Z], axis=-1) @ Q.T
    up = np.array([0.0, 0.0, 1.0])
    kw = dict(bc=(ISO, ISO, ADI, ADI, ADI, ADI), Tw=(1.0, 0.0, 0, 0, 0, 0), Tb=0.5, nu=0.06, chi=0.08, beta_g=3e-4,
              deviation=1, method=method)
    a = Curv3Oracle(Curv3Config(up=tuple(up), **kw), X, Y, Z)
    b = Curv3Oracle(Curv3Config(up=tuple(Q @ up), **kw), P[..., 0], P[..., 1], P[..., 2])
    rho, u, T = inputs.random_state(a.N, 3, seed=73)
    a.set_prim(rho, u, T)
    b.set_prim(rho, (Q @ u), T)
    a.step(30)
    b.step(30)
    ua = Q @ np.vstack([a.prim(f) for f in (1, 2, 3)])
    ub = np.vstack([b.prim(f) for f in (1, 2, 3)])
    assert np.abs(ub - ua).max() <= 1e-11 * np.abs(ua).max()
    assert np.abs(b.prim(0) - a.prim(0)).max() <= 1e-13
    assert np.abs(b.prim(4) - a.prim(4)).max() <= 1e-12


def _wedge(nth, nr=6, nz=5, dth=0.15, dev=0, method=RTLBFS, bc=(ISO, ISO, PER, PER, ADI, ADI), beta_g=4e-4):
    X, Y, Z = inputs.annulus_wedge(nr, nth, nz, 8.0, 14.0, 5.0, dth)
    cfg = Curv3Config(bc=bc, rot=(0.0, nth * dth, 0.0), Tw=(1.0, 0.0, 0, 0, 0, 0), up=(0, 0, 1), Tb=0.5,
                      nu=0.06, chi=0.08, beta_g=beta_g, deviation=dev, method=method)
    return Curv3Oracle(cfg, X, Y, Z)


@pytest.mark.parametrize("method", [RTLBFS, TLBFS])
@pytest.mark.parametrize("dev", [0, 1])
def test_one_cell_wedge_equals_every_cell_of_a_four_cell_wedge(method, dev):
    """Axisymmetric data (u_r, u_theta, u_z and T functions of (r, z) only):
    the one-cell wedge sees its azimuthal neighbours as its own rotated images,
    the four-cell wedge has three real inner azimuthal faces per row."""
    one = _wedge(1, dev=dev, method=method)
    four = _wedge(4, dev=dev, method=method)
    g = inputs.rng(79)
    nr, nz = 6, 5
    rho = 1.0 + g.uniform(-1e-3, 1e-3, (nz, nr))
    ur, ut, uz = (g.uniform(-0.02, 0.02, (nz, nr)) for _ in range(3))
    T = 0.5 + g.uniform(-0.2, 0.2, (nz, nr))

    def state(o, nth):
        cx, cy, _, _ = o.cells()
        th = np.arctan2(cy, cx)
        rep = lambda f: np.repeat(f[:, None, :], nth, axis=1).reshape(-1)
        u = np.vstack([rep(ur) * np.cos(th) - rep(ut) * np.sin(th), rep(ur) * np.sin(th) + rep(ut) * np.cos(th),
                       rep(uz)])
        o.set_prim(rep(rho), u, rep(T))
        return th

    state(one, 1)
    th4 = state(four, 4)
    one.step(40)
    four.step(40)

    def polar(o, th):
        ux, uy, uz_ = o.prim(1), o.prim(2), o.prim(3)
        return np.vstack([o.prim(0), ux * np.cos(th) + uy * np.sin(th), -ux * np.sin(th) + uy * np.cos(th), uz_,
                          o.prim(4)])

    cx1, cy1, _, _ = one.cells()
    a = polar(one, np.arctan2(cy1, cx1))                     # (5, nz*nr)
    b = polar(four, th4).reshape(5, nz, 4, nr)
    for jj in range(4):
        d = np.abs(b[:, :, jj, :].reshape(5, -1) - a)
        assert d.max() <= 1e-12 * np.abs(a).max(), (jj, d.max(axis=1))


@pytest.mark.parametrize("dev", [0, 1])
def test_closed_annulus_wedge_conserves_mass_and_energy(dev):
    o = _wedge(3, dev=dev, bc=(ADI, ADI, PER, PER, ADI, ADI))
    rho, u, T = inputs.random_state(o.N, 3, seed=83)
    o.set_prim(rho, u, T)
    I0 = o.integrals()
    o.step(200)
    I1 = o.integrals()
    assert abs(I1["mass"] - I0["mass"]) <= 1e-13 * I0["mass"]
    assert abs(I1["energy"] - I0["energy"]) <= 1e-13 * I0["energy"]


def _conduction(k):
    nr, nz = 8 * k, 2
    ri, ro = 8.0 * k, 16.0 * k
    X, Y, Z = inputs.annulus_wedge(nr, 1, nz, ri, ro, 2.0 * k, 1.0 / ri)
    cfg = Curv3Config(bc=(ISO, ISO, PER, PER, ADI, ADI), rot=(0.0, 1.0 / ri, 0.0), Tw=(1.0, 0.0, 0, 0, 0, 0),
                      nu=0.1, chi=0.2, dt=0.5)
    o = Curv3Oracle(cfg, X, Y, Z)
    cx, cy, _, _ = o.cells()
    r = np.hypot(cx, cy)
    o.set_prim(np.ones(o.N), np.zeros(3 * o.N), np.log(r / ro) / np.log(ri / ro))
    for _ in range(60):
        o.step(400)
        if max(o.residual()) < 1e-13:
            break
    qi, Ai = o.wall_heat(0)
    qo, Ao = o.wall_heat(1)
    return ri * qi / Ai, -ro * qo / Ao, 1.0 / np.log(ro / ri)


def test_concentric_conduction_converges_to_the_closed_form():
    e = []
    for k in (1, 2):
        ni, no, exact = _conduction(k)
        assert abs(ni - no) <= 1e-9 * exact, (ni, no)  # steady: the heat entering leaves
        e.append(abs(ni - exact) / exact)
    order = np.log2(e[0] / e[1])
    assert e[0] < 0.005 and 1.7 <= order <= 2.3, (e, order)  # observed 0.11%, 0.029%: order 1.89
