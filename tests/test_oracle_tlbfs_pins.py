"""Pins of the oracle's TLBFS interface flux (Sec. 2.2, Eqs. 29-40).

The TLBFS route and the RTLBFS route of the oracle are two different
computations: lattice Boltzmann moment sums of the equilibria on one side,
finite differences of macroscopic products on the other.  Sec. 3.1 relates
them by a Taylor expansion that is exact for quadratic equilibria, up to the
one O(dt^2) term the paper drops between Eqs. 39-40 and 50-51.  The first
pin checks exactly that relation; the others check what any consistent flux
must satisfy (rest, Galilean invariance, conservation, exact conduction) and
what the paper reports for TLBFS (second order on the Gaussian hill, Fig. 7,
with an error at or below RTLBFS's; Table 1 at Ra = 1e3).
"""
import numpy as np
import pytest

import inputs
import tlbfs_route
from oracle import (INIT_CONDUCTION, PERIODIC, RTLBFS, TLBFS, WALL_ADIABATIC, WALL_ISOTHERMAL, Oracle,
                    OracleConfig, face_flux, physics_from_ra)

T0 = 0.5


def _linear_fields(rho0, grho, u0, gu, T0v, gT):
    def f(x):
        x = np.asarray(x, dtype=np.float64)
        return rho0 + grho @ x, u0 + gu @ x, T0v + gT @ x
    return f


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("case", ["const_rho", "const_u"])
@pytest.mark.parametrize("deviation", [0, 1])
def test_tlbfs_flux_is_rtlbfs_flux_plus_the_dropped_term(dim, case, deviation):
    """Quadratic equilibria: TLBFS flux - RTLBFS flux = the (tau - 0.5) 0.5
    dt^2 second-derivative term of the fourth (third) equilibrium moment,
    evaluated independently by central differences of the moments; the
    TLBFS predicted rho*, m* equal the RTLBFS ones (Eqs. 30-31 vs 46-47)."""
    g = inputs.rng(700 + dim * 10 + (case == "const_u") * 3 + deviation)
    for trial in range(4):
        axis = trial % dim
        dtl = [1.0, 0.5, 0.8, 1.3][trial]
        nu, chi = g.uniform(0.02, 0.3), g.uniform(0.02, 0.3)
        rho0 = 1.0 + g.uniform(-0.01, 0.01)
        u0 = g.uniform(-0.08, 0.08, dim)
        T0v = 0.5 + g.uniform(-0.3, 0.3)
        gT = g.uniform(-0.02, 0.02, dim)
        if case == "const_rho":
            grho = np.zeros(dim)
            gu = g.uniform(-0.01, 0.01, (dim, dim))
        else:
            grho = g.uniform(-0.003, 0.003, dim)
            gu = np.zeros((dim, dim))
        fields = _linear_fields(rho0, grho, u0, gu, T0v, gT)
        xs = g.uniform(-0.5, 0.5, dim)
        dL, dR = g.uniform(0.5, 3.0), g.uniform(0.5, 3.0)
        xL = xs.copy(); xL[axis] -= dL
        xR = xs.copy(); xR[axis] += dR

        def prim_and_grad(xc):
            rho, u, T = fields(xc)
            p = np.concatenate([[rho - 1.0 if deviation else rho], u, [T - T0 if deviation else T]])
            return p, np.vstack([grho[None, :], gu, gT[None, :]])

        pL, gL = prim_and_grad(xL)
        pR, gR = prim_and_grad(xR)
        kw = dict(dim=dim, nu=nu, chi=chi, beta_g=0.0, gravity_axis=-1, dtl=dtl, deviation=deviation)
        f_tl, p_tl = face_flux(OracleConfig(method=TLBFS, **kw), axis, pL, gL, pR, gR, dL, dR)
        f_rt, p_rt = face_flux(OracleConfig(method=RTLBFS, **kw), axis, pL, gL, pR, gR, dL, dR)
        corr = tlbfs_route.tlbfs_face(dim, fields, xs, axis, dtl, nu, chi)[2]
        scale = np.abs(f_tl).max() + 1e-3
        assert np.abs(f_tl - (f_rt + corr)).max() <= 2e-13 * scale, (f_tl, f_rt, corr)
        assert np.abs(p_tl[:dim + 1] - p_rt[:dim + 1]).max() <= 1e-13 * np.abs(p_rt).max()


def test_tlbfs_rest_uniform_flow_and_conservation():
    """Rest at T_ref with gravity, and uniform flow in a periodic box: steady
    to round-off (the moment sums of Eqs. 30-32 and 38-40 reproduce rho and
    c_s^2 rho only to rounding, so unlike the RTLBFS form the rest state is
    not bitwise fixed).  Closed adiabatic box from a random state: mass and
    energy conserved to round-off.  Plain and deviation storage."""
    for dev in (0, 1):
        o = Oracle(OracleConfig(n=(12, 10), stretch=(1.5, 1.5), bc=(WALL_ADIABATIC, WALL_ISOTHERMAL,
                   WALL_ADIABATIC, WALL_ISOTHERMAL, PERIODIC, PERIODIC), Tw=(0,) * 6, gravity_axis=1, nu=0.1,
                   chi=0.14, beta_g=1e-3, deviation=dev, method=TLBFS))
        before = [o.stored(f) for f in range(4)]
        o.step(300)
        for f in range(4):
            assert np.abs(o.stored(f) - before[f]).max() <= 1e-14, f

        N = 10
        o = Oracle(OracleConfig(n=(N, 12), bc=(PERIODIC,) * 6, gravity_axis=-1, nu=0.05, chi=0.07, deviation=dev,
                                method=TLBFS))
        u = np.zeros((2, N * 12)); u[0] = 0.05; u[1] = 0.03
        o.set_prim(np.ones(N * 12), u, np.full(N * 12, 0.7))
        before = [o.stored(f) for f in range(4)]
        o.step(200)
        for f in range(4):
            assert np.abs(o.stored(f) - before[f]).max() <= 1e-14 * max(1.0, np.abs(before[f]).max())

    N = 16
    o = Oracle(OracleConfig(n=(N, N), stretch=(1.5, 1.5), bc=(WALL_ADIABATIC,) * 4 + (PERIODIC,) * 2,
               Tw=(0,) * 6, gravity_axis=1, nu=0.05, chi=0.07, beta_g=1e-3, method=TLBFS))
    rho, u, T = inputs.random_state(N * N, 2, seed=5)
    o.set_prim(rho, u, T)
    E0, M0 = o.integrals()["energy"], o.integrals()["mass"]
    o.step(500)
    assert abs(o.integrals()["energy"] - E0) / E0 <= 1e-13
    assert abs(o.integrals()["mass"] - M0) / M0 <= 1e-13


@pytest.mark.parametrize("dim", [2, 3])
def test_tlbfs_conduction_is_exactly_steady(dim):
    """The linear conduction profile has quadratic (here linear) equilibria and
    no flow, so the TLBFS flux is the exact conductive flux: steady, Nu = 1."""
    bc, Tw, gax = inputs.dhc_bc(dim)
    n = (12, 10) if dim == 2 else (8, 6, 5)
    cfg = OracleConfig(dim=dim, n=n, stretch=(1.5,) * 3, bc=bc, Tw=Tw, gravity_axis=gax, nu=0.1, chi=0.13,
                       beta_g=0.0, init=INIT_CONDUCTION, method=TLBFS)
    o = Oracle(cfg)
    before = [o.stored(f) for f in range(dim + 2)]
    o.step(200)
    for f in range(dim + 2):
        assert np.abs(o.stored(f) - before[f]).max() <= 1e-13
    nu_ = o.nusselt()
    for k in ("hot_avg", "cold_avg", "volume"):
        assert abs(nu_[k] - 1.0) <= 1e-12, (k, nu_[k])


def _hill_error(N, method):
    L = N / 2.0
    chi = 0.1
    u0 = 10.0 * chi / L
    o = Oracle(OracleConfig(n=(N, N), bc=(PERIODIC,) * 6, gravity_axis=-1, nu=chi, chi=chi, dtl=0.5, dt=1.0,
                            method=method))
    xc, _ = o.axis(0)
    yc, _ = o.axis(1)
    u = np.zeros((2, N * N)); u[0] = u0
    o.set_prim(np.ones(N * N), u, inputs.gaussian_hill(xc, yc, L, 0.0, chi, u0))
    steps = int(round(0.005 * L * L / chi))
    o.step(steps)
    Ta = inputs.gaussian_hill(xc, yc, L, steps * 1.0, chi, u0)
    return np.sqrt(np.mean((o.grid(o.prim(3)) - Ta) ** 2))


def test_tlbfs_gaussian_hill_second_order_and_not_less_accurate():
    """Fig. 7: TLBFS converges at order near 2 on the Gaussian hill, and
    RTLBFS's error is above TLBFS's (the paper calls it slightly higher and
    prints no numbers; here the ratio is about 2.4 at 120^2, the size of the
    O(dt^2) term RTLBFS drops with dt_lattice = 0.5 and tau_g = 1.1)."""
    e = [_hill_error(N, TLBFS) for N in (60, 120)]
    order = np.log(e[0] / e[1]) / np.log(2.0)
    assert 1.8 <= order <= 2.2, (e, order)
    e_rt = _hill_error(120, RTLBFS)
    assert e[1] < e_rt < 4.0 * e[1], (e[1], e_rt)


def test_tlbfs_cavity_ra1e3_matches_table1():
    """Sec. 4.2, Table 1 at Ra = 1e3 on a 32^2 uniform mesh: the average
    Nusselt number of TLBFS within 2% of the printed 1.118."""
    N = 32
    bc, Tw, gax = inputs.dhc_bc(2)
    nu, chi, bg = physics_from_ra(1e3, 0.71, 0.1, float(N))
    o = Oracle(OracleConfig(n=(N, N), bc=bc, Tw=Tw, gravity_axis=gax, nu=nu, chi=chi, beta_g=bg, dtl=1.0,
                            dt=min(0.5, 0.15 / max(nu, chi)), method=TLBFS))
    for _ in range(40):
        o.step(500)
        if max(o.residual()) < 1e-9:
            break
    assert max(o.residual()) < 1e-9
    nu_ = o.nusselt()
    assert abs(nu_["volume"] - 1.118) <= 0.02 * 1.118, nu_
    assert abs(nu_["hot_avg"] - nu_["cold_avg"]) <= 1e-4 * nu_["hot_avg"], nu_
