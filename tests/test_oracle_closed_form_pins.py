"""Closed-form pins of the oracle's Eq. 65 residual, Eq. 69 volume Nusselt
number, wall closure and buoyancy placement.

Each expected value below is derived by hand from the scheme's definition
(Sec. 3.2, Eqs. 29, 55-59, 64) for a state simple enough to be solved
exactly, never read back from the oracle:

* a uniform buoyant state in a periodic box only accelerates, so the Eq. 65
  velocity ratio has a closed form and the temperature ratio is zero;
* a single Fourier temperature mode in a periodic box at rest evolves by the
  amplification factor of the linear diffusion stencil that Eqs. 29, 55, 56
  and 59 build, which gives the Eq. 65 temperature ratio with the absolute
  temperature in the denominator;
* a state with uniform velocity, uniform density and a linear temperature
  has an Eq. 69 integral that is elementary;
* the body-force driven channel has a discrete steady state known exactly:
  the parabola shifted by F d^2 / (2 nu), with d the half-cell wall distance
  of the one-sided wall stress.
"""
import numpy as np
import pytest

import inputs
from oracle import (INIT_CONDUCTION, PERIODIC, WALL_ADIABATIC, WALL_ISOTHERMAL, Oracle, OracleConfig,
                    physics_from_ra)

T_REF = 0.5  # (T_h + T_l) / 2 with T_l = 0, T_h = 1


# ------------------------------------------------------------- Eq. 65 ----

@pytest.mark.parametrize("dev", [0, 1])
def test_eq65_velocity_ratio_of_uniformly_accelerated_state(dev):
    """Fully periodic box, rho = 1, uniform u0 and T1 != T_ref, gravity along
    x.  Every face sees the same lattice data, so all fluxes cancel and only
    the Eq. 64 source acts: u_x grows by dt beta_g (T1 - T_ref) per step, T
    stays put.  Eq. 65 then reads
        res_u = (|u^{n+1}| - |u^n|) / |u^{n+1}|,   res_T = 0.
    A denominator at time level n, or a missing absolute value, fails."""
    N, M, bg, dt, T1 = 6, 5, 1e-3, 0.5, 0.8
    u0 = (0.001, 0.002)
    o = Oracle(OracleConfig(n=(N, M), bc=(PERIODIC,) * 6, gravity_axis=0, nu=0.1, chi=0.1, beta_g=bg, dt=dt,
                            deviation=dev))
    u = np.zeros((2, N * M))
    u[0], u[1] = u0
    o.set_prim(np.ones(N * M), u, np.full(N * M, T1))
    inc = dt * bg * (T1 - T_REF)
    done = 0
    for steps in (1, 6):
        o.step(steps)
        done += steps
        new = np.hypot(u0[0] + done * inc, u0[1])
        old = np.hypot(u0[0] + (done - 1) * inc, u0[1])
        res_u, res_T = o.residual()
        assert abs(res_u / ((new - old) / new) - 1.0) < 1e-12, (done, res_u)
        assert res_T == 0.0
        assert np.abs(o.prim(1) - (u0[0] + done * inc)).max() < 1e-15
        assert np.abs(o.prim(3) - T1).max() < 1e-15


@pytest.mark.parametrize("dev", [0, 1])
@pytest.mark.parametrize("dtl", [1.0, 0.5, 0.8])
def test_eq65_temperature_ratio_of_a_fourier_mode(dev, dtl):
    """Periodic box at rest, rho = 1, no gravity, T = Tm + A cos(k x) with
    k = 2 pi / N on unit cells.  With m = 0 and uniform rho the predicted
    mass flux vanishes and Eq. 59 reduces to F_e = -chi D_n e.  Eq. 29
    reconstructs the +-h lattice nodes from the two cells' Eq. 55 gradients
    (central, from Eq. 56 midpoint face values), so on a mode e_j = exp(ikj)
        D_n e(j + 1/2) = [e^{ik} - 1 + (h - 1/2) i sin k (e^{ik} + 1)] e_j / (2h)
    and the update multiplies the mode by
        G = 1 + dt chi [cos k - 1 - (h - 1/2) sin^2 k] / h.
    After n steps Eq. 65 gives, with the absolute temperature summing to
    N M Tm,
        res_T = |A G^{n-1} (G - 1)| sum_i |cos k x_i| / (N Tm).
    Using T - T_ref in the sum (a near-zero denominator here, Tm = 0.7
    keeps it away from zero but different) or a wrong reconstruction offset
    fails; plain and deviation storage must agree."""
    N, M, A, Tm, dt, chi = 16, 4, 0.05, 0.7, 0.5, 0.2
    o = Oracle(OracleConfig(n=(N, M), bc=(PERIODIC,) * 6, gravity_axis=-1, nu=0.1, chi=chi, beta_g=0.0, dtl=dtl,
                            dt=dt, deviation=dev))
    xc, _ = o.axis(0)
    k = 2.0 * np.pi / N
    o.set_prim(np.ones(N * M), np.zeros((2, N * M)), np.tile(Tm + A * np.cos(k * xc), M))
    G = 1.0 + dt * chi * (np.cos(k) - 1.0 - (dtl - 0.5) * np.sin(k) ** 2) / dtl
    done = 0
    for steps in (1, 4):
        o.step(steps)
        done += steps
        expect = abs(A * G ** (done - 1) * (G - 1.0)) * np.abs(np.cos(k * xc)).sum() / (N * Tm)
        res_u, res_T = o.residual()
        assert res_u == 0.0
        assert abs(res_T / expect - 1.0) < 1e-12, (done, res_T, expect)
        T = o.grid(o.prim(3))
        assert np.abs(T - (Tm + A * G ** done * np.cos(k * xc))[None, :]).max() < 1e-15


# ------------------------------------------------------------- Eq. 69 ----

@pytest.mark.parametrize("dev", [0, 1])
@pytest.mark.parametrize("stretch", [0.0, 1.5])
def test_eq69_volume_nusselt_of_uniform_drift_over_linear_temperature(dev, stretch):
    """Cavity geometry (hot x = 0 at T = 1, cold x = L at T = 0), state set
    to rho = 1.2, u = (U, V) uniform and the conduction profile T = 1 - x/L.
    Eq. 56 face values and Eq. 55 gradients are exact for a linear T, and
    the mean of T over the box is 1/2, so Eq. 69 gives
        Nu_a = L/(chi dT L^2) * int (u T - chi dT/dx) = 1 + U L / (2 chi)
    with no density factor; every wall Nusselt number is exactly 1."""
    N, chi, U, V, rho = 12, 0.13, 0.004, -0.003, 1.2
    bc, Tw, gax = inputs.dhc_bc(2)
    o = Oracle(OracleConfig(n=(N, N + 2), stretch=(stretch,) * 2, bc=bc, Tw=Tw, gravity_axis=gax, nu=0.1, chi=chi,
                            beta_g=0.0, deviation=dev))
    xc, wx = o.axis(0)
    L = wx.sum()
    cells = N * (N + 2)
    u = np.zeros((2, cells))
    u[0], u[1] = U, V
    o.set_prim(np.full(cells, rho), u, np.tile(1.0 - xc / L, N + 2))
    nu_ = o.nusselt()
    assert abs(nu_["volume"] - (1.0 + U * L / (2.0 * chi))) < 1e-12
    for k in ("hot_avg", "hot_max", "cold_avg", "cold_max"):
        assert abs(nu_[k] - 1.0) < 1e-12, k


# --------------------------------------------------- wall closure (S6) ----

def _channel(H, dev=0, dtl=1.0, nu=0.4, umax=0.01, T1=0.8):
    """Plane channel: periodic along x (4 cells), no-slip adiabatic walls at
    y = 0 and y = H (unit cells), uniform T1 with gravity along x, so the
    Eq. 64 force F = beta_g (T1 - T_ref) drives the flow.  Started from the
    continuum parabola and run to a bitwise steady state."""
    NX = 4
    F = 8.0 * nu * umax / H ** 2
    dt = min(0.5, 0.15 / nu)
    o = Oracle(OracleConfig(n=(NX, H), bc=(PERIODIC, PERIODIC, WALL_ADIABATIC, WALL_ADIABATIC, PERIODIC, PERIODIC),
                            Tw=(0.0,) * 6, gravity_axis=0, nu=nu, chi=nu, beta_g=F / (T1 - T_REF), dt=dt, dtl=dtl,
                            deviation=dev))
    yc, _ = o.axis(1)
    parabola = F * yc * (H - yc) / (2.0 * nu)
    u = np.zeros((2, NX * H))
    u[0] = np.repeat(parabola, NX)
    o.set_prim(np.ones(NX * H), u, np.full(NX * H, T1))
    o.step(int(3.0 * H * H / (nu * dt)))
    return o, F, parabola


@pytest.mark.parametrize("dev", [0, 1])
@pytest.mark.parametrize("dtl", [1.0, 0.6])
def test_wall_shear_channel_discrete_steady_state(dev, dtl):
    """S6 wall stress -nu (-m_t / d) with d the half-cell distance.  For a
    quadratic profile the interior Eq. 29 lattice derivative is exact on
    uniform cells, and a global force balance fixes the wall stress at
    F H / 2.  The discrete steady state is therefore the parabola
    F y (H - y) / (2 nu) shifted up by F d^2 / (2 nu), d = 1/2, with rho = 1,
    v = 0 and T = T1 exactly.  That makes the error against the continuum
    profile exactly u_max / H^2 relative: second order.  A wall distance of
    one cell, or a missing factor in the wall shear, moves the shift."""
    errs = []
    for H in (8, 16, 32):
        o, F, parabola = _channel(H, dev=dev, dtl=dtl)
        ux = o.grid(o.prim(1))
        umax = F * H * H / (8.0 * 0.4)
        assert np.abs(ux - (parabola + F * 0.25 / (2.0 * 0.4))[:, None]).max() < 1e-11 * umax
        assert np.abs(o.prim(2)).max() == 0.0
        assert np.abs(o.prim(0) - 1.0).max() < 1e-15 and np.abs(o.prim(3) - 0.8).max() < 1e-15
        errs.append(np.abs(ux[:, 0] - parabola).max())
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(orders - 2.0) < 1e-6), orders


# ------------------------------------------ buoyancy placement (S5), P5b ----

def _rb(NX, NY, noise, steps, force_in_predictor=1):
    bc, Tw, gax = inputs.rb_bc()
    nu, chi, bg = physics_from_ra(1000.0, 0.71, 0.1, float(NY))
    o = Oracle(OracleConfig(n=(NX, NY), bc=bc, Tw=Tw, gravity_axis=gax, nu=nu, chi=chi, beta_g=bg,
                            init=INIT_CONDUCTION, seed=3, noise_amp=noise, force_in_predictor=force_in_predictor))
    o.step(steps)
    return o


def test_rayleigh_benard_below_onset_returns_to_hydrostatic_conduction():
    """Ra = 1000 < 1708 in the 2:1 periodic box.  (i) A 1e-3 temperature
    noise decays onto the noise-free run.  (ii) The noise-free state is
    steady and x-invariant.  (iii) Its only velocity is the wall-row
    current that the S6 closure leaves in a hydrostatic state (pressure
    c_s^2 rho_P at the wall, not extrapolated); away from the walls the
    fluid is at rest to 1e-6 of V_c, and the current and Nu - 1 shrink
    under refinement.  (iv) With the paper-literal force placement (update
    only, no force in the predicted momentum) the interior is not at rest:
    a spurious current 100 times larger remains, which is the reason for
    the S5 reading."""
    Vc = 0.1
    a = _rb(32, 16, 1e-3, 14000)
    b = _rb(32, 16, 0.0, 14000)
    assert max(np.abs(a.prim(f) - b.prim(f)).max() for f in range(4)) < 1e-8
    assert max(b.residual()) < 1e-11
    assert np.abs(b.prim(1)).max() < 1e-25
    v = b.grid(b.prim(2))
    assert np.abs(v - v[:, :1]).max() < 1e-20
    interior = np.abs(v[3:-3]).max()
    assert interior < 1e-5 * Vc, interior
    coarse = _rb(16, 8, 0.0, 14000)
    nb, nc = b.nusselt(), coarse.nusselt()
    for k in ("hot_avg", "cold_avg", "volume"):
        assert 0.0 < nb[k] - 1.0 < 0.5 * (nc[k] - 1.0), (k, nb[k], nc[k])
    assert np.abs(v).max() < 0.5 * np.abs(coarse.prim(2)).max()
    lit = _rb(32, 16, 0.0, 14000, force_in_predictor=0)
    assert np.abs(lit.grid(lit.prim(2))[3:-3]).max() > 100.0 * interior
