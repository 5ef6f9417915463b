"""GPU parity: the HIP kernels (through the C ABI) against the FP64 oracle.

Element-by-element comparison of the absolute primitive fields on the same
seeded inputs.  Tolerance for the FP64 paths (RTLBFS and TLBFS): max |gpu -
oracle| / scale <= 1e-12 per field.  The scale is max |oracle| for rho and
T.  The velocity components share one scale, the largest of max |oracle
u_a| over the components (the flow speed).  That speed is floored at V_c
(= Ma, the characteristic velocity of Eq. 63) while the flow is still
developing.  The long horizons (the 64^2 cavity at 20,000 steps, the 256^2
cavity's 2,000-step prefix, the 48^3 cube) drop the floor.  The kernels
contract multiply-adds and sum fluxes in a different order.  In plain storage
the rounding of rho ~ 1 (1e-16) enters the pressure gradient every step, so
early in a run, when |u| << V_c, the velocity differences against max |u|
alone reflect that rounding, not the scheme.  The FP32 deviation path is
compared against the oracle's FP64 deviation form with a tolerance derived
from FP32 rounding, and on Nusselt numbers at steady state (1e-4 relative).
"""
import numpy as np
import pytest

import inputs
import paper_2202_13449_amd as rt
from oracle import INIT_CONDUCTION, INIT_REST, Oracle, OracleConfig, physics_from_ra, mesh_nodes

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
TLBFS_TOL = FP64_TOL  # measured about 3e-15, like RTLBFS


def make_pair(dim, n, stretch, kind, Tdev, gaxis, Ra=1e4, Pr=0.71, Ma=0.1, precision=rt.FP64_PLAIN, seed=1,
              noise=1e-3, init=INIT_REST, dtl=1.0, dt=0.0, residual_every=100, graph_steps=0, L_axis=None,
              method=rt.METHOD_RTLBFS, tile=0):
    """A GPU solver and an oracle run of the same problem (the oracle is given
    the parameters the library derived, read back through rtlbfs_get_info)."""
    s = rt.Solver(dim, n, stretch, kind, Tdev, gaxis, Ra=Ra, Pr=Pr, Ma=Ma, precision=precision, seed=seed,
                  noise_amp=noise, init=init, dtl=dtl, dt=dt, residual_every=residual_every,
                  graph_steps=graph_steps, method=method, tile=tile)
    info = s.info
    # independent derivation of Eq. 63 on the oracle side
    La = info.L
    nu, chi, bg = physics_from_ra(Ra, Pr, Ma, La)
    assert abs(nu - info.nu) <= 1e-14 * nu and abs(chi - info.chi) <= 1e-14 * chi
    assert abs(bg - info.beta_g) <= 1e-14 * bg
    cfg = OracleConfig(dim=dim, n=tuple(n) + (1,) * (3 - len(n)), stretch=tuple(stretch) + (0.0,) * (3 - len(stretch)),
                       bc=tuple(kind) + (0,) * (6 - len(kind)), Tw=tuple(Tdev) + (0.0,) * (6 - len(Tdev)),
                       gravity_axis=gaxis, nu=nu, chi=chi, beta_g=bg, dtl=info.dtl, dt=info.dt,
                       deviation=0 if precision == rt.FP64_PLAIN else 1, init=init, seed=seed, noise_amp=noise,
                       method=method)
    return s, Oracle(cfg)


def field_rel(s, o, dim, Vc=0.1):
    """max |gpu - oracle| / scale per absolute primitive.  The scale is
    max |oracle| (P14) for rho and T; the velocity is one vector field, so
    its components share the scale max_a max |oracle u_a| (the largest speed
    component), floored at Vc.  Vc = 0 gives the plain P14 scale, used once
    the flow is developed."""
    prim = [o.prim(f) for f in range(dim + 2)]
    speed = max(float(np.abs(prim[f]).max()) for f in range(1, dim + 1))
    out = []
    for f in range(dim + 2):
        a, b = s.field(f), prim[f]
        scale = max(speed, Vc) if 1 <= f <= dim else float(np.abs(b).max())
        out.append(float(np.abs(a - b).max() / max(scale, 1e-300)))
    return out


DHC2 = dict(kind=(1, 1, 2, 2), Tdev=(0.5, -0.5, 0.0, 0.0), gaxis=1)


def test_initial_state_is_identical():
    """Both sides implement SplitMix64 and the conduction profile from their
    definitions: the uploaded initial state matches the oracle's bit for bit."""
    for prec in (rt.FP64_PLAIN, rt.FP64_DEV):
        s, o = make_pair(2, (40, 24), (1.5, 1.5), **DHC2, precision=prec, init=INIT_CONDUCTION, noise=1e-3, seed=9)
        for f in range(4):
            assert np.array_equal(s.stored(f), o.stored(f)), (prec, f)


@pytest.mark.parametrize("prec", [rt.FP64_PLAIN, rt.FP64_DEV])
@pytest.mark.parametrize("shape,stretch", [((64, 64), (0.0, 0.0)), ((70, 45), (1.5, 1.5)), ((33, 9), (0.0, 0.0))])
def test_fp64_cavity_parity(prec, shape, stretch):
    """Differentially heated cavity, several tiles with ragged tails,
    uniform and stretched: fields after 600 steps within 1e-12."""
    s, o = make_pair(2, shape, stretch, **DHC2, Ra=1e5, precision=prec, noise=1e-3)
    s.step(600)
    o.step(600)
    rel = field_rel(s, o, 2)
    assert max(rel) <= FP64_TOL, rel


def test_fp64_c1_parity_1000_steps_and_diagnostics():
    """64^2 uniform cavity at Ra = 1e3 (the small configuration): fields,
    Eq. 65 residual, Nusselt numbers and mass after 1000 steps."""
    s, o = make_pair(2, (64, 64), (0.0, 0.0), **DHC2, Ra=1e3, noise=1e-6)
    s.step(1000)
    o.step(1000)
    assert max(field_rel(s, o, 2)) <= FP64_TOL
    ru, rT = s.residual()
    ou, oT = o.residual()
    assert abs(ru - ou) <= 1e-9 * ou and abs(rT - oT) <= 1e-9 * oT
    a, b = s.nusselt(), o.nusselt()
    for k in a:
        assert abs(a[k] - b[k]) <= 1e-11 * abs(b[k]), (k, a[k], b[k])
    ig, io = s.integrals(), o.integrals()
    assert abs(ig["volume"] - io["volume"]) <= 1e-12 * io["volume"]
    assert abs(ig["mass_dev"] - io["mass_dev"]) <= 1e-12 * io["volume"]


def test_fp64_c1_parity_20000_steps():
    """The small configuration over a long horizon: the 64^2 uniform cavity at
    Ra = 1e3 for 20,000 steps (t* = 62, most of the way to steady state),
    fields within 1e-12 of the oracle.  The oracle needs about a minute."""
    s, o = make_pair(2, (64, 64), (0.0, 0.0), **DHC2, Ra=1e3, noise=1e-6)
    s.step(20000)
    o.step(20000)
    rel = field_rel(s, o, 2, Vc=0.0)
    print("64^2, 20000 steps: rel (P14 scale)", rel, flush=True)
    assert max(np.abs(o.prim(1)).max(), np.abs(o.prim(2)).max()) > 0.01  # developed: u L / chi ~ 3.6
    assert max(rel) <= FP64_TOL, rel


def test_fp64_periodic_rayleigh_benard_parity():
    """Rayleigh-Benard box periodic in x (wrapped halos, ragged periodic
    tiles): 400 steps."""
    bc, Tw, g = inputs.rb_bc()
    s, o = make_pair(2, (72, 20), (0.0, 0.0), bc[:4], Tw[:4], g, Ra=1e6, init=INIT_CONDUCTION, noise=1e-3, seed=3)
    s.step(400)
    o.step(400)
    rel = field_rel(s, o, 2)
    assert max(rel) <= FP64_TOL, rel


def test_fp64_fully_periodic_gaussian_hill_parity():
    """Periodic box with given nu/chi, dtl = 0.5, Delta t = 1 (the Sec. 4.1
    set-up) starting from the Gaussian hill."""
    N = 40
    L = N / 2.0
    chi = 0.1
    u0 = 10.0 * chi / L
    s = rt.Solver(2, (N, N), (0, 0), (0, 0, 0, 0), (0, 0, 0, 0), -1, phys_given=1, nu=chi, chi=chi, beta_g=0.0,
                  dtl=0.5, dt=1.0)
    o = Oracle(OracleConfig(n=(N, N), bc=(0,) * 6, gravity_axis=-1, nu=chi, chi=chi, dtl=0.5, dt=1.0))
    xc, _ = o.axis(0)
    yc, _ = o.axis(1)
    u = np.zeros((2, N * N))
    u[0] = u0
    T = inputs.gaussian_hill(xc, yc, L, 0.0, chi, u0).reshape(-1)
    s.set_state(np.ones(N * N), u, T)
    o.set_prim(np.ones(N * N), u, T)
    s.step(80)
    o.step(80)
    assert max(field_rel(s, o, 2)[1:]) <= FP64_TOL  # rho stays exactly 1 on both


def test_fp64_random_state_parity_all_boundary_kinds():
    """Random smooth-ish state, mixed walls (isothermal, adiabatic) and
    gravity along x: 200 steps."""
    s, o = make_pair(2, (37, 29), (1.2, 0.0), (1, 2, 2, 1), (0.3, 0.0, 0.0, -0.2), 0, Ra=1e5)
    rho, u, T = inputs.random_state(37 * 29, 2, seed=11)
    s.set_state(rho, u, T)
    o.set_prim(rho, u, T)
    s.step(200)
    o.step(200)
    assert max(field_rel(s, o, 2)) <= FP64_TOL


def test_graph_replay_equals_direct_launches():
    """Chunks replayed from captured HIP graphs give exactly the same state as
    kernels launched one by one, over several replays with host work in
    between."""
    args = (2, (48, 40), (0, 0), DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"])
    a = rt.Solver(*args, Ra=1e5, noise_amp=1e-3, seed=2, residual_every=25, graph_steps=0)
    b = rt.Solver(*args, Ra=1e5, noise_amp=1e-3, seed=2, residual_every=25, graph_steps=-1)
    for _ in range(4):
        a.step(50)
        b.step(50)
        assert a.residual() == b.residual()
        for f in range(4):
            assert np.array_equal(a.stored(f), b.stored(f))
    a.step(37)  # partial chunk + parity flip
    b.step(37)
    for f in range(4):
        assert np.array_equal(a.stored(f), b.stored(f))
    # two steps per launch: odd chunks (residual_every = 25) replayed from
    # graphs and launched directly
    c = rt.Solver(*args, Ra=1e5, noise_amp=1e-3, seed=2, residual_every=25, graph_steps=0, tile=6)
    e = rt.Solver(*args, Ra=1e5, noise_amp=1e-3, seed=2, residual_every=25, graph_steps=-1, tile=6)
    r = rt.Solver(*args, Ra=1e5, noise_amp=1e-3, seed=2, residual_every=25, graph_steps=0, tile=1)
    for n in (50, 50, 37, 1, 25):
        for x in (c, e, r):
            x.step(n)
        assert c.residual() == e.residual()
        # the FP64 partial sums are reduced in a different order (other block size)
        assert np.allclose(c.residual(), r.residual(), rtol=1e-13, atol=0)
        for f in range(4):
            assert np.array_equal(c.stored(f), e.stored(f))
            assert np.array_equal(c.stored(f), r.stored(f))


def test_every_tile_shape_gives_the_same_state():
    """The per-cell arithmetic does not depend on the launch shape: all 2D
    tiles, one or two steps per launch (the two-step launches recompute the
    halo ring of their first step), and the autotuned choice produce
    bit-identical states, in FP32 with stochastic rounding and in FP64, on a
    walled and on a periodic box, also for step counts the two-step shapes
    must finish with a one-step launch."""
    cases = [((2, (70, 45), (1.5, 1.5), DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"]), dict(Ra=1e5)),
             ((2, (52, 20), (0.0, 0.0), (0, 0, 1, 1), (0.0, 0.0, 0.5, -0.5), 1),
              dict(Ra=1e6, init=INIT_CONDUCTION))]
    for args, kw in cases:
        for prec in (rt.FP32_DEV, rt.FP64_PLAIN):
            ref = None
            for tile in range(0, 10):
                s = rt.Solver(*args, noise_amp=1e-3, seed=4, tile=tile, precision=prec, residual_every=20, **kw)
                if tile == 0:
                    tm = list(s.info.tune_ms)[:9]
                    assert all(t > 0 for t in tm), tm
                assert s.info.steps_per_launch == (2 if tile >= 6 else 1 if tile >= 1 else s.info.steps_per_launch)
                s.step(120)
                s.step(7)  # odd: ends with a one-step launch on the two-step shapes
                st = [s.stored(f) for f in range(4)]
                res = s.residual()
                if ref is None:
                    ref = (st, res)
                for f in range(4):
                    assert np.array_equal(st[f], ref[0][f]), (prec, tile, f)
                # same state; the Eq. 65 sums only differ in reduction order
                assert np.allclose(res, ref[1], rtol=1e-13, atol=0), (prec, tile, res, ref[1])


def test_rest_state_bitwise_and_mass_conservation_on_gpu():
    s = rt.Solver(2, (40, 30), (1.5, 1.5), (2, 1, 2, 1), (0, 0, 0, 0), 1, Ra=1e5)
    before = [s.stored(f) for f in range(4)]
    s.step(300)
    for f in range(4):
        assert np.array_equal(s.stored(f), before[f])
    s, o = make_pair(2, (40, 30), (1.5, 1.5), **DHC2, Ra=1e6, noise=1e-2)
    m0 = s.integrals()["mass_dev"]
    s.step(2000)
    vol = s.integrals()["volume"]
    assert abs(s.integrals()["mass_dev"] - m0) <= 1e-13 * vol


def test_minimum_mesh_and_single_tile():
    s, o = make_pair(2, (4, 4), (0, 0), **DHC2, Ra=1e4)
    s.step(50)
    o.step(50)
    assert max(field_rel(s, o, 2)) <= FP64_TOL


def test_empty_and_invalid_calls_on_a_live_handle():
    """Degenerate calls on a live handle: zero steps leave the state bit for
    bit; a negative step count, a short output buffer and a field index out
    of range are EINVAL and change nothing; the handle keeps working, and a
    one-step call after them matches the oracle (one step in a two-step
    shape runs the one-step launch of the same tile)."""
    import ctypes as C

    s, o = make_pair(2, (20, 12), (1.2, 0.0), **DHC2, Ra=1e4, tile=6)
    s.step(7)
    o.step(7)
    before = [s.stored(f).copy() for f in range(4)]
    s.step(0)
    lib, h = s._lib, s._h
    assert lib.rtlbfs_step(h, -1) == rt.EINVAL
    buf = np.zeros(s.cells)
    assert lib.rtlbfs_get_field(h, 0, buf.ctypes.data_as(C.POINTER(C.c_double)), s.cells - 1) == rt.EINVAL
    assert lib.rtlbfs_get_field(h, 4, buf.ctypes.data_as(C.POINTER(C.c_double)), s.cells) == rt.EINVAL
    for f in range(4):
        assert np.array_equal(s.stored(f), before[f])
    s.step(1)
    o.step(1)
    assert max(field_rel(s, o, 2)) <= FP64_TOL


@pytest.mark.parametrize("prec", [rt.FP32_DEV, rt.FP64_PLAIN])
def test_checkpoint_restore_continues_bit_for_bit(prec):
    """A run stopped after 200 steps (taken in uneven calls), checkpointed
    (stored fields, step counter, mass-correction phase and reference mass)
    and restored into a new handle created with another seed and noise,
    continues exactly as the uninterrupted 350-step run: every stored field
    and the Eq. 65 residual, FP32 (stochastic rounding keyed by the step
    counter, mass correction every 100 steps) and FP64, 2D and 3D."""
    cases = [(2, (48, 40), (1.5, 1.5), DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"]),
             (3, (12, 10, 9), (1.8, 1.8, 1.8), DHC3["kind"], DHC3["Tdev"], DHC3["gaxis"])]
    for args in cases:
        kw = dict(Ra=1e5, precision=prec, residual_every=50, mass_fix_every=100)
        a = rt.Solver(*args, seed=3, noise_amp=1e-3, **kw)
        a.step(350)
        b = rt.Solver(*args, seed=3, noise_amp=1e-3, **kw)
        b.step(130)
        b.step(70)
        stored, ck = b.checkpoint()
        assert ck.steps == 200
        b.close()
        c = rt.Solver(*args, seed=99, noise_amp=5e-3, **kw)
        c.restore(stored, ck)
        c.step(150)
        for f in range(args[0] + 2):
            assert np.array_equal(a.stored(f), c.stored(f)), (args[1], f)
        assert a.residual() == c.residual()
        assert c.checkpoint()[1].steps == 350


@pytest.mark.parametrize("prec", [rt.FP64_PLAIN, rt.FP32_DEV])
def test_two_runs_are_bitwise_identical(prec):
    """Determinism: two handles of the same problem, stepped alike, hold the
    same stored state bit for bit, and the FP64 diagnostics (Eq. 65 residual,
    Nusselt numbers, integrals) are equal; the reductions run in a fixed
    order and the stochastic rounding is keyed by (cell, step, field)."""
    args = (2, (40, 28), (1.3, 1.3), DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"])
    a = rt.Solver(*args, Ra=1e5, precision=prec, seed=3, noise_amp=1e-3, residual_every=50)
    b = rt.Solver(*args, Ra=1e5, precision=prec, seed=3, noise_amp=1e-3, residual_every=50)
    a.step(300)
    b.step(130)
    b.step(170)
    for f in range(4):
        assert np.array_equal(a.stored(f), b.stored(f)), f
    assert a.residual() == b.residual()
    assert a.nusselt() == b.nusselt()
    assert a.integrals() == b.integrals()


def test_divergence_is_reported_and_clears():
    """Failure detection, forced from the host: a state moving at Mach 0.69
    (above the default guard of 0.5), and then one with a NaN temperature,
    makes the synchronising call after the next residual step return
    EDIVERGED without stopping the handle; a valid state clears the flag at
    the following residual step."""
    s = rt.Solver(2, (32, 32), (0.0, 0.0), DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"], Ra=1e4, residual_every=1)
    n = s.cells
    s.step(3)
    s.sync()
    u = np.zeros(2 * n)
    u[:n] = 0.4  # |u| / c_s = 0.69
    s.set_state(np.ones(n), u, np.full(n, 0.5))
    s.step(1)
    with pytest.raises(rt.RtlbfsError) as e:
        s.sync()
    assert e.value.code == rt.EDIVERGED
    s.set_state(np.ones(n), np.zeros(2 * n), np.full(n, 0.5))
    s.step(1)
    s.sync()
    T = np.full(n, 0.5)
    T[n // 3] = np.nan
    s.set_state(np.ones(n), np.zeros(2 * n), T)
    s.step(1)
    with pytest.raises(rt.RtlbfsError) as e:
        s.sync()
    assert e.value.code == rt.EDIVERGED
    s.set_state(np.ones(n), np.zeros(2 * n), np.full(n, 0.5))
    s.step(2)
    s.sync()
    assert np.isfinite(s.field(3)).all()


_FULL_SIZE_ORACLE = {}


@pytest.mark.timeout(600)
@pytest.mark.parametrize("tile", [0, 6])
def test_c2_full_size_prefix_fp64(tile):
    """256^2 tanh (phi = 1.5) cavity at Ra = 1e6, the benchmarked
    configuration, in the autotuned launch shape and in 16x16 with two steps
    per launch: the 2,000-step prefix compared cell by cell with the oracle
    (one oracle run, about 90 s, serves both shapes), on P14's scale
    max |oracle| for every field."""
    s, o = make_pair(2, (256, 256), (1.5, 1.5), **DHC2, Ra=1e6, noise=1e-6, tile=tile)
    print("C2 prefix, tile", (s.info.tile_x, s.info.tile_y, s.info.steps_per_launch), flush=True)
    s.step(2000)
    if "fp64" not in _FULL_SIZE_ORACLE:
        o.step(2000)
        _FULL_SIZE_ORACLE["fp64"] = o
    o = _FULL_SIZE_ORACLE["fp64"]
    rel = field_rel(s, o, 2, Vc=0.0)
    print("C2 prefix 2000 steps: rel (P14 scale)", rel, "u max", np.abs(o.prim(1)).max(), flush=True)
    assert max(rel) <= FP64_TOL, rel


@pytest.mark.parametrize("tile", [0, 6])
def test_c2_full_size_fp32_in_the_benchmarked_configuration(tile):
    """The benchmark workload itself: 256^2 tanh cavity, Ra = 1e6, FP32
    deviation storage with stochastic rounding, 200 steps against the FP64
    oracle cell by cell; in the autotuned launch shape and in 16x16 with two
    steps per launch (the shape the autotuner usually picks on this size).
    Besides the usual scale (V_c for velocities), every field is held to its
    own maximum, since the flow is still weak this early."""
    s, o = make_pair(2, (256, 256), (1.5, 1.5), **DHC2, Ra=1e6, noise=1e-6, precision=rt.FP32_DEV, tile=tile)
    if tile == 6:
        assert (s.info.tile_x, s.info.tile_y, s.info.steps_per_launch) == (16, 16, 2)
    s.step(200)
    if "fp32" not in _FULL_SIZE_ORACLE:  # the oracle run does not depend on the launch shape
        o.step(200)
        _FULL_SIZE_ORACLE["fp32"] = o
    o = _FULL_SIZE_ORACLE["fp32"]
    rel = field_rel(s, o, 2)
    own = [float(np.abs(s.field(f) - o.prim(f)).max() / np.abs(o.prim(f)).max()) for f in (1, 2, 3)]
    r_gpu, r_orc = s.stored(0), o.stored(0)
    r_rel = float(np.abs(r_gpu - r_orc).max() / np.abs(r_orc).max())
    print("tile", (s.info.tile_x, s.info.tile_y, s.info.steps_per_launch), "r", r_rel, "rel", rel, "own", own)
    assert r_rel <= 1e-5
    assert max(rel[1:]) <= 1e-4, rel
    assert max(own) <= 1e-5, own  # measured: about 4e-7


def step_from_gpu_state(s, o, dim, nsteps):
    """Hand the GPU's stored fields to the oracle (FP32 values are exact in
    FP64; both sides store r = rho - 1 or rho, m, theta = rho (T - T0) or
    the plain energy alike), then advance both by nsteps."""
    for f in range(dim + 2):
        o.set_stored(f, s.stored(f))
    s.step(nsteps)
    o.step(nsteps)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", [rt.FP64_PLAIN, rt.FP32_DEV])
def test_c3_full_size_steps_from_a_developed_state(prec):
    """The 1024 x 512 periodic Rayleigh-Benard box at Ra = 1e8 as the
    benchmark runs it (conduction profile plus 1e-3 noise, seed 3, the
    autotuned launch shape, graph-replayed chunks): after 20,000 GPU steps
    the state is handed to the oracle and both advance 4 steps.  Every cell
    of every field is compared on P14's scale, max |oracle|, which needs a
    developed flow: a few hundred steps from rest the velocity is still at
    the level of the rounding of the hydrostatic balance.  1e-12 in FP64; in
    FP32 the GPU's own rounding of 4 steps, held to 1e-6."""
    s, o = make_pair(2, (1024, 512), (0.0, 0.0), (0, 0, 1, 1), (0.0, 0.0, 0.5, -0.5), 1, Ra=1e8, noise=1e-3,
                     seed=3, init=INIT_CONDUCTION, precision=prec)
    print("C3 full size, tile", (s.info.tile_x, s.info.tile_y, s.info.steps_per_launch), flush=True)
    s.step(20000)
    step_from_gpu_state(s, o, 2, 4)
    rel = field_rel(s, o, 2, Vc=0.0)
    print("C3 4 steps from step 20000:", rel, "max |u|", float(np.abs(o.prim(1)).max()), flush=True)
    assert max(rel) <= (FP64_TOL if prec == rt.FP64_PLAIN else 1e-6), rel


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", [rt.FP64_PLAIN, rt.FP32_DEV])
def test_c5_full_size_step_from_a_developed_state(prec):
    """The 192^3 tanh (phi = 1.8) cube at Ra = 1e6 as the benchmark runs it
    (the default 4 x 4 x 4 tiles, graph-replayed chunks): after 3,000 GPU
    steps (the wall layers developed; P14's scale max |oracle| needs them)
    the state is handed to the oracle and both advance one step.  All
    7,077,888 cells of every field are compared on that scale: 1e-12 in
    FP64, 1e-6 in FP32."""
    s, o = make_pair(3, (192, 192, 192), (1.8, 1.8, 1.8), (1, 1, 2, 2, 2, 2), (-0.5, 0.5, 0, 0, 0, 0), 2, Ra=1e6,
                     noise=1e-6, precision=prec)
    print("C5 full size, tile", (s.info.tile_x, s.info.tile_y, s.info.tile_z), flush=True)
    s.step(3000)
    step_from_gpu_state(s, o, 3, 1)
    rel = field_rel(s, o, 3, Vc=0.0)
    print("C5 1 step from step 3000:", rel, "max |u|", float(np.abs(o.prim(1)).max()), flush=True)
    assert max(rel) <= (FP64_TOL if prec == rt.FP64_PLAIN else 1e-6), rel
    o.close()


@pytest.mark.parametrize("prec", [rt.FP64_PLAIN, rt.FP64_DEV])
def test_buoyancy_in_the_update_only_parity(prec):
    """The paper-literal placement of Eq. 64 (force in the cell update only,
    opts.buoyancy_update_only = 1) against the oracle with the force left
    out of the predicted momentum: a stretched cavity and the periodic
    Rayleigh-Benard box, 600 steps, fields within 1e-12.  The two placements
    differ by far more than that (checked on the oracle)."""
    cases = [((2, (40, 30), (1.5, 1.5), DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"]), dict(Ra=1e5, noise=1e-3)),
             ((2, (48, 20), (0.0, 0.0), (0, 0, 1, 1), (0.0, 0.0, 0.5, -0.5), 1),
              dict(Ra=5e4, noise=1e-3, init=INIT_CONDUCTION, seed=3))]
    for args, kw in cases:
        s = rt.Solver(*args, Ra=kw["Ra"], precision=prec, seed=kw.get("seed", 1), noise_amp=kw["noise"],
                      init=kw.get("init", INIT_REST), buoyancy_update_only=1)
        info = s.info
        nu, chi, bg = physics_from_ra(kw["Ra"], 0.71, 0.1, info.L)
        cfg = dict(n=args[1], stretch=args[2], bc=tuple(args[3]) + (0, 0), Tw=tuple(args[4]) + (0.0, 0.0),
                   gravity_axis=args[5], nu=nu, chi=chi, beta_g=bg, dtl=info.dtl, dt=info.dt,
                   deviation=0 if prec == rt.FP64_PLAIN else 1, init=kw.get("init", INIT_REST),
                   seed=kw.get("seed", 1), noise_amp=kw["noise"])
        lit = Oracle(OracleConfig(force_in_predictor=0, **cfg))
        pred = Oracle(OracleConfig(force_in_predictor=1, **cfg))
        s.step(600)
        lit.step(600)
        pred.step(600)
        rel = field_rel(s, lit, 2)
        apart = max(float(np.abs(lit.prim(f) - pred.prim(f)).max() / max(np.abs(pred.prim(f)).max(), 0.1))
                    for f in (1, 2))
        print("update-only force:", args[1], "rel", rel, "placements differ by", apart, flush=True)
        assert apart > 1e-6
        assert max(rel) <= FP64_TOL, rel


@pytest.mark.parametrize("shape,stretch", [((64, 64), (0.0, 0.0)), ((256, 256), (1.5, 1.5))])
def test_fp32_mass_drift_fix_on_cartesian_meshes(shape, stretch):
    """P3 for the FP32 deviation storage on the Cartesian path: with the
    mass-drift correction (every 1,000 steps, the default) the total mass
    stays within 1e-7 of its initial value over 20,000 steps, checked after
    every 2,000; the FP64 integral is formed on the device from the FP32
    fields."""
    s = rt.Solver(2, shape, stretch, DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"], Ra=1e6, precision=rt.FP32_DEV,
                  seed=1, noise_amp=1e-6, mass_fix_every=1000)
    i0 = s.integrals()
    M0 = i0["volume"] + i0["mass_dev"]
    worst = 0.0
    for _ in range(10):
        s.step(2000)
        i = s.integrals()
        worst = max(worst, abs(i["mass_dev"] - i0["mass_dev"]) / M0)
    print("FP32 mass drift", shape, worst, flush=True)
    assert worst <= 1e-7, worst


# ------------------------------------------------------------- 3D --------

DHC3 = dict(kind=(1, 1, 2, 2, 2, 2), Tdev=(-0.5, 0.5, 0, 0, 0, 0), gaxis=2)


@pytest.mark.parametrize("prec", [rt.FP64_PLAIN, rt.FP64_DEV])
def test_fp64_3d_cavity_parity(prec):
    """3D cubic cavity (cold x = 0, hot x = L, gravity +z), stretched mesh,
    ragged tiles in every direction: 120 steps."""
    s, o = make_pair(3, (19, 13, 10), (1.8, 1.8, 1.8), **DHC3, Ra=1e5, precision=prec, noise=1e-3)
    s.step(120)
    o.step(120)
    rel = field_rel(s, o, 3)
    assert max(rel) <= FP64_TOL, rel


@pytest.mark.timeout(300)
def test_fp64_3d_48cube_tanh_parity_200_steps():
    """A 48^3 tanh (phi = 1.8) cubic cavity at Ra = 1e5, 200 steps: twelve
    4x4x4 tiles along each axis, fields within 1e-12 on P14's scale
    max |oracle|.  The oracle needs about a minute."""
    s, o = make_pair(3, (48, 48, 48), (1.8, 1.8, 1.8), **DHC3, Ra=1e5, noise=1e-3)
    s.step(200)
    o.step(200)
    rel = field_rel(s, o, 3, Vc=0.0)
    print("48^3 tanh, 200 steps: rel (P14 scale)", rel, "|u| max",
          max(np.abs(o.prim(f)).max() for f in (1, 2, 3)), flush=True)
    assert max(rel) <= FP64_TOL, rel


def test_fp64_3d_periodic_and_diagnostics():
    s, o = make_pair(3, (12, 10, 9), (0, 0, 0), (0, 0, 1, 1, 2, 2), (0, 0, 0.5, -0.5, 0, 0), 1, Ra=5e4,
                     init=INIT_CONDUCTION, noise=1e-2)
    s.step(100)
    o.step(100)
    rel = field_rel(s, o, 3)
    assert max(rel) <= FP64_TOL, rel
    a, b = s.nusselt(), o.nusselt()
    for k in a:
        assert abs(a[k] - b[k]) <= 1e-11 * abs(b[k]), k


# ------------------------------------------------------------- FP32 ------

def test_fp32_deviation_short_horizon_fields():
    """FP32 deviation storage against the oracle's FP64 deviation form:
    200 steps of a developing Ra = 1e5 cavity; the deviation variables keep
    the FP32 rounding at ~1e-7 of the field scale."""
    s, o = make_pair(2, (48, 48), (1.5, 1.5), **DHC2, Ra=1e5, precision=rt.FP32_DEV, noise=1e-3)
    s.step(200)
    o.step(200)
    rel = field_rel(s, o, 2)
    # rho ~ 1: compare the deviation r instead
    r_gpu, r_orc = s.stored(0), o.stored(0)
    assert np.abs(r_gpu - r_orc).max() <= 1e-5 * np.abs(r_orc).max()
    assert max(rel[1:]) <= 1e-4, rel


def test_fp32_deviation_nusselt_at_steady_state():
    """At steady state (Ra = 1e3, 32^2) the FP32 deviation path reproduces the
    FP64 oracle's Nusselt numbers within 1e-4 relative."""
    s, o = make_pair(2, (32, 32), (0, 0), **DHC2, Ra=1e3, precision=rt.FP32_DEV, noise=1e-6)
    o.step(12000)
    s.step(12000)
    a, b = s.nusselt(), o.nusselt()
    for k in ("hot_avg", "cold_avg", "volume", "hot_max", "cold_max"):
        assert abs(a[k] - b[k]) <= 1e-4 * abs(b[k]), (k, a[k], b[k])


def test_fp32_stochastic_rounding_removes_the_steady_state_bias():
    """Near steady state the FP32 increments fall below half an ulp of the
    stored deviation variables; round-to-nearest then stalls the slow modes
    and biases the converged Nusselt number, while stochastic rounding of the
    update is unbiased.  128^2 tanh cavity at Ra = 1e5 run until the FP64
    residual is below 1e-8: FP32 (stochastic) Nusselt numbers within 1e-4 of
    FP64, and closer than round-to-nearest."""
    args = (2, (128, 128), (1.5, 1.5), DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"])
    kw = dict(Ra=1e5, noise_amp=1e-6, seed=1, residual_every=1000)
    ref = rt.Solver(*args, precision=rt.FP64_PLAIN, **kw)
    n = 0
    while n < 2_000_000:
        ref.step(20000)
        n += 20000
        if max(ref.residual()) < 1e-8:
            break
    assert max(ref.residual()) < 1e-8
    sr = rt.Solver(*args, precision=rt.FP32_DEV, **kw)
    rn = rt.Solver(*args, precision=rt.FP32_DEV, round_nearest=1, **kw)
    sr.step(n)
    rn.step(n)
    a, b, c = ref.nusselt(), sr.nusselt(), rn.nusselt()
    for k in ("hot_avg", "cold_avg", "volume"):
        e_sr = abs(b[k] - a[k]) / abs(a[k])
        e_rn = abs(c[k] - a[k]) / abs(a[k])
        assert e_sr <= 1e-4, (k, e_sr)
        assert e_sr < e_rn, (k, e_sr, e_rn)


# ------------------------------------------------------------------ TLBFS --

@pytest.mark.parametrize("prec", [rt.FP64_PLAIN, rt.FP64_DEV])
@pytest.mark.parametrize("shape,stretch", [((64, 64), (0.0, 0.0)), ((70, 45), (1.5, 1.5))])
def test_tlbfs_fp64_cavity_parity(prec, shape, stretch):
    """The TLBFS interface flux (Sec. 2.2) on the GPU against the oracle's,
    same cavity set-up as the RTLBFS parity runs."""
    s, o = make_pair(2, shape, stretch, Ra=1e5, precision=prec, method=rt.METHOD_TLBFS, **DHC2)
    s.step(300)
    o.step(300)
    rel = field_rel(s, o, 2)
    print("TLBFS", shape, prec, "rel", rel, flush=True)
    assert max(rel) <= TLBFS_TOL, rel


def test_tlbfs_fp64_periodic_rayleigh_benard_and_random_state():
    bc = (0, 0, 1, 1)
    s, o = make_pair(2, (48, 24), (0.0, 0.0), bc, (0.0, 0.0, 0.5, -0.5), 1, Ra=5e4, init=INIT_CONDUCTION,
                     method=rt.METHOD_TLBFS)
    s.step(400)
    o.step(400)
    rel = field_rel(s, o, 2)
    print("TLBFS RB rel", rel, flush=True)
    assert max(rel) <= TLBFS_TOL, rel
    N = 33 * 21
    kind = (1, 2, 2, 1)
    s, o = make_pair(2, (33, 21), (1.5, 0.0), kind, (0.3, 0.0, 0.0, -0.2), 0, Ra=1e4, method=rt.METHOD_TLBFS,
                     precision=rt.FP64_DEV)
    rho, u, T = inputs.random_state(N, 2, seed=11)
    s.set_state(rho, u, T)
    o.set_prim(rho, u, T)
    s.step(50)
    o.step(50)
    rel = field_rel(s, o, 2)
    print("TLBFS random state rel", rel, flush=True)
    assert max(rel) <= TLBFS_TOL, rel


@pytest.mark.parametrize("prec", [rt.FP64_PLAIN, rt.FP64_DEV])
def test_tlbfs_fp64_3d_cavity_parity(prec):
    s, o = make_pair(3, (20, 14, 12), (1.5, 1.5, 1.5), (1, 1, 2, 2, 2, 2), (0.5, -0.5, 0, 0, 0, 0), 2, Ra=1e5,
                     precision=prec, method=rt.METHOD_TLBFS)
    s.step(150)
    o.step(150)
    rel = field_rel(s, o, 3)
    print("TLBFS 3D", prec, "rel", rel, flush=True)
    assert max(rel) <= TLBFS_TOL, rel


def test_tlbfs_two_step_launches_equal_one_step_launches():
    """TLBFS through the two-step launch shapes gives the same bits as through
    the one-step ones (FP32 with stochastic rounding and FP64 deviation)."""
    args = (2, (52, 36), (1.5, 1.5), DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"])
    for prec in (rt.FP32_DEV, rt.FP64_DEV):
        ref = None
        for tile in (2, 6, 7, 9):  # 16x16/1, 16x16/2, 32x8/2, 8x8/2
            s = rt.Solver(*args, Ra=1e5, noise_amp=1e-3, seed=6, tile=tile, precision=prec,
                          method=rt.METHOD_TLBFS, residual_every=30)
            s.step(91)
            st = [s.stored(f) for f in range(4)]
            if ref is None:
                ref = st
            for f in range(4):
                assert np.array_equal(st[f], ref[f]), (prec, tile, f)


def test_tlbfs_fp32_short_horizon_and_tiles():
    """FP32 deviation TLBFS against the FP64 oracle over a short horizon, and
    every tile shape gives the same state."""
    s, o = make_pair(2, (70, 45), (1.5, 1.5), Ra=1e5, precision=rt.FP32_DEV, method=rt.METHOD_TLBFS, **DHC2)
    s.step(500)
    o.step(500)
    assert max(field_rel(s, o, 2)) <= 1e-4
    ref = None
    for tile in range(1, 6):
        t = rt.Solver(2, (70, 45), (1.5, 1.5), DHC2["kind"], DHC2["Tdev"], DHC2["gaxis"], Ra=1e5,
                      precision=rt.FP32_DEV, seed=1, noise_amp=1e-3, tile=tile, method=rt.METHOD_TLBFS)
        t.step(200)
        st = [t.stored(f) for f in range(4)]
        if ref is None:
            ref = st
        for a, b in zip(st, ref):
            assert np.array_equal(a, b)


def test_3d_column_kernels_agree_with_the_tile_kernel_and_the_oracle():
    """The 3D step by marching columns (16x8 and 8x8 columns, segments of 32
    to 96 planes; opts.tile 2..6) against the 4x4x4 tile kernel (opts.tile 1,
    the default) over 60 steps: both methods, FP32 with stochastic rounding
    and both FP64 storages, ragged columns and segments, walls on every side,
    a periodic x axis, and a periodic z axis shorter than one segment.  The
    per-face and per-cell arithmetic is shared, but the two kernels are
    compiled with different multiply-add contractions, which moves the last
    bit of a few cells; after one step the states are identical, after 60
    they agree to 1e-12 of the field scale in FP64 and 1e-6 in FP32.  In
    FP64 the columns also match the oracle to 1e-12."""
    cases = [((3, (37, 21, 70), (1.8, 1.8, 1.8), (1, 1, 2, 2, 2, 2), (-0.5, 0.5, 0, 0, 0, 0), 2), dict(Ra=1e5)),
             ((3, (24, 11, 9), (0.0, 0.0, 0.0), (0, 0, 1, 1, 2, 2), (0, 0, 0.5, -0.5, 0, 0), 1),
              dict(Ra=5e4, init=INIT_CONDUCTION)),
             ((3, (18, 13, 5), (0.0, 1.5, 0.0), (1, 1, 2, 2, 0, 0), (0.5, -0.5, 0, 0, 0, 0), 1), dict(Ra=2e4))]
    for args, kw in cases:
        for prec in (rt.FP32_DEV, rt.FP64_PLAIN, rt.FP64_DEV):
            for method in (rt.METHOD_RTLBFS, rt.METHOD_TLBFS):
                tol = 1e-6 if prec == rt.FP32_DEV else 1e-12
                for steps in (1, 60):
                    ref = None
                    for tile in range(1, 7):
                        s = rt.Solver(*args, noise_amp=1e-3, seed=7, tile=tile, precision=prec, method=method,
                                      residual_every=25, **kw)
                        s.step(steps)
                        st = [s.stored(f) for f in range(5)]
                        if ref is None:
                            ref = st
                            assert (s.info.tile_x, s.info.tile_y, s.info.tile_z) == (4, 4, 4)
                            continue
                        for f in range(5):
                            if steps == 1:
                                assert np.array_equal(st[f], ref[f]), (args[1], prec, method, tile, f)
                            scale = max(float(np.abs(ref[f]).max()), 1e-3 if f == 0 else 1e-2)
                            assert np.abs(st[f] - ref[f]).max() <= tol * scale, (args[1], prec, method, tile, f)
    for tile in (3, 6):
        s, o = make_pair(3, (19, 13, 10), (1.8, 1.8, 1.8), **DHC3, Ra=1e5, noise=1e-3, tile=tile)
        s.step(120)
        o.step(120)
        rel = field_rel(s, o, 3)
        assert max(rel) <= FP64_TOL, (tile, rel)
