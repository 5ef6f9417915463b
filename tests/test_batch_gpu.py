"""Batched stepping: members of one batch (one kernel launch per step over
all members' tiles) against single-domain solvers and the oracle."""
import numpy as np
import pytest

import paper_2202_13449_amd as rt
from oracle import Oracle, OracleConfig, physics_from_ra

pytestmark = pytest.mark.gpu

KIND = (1, 1, 2, 2)
TDEV = (0.5, -0.5, 0.0, 0.0)
MEMBERS = [  # (n, stretch, Ra, Pr): uneven sizes, ragged tiles, both mesh kinds
    ((64, 64), (0.0, 0.0), 1e3, 0.71),
    ((40, 24), (1.5, 1.5), 1e5, 7.0),
    ((128, 96), (1.5, 0.0), 3e6, 0.71),
    ((33, 9), (0.0, 0.0), 2e4, 0.71),
]


def make_batch(precision, members=MEMBERS, **kw):
    meshes = [rt.make_mesh(2, n, st) for n, st, _, _ in members]
    bcs = [rt.make_bc(KIND, TDEV, 1) for _ in members]
    return rt.Batch(meshes, [m[2] for m in members], [m[3] for m in members], bcs, Ma=0.1, precision=precision,
                    seed=5, noise_amp=1e-3, **kw)


def single(member, precision, **kw):
    n, st, Ra, Pr = member
    return rt.Solver(2, n, st, KIND, TDEV, 1, Ra=Ra, Pr=Pr, Ma=0.1, precision=precision, seed=5, noise_amp=1e-3,
                     tile=4, **kw)  # 16x8, the batch tile


@pytest.mark.parametrize("precision", [rt.FP64_PLAIN, rt.FP32_DEV])
def test_batch_members_equal_single_domain_runs(precision):
    """Each member of the batch is bit-identical to a single-domain solver of
    the same problem (same 16x8 tile arithmetic, own Delta-t and parameters),
    including the residual, the Nusselt numbers and the FP32 mass fix."""
    b = make_batch(precision, residual_every=50, mass_fix_every=100)
    b.step(350)
    for k, m in enumerate(MEMBERS):
        s = single(m, precision, residual_every=50, mass_fix_every=100)
        s.step(350)
        for f in range(4):
            assert np.array_equal(b.field(k, f), s.field(f)), (k, f)
        assert b.residual(k) == s.residual()
        nb, ns = b.nusselt(k), s.nusselt()
        for key in nb:
            assert nb[key] == ns[key], (k, key)
        ib, isg = b.info(k), s.info
        assert ib.dt == isg.dt and ib.nu == isg.nu and ib.cells == isg.cells


def test_batch_member_matches_oracle():
    b = make_batch(rt.FP64_PLAIN)
    b.step(300)
    n, st, Ra, Pr = MEMBERS[1]
    info = b.info(1)
    nu, chi, bg = physics_from_ra(Ra, Pr, 0.1, info.L)
    o = Oracle(OracleConfig(n=n, stretch=st, bc=KIND + (0, 0), Tw=TDEV + (0, 0), gravity_axis=1, nu=nu, chi=chi,
                            beta_g=bg, dtl=info.dtl, dt=info.dt, seed=5, noise_amp=1e-3))
    o.step(300)
    for f in range(4):
        a, c = b.field(1, f), o.prim(f)
        scale = max(np.abs(c).max(), 0.1 if f in (1, 2) else 0.0)
        assert np.abs(a - c).max() <= 1e-12 * scale, f


def test_batch_graph_replay_equals_direct_launches():
    a = make_batch(rt.FP32_DEV, residual_every=20, graph_steps=0)
    c = make_batch(rt.FP32_DEV, residual_every=20, graph_steps=-1)
    a.step(130)
    c.step(130)
    for k in range(len(MEMBERS)):
        for f in range(4):
            assert np.array_equal(a.field(k, f), c.field(k, f))


def test_batch_with_a_512_tanh_member_equals_single_handles():
    """A 512^2 tanh (phi = 1.5) cavity at Ra = 1e6, the largest member size
    of the 256-cavity workload, batched with a small uniform one: both equal
    their single-domain runs bit for bit (FP32 with stochastic rounding and
    the mass fix, and FP64)."""
    members = [((512, 512), (1.5, 1.5), 1e6, 0.71), ((64, 64), (0.0, 0.0), 1e4, 7.0)]
    for precision in (rt.FP32_DEV, rt.FP64_PLAIN):
        b = make_batch(precision, members=members, residual_every=40, mass_fix_every=100)
        b.step(230)
        for k, m in enumerate(members):
            s = single(m, precision, residual_every=40, mass_fix_every=100)
            s.step(230)
            for f in range(4):
                assert np.array_equal(b.field(k, f), s.field(f)), (precision, k, f)
            assert b.residual(k) == s.residual()


@pytest.mark.timeout(600)
def test_full_256_cavity_work_list_equals_single_handles():
    """The benchmarked batch itself: the 256 seeded cavities (side 64 to 512,
    Ra 1e3 to 1e7, Pr 0.71 or 7, uniform or tanh; about 2.3e7 cells) in one
    launch per step, FP32 deviation storage.  After 30 steps every member
    equals its own single-domain run bit for bit, and the largest member
    (512^2) matches the FP64 oracle cell by cell on each field's own scale
    (1e-5; FP32 storage with stochastic rounding)."""
    from paper_2202_13449_amd.workloads import batch_cavities, total_cells

    wl = batch_cavities(256, seed=4)
    members = [((m["n"], m["n"]), (m["stretch"], m["stretch"]), m["Ra"], m["Pr"]) for m in wl]
    b = make_batch(rt.FP32_DEV, members=members, residual_every=10)
    print("C4 work list:", len(members), "members,", total_cells(wl), "cells", flush=True)
    b.step(30)
    for k, m in enumerate(members):
        s = single(m, rt.FP32_DEV, residual_every=10)
        s.step(30)
        for f in range(4):
            assert np.array_equal(b.field(k, f), s.field(f)), (k, m, f)
        s.close()
    # The largest member (a 512^2 cavity) against the FP64 oracle, cell by cell.
    k = max(range(len(members)), key=lambda j: members[j][0][0] * members[j][0][1])
    n, st, Ra, Pr = members[k]
    info = b.info(k)
    nu, chi, bg = physics_from_ra(Ra, Pr, 0.1, info.L)
    o = Oracle(OracleConfig(n=n, stretch=st, bc=KIND + (0, 0), Tw=TDEV + (0, 0), gravity_axis=1, nu=nu, chi=chi,
                            beta_g=bg, dtl=info.dtl, dt=info.dt, deviation=1, seed=5, noise_amp=1e-3))
    o.step(30)
    own = [float(np.abs(b.field(k, f) - o.prim(f)).max() / np.abs(o.prim(f)).max()) for f in range(4)]
    print("C4 largest member", members[k], "FP32 vs oracle, own scale:", own, flush=True)
    assert max(own) <= 1e-5, own
