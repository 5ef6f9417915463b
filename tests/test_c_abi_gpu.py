"""The C ABI used from plain C: tests/abi_c/abi_check (built by build() with
gcc against include/rtlbfs.h and librtlbfs.so) runs a cavity with a
library-owned workspace on the null stream, a two-member batch, a 2D
body-fitted O-mesh annulus (heated wall, far field, buoyancy) and a 3D
annulus wedge closed by a rotation, in a process without torch or Python.
Its results must equal the binding's runs of the same problems bit for bit
(the meshes are read back from the files the program wrote)."""
import json
import os
import subprocess

import numpy as np
import pytest

import paper_2202_13449_amd as rt

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(__file__), "abi_c", "abi_check")


def test_plain_c_program_matches_the_binding(tmp_path):
    if not os.path.exists(EXE):
        pytest.skip("tests/abi_c/abi_check is not built (run build())")
    n, Ra, steps = 48, 1e4, 500
    out_T = str(tmp_path / "T.bin")
    r = subprocess.run([EXE, str(n), repr(Ra), str(steps), out_T], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    res = json.loads(r.stdout.strip().splitlines()[-1])
    T_c = np.fromfile(out_T, dtype=np.float64)

    s = rt.Solver(2, (n, n), (0.0, 0.0), (1, 1, 2, 2), (0.5, -0.5, 0.0, 0.0), 1, Ra=Ra, Pr=0.71, Ma=0.1,
                  seed=1, noise_amp=1e-6)
    s.step(steps)
    assert np.array_equal(s.field(3), T_c)
    nu = s.nusselt()
    assert abs(nu["hot_avg"] - res["nu_hot"]) <= 1e-13 * abs(nu["hot_avg"])
    assert abs(nu["volume"] - res["nu_volume"]) <= 1e-13 * abs(nu["volume"])
    assert np.allclose(s.residual(), (res["res_u"], res["res_T"]), rtol=1e-13, atol=0)
    assert res["bad_field_rc"] == rt.EINVAL
    assert res["batch_diverged"] == [0, 0]
    assert res["batch_nu_hot0"] > 1.0
    assert res["curv_nusselt_rc"] == rt.EUNSUPPORTED

    base = out_T
    ni, nj = 36, 14
    cx = np.fromfile(base + ".cx").reshape(nj + 1, ni + 1)
    cy = np.fromfile(base + ".cy").reshape(nj + 1, ni + 1)
    c = rt.CurvSolver(cx, cy, (rt.PERIODIC, rt.PERIODIC, rt.WALL_ISOTHERMAL, rt.FARFIELD), Tw=(0, 0, 1.0, 0),
                      up=(0.0, 1.0), T_ref=0.0, u_inf=(0.0, 0.04), T_inf=0.0, nu=0.08, chi=0.11, beta_g=4e-5, dt=0.5)
    c.step(steps)
    assert list(c.wall_heat(2)) == res["curv_wall_heat"]

    nr, nz = 8, 10
    x3, y3, z3 = (np.fromfile(base + e).reshape(nz + 1, 2, nr + 1) for e in (".c3x", ".c3y", ".c3z"))
    w = rt.Curv3Solver(x3, y3, z3, (rt.WALL_ISOTHERMAL, rt.WALL_ISOTHERMAL, rt.PERIODIC, rt.PERIODIC,
                                    rt.WALL_ADIABATIC, rt.WALL_ADIABATIC), rot=(0.0, 0.1, 0.0),
                       Tw=(1.0, 0, 0, 0, 0, 0), up=(0.0, 0.0, 1.0), T_ref=0.5, nu=0.06, chi=0.08, beta_g=5e-4, dt=0.5)
    w.step(steps)
    assert list(w.wall_heat(0)) == res["curv3_wall_heat"]
