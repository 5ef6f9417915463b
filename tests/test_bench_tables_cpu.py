"""Host-side helpers of the high-Ra cavity workload (Sec. 4.2, Tables 2-3):
the Eq. 74 stretching solved for the printed first-cell size, the parabolic
peak refinement, and the table quantities of a pure-conduction state, whose
mid-plane Nusselt number is 1 exactly and whose streamfunction and
velocities vanish."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import paper_2202_13449_amd as rt  # noqa: E402


@pytest.mark.parametrize("Ra", sorted(bench.TABLES_2_3))
def test_stretch_gives_the_printed_first_cell(Ra):
    case = bench.TABLES_2_3[Ra]
    phi = bench.stretch_for_first_cell(rt, case["n"], case["first_over_L"])
    x, L = rt.mesh_nodes(case["n"], phi)
    assert abs((x[1] - x[0]) / L - case["first_over_L"]) < 1e-12
    assert abs(x[-1] - L) < 1e-9 * L


def test_peak_of_a_parabola_on_an_uneven_grid():
    xs = np.cumsum(np.r_[0.0, np.random.default_rng(5).uniform(0.05, 0.2, 15)])
    ys = 3.0 - 2.0 * (xs - 0.8137) ** 2
    pos, val = bench._peak(xs, ys)
    assert abs(val - 3.0) < 1e-12 and abs(pos - 0.8137) < 1e-12


def test_conduction_state_has_unit_midplane_nusselt():
    n = 300
    phi = bench.stretch_for_first_cell(rt, n, 4e-4)
    x, L = rt.mesh_nodes(n, phi)
    xc = 0.5 * (x[:-1] + x[1:])

    class Fake:
        class info:
            chi = 0.0666

        fields = [np.ones(n * n), np.zeros(n * n), np.zeros(n * n), np.tile(1.0 - xc / L, n)]

        def field(self, f):
            return self.fields[f]

        def grid(self, v):
            return v.reshape(n, n)

    q = bench.table23_quantities(rt, Fake(), n, phi)
    assert abs(q["nu_half"] - 1.0) < 1e-12
    assert q["psi_max"] == 0.0 and q["u_max"] == 0.0 and q["v_max"] == 0.0
