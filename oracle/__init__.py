"""Plain FP64 CPU oracle of the RTLBFS time step, with the TLBFS face flux as an
alternative (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
import this package.  It shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    INIT_CONDUCTION, INIT_REST, PERIODIC, RTLBFS, TLBFS, WALL_ADIABATIC, WALL_ISOTHERMAL, Oracle, OracleConfig,
    face_flux, face_flux_frame,
    mesh_nodes, physics_from_ra, splitmix_uniform)
from .curvilinear import FARFIELD, Curv3Config, Curv3Oracle, CurvConfig, CurvOracle  # noqa: F401,E402
