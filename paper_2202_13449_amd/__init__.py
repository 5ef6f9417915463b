"""MI355X (gfx950) implementation of the RTLBFS time step (arXiv 2202.13449).

The compute path is the HIP library librtlbfs.so (C ABI in include/rtlbfs.h);
`rtlbfs` is its thin ctypes binding.
"""
from .rtlbfs import (  # noqa: F401
    EDIVERGED, EINVAL, EUNSUPPORTED, FARFIELD, FP32_DEV, FP64_DEV, FP64_PLAIN, INIT_CONDUCTION, INIT_REST,
    METHOD_RTLBFS, METHOD_TLBFS, OK, PERIODIC,
    WALL_ADIABATIC, WALL_ISOTHERMAL, Batch, Curv3Solver, CurvSolver, RtlbfsError, Solver, load_library, make_bc, make_mesh,
    make_opts,
    mesh_nodes, residual_states, strerror)
