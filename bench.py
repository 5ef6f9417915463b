"""Throughput of the RTLBFS time step on one MI355X.

Headline workload: 2D differentially heated cavity, 256 x 256 tanh-stretched
mesh (phi = 1.5 on both axes, finest cell = 1), Ra = 1e6, Pr = 0.71,
V_c = 0.1, hot / cold isothermal side walls, adiabatic top / bottom, fluid
at rest with seeded 1e-6 temperature noise.  One step is one full RTLBFS
time step (face lattice predictor, fluxes, divergence, update) with its FP64
reductions at their cadence (Eq. 65 residual every 100 steps, mass-drift
correction every 1000 steps), replayed from captured HIP graphs.  `value` is
the FP32 deviation-storage path over exactly `steps` timed steps; the FP64
plain path is timed beside it.  Inputs are resident in HBM before each timed
region starts.

The same JSON line carries
- `roofline`: the dominant kernel's algorithmic rate against the FP32
  vector peak, its HBM fraction and, while the kernel is unchanged, the
  HBM traffic the counters measured;
- `fixed_nu_error`: FP64 run to steady state (both Eq. 65 ratios below
  1e-8), FP32 run for the same steps, the relative Nusselt differences;
- `legs`: the 256-cavity batch (FP32 and FP64 batches and the 256
  problems as separate handles) and the 192^3 cube (FP32 and FP64), each
  with its HBM and ALU fractions and counter traffic ratio;
- `cpu_baseline`: the FP64 oracle timed on a bounded sample.

Other workloads are selected with --workload / --batch.
"""
import argparse
import math
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_CELLS_SIDE = 256
STRETCH = 1.5
RA, PR, MA = 1e6, 0.71, 0.1
KIND = (1, 1, 2, 2)           # isothermal x walls, adiabatic y walls
TDEV = (0.5, -0.5, 0.0, 0.0)  # hot at x = 0
GAXIS = 1
BYTES_PER_CELL = {"f32": 4 * 4 * 2, "f64": 4 * 8 * 2}  # read + write of the 4 stored fields
HBM_PEAK_GBS = 8000.0
# Published MI355X vector peaks.  FP32 157.3 TFLOP/s = 256 CU x 4 SIMD x 16
# lanes x 2 (FMA) x 2 (packed FP32) x 2.4 GHz; without packed FP32
# instructions (which the build disables) the FP32 ceiling is half, 78.6.
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_NONPACKED_PEAK_TFLOPS = 78.6
FP64_VECTOR_PEAK_TFLOPS = 78.6
# Algorithmic flops per cell-update: the operation count of one time step of
# the method in the paper's plain FP64 nodal form (the differences of Eqs.
# 46-48 taken node by node, as the oracle does), counted on the library's
# face_flux_nodes with a counting number type (tests/test_flops_cpu.py): 2D,
# two faces of 407 + Eq. 55 gradients 64 (4 primitives x 2 axes x 8) +
# primitives 4 + area weighting 8 + update and buoyancy 23 = 913; 3D, three
# faces of 840 + gradients 120 + primitives, weighting and update about 30 =
# 2670.  The deviation storage adds 21 per 2D face (31 in 3D) and the FP32
# stochastic rounding 6 per stored field; both are implementation overhead
# and are not counted.
ALG_FLOPS_PER_CELL = {2: 2 * 407 + 64 + 4 + 8 + 23, 3: 3 * 840 + 120 + 30}
# What the kernels execute per cell-update on owned faces with the column form
# of the face flux (face_flux: 313 / 299 per 2D face, 542 / 528 per 3D face,
# deviation / plain), reported beside the algorithmic figure.
EXEC_FLOPS_PER_CELL = {(2, "f32"): 2 * 313 + 64 + 5 + 8 + 23 + 24, (2, "f64"): 2 * 299 + 64 + 4 + 8 + 23,
                       (3, "f32"): 3 * 542 + 150, (3, "f64"): 3 * 528 + 150}
BYTES_PER_CELL_3D = {"f32": 5 * 4 * 2, "f64": 5 * 8 * 2}
CSRC = os.path.join(ROOT, "paper_2202_13449_amd", "csrc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_k_step2d_fp32_cavity256.json")
TRAFFIC_FILE_BATCH = os.path.join(ROOT, "profiles", "traffic_k_batch_step2d_256cavities.json")
TRAFFIC_FILE_3D = os.path.join(ROOT, "profiles", "traffic_k_step3d_cube192.json")
TRAFFIC_FILE_PROXY = os.path.join(ROOT, "profiles", "traffic_k_step2d_fp32_proxy4788.json")


def sources_sha256(headers, api_file, kernel) -> str:
    """Hash of what defines one step kernel (its device headers, its
    __global__ wrapper in `api_file` and the compile flags of build.py), so
    stored counter data is used only while that kernel is unchanged."""
    import hashlib
    import re

    h = hashlib.sha256()
    for name in headers:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(CSRC, api_file)) as f:
        api = f.read()
    m = re.search(r"template <[^\n]*>\n__global__[^\n]*" + kernel + r"\(.*?\n}\n", api, re.S)
    if not m:
        raise RuntimeError(f"{kernel} wrapper not found in {api_file}")
    h.update(kernel.encode() + b"\0" + m.group(0).encode())
    with open(os.path.join(ROOT, "paper_2202_13449_amd", "build.py")) as f:
        build = f.read()
    fm = re.search(r"flags = \[.*?\]", build, re.S)  # the code-generation flags, not the file lists
    if not fm:
        raise RuntimeError("compile flags not found in build.py")
    h.update(b"build flags\0" + fm.group(0).encode())
    return h.hexdigest()


def kernel_sources_sha256() -> str:
    return sources_sha256(("rtlbfs_device.h", "step2d.h"), "rtlbfs_api.hip", "k_step2d")


def batch_sources_sha256() -> str:
    return sources_sha256(("rtlbfs_device.h", "step2d.h"), "rtlbfs_batch.hip", "k_batch_step2d")


def cube_sources_sha256() -> str:
    return sources_sha256(("rtlbfs_device.h", "step3d.h"), "rtlbfs_api.hip", "k_step3d")


def stored_traffic(path, sha, key):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, each scaled by its
    copy-kernel calibration) from a committed counter summary; None when the
    kernel changed since the counters were taken or no entry exists."""
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256") != sha:
        return None
    return t.get("bytes_per_launch_by_tile", {}).get(key)


def measured_traffic(tile):
    """Traffic of the 2D step kernel in launch shape `tile` (tile x, tile y,
    steps per launch)."""
    key = f"{tile[0]}x{tile[1]}" + ("" if tile[2] == 1 else f"/{tile[2]}")
    return stored_traffic(TRAFFIC_FILE, kernel_sources_sha256(), key)


# opts.tile of each 2D launch shape (tile x, tile y, steps per launch)
TILES_2D = {(32, 8, 1): 1, (16, 16, 1): 2, (64, 4, 1): 3, (16, 8, 1): 4, (8, 8, 1): 5,
            (16, 16, 2): 6, (32, 8, 2): 7, (16, 8, 2): 8, (8, 8, 2): 9}


def launch_shape(info):
    return (info.tile_x, info.tile_y, info.steps_per_launch)


def make_solver(rt, precision, residual_every=100, mass_fix_every=1000, tile=0):
    return rt.Solver(2, (N_CELLS_SIDE, N_CELLS_SIDE), (STRETCH, STRETCH), KIND, TDEV, GAXIS, Ra=RA, Pr=PR, Ma=MA,
                     precision=precision, seed=1, noise_amp=1e-6, residual_every=residual_every,
                     mass_fix_every=mass_fix_every, tile=tile)


KERNEL_CHUNK = 2000


def time_step_kernel(rt, torch, precision, steps, warmup, tile):
    """Average duration of one step-kernel launch: the same workload and tile
    with the reductions moved out of the way (Eq. 65 residual on one step in
    KERNEL_CHUNK, no mass fix), timed with events on the solver's stream."""
    s = make_solver(rt, precision, residual_every=KERNEL_CHUNK, mass_fix_every=-1, tile=tile)
    s.step(max(warmup, KERNEL_CHUNK))
    s.sync()
    steps = max(KERNEL_CHUNK, steps - steps % KERNEL_CHUNK)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    s.sync()
    return e0.elapsed_time(e1) / steps, list(launch_shape(s.info))


def time_path(rt, torch, precision, steps, warmup):
    s = make_solver(rt, precision)
    s.step(warmup)
    s.sync()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    s.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    s.sync()  # raises on divergence
    ms = e0.elapsed_time(e1)
    nu = s.nusselt()
    res = s.residual()
    return dict(solver=s, event_ms=ms, wall_s=wall, nu=nu, res=res)


def field_comparison(s32, s64):
    """Both runs after the same number of steps: velocity maxima (u on the
    vertical mid-line x = L/2, v on the horizontal mid-line y = L/2, as in
    Table 1, scaled by L/chi) and the relative L2 error of the FP32 velocity
    and temperature fields against FP64."""
    n = N_CELLS_SIDE
    h = n // 2
    L, chi = s64.info.L, s64.info.chi
    out = {}
    for name, s in (("fp32", s32), ("fp64", s64)):
        u = s.field(1).reshape(n, n)
        v = s.field(2).reshape(n, n)
        out[name] = {"u_max_L_over_chi": float(0.5 * (u[:, h - 1] + u[:, h]).max() * L / chi),
                     "v_max_L_over_chi": float(0.5 * (v[h - 1, :] + v[h, :]).max() * L / chi)}
    vel32 = np.stack([s32.field(1), s32.field(2)])
    vel64 = np.stack([s64.field(1), s64.field(2)])
    T32, T64 = s32.field(3), s64.field(3)
    out["rel_l2_velocity"] = float(np.linalg.norm(vel32 - vel64) / np.linalg.norm(vel64))
    out["rel_l2_temperature"] = float(np.linalg.norm(T32 - T64) / np.linalg.norm(T64))
    return out


def batch_bench(rt, torch, steps, warmup, sequential=True):
    """256 seeded cavities (sides 64..512, Ra 1e3..1e7, Pr 0.71/7, uniform or
    tanh): the batched handle (one launch per step over all members) against
    the same 256 problems stepped as separate single-domain handles."""
    from paper_2202_13449_amd.workloads import (CAVITY_GRAVITY, CAVITY_KIND, CAVITY_TDEV, batch_cavities,
                                                total_cells)

    members = batch_cavities()
    cells = total_cells(members)
    meshes = [rt.make_mesh(2, (m["n"], m["n"]), (m["stretch"], m["stretch"])) for m in members]
    bcs = [rt.make_bc(CAVITY_KIND, CAVITY_TDEV, CAVITY_GRAVITY) for _ in members]
    b = rt.Batch(meshes, [m["Ra"] for m in members], [m["Pr"] for m in members], bcs, Ma=MA,
                 precision=rt.FP32_DEV, seed=4, noise_amp=1e-6, residual_every=100, mass_fix_every=1000)
    stream = torch.cuda.current_stream()
    b.step(warmup)
    b.sync()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    b.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    b.sync()
    ms_batch = e0.elapsed_time(e1) / steps
    nu32 = [b.nusselt(k)["hot_avg"] for k in range(len(members))]
    del b
    torch.cuda.empty_cache()
    # the same batch in FP64 plain storage for the same number of steps: the
    # FP32 members' wall Nusselt numbers against FP64
    b64 = rt.Batch(meshes, [m["Ra"] for m in members], [m["Pr"] for m in members], bcs, Ma=MA,
                   precision=rt.FP64_PLAIN, seed=4, noise_amp=1e-6, residual_every=100)
    b64.step(warmup + steps)
    nu64 = [b64.nusselt(k)["hot_avg"] for k in range(len(members))]
    del b64
    torch.cuda.empty_cache()
    nu_err = [abs(a - c) / abs(c) for a, c in zip(nu32, nu64)]
    bpl = BYTES_PER_CELL["f32"] * cells
    out = {"metric": "cell-updates/s", "workload": "256 batched 2D cavities (seed 4), FP32 deviation",
           "cells": cells, "steps": steps, "warmup": warmup,
           "batched": {"ms_per_step": ms_batch, "value": cells / (ms_batch * 1e-3),
                       "hbm_gbs": bpl / (ms_batch * 1e-3) / 1e9,
                       "frac": bpl / (ms_batch * 1e-3) / 1e9 / HBM_PEAK_GBS},
           "nu_hot_rel_diff_fp32_vs_fp64": {"max": max(nu_err), "median": float(np.median(nu_err)),
                                            "members_above_1e-4": int(sum(e > 1e-4 for e in nu_err)),
                                            "steps": warmup + steps}}
    if not sequential:
        return out
    singles = [rt.Solver(2, (m["n"], m["n"]), (m["stretch"], m["stretch"]), CAVITY_KIND, CAVITY_TDEV,
                         CAVITY_GRAVITY, Ra=m["Ra"], Pr=m["Pr"], Ma=MA, precision=rt.FP32_DEV, seed=4,
                         noise_amp=1e-6, residual_every=100, mass_fix_every=1000) for m in members]
    seq_steps = max(100, steps // 10)
    for s in singles:
        s.step(100)
    torch.cuda.synchronize()
    e0.record(stream)
    for s in singles:
        s.step(seq_steps)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1) / seq_steps
    out["sequential_256_handles"] = {"ms_per_step": ms_seq, "value": cells / (ms_seq * 1e-3), "steps": seq_steps}
    out["speedup_batched_vs_sequential"] = ms_seq / ms_batch
    return out


def batch_steady_bench(rt, torch, steps, warmup, total=200_000, chunk=10_000, tol=1e-8):
    """The fixed-Nu-error check of the 256-cavity batch: FP64 plain and FP32
    deviation batches advanced together in chunks to `total` steps; members
    whose FP64 Eq. 65 ratios are both below `tol` are steady, and for them
    the FP32 Nusselt numbers are compared with FP64.  Progress goes to
    stderr after every chunk."""
    from paper_2202_13449_amd.workloads import (CAVITY_GRAVITY, CAVITY_KIND, CAVITY_TDEV, batch_cavities,
                                                total_cells)

    members = batch_cavities()
    meshes = [rt.make_mesh(2, (m["n"], m["n"]), (m["stretch"], m["stretch"])) for m in members]
    bcs = [rt.make_bc(CAVITY_KIND, CAVITY_TDEV, CAVITY_GRAVITY) for _ in members]
    kw = dict(Ma=MA, seed=4, noise_amp=1e-6, residual_every=1000)
    b64 = rt.Batch(meshes, [m["Ra"] for m in members], [m["Pr"] for m in members], bcs, precision=rt.FP64_PLAIN,
                   **kw)
    b32 = rt.Batch(meshes, [m["Ra"] for m in members], [m["Pr"] for m in members], bcs, precision=rt.FP32_DEV,
                   mass_fix_every=1000, **kw)
    done = 0
    t0 = time.perf_counter()
    while done < total:
        b64.step(chunk)
        b32.step(chunk)
        for b in (b64, b32):
            try:
                b.sync()
            except rt.RtlbfsError as e:  # a diverged member does not stop the others
                if e.code != rt.EDIVERGED:
                    raise
        done += chunk
        res = b64.residuals()
        print(f"batch steady: {done} steps, {int((res.max(axis=1) < tol).sum())} of {len(members)} FP64 members "
              f"below {tol:g}, {time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    res64 = b64.residuals()
    div = b64.diverged() | b32.diverged()
    steady = [k for k in range(len(members)) if not div[k] and max(res64[k]) < tol]
    rows = []
    for k in steady:
        a, c = b32.nusselt(k), b64.nusselt(k)
        rows.append({"member": k, "n": members[k]["n"], "stretch": members[k]["stretch"], "Ra": members[k]["Ra"],
                     "Pr": members[k]["Pr"], "nu_fp64": c, "fp64_residual": list(res64[k]),
                     "nu_rel_diff": {q: abs(a[q] - c[q]) / abs(c[q]) for q in c}})
    worst = max((max(r["nu_rel_diff"].values()) for r in rows), default=None)
    return {"workload": "256 batched cavities, FP32 vs FP64 at steady state", "cells": total_cells(members),
            "steps": done, "tol": tol, "steady_members": len(steady), "members": len(members),
            "diverged_members": [int(k) for k in np.nonzero(div)[0]],
            "max_nu_rel_diff_steady": worst,
            "members_above_1e-4": int(sum(max(r["nu_rel_diff"].values()) > 1e-4 for r in rows)),
            "rows": rows, "seconds": time.perf_counter() - t0}


def timed(torch, solver, steps):
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    solver.step(steps)
    e1.record(stream)
    torch.cuda.synchronize()
    solver.sync()
    return e0.elapsed_time(e1) / steps


# C3: the stability test is 200,000 steps; the run then continues so the
# time averages have a stated statistical error.  Samples every 100 steps
# resolve the box's acoustic period (2 H / c_s, about 3,500 steps for
# H = 512, and its harmonics), which sampling every 1,000 steps aliased.
RB_PASS_STEPS, RB_TOTAL_STEPS, RB_AVG_STEPS, RB_SAMPLE_EVERY, RB_BLOCKS = 200_000, 1_200_000, 1_000_000, 100, 20


def batch_means(x, blocks):
    """Mean and its standard error from `blocks` contiguous block means (the
    blocks are long against the correlation time of the samples)."""
    x = np.asarray(x, dtype=np.float64)
    m = len(x) // blocks
    bm = x[:m * blocks].reshape(blocks, m).mean(axis=1)
    return float(bm.mean()), float(bm.std(ddof=1) / math.sqrt(blocks))


def rb_bench(rt, torch, steps, warmup):
    """1024 x 512 Rayleigh-Benard box, periodic in x, Ra = 1e8 on H = 512,
    conduction profile plus 1e-3 seeded noise, FP32 deviation storage: the
    throughput over `steps`; the stability criterion at 200,000 steps
    (finite, max |u| < 0.3); then the run continued to 1.2M steps with the
    wall and volume (Eq. 69 along the vertical) Nusselt numbers sampled
    every 100 steps over the last 1M, as means with batch-means standard
    errors."""
    s = rt.Solver(2, (1024, 512), (0, 0), (0, 0, 1, 1), (0, 0, 0.5, -0.5), 1, Ra=1e8, Pr=0.71, Ma=MA,
                  precision=rt.FP32_DEV, init=rt.INIT_CONDUCTION, seed=3, noise_amp=1e-3)
    s.step(warmup)
    ms = timed(torch, s, steps)
    done = warmup + steps
    s.step(RB_PASS_STEPS - done)
    done = RB_PASS_STEPS
    s.sync()
    u, v = s.field(1), s.field(2)
    umax = float(np.sqrt(u * u + v * v).max())
    keys = ("hot_avg", "cold_avg", "volume")
    samples = {k: [] for k in keys}
    t0 = time.perf_counter()
    while done < RB_TOTAL_STEPS:
        s.step(RB_SAMPLE_EVERY)
        done += RB_SAMPLE_EVERY
        if done > RB_TOTAL_STEPS - RB_AVG_STEPS:
            nu = s.nusselt()
            for k in keys:
                samples[k].append(nu[k])
    s.sync()
    u2, v2 = s.field(1), s.field(2)
    stats = {}
    for k in keys:
        m, se = batch_means(samples[k], RB_BLOCKS)
        stats[k] = {"mean": m, "stderr": se, "std": float(np.std(samples[k]))}
    cells = 1024 * 512
    return {"workload": "rb1024x512 Ra=1e8 FP32", "cells": cells, "steps_timed": steps, "ms_per_step": ms,
            "value": cells / (ms * 1e-3), "hbm_gbs": BYTES_PER_CELL["f32"] * cells / (ms * 1e-3) / 1e9,
            "pass_steps": RB_PASS_STEPS, "finite": bool(np.isfinite(umax)), "umax": umax,
            "pass": bool(np.isfinite(umax) and umax < 0.3),
            "total_steps": done, "umax_end": float(np.sqrt(u2 * u2 + v2 * v2).max()),
            "nu_time_avg": stats, "nu_samples": len(samples["volume"]), "sample_every": RB_SAMPLE_EVERY,
            "avg_window_steps": RB_AVG_STEPS, "batch_means_blocks": RB_BLOCKS,
            "seconds_sampling": time.perf_counter() - t0, "tile": list(launch_shape(s.info))}


TILE = 0  # --tile: opts.tile of the cube192 and proxy2d workloads (0: the library's default)


def cube_bench(rt, torch, steps, warmup):
    """192^3 tanh (phi = 1.8) cubic cavity, Ra = 1e6: FP32 deviation and FP64
    plain throughput (launch shape --tile)."""
    out = {"workload": "cube192 tanh1.8 Ra=1e6", "cells": 192 ** 3, "tile": TILE}
    for name, prec, bpc in (("fp32_dev", rt.FP32_DEV, 40), ("fp64_plain", rt.FP64_PLAIN, 80)):
        s = rt.Solver(3, (192, 192, 192), (1.8, 1.8, 1.8), (1, 1, 2, 2, 2, 2), (-0.5, 0.5, 0, 0, 0, 0), 2, Ra=1e6,
                      Pr=0.71, Ma=MA, precision=prec, seed=1, noise_amp=1e-6, tile=TILE)
        s.step(warmup)
        ms = timed(torch, s, steps)
        out[name] = {"ms_per_step": ms, "value": 192 ** 3 / (ms * 1e-3),
                     "hbm_gbs": bpc * 192 ** 3 / (ms * 1e-3) / 1e9, "nu": s.nusselt()}
        del s
        torch.cuda.empty_cache()
    return out


def proxy2d_bench(rt, torch, steps, warmup, n=4788):
    """One 4788 x 4788 uniform cavity (22.9M cells, the 256-cavity batch's
    total) at Ra = 1e7 in FP32 deviation storage with the batch's 16 x 8
    one-step tile (--tile 4): the batch kernel's per-tile arithmetic on a
    single domain, for HBM counters and as a throughput reference."""
    s = rt.Solver(2, (n, n), (0.0, 0.0), KIND, TDEV, GAXIS, Ra=1e7, Pr=PR, Ma=MA, precision=rt.FP32_DEV, seed=1,
                  noise_amp=1e-6, tile=TILE or 4, residual_every=KERNEL_CHUNK, mass_fix_every=-1)
    s.step(max(warmup, 20))
    s.sync()
    ms = timed(torch, s, max(steps, 50))
    cells = n * n
    return {"workload": f"cavity {n}x{n} uniform Ra=1e7 FP32, single domain", "cells": cells,
            "tile": list(launch_shape(s.info)), **rates(cells, ms, 2, "f32")}


TABLE5 = {1e3: {"u_max": 0.132, "z": 0.185, "w_max": 0.133, "x": 0.825, "Nu_m": 1.089, "Nu_o": 1.071},
          1e4: {"u_max": 0.198, "z": 0.175, "w_max": 0.220, "x": 0.885, "Nu_m": 2.251, "Nu_o": 2.055},
          1e5: {"u_max": 0.141, "z": 0.147, "w_max": 0.245, "x": 0.936, "Nu_m": 4.613, "Nu_o": 4.337},
          1e6: {"u_max": 0.0812, "z": 0.138, "w_max": 0.257, "x": 0.963, "Nu_m": 8.882, "Nu_o": 8.643}}
# Step cap per Ra: at Ra 1e3 and 1e4 the 80^3 cube is diffusion-dominated
# (Delta t = 0.15 / chi is 0.10 and 0.32, one diffusion time L^2 / chi about
# 1e6 steps), so it needs several times the steps of the convective cases.
CUBE80_MAX_STEPS = {1e3: 4_000_000, 1e4: 3_000_000, 1e5: 800_000, 1e6: 1_400_000}
# Stopping rule: relative change of the hot-wall Nu per 20,000-step chunk.  At
# Ra = 1e6 Nu still creeps up by about 3e-5 per chunk near 500,000 steps and
# settles only near 900,000.
CUBE80_TOL = {1e3: 2e-5, 1e4: 2e-5, 1e5: 2e-5, 1e6: 1e-6}
# No plateau test before this many steps: from rest, the hot-wall Nusselt
# number first falls (conduction) and then rises (convection), and passes a
# minimum where its change per chunk vanishes; at Ra 1e3 and 1e4 that minimum
# comes long before the steady state, which takes about two diffusion times.
CUBE80_MIN_STEPS = {1e3: 2_000_000, 1e4: 2_000_000, 1e5: 0, 1e6: 0}
CUBE80_CASES = tuple(sorted(TABLE5))  # --ra selects one


def _peak(xc, f):
    """Maximum of samples f at nodes xc by the parabola through the largest
    sample and its two neighbours: (position, value)."""
    k = int(np.argmax(f))
    k = min(max(k, 1), len(f) - 2)
    x0, x1, x2 = xc[k - 1:k + 2]
    y0, y1, y2 = f[k - 1:k + 2]
    A = np.array([[x0 * x0, x0, 1.0], [x1 * x1, x1, 1.0], [x2 * x2, x2, 1.0]])
    a, b, c = np.linalg.solve(A, [y0, y1, y2])
    if a >= 0:
        return float(xc[int(np.argmax(f))]), float(f.max())
    xm = -b / (2 * a)
    return float(xm), float(a * xm * xm + b * xm + c)


def cube_table5_bench(rt, torch, steps, warmup, n=80, chunk=20_000):
    """The 3D cubic cavity of the paper's Sec. 4.4 on its 80^3 tanh mesh (phi =
    1.8), Ra = 1e3 ... 1e6, FP32 deviation storage, run until the hot-wall
    Nusselt number changes by less than CUBE80_TOL (relative) over a chunk.  Reported
    against the printed 'Present' values: u_max / V_c on the vertical centre
    line (x = y = L/2) and its height, w_max / V_c on the horizontal centre
    line (y = z = L/2) and its position, Nu_m on the line x = L, y = L/2
    (Eq. 75) and the hot-wall average Nu_o (Eq. 76)."""
    out = {"workload": f"cube{n} tanh1.8 Table 5", "cases": {}}
    x, L = rt.mesh_nodes(n, 1.8)
    xc = 0.5 * (x[1:] + x[:-1]) / L
    w_first = (x[1] - x[0])
    h = n // 2
    for Ra in CUBE80_CASES:
        max_steps, min_steps, tol = CUBE80_MAX_STEPS[Ra], CUBE80_MIN_STEPS[Ra], CUBE80_TOL[Ra]
        s = rt.Solver(3, (n, n, n), (1.8, 1.8, 1.8), (1, 1, 2, 2, 2, 2), (-0.5, 0.5, 0, 0, 0, 0), 2, Ra=Ra,
                      Pr=0.71, Ma=MA, precision=rt.FP32_DEV, seed=1, noise_amp=1e-6)
        t0 = time.perf_counter()
        done, prev, nu = 0, None, None
        while done < max_steps:
            s.step(chunk)
            done += chunk
            nu = s.nusselt()
            if done % (10 * chunk) == 0:
                print(f"# Ra {Ra:g}: {done} steps, Nu hot {nu['hot_avg']:.5f}, {time.perf_counter() - t0:.0f} s",
                      flush=True)
            if done > min_steps and prev is not None and abs(nu["hot_avg"] - prev) < tol * abs(nu["hot_avg"]):
                break
            prev = nu["hot_avg"]
        el = time.perf_counter() - t0
        sh = (n, n, n)  # (z, y, x) with x fastest
        u = s.field(1).reshape(sh)
        w = s.field(3).reshape(sh)
        T = s.field(4).reshape(sh)
        Vc = MA
        # centre lines: the mid-planes fall between cells h - 1 and h (symmetric mesh)
        u_line = u[:, h - 1:h + 1, h - 1:h + 1].mean(axis=(1, 2)) / Vc
        w_line = w[h - 1:h + 1, h - 1:h + 1, :].mean(axis=(0, 1)) / Vc
        zu, umax = _peak(xc, u_line)
        xw, wmax = _peak(xc, w_line)
        # Nu_m: hot wall at x = L (T = 1), one-sided gradient over the half cell
        Twall = 1.0
        dTdx = (Twall - T[:, h - 1:h + 1, n - 1].mean(axis=1)) / (0.5 * w_first)
        dz = np.diff(x) / L
        Nu_m = float(np.sum(dTdx * L * dz))
        out["cases"][f"{Ra:g}"] = {
            "steps": done, "seconds": el, "nu": nu,
            "u_max": umax, "z": zu, "w_max": wmax, "x": xw, "Nu_m": Nu_m, "Nu_o": nu["hot_avg"],
            "paper_present": TABLE5[Ra],
            "rel_diff": {k: abs(v - TABLE5[Ra][k]) / TABLE5[Ra][k]
                         for k, v in (("u_max", umax), ("w_max", wmax), ("Nu_m", Nu_m), ("Nu_o", nu["hot_avg"]))},
        }
        print(json.dumps({f"Ra={Ra:g}": out["cases"][f"{Ra:g}"]}), flush=True)
        del s
        torch.cuda.empty_cache()
    return out


def cube_solver(rt, n, prec, **kw):
    return rt.Solver(3, (n, n, n), (1.8, 1.8, 1.8), (1, 1, 2, 2, 2, 2), (-0.5, 0.5, 0, 0, 0, 0), 2, Ra=1e6,
                     Pr=0.71, Ma=MA, precision=prec, seed=1, noise_amp=1e-6, **kw)


CUBE_STEADY_BUDGET_S = 450.0  # --budget-s: wall-clock seconds of the 192^3 FP64 run


def cube_steady_bench(rt, torch, steps, warmup, n=192, coarse=80, chunk=20_000, tol=1e-8, coarse_tol=1e-6,
                      budget_s=None):
    """C5's fixed-Nu-error check: the 192^3 cube at Ra = 1e6 in FP64 plain
    and FP32 deviation at steady state.  To reach it within one run, both
    start from the same state: the 80^3 FP64 steady solution (hot-wall Nu
    changing by less than coarse_tol per chunk) interpolated trilinearly in
    the normalised coordinate onto the 192^3 cell centres (rho, u, T; lattice
    units scale with the mesh, u / V_c and rho - 1 do not).  The steady state
    does not depend on the start, only the transient is shortened.  FP64
    then runs until both Eq. 65 ratios fall below tol or budget_s runs out;
    FP32 runs the same number of steps.  Progress goes to stderr."""
    from scipy.interpolate import RegularGridInterpolator

    budget_s = CUBE_STEADY_BUDGET_S if budget_s is None else budget_s
    t0 = time.perf_counter()
    c = cube_solver(rt, coarse, rt.FP64_PLAIN, residual_every=1000)
    done, prev = 0, None
    while done < 2_000_000:
        c.step(chunk)
        done += chunk
        nu = c.nusselt()["hot_avg"]
        if done % (10 * chunk) == 0:
            print(f"cube steady: {coarse}^3 FP64 {done} steps, Nu hot {nu:.7f}, {time.perf_counter() - t0:.0f} s",
                  file=sys.stderr, flush=True)
        if prev is not None and abs(nu - prev) < coarse_tol * nu:
            break
        prev = nu
    print(f"cube steady: {coarse}^3 FP64 {done} steps, Nu hot {nu:.6f}, residual {c.residual()}, "
          f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
    xc_c, Lc = rt.mesh_nodes(coarse, 1.8)
    xf, Lf = rt.mesh_nodes(n, 1.8)
    gc = 0.5 * (xc_c[1:] + xc_c[:-1]) / Lc
    gf = 0.5 * (xf[1:] + xf[:-1]) / Lf
    Z, Y, X = np.meshgrid(gf, gf, gf, indexing="ij")
    pts = np.stack([Z.ravel(), Y.ravel(), X.ravel()], axis=1)
    del Z, Y, X
    fields = []
    for f in range(5):
        g = c.field(f).reshape(coarse, coarse, coarse)
        fields.append(RegularGridInterpolator((gc, gc, gc), g, bounds_error=False, fill_value=None)(pts))
    del pts, c
    torch.cuda.empty_cache()
    rho, u, T = fields[0], np.concatenate(fields[1:4]), fields[4]
    s64 = cube_solver(rt, n, rt.FP64_PLAIN, residual_every=1000)
    s32 = cube_solver(rt, n, rt.FP32_DEV, residual_every=1000)
    s64.set_state(rho, u, T)
    s32.set_state(rho, u, T)
    del fields, rho, u, T
    t1 = time.perf_counter()
    done = 0
    while True:
        s64.step(chunk)
        done += chunk
        r = s64.residual()
        print(f"cube steady: 192^3 FP64 {done} steps, residual {r}, Nu hot {s64.nusselt()['hot_avg']:.7f}, "
              f"{time.perf_counter() - t1:.0f} s", file=sys.stderr, flush=True)
        if max(r) < tol or time.perf_counter() - t1 > budget_s:
            break
    t64 = time.perf_counter() - t1
    t2 = time.perf_counter()
    left = done
    while left > 0:
        k = min(chunk * 5, left)
        s32.step(k)
        s32.sync()
        left -= k
        print(f"cube steady: 192^3 FP32 {done - left} steps, {time.perf_counter() - t2:.0f} s", file=sys.stderr,
              flush=True)
    a, b = s32.nusselt(), s64.nusselt()
    diff = {k: abs(a[k] - b[k]) / abs(b[k]) for k in b}
    out = {"workload": "cube192 tanh1.8 Ra=1e6, FP32 vs FP64 at steady state", "coarse_start": coarse,
           "steps": done, "steady": bool(max(s64.residual()) < tol), "fp64_residual": list(s64.residual()),
           "fp32_residual": list(s32.residual()), "nu_fp64": b, "nu_fp32": a, "nu_rel_diff": diff,
           "max_nu_rel_diff": max(diff.values()), "seconds_fp64": t64, "seconds_fp32": time.perf_counter() - t2}
    for name, x in (("fp64", s64), ("fp32", s32)):
        u = x.field(1).reshape(n, n, n)
        w = x.field(3).reshape(n, n, n)
        h = n // 2
        out[f"{name}_u_max_over_Vc"] = float(u[:, h - 1:h + 1, h - 1:h + 1].mean(axis=(1, 2)).max() / MA)
        out[f"{name}_w_max_over_Vc"] = float(w[h - 1:h + 1, h - 1:h + 1, :].mean(axis=(0, 1)).max() / MA)
    return out


def hill_bench(rt, torch, steps, warmup, sizes=(80, 120, 160, 200, 240)):
    """Sec. 4.1 accuracy study (Fig. 7): the Gaussian hill advected and
    diffused on the periodic [0, 2L]^2 box (L = N/2 cells, dtl = 0.5, Delta t
    = 1, chi = 0.1 so Fo_dx = 0.1, Pe = 10, nu = chi), E_2 of Eq. 68 against
    Eq. 67 at Fo = 0.005 on the paper's five meshes, and the fitted order,
    for RTLBFS and TLBFS (Fig. 7 compares the two)."""
    out = {"workload": "Gaussian hill, Sec. 4.1", "sizes": list(sizes)}
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import inputs  # seeded inputs and the closed form of Eq. 67

    for name, prec, method in (("fp64_plain", rt.FP64_PLAIN, rt.METHOD_RTLBFS), ("fp32_dev", rt.FP32_DEV, rt.METHOD_RTLBFS),
                               ("fp64_dev", rt.FP64_DEV, rt.METHOD_RTLBFS),
                               ("tlbfs_fp64_plain", rt.FP64_PLAIN, rt.METHOD_TLBFS),
                               ("tlbfs_fp32_dev", rt.FP32_DEV, rt.METHOD_TLBFS)):
        errs = []
        for N in sizes:
            L = N / 2.0
            chi = 0.1
            u0 = 10.0 * chi / L
            s = rt.Solver(2, (N, N), (0, 0), (0, 0, 0, 0), (0, 0, 0, 0), -1, phys_given=1, nu=chi, chi=chi,
                          beta_g=0.0, dtl=0.5, dt=1.0, precision=prec, method=method)
            xc = np.arange(N) + 0.5
            u = np.zeros((2, N * N))
            u[0] = u0
            s.set_state(np.ones(N * N), u, inputs.gaussian_hill(xc, xc, L, 0.0, chi, u0).reshape(-1))
            n = int(round(0.005 * L * L / chi))
            s.step(n)
            Ta = inputs.gaussian_hill(xc, xc, L, float(n), chi, u0).reshape(-1)
            errs.append(float(np.sqrt(np.mean((s.field(3) - Ta) ** 2))))
        order = -float(np.polyfit(np.log(sizes), np.log(errs), 1)[0])
        out[name] = {"E2": errs, "order": order}
    return out


TABLE6 = {"tlbfs": 60585.58, "rtlbfs": 58864.12, "ratio": 0.9716}  # serial CPU, t* = 1, 80^3, Ra = 1e6


def methods_bench(rt, torch, steps, warmup):
    """Cost of the two interior-face fluxes on the same workloads (the paper's
    Table 6 compares RTLBFS with TLBFS by CPU time): the 256^2 tanh cavity in
    FP32 deviation and FP64 plain storage, and the 192^3 tanh cube in FP32,
    each timed as whole graph-replayed steps with the tile fixed to the one
    the autotuner picks for RTLBFS; then Table 6's own case, one t* on the
    80^3 cube at Ra = 1e6 in FP64."""
    out = {"workload": "RTLBFS vs TLBFS step cost"}
    for name, prec in (("cavity256_fp32", rt.FP32_DEV), ("cavity256_fp64", rt.FP64_PLAIN)):
        res = {}
        tile = 0
        for mname, method in (("rtlbfs", rt.METHOD_RTLBFS), ("tlbfs", rt.METHOD_TLBFS)):
            s = rt.Solver(2, (N_CELLS_SIDE, N_CELLS_SIDE), (STRETCH, STRETCH), KIND, TDEV, GAXIS, Ra=RA, Pr=PR,
                          Ma=MA, precision=prec, seed=1, noise_amp=1e-6, residual_every=KERNEL_CHUNK,
                          mass_fix_every=-1, tile=tile, method=method)
            tile = TILES_2D[launch_shape(s.info)]
            s.step(max(warmup, KERNEL_CHUNK))
            n = max(KERNEL_CHUNK, steps - steps % KERNEL_CHUNK)
            res[mname] = {"us_per_step": timed(torch, s, n) * 1e3, "tile": list(launch_shape(s.info))}
            del s
        res["rtlbfs_over_tlbfs"] = res["rtlbfs"]["us_per_step"] / res["tlbfs"]["us_per_step"]
        out[name] = res
    res = {}
    for mname, method in (("rtlbfs", rt.METHOD_RTLBFS), ("tlbfs", rt.METHOD_TLBFS)):
        s = rt.Solver(3, (192, 192, 192), (1.8, 1.8, 1.8), (1, 1, 2, 2, 2, 2), (-0.5, 0.5, 0, 0, 0, 0), 2, Ra=1e6,
                      Pr=0.71, Ma=MA, precision=rt.FP32_DEV, seed=1, noise_amp=1e-6, method=method)
        s.step(20)
        res[mname] = {"ms_per_step": timed(torch, s, 200)}
        del s
        torch.cuda.empty_cache()
    res["rtlbfs_over_tlbfs"] = res["rtlbfs"]["ms_per_step"] / res["tlbfs"]["ms_per_step"]
    out["cube192_fp32"] = res
    # Table 6's own case: t_cost of one dimensionless time unit t* = V_c t / L
    # on the 80^3 tanh cube (phi = 1.8) at Ra = 1e6, in FP64 (the paper's
    # arithmetic), started from the state after 2,000 steps.
    res = {}
    for mname, method in (("rtlbfs", rt.METHOD_RTLBFS), ("tlbfs", rt.METHOD_TLBFS)):
        s = rt.Solver(3, (80, 80, 80), (1.8, 1.8, 1.8), (1, 1, 2, 2, 2, 2), (-0.5, 0.5, 0, 0, 0, 0), 2, Ra=1e6,
                      Pr=0.71, Ma=MA, precision=rt.FP64_PLAIN, seed=1, noise_amp=1e-6, method=method)
        s.step(2000)
        n_tstar = int(math.ceil(s.info.L / (MA * s.info.dt)))
        ms = timed(torch, s, n_tstar)
        res[mname] = {"steps_per_tstar": n_tstar, "t_cost_s": ms * n_tstar * 1e-3}
        del s
        torch.cuda.empty_cache()
    res["rtlbfs_over_tlbfs"] = res["rtlbfs"]["t_cost_s"] / res["tlbfs"]["t_cost_s"]
    res["paper_table6_serial_cpu_s"] = TABLE6
    out["cube80_fp64_tstar1"] = res
    return out


STAB_RA = (1e3, 1e4, 1e5, 1e6, 1e7, 1e8)
STAB_DTL = (0.1, 0.2, 0.3, 0.4, 0.5, 0.6, 0.7, 0.8, 0.9, 1.0)
STAB_N = (10, 20, 30, 40, 60, 80, 100)


def stability_sweep(rt, members, dtl, method, max_steps, check_every=5000, tol=1e-9):
    """Run the cavities `members` [(N, Ra)] as one FP64 batch (uniform mesh,
    Pr = 0.71, V_c = 0.1, Delta t = 0.5, lattice step dtl) until each has
    converged (both Eq. 65 ratios below tol) or diverged (NaN/Inf or Mach >
    0.5), or max_steps passed: 'C', 'D' or 'U' per member."""
    from paper_2202_13449_amd.workloads import CAVITY_GRAVITY, CAVITY_KIND, CAVITY_TDEV

    meshes = [rt.make_mesh(2, (n, n), (0.0, 0.0)) for n, _ in members]
    bcs = [rt.make_bc(CAVITY_KIND, CAVITY_TDEV, CAVITY_GRAVITY) for _ in members]
    b = rt.Batch(meshes, [ra for _, ra in members], [0.71] * len(members), bcs, Ma=MA, precision=rt.FP64_PLAIN,
                 seed=1, noise_amp=1e-6, dtl=dtl, dt=0.5, method=method, residual_every=100)
    state = ["U"] * len(members)
    done = 0
    while done < max_steps and "U" in state:
        b.step(check_every)
        done += check_every
        div = b.diverged()
        res = b.residuals()
        for k in range(len(members)):
            if state[k] != "U":
                continue
            if div[k] or not np.all(np.isfinite(res[k])):
                state[k] = "D"
            elif res[k].max() < tol:
                state[k] = "C"
    del b
    return state, done


def stability_bench(rt, torch, steps, warmup, max_steps=600_000):
    """The stability maps of Sec. 3.3 as batched launches, FP64, for RTLBFS
    and TLBFS: Fig. 4 (50^2, Delta t = 0.5, lattice step dtl x Ra) and Fig. 5
    (dtl = 1, mesh N x Ra).  Rows are printed as strings of C (converged to
    1e-9), D (diverged), U (neither within the step budget)."""
    out = {"workload": "stability maps, Sec. 3.3", "Ra": list(STAB_RA), "max_steps": max_steps}
    t0 = time.perf_counter()
    for mname, method in (("rtlbfs", rt.METHOD_RTLBFS), ("tlbfs", rt.METHOD_TLBFS)):
        fig4 = {}
        for dtl in STAB_DTL:
            st, n = stability_sweep(rt, [(50, ra) for ra in STAB_RA], dtl, method, max_steps)
            fig4[f"{dtl:.1f}"] = "".join(st)
            print(json.dumps({"fig4": mname, "dtl": dtl, "row": "".join(st), "steps": n,
                              "s": round(time.perf_counter() - t0, 1)}), flush=True)
        members = [(n, ra) for n in STAB_N for ra in STAB_RA]
        st, n = stability_sweep(rt, members, 1.0, method, max_steps)
        fig5 = {str(N): "".join(st[i * len(STAB_RA):(i + 1) * len(STAB_RA)]) for i, N in enumerate(STAB_N)}
        print(json.dumps({"fig5": mname, "rows": fig5, "steps": n, "s": round(time.perf_counter() - t0, 1)}),
              flush=True)
        out[mname] = {"fig4_dtl_by_Ra": fig4, "fig5_N_by_Ra": fig5}
    a4 = "".join(out["rtlbfs"]["fig4_dtl_by_Ra"].values())
    b4 = "".join(out["tlbfs"]["fig4_dtl_by_Ra"].values())
    a5 = "".join(out["rtlbfs"]["fig5_N_by_Ra"].values())
    b5 = "".join(out["tlbfs"]["fig5_N_by_Ra"].values())
    out["agreement_fig4"] = sum(x == y for x, y in zip(a4, b4)) / len(a4)
    out["agreement_fig5"] = sum(x == y for x, y in zip(a5, b5)) / len(a5)
    out["seconds"] = time.perf_counter() - t0
    return out


def steady_bench(rt, torch, steps, warmup, tol=1e-8, max_steps=4_000_000, chunk=20000):
    """The 256^2 cavity run to steady state: FP64 plain until both Eq. 65
    ratios are below tol, then FP32 deviation for the same number of steps;
    Nusselt numbers and velocity maxima of both (the fixed-Nu-error check)."""
    res = {}
    s64 = make_solver(rt, rt.FP64_PLAIN)
    n = 0
    t0 = time.perf_counter()
    while n < max_steps:
        s64.step(chunk)
        n += chunk
        if max(s64.residual()) < tol:
            break
    res["fp64_plain"] = {"steps": n, "residual": s64.residual(), "nu": s64.nusselt(),
                         "seconds": time.perf_counter() - t0}
    s32 = make_solver(rt, rt.FP32_DEV)
    t0 = time.perf_counter()
    s32.step(n)
    res["fp32_dev"] = {"steps": n, "residual": s32.residual(), "nu": s32.nusselt(),
                       "seconds": time.perf_counter() - t0}
    a, b = res["fp32_dev"]["nu"], res["fp64_plain"]["nu"]
    res["nu_rel_diff"] = {k: abs(a[k] - b[k]) / abs(b[k]) for k in b}
    L = s64.info.L
    chi = s64.info.chi
    for name, s in (("fp64_plain", s64), ("fp32_dev", s32)):
        u = s.grid(s.field(1))
        v = s.grid(s.field(2))
        res[name]["umax_mid_uL_over_chi"] = float(0.5 * (u[:, 127] + u[:, 128]).max() * L / chi)
        res[name]["vmax_mid_vL_over_chi"] = float(0.5 * (v[127, :] + v[128, :]).max() * L / chi)
    res["workload"] = "cavity256 tanh1.5 Ra=1e6 to steady state"
    return res


# High-Ra cavities of Sec. 4.2 (Tables 2 and 3): the paper gives the mesh
# size and the wall distance of the first cell (0.0004 L on 300^2 at Ra =
# 1e7, 0.0002 L on 400^2 at Ra = 1e8) but not the stretching law; the Eq. 74
# tanh law is used with phi solved for that first cell.  Printed values: the
# "Present" column and the pseudospectral column (Quere) of each table.
TABLES_2_3 = {
    1e7: {"n": 300, "first_over_L": 4e-4,
          "present": {"psi_max": 30.121, "psi_x": 0.0862, "psi_y": 0.5584, "nu_half": 16.510,
                      "u_max": 148.08, "u_y": 0.8802, "v_max": 699.21, "v_x": 0.0213},
          "pseudospectral": {"psi_max": 30.165, "psi_x": 0.086, "psi_y": 0.556, "nu_half": 16.52,
                             "u_max": 148.59, "u_y": 0.879, "v_max": 699.18, "v_x": 0.021}},
    1e8: {"n": 400, "first_over_L": 2e-4,
          "present": {"psi_max": 53.823, "psi_x": 0.0488, "psi_y": 0.5516, "nu_half": 30.220,
                      "u_max": 312.734, "u_y": 0.9303, "v_max": 2222.8, "v_x": 0.0118},
          "pseudospectral": {"psi_max": 53.85, "psi_x": 0.048, "psi_y": 0.553, "nu_half": 30.225,
                             "u_max": 321.9, "u_y": 0.928, "v_max": 2222.0, "v_x": 0.012}},
}
HIGHRA_BUDGET_S = 240.0   # wall-clock budget per case (--budget-s)
HIGHRA_CASES = (1e7, 1e8)  # --ra selects one


def stretch_for_first_cell(rt, n, first_over_L):
    """phi of the Eq. 74 tanh law whose first cell is first_over_L of the
    length (bisection; the length in first-cell units grows with phi)."""
    lo, hi = 0.1, 6.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if 1.0 / rt.mesh_nodes(n, mid)[1] > first_over_L:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def table23_quantities(rt, s, n, phi):
    """The quantities of Tables 2 and 3 from the absolute primitive fields:
    |psi/chi|_max and its position (psi = integral of u dy from the bottom
    wall, at the cell columns), Nu along x = L/2 (integral of rho u T -
    chi dT/dx over y, divided by chi; dT = 1), and the maxima of u L/chi
    along x = L/2 and v L/chi along y = L/2 with their positions (parabolic
    refinement around the largest cell value)."""
    x, L = rt.mesh_nodes(n, phi)
    xc, dx = 0.5 * (x[:-1] + x[1:]), np.diff(x)
    chi = s.info.chi
    rho, u, v, T = (s.grid(s.field(f)) for f in range(4))  # [row j (y), column i (x)]
    m = n // 2  # x = L/2 lies between columns m - 1 and m (symmetric mesh)
    q = 0.5 * (rho[:, m - 1] * u[:, m - 1] * T[:, m - 1] + rho[:, m] * u[:, m] * T[:, m])
    q -= chi * (T[:, m] - T[:, m - 1]) / (xc[m] - xc[m - 1])
    nu_half = float(np.sum(q * dx) / chi)
    uy, um = _peak(xc / L, 0.5 * (u[:, m - 1] + u[:, m]) * L / chi)
    vx, vm = _peak(xc / L, 0.5 * (v[m - 1, :] + v[m, :]) * L / chi)
    psi = np.abs(np.cumsum(u * dx[:, None], axis=0)) / chi  # at the top face of each cell
    j, i = np.unravel_index(int(np.argmax(psi)), psi.shape)
    return {"psi_max": float(psi[j, i]), "psi_x": float(xc[i] / L), "psi_y": float(x[j + 1] / L),
            "nu_half": nu_half, "u_max": um, "u_y": uy, "v_max": vm, "v_x": vx}


def dhc_highra_bench(rt, torch, steps, warmup, tol=1e-8, chunk=100_000, plateau=2e-5):
    """Cavities of Tables 2 and 3 in FP32 deviation storage, run from rest
    (plus 1e-6 noise) to steady state or until the time budget per case is
    spent, with a progress line every 10 chunks; then the table quantities
    beside the printed ones.  Steady: both Eq. 65 ratios below tol, or the
    hot-wall Nusselt number changing by less than `plateau` (relative) over
    three successive progress lines.  Stochastically rounded FP32 holds the
    Eq. 65 ratios at a floor of a few 1e-8 once the flow is steady, which the
    plateau test allows for."""
    out = {"workload": "2D cavity at Ra 1e7 (300^2) and 1e8 (400^2), Sec. 4.2 Tables 2-3"}
    for Ra in HIGHRA_CASES:
        case = TABLES_2_3[Ra]
        n = case["n"]
        phi = stretch_for_first_cell(rt, n, case["first_over_L"])
        s = rt.Solver(2, (n, n), (phi, phi), KIND, TDEV, GAXIS, Ra=Ra, Pr=PR, Ma=MA, precision=rt.FP32_DEV,
                      seed=1, noise_amp=1e-6, residual_every=chunk, mass_fix_every=1000)
        steps_per_tstar = s.info.L / (MA * s.info.dt)
        done, t0, res = 0, time.perf_counter(), (1.0, 1.0)
        history, steady = [], False
        while time.perf_counter() - t0 < HIGHRA_BUDGET_S:
            s.step(chunk)
            done += chunk
            res = s.residual()
            if max(res) < tol:
                steady = True
            if done % (10 * chunk) == 0 or steady:
                nu = s.nusselt()["hot_avg"]
                history.append(nu)
                print(f"# Ra {Ra:.0e}: {done} steps (t* {done / steps_per_tstar:.1f}), residual {res[0]:.2e} "
                      f"{res[1]:.2e}, Nu hot {nu:.5f}, {time.perf_counter() - t0:.0f} s", flush=True)
                last = history[-4:]
                if len(last) == 4 and max(abs(a - b) for a, b in zip(last, last[1:])) < plateau * abs(nu):
                    steady = True
            if steady:
                break
        got = table23_quantities(rt, s, n, phi)
        pres = case["present"]
        out[f"ra{Ra:.0e}"] = {"n": n, "phi": phi, "L": s.info.L, "steps": done, "tstar": done / steps_per_tstar,
                              "residual": list(res), "steady": steady,
                              "seconds": time.perf_counter() - t0, "ours": got, "paper_present": pres,
                              "paper_pseudospectral": case["pseudospectral"],
                              "rel_diff_vs_present": {k: (got[k] - pres[k]) / pres[k] for k in pres},
                              "nu_walls": s.nusselt(), "tile": list(launch_shape(s.info))}
        del s
        torch.cuda.empty_cache()
    return out


# Body-fitted meshes (Sec. 4.3).  Flops per cell-update of the curvilinear
# step kernel in the nodal form: two faces (545 FP32-deviation / 523
# FP64-plain each: the frame rotation, shift and flux the kernels run, 430 /
# 415 by tests/test_flops_cpu.py, plus the 115 / 108 by which the nodal face
# flux exceeds the column form) + Eq. 55 Gauss gradients over four faces 152
# (4 x (4 Eq. 56 values x 4 + normals 4 + 4 x 2 x 2 accumulations) + 8 area
# scalings) + primitives 5 (4) + update and buoyancy 32 (31) + stochastic
# rounding 24.  Bytes per cell: state read and written (32 / 64) + two face
# records of 8 values (64 / 128) + 1/dV (4 / 8).
FLOPS_PER_CELL_CURV = {"f32": 2 * 545 + 152 + 5 + 32 + 24, "f64": 2 * 523 + 152 + 4 + 31}
EXEC_FLOPS_PER_CELL_CURV = {"f32": 2 * 430 + 152 + 5 + 32 + 24, "f64": 2 * 415 + 152 + 4 + 31}
BYTES_PER_CELL_CURV = {"f32": 32 + 64 + 4, "f64": 64 + 128 + 8}
TABLE4 = {0.0: (2.438, 43.65), 100.0: (2.653, 29.91), 800.0: (3.202, 0.0), 1600.0: (3.508, 0.0)}


def cylinder_solver(rt, Gr, precision, **opts):
    """The heated cylinder of Sec. 4.3 on its 450 x 300 O-mesh (lengths in
    units of the first cell, D = 1/0.003): Re = 20 and Pr = 0.7 give nu and
    chi from u_inf = 0.1 c_s (Eq. 70), Gr gives beta g (Eq. 71, dT = 1);
    free stream along +y against gravity, T_wall = 1, T_inf = T_ref = 0.
    The buoyant plume reaches |u| ~ 0.3 at Gr = 1600, so the divergence
    guard sits at Mach 0.9."""
    from paper_2202_13449_amd.workloads import CYLINDER, cylinder_mesh

    x, y, D = cylinder_mesh()
    u_inf = CYLINDER["u_inf_cs"] * (1.0 / 3.0) ** 0.5
    nu = u_inf * D / CYLINDER["Re"]
    chi = nu / CYLINDER["Pr"]
    s = rt.CurvSolver(np.array(x), np.array(y), (rt.PERIODIC, rt.PERIODIC, rt.WALL_ISOTHERMAL, rt.FARFIELD),
                      Tw=(0.0, 0.0, CYLINDER["T_wall"], 0.0), up=(0.0, 1.0), T_ref=CYLINDER["T_inf"],
                      u_inf=(0.0, u_inf), T_inf=CYLINDER["T_inf"], nu=nu, chi=chi, beta_g=Gr * nu * nu / D ** 3,
                      precision=precision, max_mach=0.9, **opts)
    return s, D, u_inf


def cylinder_nu_and_separation(s):
    """Eq. 73 average Nusselt number (dT = 1) and the separation angle in
    degrees from the rear stagnation point: where the tangential velocity of
    the first cell layer changes sign on the half of the cylinder from the
    front (theta = -90 deg) to the rear (+90 deg) stagnation point; 0 when
    the flow stays attached."""
    q, _ = s.wall_heat(2)
    ni = s.shape[0]
    cx, cy, _ = s.geometry()
    th = np.arctan2(cy[:ni], cx[:ni])
    ut = -s.field(1)[:ni] * np.sin(th) + s.field(2)[:ni] * np.cos(th)
    half = np.where((th > -np.pi / 2) & (th < np.pi / 2))[0]
    half = half[np.argsort(th[half])]
    v, t = ut[half], th[half]
    neg = np.where(v < 0.0)[0]
    sep = 0.0
    if len(neg) and neg[0] > 0:
        k = neg[0]
        ts = t[k - 1] + (t[k] - t[k - 1]) * v[k - 1] / (v[k - 1] - v[k])
        sep = 90.0 - float(np.degrees(ts))
    return q / np.pi, sep


def cylinder_bench(rt, torch, steps, warmup):
    """Throughput of the body-fitted step kernel on the Sec. 4.3 mesh
    (135,000 cells), Gr = 100, FP32 deviation and FP64 plain, with the
    reductions moved aside (residual once per KERNEL_CHUNK steps, no mass
    fix); roofline of the FP32 kernel against the FP32 vector peak."""
    out = {"workload": "cylinder 450x300 O-mesh Re=20 Gr=100 (Sec. 4.3)", "cells": 450 * 300}
    for name, prec, key in (("fp32_dev", rt.FP32_DEV, "f32"), ("fp64_plain", rt.FP64_PLAIN, "f64")):
        s, _, _ = cylinder_solver(rt, 100.0, prec, residual_every=KERNEL_CHUNK, mass_fix_every=-1)
        s.step(max(warmup, KERNEL_CHUNK))
        s.sync()
        n = max(KERNEL_CHUNK, steps - steps % KERNEL_CHUNK)
        ms = timed(torch, s, n)
        cells = s.cells
        tf = FLOPS_PER_CELL_CURV[key] * cells / (ms * 1e-3) / 1e12
        peak = FP32_VECTOR_PEAK_TFLOPS if key == "f32" else FP64_VECTOR_PEAK_TFLOPS
        out[name] = {"ms_per_step": ms, "value": cells / (ms * 1e-3), "kernel_us": ms * 1e3, "tflops": tf,
                     "tile": [s.info.tile_x, s.info.tile_y],
                     "frac": tf / peak, "peak": peak, "flops_per_cell": FLOPS_PER_CELL_CURV[key],
                     "executed_flops_per_cell": EXEC_FLOPS_PER_CELL_CURV[key],
                     "bytes_per_cell": BYTES_PER_CELL_CURV[key],
                     "hbm_gbs": BYTES_PER_CELL_CURV[key] * cells / (ms * 1e-3) / 1e9}
        if key == "f32":
            out[name]["frac_nonpacked"] = tf / FP32_NONPACKED_PEAK_TFLOPS
        del s
        torch.cuda.empty_cache()
    return out


def cylinder_table4_bench(rt, torch, steps, warmup, chunk=200_000, max_steps=4_000_000, window=5):
    """Sec. 4.3, Table 4: each Gr from the free stream, FP32 deviation
    storage, until the Eq. 73 Nusselt number moves by less than 2e-5
    relative over `chunk` steps (at most max_steps); the reported values are
    the means over the last `window` samples.  Gr = 1600 drifts slowly
    instead of settling (heat and mass collect where the buoyant plume meets
    the far-field ghosts), so its window is taken at t* = t u_inf / D in
    [25, 45], a plateau before the drift sets in; its final value is
    reported beside it."""
    rows = {}
    for Gr, (nu_ref, sep_ref) in TABLE4.items():
        s, D, u_inf = cylinder_solver(rt, Gr, rt.FP32_DEV, residual_every=1000)
        dt = s.info.dt
        hist = []
        done = 0
        t0 = time.perf_counter()
        while done < max_steps:
            s.step(chunk)
            done += chunk
            nu, sep = cylinder_nu_and_separation(s)
            hist.append((done * dt * u_inf / D, nu, sep))
            if Gr < 1600.0 and len(hist) > window and abs(hist[-1][1] - hist[-2][1]) < 2e-5 * nu:
                break
            if Gr >= 1600.0 and hist[-1][0] > 45.0:
                break
        sel = [h for h in hist if 25.0 <= h[0] <= 45.0] if Gr >= 1600.0 else hist[-window:]
        nu_m = float(np.mean([h[1] for h in sel]))
        sep_m = float(np.mean([h[2] for h in sel]))
        rows[str(int(Gr))] = {"Nu": nu_m, "Nu_paper": nu_ref, "Nu_rel_err": abs(nu_m - nu_ref) / nu_ref,
                              "theta_s": sep_m, "theta_s_paper": sep_ref, "steps": done, "t_star": hist[-1][0],
                              "final": {"Nu": hist[-1][1], "theta_s": hist[-1][2]},
                              "residual": s.residual(), "seconds": time.perf_counter() - t0}
        print(json.dumps({"Gr": Gr, **rows[str(int(Gr))]}), flush=True)
        del s
        torch.cuda.empty_cache()
    return {"workload": "cylinder Table 4 (Re=20, Pr=0.7, Gr 0/100/800/1600), FP32 deviation", "rows": rows}


TABLE7 = {1e4: (3.212, 3.222), 1e5: (5.791, 5.810)}


def annulus_solver(rt, Ra, precision, **opts):
    """The Sec. 4.5 wedge (120 x 1 x 240, rotation-closed, wedge angle 1/R_i),
    Pr = 0.71, V_c = 0.1 (Eq. 77: beta g = V_c^2 / (dT (R_o - R_i)))."""
    import math

    from paper_2202_13449_amd.workloads import annulus_mesh

    x, y, z, Ri, Ro, H, dth = annulus_mesh()
    L, Vc, Pr = Ro - Ri, 0.1, 0.71
    nu = Vc * L * math.sqrt(Pr / Ra)
    s = rt.Curv3Solver(np.array(x), np.array(y), np.array(z), (rt.WALL_ISOTHERMAL, rt.WALL_ISOTHERMAL, rt.PERIODIC,
                       rt.PERIODIC, rt.WALL_ADIABATIC, rt.WALL_ADIABATIC), rot=(0.0, dth, 0.0),
                       Tw=(1.0, 0.0, 0, 0, 0, 0), up=(0.0, 0.0, 1.0), T_ref=0.5, nu=nu, chi=nu / Pr,
                       beta_g=Vc * Vc / L, precision=precision, noise_amp=1e-6, seed=1, **opts)
    return s, Ri, Ro


def annulus_bench(rt, torch, steps, warmup):
    """Time per step of the body-fitted 3D step on the Sec. 4.5 wedge (28,800
    cells), Ra = 1e5, FP32 deviation and FP64 plain, residual once per
    KERNEL_CHUNK steps: the fused single-layer kernel (one launch per step,
    the default on this mesh) and, for comparison, the three-launch path
    (opts.tile = 1)."""
    out = {"workload": "annulus 120x1x240 wedge Ra=1e5 (Sec. 4.5)", "cells": 120 * 240}
    for name, prec, tile in (("fp32_dev", rt.FP32_DEV, 0), ("fp64_plain", rt.FP64_PLAIN, 0),
                             ("fp32_dev_three_kernels", rt.FP32_DEV, 1), ("fp64_plain_three_kernels", rt.FP64_PLAIN, 1)):
        s, _, _ = annulus_solver(rt, 1e5, prec, residual_every=KERNEL_CHUNK, mass_fix_every=-1, tile=tile)
        s.step(max(warmup, KERNEL_CHUNK))
        s.sync()
        ms = timed(torch, s, max(KERNEL_CHUNK, steps - steps % KERNEL_CHUNK))
        out[name] = {"ms_per_step": ms, "value": s.cells / (ms * 1e-3), "tile": [s.info.tile_x, s.info.tile_z]}
        del s
        torch.cuda.empty_cache()
    return out


def annulus_table7_bench(rt, torch, steps, warmup, chunk=100_000, max_steps=1_500_000):
    """Sec. 4.5, Table 7: the 120 x 1 x 240 annulus wedge (one azimuthal cell,
    rotation-closed, wedge angle 1/R_i), Pr = 0.71, V_c = 0.1 (Eq. 77),
    FP32 deviation storage, from rest until the inner Nusselt number moves by
    less than 1e-6 relative over `chunk` steps; Eq. 78 on both cylinders as
    R (T_w - T_P)/d averaged over the wall.  Also the time per step of the
    three body-fitted 3D kernels."""
    rows = {}
    for Ra, (ni_ref, no_ref) in TABLE7.items():
        s, Ri, Ro = annulus_solver(rt, Ra, rt.FP32_DEV, residual_every=1000)
        done, prev = 0, None
        t0 = time.perf_counter()
        while done < max_steps:
            s.step(chunk)
            done += chunk
            qi, Ai = s.wall_heat(0)
            qo, Ao = s.wall_heat(1)
            nui, nuo = Ri * qi / Ai, -Ro * qo / Ao
            if prev is not None and abs(nui - prev) < 1e-6 * nui:
                break
            prev = nui
        ms = timed(torch, s, max(steps, 1000))
        rows[f"{Ra:.0e}"] = {"Nu_i": nui, "Nu_i_paper": ni_ref, "Nu_o": nuo, "Nu_o_paper": no_ref,
                             "Nu_i_rel_err": abs(nui - ni_ref) / ni_ref, "Nu_o_rel_err": abs(nuo - no_ref) / no_ref,
                             "steps": done, "residual": s.residual(), "seconds": time.perf_counter() - t0,
                             "ms_per_step": ms, "cell_updates_per_s": s.cells / (ms * 1e-3)}
        del s
        torch.cuda.empty_cache()
    return {"workload": "annulus Table 7 (Ar=2, eta=2, Pr=0.71, 120x1x240 wedge), FP32 deviation", "rows": rows}


def rates(cells, ms, dim, prec):
    """Algorithmic HBM and ALU rates of one step over `cells` in `ms`."""
    bpc = (BYTES_PER_CELL if dim == 2 else BYTES_PER_CELL_3D)[prec]
    gbs = bpc * cells / (ms * 1e-3) / 1e9
    tf = ALG_FLOPS_PER_CELL[dim] * cells / (ms * 1e-3) / 1e12
    peak = FP32_VECTOR_PEAK_TFLOPS if prec == "f32" else FP64_VECTOR_PEAK_TFLOPS
    out = {"ms_per_step": ms, "value": cells / (ms * 1e-3), "hbm_gbs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
           "alu_tflops": tf, "alu_frac": tf / peak,
           "executed_tflops": EXEC_FLOPS_PER_CELL[(dim, prec)] * cells / (ms * 1e-3) / 1e12}
    if prec == "f32":
        out["alu_frac_nonpacked"] = tf / FP32_NONPACKED_PEAK_TFLOPS
    return out


def headline(rt, torch, args):
    """The 256^2 tanh cavity: FP32 deviation (`value`) and FP64 plain, each
    over exactly `steps` timed steps; the dominant kernel's launch time for
    the roofline."""
    cells = N_CELLS_SIDE * N_CELLS_SIDE
    r32 = time_path(rt, torch, rt.FP32_DEV, args.steps, args.warmup)
    ms32 = r32["event_ms"] / args.steps
    out = {
        "metric": "cell-updates/s",
        "value": cells / (ms32 * 1e-3),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D differentially heated cavity 256x256 tanh (phi=1.5) Ra=1e6 Pr=0.71 "
                               "FP32 deviation storage, FP64 reductions",
                   "cells": cells, "residual_every": 100, "mass_fix_every": 1000},
    }
    # Dominant kernel: the FP32 step kernel.  Its algorithmic intensity is
    # 913 flop / 32 B = 29 flop/B, above the FP32 ridge (157.3 / 8 = 20), so
    # the vector ALU roofline is the lower one; the metric's HBM fraction is
    # reported beside it (hbm_frac).
    tile32 = launch_shape(r32["solver"].info)
    kms, ktile = time_step_kernel(rt, torch, rt.FP32_DEV, args.steps, args.warmup, TILES_2D[tile32])
    k = rates(cells, kms, 2, "f32")
    out["roofline"] = {"bound": "alu", "achieved": k["alu_tflops"], "peak": FP32_VECTOR_PEAK_TFLOPS,
                       "unit": "TFLOP/s", "frac": k["alu_frac"], "traffic": measured_traffic(ktile),
                       "peak_nonpacked": FP32_NONPACKED_PEAK_TFLOPS, "frac_nonpacked": k["alu_frac_nonpacked"],
                       "kernel": "k_step2d<float, deviation>", "kernel_us": kms * 1e3, "kernel_tile": ktile,
                       "steps_per_launch": ktile[2], "launch_us": kms * 1e3 * ktile[2],
                       "flops_per_cell": ALG_FLOPS_PER_CELL[2], "executed_flops_per_cell": EXEC_FLOPS_PER_CELL[(2, "f32")],
                       "executed_tflops": k["executed_tflops"], "bytes_per_cell": BYTES_PER_CELL["f32"],
                       "hbm_achieved_gbs": k["hbm_gbs"], "hbm_frac": k["hbm_frac"]}
    out["hbm_roofline_frac"] = k["hbm_frac"]
    out["nu_fp32"] = r32["nu"]
    out["tile"] = list(tile32)
    if not args.fp32_only:
        r64 = time_path(rt, torch, rt.FP64_PLAIN, args.steps, args.warmup)
        ms64 = r64["event_ms"] / args.steps
        out["fp64_plain"] = rates(cells, ms64, 2, "f64")
        out["speedup_fp32_vs_fp64"] = ms64 / ms32
    return out


def steady_nu_error(rt, tol=1e-8, max_steps=4_000_000, chunk=20_000):
    """The fixed-Nu-error check on the benchmark workload: FP64 plain run
    until both Eq. 65 ratios are below `tol` (steady state), FP32 deviation
    run for the same number of steps; relative Nusselt differences, the
    Table 1 velocity maxima of both and the FP32 field errors."""
    s64 = make_solver(rt, rt.FP64_PLAIN)
    n = 0
    t0 = time.perf_counter()
    while n < max_steps:
        s64.step(chunk)
        n += chunk
        if max(s64.residual()) < tol:
            break
    t64 = time.perf_counter() - t0
    s32 = make_solver(rt, rt.FP32_DEV)
    t0 = time.perf_counter()
    s32.step(n)
    s32.sync()
    t32 = time.perf_counter() - t0
    a, b = s32.nusselt(), s64.nusselt()
    return {"steps": n, "steady": bool(max(s64.residual()) < tol), "fp64_residual": list(s64.residual()),
            "fp32_residual": list(s32.residual()), "nu_fp64": b, "nu_fp32": a,
            "nu_rel_diff_fp32_vs_fp64": {k: abs(a[k] - b[k]) / abs(b[k]) for k in b},
            "max_nu_rel_diff": max(abs(a[k] - b[k]) / abs(b[k]) for k in b),
            "fields_fp32_vs_fp64": field_comparison(s32, s64), "seconds_fp64": t64, "seconds_fp32": t32}


def batch_leg(rt, torch, steps, warmup):
    """The 256 seeded cavities (about 2.3e7 cells) in one launch per step:
    FP32 deviation and FP64 plain batches, and the same 256 problems as
    separate FP32 handles stepped one after another."""
    from paper_2202_13449_amd.workloads import (CAVITY_GRAVITY, CAVITY_KIND, CAVITY_TDEV, batch_cavities,
                                                total_cells)

    members = batch_cavities()
    cells = total_cells(members)
    meshes = [rt.make_mesh(2, (m["n"], m["n"]), (m["stretch"], m["stretch"])) for m in members]
    bcs = [rt.make_bc(CAVITY_KIND, CAVITY_TDEV, CAVITY_GRAVITY) for _ in members]
    nsteps = max(steps, 200)
    out = {"workload": "256 batched 2D cavities (seed 4): sides 64-512, Ra 1e3-1e7, Pr 0.71/7, uniform or tanh",
           "cells": cells, "steps": nsteps}
    for name, prec, tag in (("fp32_dev", rt.FP32_DEV, "f32"), ("fp64_plain", rt.FP64_PLAIN, "f64")):
        b = rt.Batch(meshes, [m["Ra"] for m in members], [m["Pr"] for m in members], bcs, Ma=MA, precision=prec,
                     seed=4, noise_amp=1e-6, residual_every=100, mass_fix_every=1000)
        b.step(max(warmup, 20))
        b.sync()
        ms = timed(torch, b, nsteps)
        out[name] = rates(cells, ms, 2, tag)
        del b
        torch.cuda.empty_cache()
    t = stored_traffic(TRAFFIC_FILE_BATCH, batch_sources_sha256(), "16x8")
    out["fp32_dev"]["traffic"] = t
    out["fp32_dev"]["traffic_ratio"] = (t / (BYTES_PER_CELL["f32"] * cells)) if t else None
    # The batch kernel's per-tile arithmetic (16 x 8 one-step tiles) counted on
    # one 4788^2 domain of the same total size: HBM bytes over algorithmic.
    try:
        with open(TRAFFIC_FILE_PROXY) as f:
            tp = json.load(f)
        if tp.get("kernel_sources_sha256") == kernel_sources_sha256():
            out["fp32_dev"]["traffic_ratio_single_domain_proxy"] = tp["bytes_per_launch"] / tp["algorithmic_bytes_per_step"]
    except (OSError, ValueError, KeyError):
        pass
    out["speedup_fp32_vs_fp64"] = out["fp64_plain"]["ms_per_step"] / out["fp32_dev"]["ms_per_step"]
    singles = [rt.Solver(2, (m["n"], m["n"]), (m["stretch"], m["stretch"]), CAVITY_KIND, CAVITY_TDEV,
                         CAVITY_GRAVITY, Ra=m["Ra"], Pr=m["Pr"], Ma=MA, precision=rt.FP32_DEV, seed=4,
                         noise_amp=1e-6, residual_every=100, mass_fix_every=1000) for m in members]
    for x in singles:
        x.step(100)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for x in singles:
        x.step(100)
    e1.record(stream)
    torch.cuda.synchronize()
    ms_seq = e0.elapsed_time(e1) / 100
    out["sequential_256_handles_fp32"] = {"ms_per_step": ms_seq, "value": cells / (ms_seq * 1e-3)}
    out["speedup_batched_vs_sequential"] = ms_seq / out["fp32_dev"]["ms_per_step"]
    del singles
    torch.cuda.empty_cache()
    return out


def cube_leg(rt, torch, steps, warmup):
    """192^3 tanh (phi = 1.8) cubic cavity at Ra = 1e6, FP32 deviation and
    FP64 plain, over at least 200 timed steps (two graph-replayed chunks with
    their residual steps, as a long run takes them)."""
    cells = 192 ** 3
    nsteps = max(steps, 200)
    out = {"workload": "3D differentially heated cube 192^3 tanh (phi=1.8) Ra=1e6 Pr=0.71", "cells": cells,
           "steps": nsteps}
    for name, prec, tag in (("fp32_dev", rt.FP32_DEV, "f32"), ("fp64_plain", rt.FP64_PLAIN, "f64")):
        s = rt.Solver(3, (192, 192, 192), (1.8, 1.8, 1.8), (1, 1, 2, 2, 2, 2), (-0.5, 0.5, 0, 0, 0, 0), 2, Ra=1e6,
                      Pr=0.71, Ma=MA, precision=prec, seed=1, noise_amp=1e-6)
        s.step(max(warmup, 10))
        s.sync()
        ms = timed(torch, s, nsteps)
        out[name] = rates(cells, ms, 3, tag)
        t = stored_traffic(TRAFFIC_FILE_3D, cube_sources_sha256(), tag)
        out[name]["traffic"] = t
        out[name]["traffic_ratio"] = (t / (BYTES_PER_CELL_3D[tag] * cells)) if t else None
        del s
        torch.cuda.empty_cache()
    out["speedup_fp32_vs_fp64"] = out["fp64_plain"]["ms_per_step"] / out["fp32_dev"]["ms_per_step"]
    return out


def cpu_baseline(seconds_target=15.0):
    """The FP64 oracle, as written, on a bounded sample of the same workload."""
    from oracle import Oracle, OracleConfig, physics_from_ra, mesh_nodes

    _, L = mesh_nodes(N_CELLS_SIDE, STRETCH)
    nu, chi, bg = physics_from_ra(RA, PR, MA, L)
    o = Oracle(OracleConfig(n=(N_CELLS_SIDE, N_CELLS_SIDE), stretch=(STRETCH, STRETCH), bc=KIND + (0, 0),
                            Tw=TDEV + (0, 0), gravity_axis=GAXIS, nu=nu, chi=chi, beta_g=bg, dtl=1.0,
                            dt=min(0.5, 0.15 / max(nu, chi)), seed=1, noise_amp=1e-6))
    t0 = time.perf_counter()
    o.step(2)
    per_step = (time.perf_counter() - t0) / 2
    steps = max(5, int(seconds_target / per_step))
    t0 = time.perf_counter()
    o.step(steps)
    el = time.perf_counter() - t0
    cells = N_CELLS_SIDE * N_CELLS_SIDE
    return {"value": cells * steps / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} steps of the 256x256 tanh cavity (Ra=1e6), plain FP64 C oracle, one thread, "
                      f"{el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--warmup", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fp32-only", action="store_true", help="time only the FP32 path (profiling runs)")
    ap.add_argument("--no-sequential", action="store_true",
                    help="with --batch: skip the 256 single-domain handles (profiling runs)")
    ap.add_argument("--batch", action="store_true",
                    help="time the 256-cavity batch (one launch per step) against 256 sequential single-domain runs")
    ap.add_argument("--workload", default="cavity256", choices=["cavity256", "rb1024", "cube192", "cube192_steady", "proxy2d", "steady256", "cube80", "hill", "methods",
                                                           "stability", "cylinder", "cylinder_table4", "annulus", "annulus_table7",
                                                           "dhc_highra"],
                    help="cavity256: the benchmark line; rb1024: 1024x512 Rayleigh-Benard, Ra=1e8; cube192: 192^3 "
                         "tanh cube, Ra=1e6; steady256: the 256^2 cavity to steady state, FP32 vs FP64 Nusselt; "
                         "cube80: the 80^3 cubic cavity at Ra 1e3 ... 1e6 to steady state against Table 5; "
                         "hill: the Gaussian-hill convergence study of Sec. 4.1; methods: RTLBFS vs TLBFS step cost; "
                         "stability: the stability maps of Figs. 4-5 as batched runs; cylinder: the body-fitted "
                         "step on the 450x300 O-mesh of Sec. 4.3; cylinder_table4: Table 4, Gr 0..1600; "
                         "annulus: the body-fitted 3D step on the 120x1x240 wedge of Sec. 4.5; "
                         "annulus_table7: that annulus against Table 7; dhc_highra: the cavities of Tables 2-3 "
                         "(Ra 1e7 on 300^2, Ra 1e8 on 400^2) to steady state or --budget-s")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (5 times) to calibrate HBM counters")
    ap.add_argument("--ra", type=float, default=None,
                    help="dhc_highra (1e7 or 1e8) and cube80 (1e3 ... 1e6): run only this Rayleigh number")
    ap.add_argument("--budget-s", type=float, default=None,
                    help="dhc_highra: wall-clock seconds per case; cube192_steady: seconds of the 192^3 FP64 run")
    ap.add_argument("--tile", type=int, default=0, help="cube192 / proxy2d: opts.tile of the solver")
    ap.add_argument("--steady-steps", type=int, default=0,
                    help="with --batch: advance FP64 and FP32 batches this many steps and compare the Nusselt "
                         "numbers of the members that reached steady state")
    args = ap.parse_args()
    global HIGHRA_CASES, HIGHRA_BUDGET_S, CUBE80_CASES, TILE, CUBE_STEADY_BUDGET_S
    TILE = args.tile
    if args.ra is not None:
        if args.workload == "cube80":
            if args.ra not in TABLE5:
                ap.error("--ra must be 1e3, 1e4, 1e5 or 1e6 for cube80")
            CUBE80_CASES = (args.ra,)
        else:
            if args.ra not in TABLES_2_3:
                ap.error("--ra must be 1e7 or 1e8")
            HIGHRA_CASES = (args.ra,)
    if args.budget_s is not None:
        HIGHRA_BUDGET_S = args.budget_s
        CUBE_STEADY_BUDGET_S = args.budget_s
    if args.gpus != 1:
        print("bench.py measures one GPU: the RTLBFS step of one domain runs on a single MI355X; "
              "multi-GPU sharding is not implemented (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2202_13449_amd as rt

    torch.cuda.set_device(0)
    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "launches": 5}), flush=True)
        return
    if args.batch:
        if args.steady_steps:
            print(json.dumps(batch_steady_bench(rt, torch, args.steps, args.warmup, total=args.steady_steps)),
                  flush=True)
            return
        print(json.dumps(batch_bench(rt, torch, args.steps, args.warmup, sequential=not args.no_sequential)),
              flush=True)
        return
    if args.workload != "cavity256":
        fn = {"rb1024": rb_bench, "cube192": cube_bench, "cube192_steady": cube_steady_bench, "proxy2d": proxy2d_bench,
              "steady256": steady_bench,
              "cube80": cube_table5_bench, "hill": hill_bench, "methods": methods_bench,
              "stability": stability_bench, "cylinder": cylinder_bench,
              "cylinder_table4": cylinder_table4_bench, "annulus": annulus_bench,
              "annulus_table7": annulus_table7_bench, "dhc_highra": dhc_highra_bench}[args.workload]
        print(json.dumps(fn(rt, torch, args.steps, args.warmup)), flush=True)
        return
    out = headline(rt, torch, args)
    if not args.fp32_only:
        out["fixed_nu_error"] = steady_nu_error(rt)
        out["legs"] = {"batched_256_cavities": batch_leg(rt, torch, args.steps, args.warmup),
                       "cube192": cube_leg(rt, torch, args.steps, args.warmup)}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
