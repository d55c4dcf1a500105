#!/usr/bin/env python3
"""Throughput of third-order semi-Lagrangian advection on one MI355X.

Workload (default): one FP32 scalar on a periodic 512^3 grid (sum of 8
seeded Gaussians, sigma in [0.05, 0.15] of the box), steady ABC velocity
(A = B = C = 1) on [0, 2 pi)^3, CFL 0.9, the third-order scheme.  A "step"
is one full time step of the scheme over the whole grid (all interpolation
calls of all three axis sweeps).  Inputs are resident in HBM before the
timed region starts.

Prints one JSON line: Gcell-updates/s over exactly --steps steps, the
roofline of the dominant kernel (per-launch durations from HIP events
recorded by the library on its stream during the timed region), the HBM
traffic from rocprofv3 counters when they were taken on the current kernel
source, and the FP64 CPU oracle timed on a bounded sample of the same
workload.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import resource
import sys
import time
import traceback

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "Gcell-updates/s + %HBM peak, 3rd-order 512³ FP32; learned vs plain at equal L2"
HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
CSRC = os.path.join(ROOT, "paper_1606_06117_amd", "csrc")
# source file holding each kernel kind (counters are stale once it changes)
KERNEL_SRC = {"cec3d": "cec3d_kernel.hip", "learned": "mlp_kernels.hip"}


def algorithmic_bytes(kind: str, ncells: int, ndim: int) -> int:
    """Bytes a launch of ``kind`` must move at minimum over ``ncells`` cells.

    A whole step reads phi and the ndim velocity planes and writes phi:
    (8 + 4 ndim) B per cell.  One axis sweep reads phi and its velocity plane
    and writes phi: 12 B per cell; the fused x and y sweeps read phi and two
    planes: 16 B.  A copy reads and writes 4 B each.
    """
    per_cell = {"cir": 8 + 4 * ndim, "fec": 8 + 4 * ndim, "bec": 8 + 4 * ndim,
                "cec3d": 8 + 4 * ndim, "sweep_x": 12, "sweep_y": 12, "sweep_z": 12,
                "sweep_xy": 16, "copy": 8}[kind]
    return per_cell * ncells


def source_hash(kind: str) -> str:
    with open(os.path.join(CSRC, KERNEL_SRC.get(kind, "advect_kernels.hip")), "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()[:16]


def measured_traffic(kind: str, workload: str):
    """HBM bytes per launch from committed rocprofv3 counters, if still current."""
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    entry = data.get(workload, {}).get(kind)
    if not entry or entry.get("source_sha256_16") != source_hash(kind):
        return None
    if kind == "cec3d":
        from paper_1606_06117_amd import native
        if entry.get("variant") != native.CEC3D_DEFAULT:
            return None  # counters of another implementation of the fused step
    return entry.get("bytes_per_launch")


def cpu_baseline(phi, u, dx, dt, scheme, edge, steps):
    """The FP64 oracle timed on a periodic sub-box of the same inputs."""
    import numpy as np
    import oracle
    sub = phi[:edge, :edge, :edge].astype(np.float64)
    usub = np.ascontiguousarray(u[:, :edge, :edge, :edge])
    c0 = resource.getrusage(resource.RUSAGE_SELF)
    t0 = time.perf_counter()
    oracle.advect(sub, usub, dx, dt, scheme, steps)
    wall = time.perf_counter() - t0
    c1 = resource.getrusage(resource.RUSAGE_SELF)
    cpu = (c1.ru_utime - c0.ru_utime) + (c1.ru_stime - c0.ru_stime)
    cores = max(1, int(round(cpu / wall)))
    return {
        "value": edge**3 * steps / wall / 1e9,
        "unit": "Gcell-updates/s",
        "cores": cores,
        "kind": "oracle",
        "sample": f"FP64 NumPy oracle, {edge}^3 periodic sub-box of the same inputs, "
                  f"{steps} steps of the same scheme ({wall:.1f} s wall, host has {os.cpu_count()} CPUs)",
    }


def cpu_all_cores(phi, u, dx, dt, scheme, edge, zedge, steps, workers):
    """The same oracle over z-slabs with halos in ``workers`` processes.

    The sample is a periodic ``zedge x edge x edge`` sub-box of the same
    inputs; each step every worker advances one slab plus the planes one step
    can read, so the result is the one-process result bit for bit.
    """
    import numpy as np
    from oracle import slabs
    sub = phi[:zedge, :edge, :edge].astype(np.float64)
    usub = np.ascontiguousarray(u[:, :zedge, :edge, :edge])
    p0 = resource.getrusage(resource.RUSAGE_SELF)
    c0 = resource.getrusage(resource.RUSAGE_CHILDREN)
    with slabs.SlabPool(usub, dx, dt, scheme, workers) as pool:
        t0 = time.perf_counter()
        pool.advect(sub, steps)
        wall = time.perf_counter() - t0
        used, halo = pool.workers, pool.halo
    p1 = resource.getrusage(resource.RUSAGE_SELF)
    c1 = resource.getrusage(resource.RUSAGE_CHILDREN)
    cpu = sum(b.ru_utime - a.ru_utime + b.ru_stime - a.ru_stime for a, b in ((p0, p1), (c0, c1)))
    return {
        "value": zedge * edge * edge * steps / wall / 1e9,
        "unit": "Gcell-updates/s",
        "cores": used,
        "busy_cores": round(cpu / wall, 1),
        "sample": f"FP64 NumPy oracle over {used} z-slabs (+{halo} halo planes each side) in "
                  f"{used} processes, {zedge}x{edge}x{edge} periodic sub-box of the same inputs, "
                  f"{steps} steps ({wall:.1f} s wall; busy cores include pool start-up)",
    }


def cpu_scheme_parity(ctx, size, cfl, steps, workers):
    """Every scheme's error against the FP64 oracle on a whole workload.

    The 3D problem of 8 Gaussians under the ABC flow at ``size``^3 and CFL
    ``cfl``: each scheme runs ``steps`` steps on the GPU and in the oracle
    (over z-slabs in ``workers`` processes, the one-process result bit for
    bit), and the two results are compared on every cell: relative L2, and
    max |gpu - oracle| relative to max |phi0|.  The oracle's wall time is
    reported with it (FP64 NumPy, same unit as the GPU figures).
    """
    import numpy as np
    import torch
    from oracle import norms as onorms
    from oracle import slabs
    from paper_1606_06117_amd import native
    from paper_1606_06117_amd import workloads as W
    shape = (size,) * 3
    phi0 = W.random_gaussians_torch(shape, 8, 2000, "cuda:0").cpu().numpy()  # random_gaussians' values
    u = W.abc_velocity(shape)
    dx = (2 * math.pi / size,) * 3
    dt = W.abc_dt(shape, cfl)
    dev = torch.device("cuda:0")
    ud = torch.from_numpy(u).to(dev)
    scale = float(np.max(np.abs(phi0)))
    rows = []
    for name in ("cir", "fec", "bec", "cec"):
        p = torch.from_numpy(phi0).to(dev)
        ctx.advect(p, ud, dx, dt, native.SCHEMES[name], steps)
        torch.cuda.synchronize()
        ctx.check()
        got = p.cpu().numpy().astype(np.float64)
        with slabs.SlabPool(u, dx, dt, native.SCHEMES[name], workers) as pool:
            t0 = time.perf_counter()
            ref = pool.advect(phi0, steps)
            wall = time.perf_counter() - t0
            used = pool.workers
        rows.append({"scheme": name, "relL2_vs_oracle": onorms.rel_l2(got, ref),
                     "linf_vs_oracle_rel": onorms.linf(got, ref) / scale,
                     "bound_relL2": 1e-5 * steps,
                     "oracle_seconds": round(wall, 2), "oracle_processes": used,
                     "oracle_gcell_updates_per_s": size**3 * steps / wall / 1e9})
    del ud
    torch.cuda.empty_cache()
    return {"workload": f"{size}^3, 8 Gaussians (seed 2000), ABC velocity, CFL {cfl}, {steps} steps "
                        f"per scheme; GPU FP32 against the FP64 oracle on every cell",
            "runs": rows}


def copy_probe(reps: int, warmup: int) -> int:
    """Copy a 512 MiB FP32 buffer ``reps`` times (read 512 MiB + write 512 MiB each)."""
    import torch
    n = 128 * 1024 * 1024
    src = torch.ones(n, device="cuda:0", dtype=torch.float32)
    dst = torch.empty_like(src)
    for _ in range(max(1, warmup)):
        dst.copy_(src)
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    moved = 2 * 4 * n
    print(json.dumps({"probe": "copy", "bytes_read_per_copy": 4 * n, "bytes_written_per_copy": 4 * n,
                      "ms_per_copy": ms, "GBps": moved / (ms / 1e3) / 1e9,
                      "frac_of_peak": moved / (ms / 1e3) / 1e9 / HBM_PEAK_GBS}), flush=True)
    return 0


def learned_probe(size: int, reps: int, warmup: int) -> int:
    """Time the learned step alone (CIR pass + correction) at ``size``^3 with
    seeded random weights (the limiter keeps the field bounded whatever the
    network outputs): per-kind kernel times, and the correction's share of
    the matrix cores' BF16 peak at 12 416 FLOP per node."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    from paper_1606_06117_amd import native
    from paper_1606_06117_amd import workloads as W
    shape = (size,) * 3
    dev = torch.device("cuda:0")
    phi = W.random_gaussians_torch(shape, 8, 2000, dev)
    u = W.abc_velocity_torch(shape, dev)
    dx = (2 * math.pi / size,) * 3
    dt = W.abc_dt(shape, 0.9)
    ctx = native.Context(0)
    model = native.Model(ctx)
    rng = np.random.default_rng(5)
    model.set_params((rng.standard_normal(native.MLP_PARAMS) * 0.2).astype(np.float32))
    model.set_courant_range(1.0)
    # at least 30 warm-up steps (about 15 ms of GPU work): the clocks of an
    # idle GPU take that long to come up
    native.advect_learned(ctx, model, phi, u, dx, dt, max(30, warmup), courant_max=0.9)
    torch.cuda.synchronize()
    ctx.timing(True)
    native.advect_learned(ctx, model, phi, u, dx, dt, reps, step0=warmup, courant_max=0.9)
    torch.cuda.synchronize()
    times = ctx.timing_read()
    ctx.timing(False)
    per = {k: v[1] / v[0] for k, v in times.items()}
    flops = 12416 * size**3
    print(json.dumps({"probe": "learned", "grid": [size] * 3, "steps": reps, "per_kind_ms": per,
                      "ms_per_step": sum(per.values()),
                      "mfma_frac": flops / (per["learned"] * 1e-3) / 2.5e15}), flush=True)
    model.close()
    ctx.close()
    return 0


def train_probe(rows: int, reps: int, warmup: int) -> int:
    """Time training steps alone (forward, backward, gradient reduction and
    Adam) on ``rows`` seeded random feature rows and targets: microseconds
    per step (HIP events), and the steps' share of the matrix cores' BF16
    peak at 32 768 FLOP of matrix products per row (12 288 forward, 20 480
    backward)."""
    import numpy as np
    import torch
    sys.path.insert(0, ROOT)
    from paper_1606_06117_amd import native
    ctx = native.Context(0)
    model = native.Model(ctx)
    rng = np.random.default_rng(7)
    model.set_params((rng.standard_normal(native.MLP_PARAMS) * 0.1).astype(np.float32))
    x = rng.standard_normal((rows, native.MLP_INPUTS)).astype(np.float32)
    x[:, 30:] = 0.0
    feats = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).cuda()
    target = torch.from_numpy(rng.standard_normal(rows).astype(np.float32)).cuda()
    for _ in range(max(50, warmup)):
        model.train_step(feats, target, 1e-4)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        model.train_step(feats, target, 1e-4)
    b.record()
    torch.cuda.synchronize()
    us = a.elapsed_time(b) * 1e3 / reps
    print(json.dumps({"probe": "train", "rows": rows, "steps": reps, "us_per_step": us,
                      "mfma_frac_step": 32768 * rows / (us * 1e-6) / 2.5e15}), flush=True)
    model.close()
    ctx.close()
    return 0


def learned_section(ctx, size, fields, steps_per_field, cells, iters, batch, lr, rounds):
    """Learned correction vs the plain third-order scheme on the time-modulated
    ABC flow (CFL 0.9 at peak amplitude): training on pairs from the GPU
    third-order scheme, then error against the exact field after whole
    modulation periods, time per step, and the speedup at equal error: the
    learned run's cost against the plain scheme's cost interpolated at the
    same error, over plain runs at several time steps on the same grid and on
    coarser grids of the same physical problem."""
    from paper_1606_06117_amd import learned as Lr
    shape = (size, size, size)
    model, pairs, hists, pairs_s, train_s = Lr.train_rollout(
        ctx, shape, fields=list(range(4000, 4000 + fields)), steps_per_field=steps_per_field,
        cells_per_snapshot=cells, cfl=0.9, seed=4500, rounds=rounds, iters=iters, batch=batch, lr=lr,
        log_every=max(1, iters // 10))
    hist = [h for hh in hists for h in hh]
    ev = Lr.evaluate(ctx, model, shape, seed=4100, periods=2, cfl=0.9)
    # cost-to-error curve of the plain scheme: a period in 50..200 steps
    plain = []
    for spp in (200, 100, 75, 60):
        err, secs = Lr.error_at_cfl(ctx, shape, 4100, 0.9, spp, 2)
        plain.append((err, secs, 0.9 * Lr.PERIOD / spp))
    # and of the same physical problem on coarser grids (same time step)
    coarse = []
    for n in (32, 48, 64, 96, 128):
        if n < size:
            err, secs = Lr.error_at_resolution(ctx, n, size, 4100, 0.9, 2)
            coarse.append((err, secs, n))
    # the learned model at its training Courant number, below it, and above
    # the range it was trained on (there it must fall back to the plain scheme)
    learned_pts = []
    for spp in (200, Lr.PERIOD, 67):
        fb = []
        err, secs = Lr.error_at_cfl(ctx, shape, 4100, 0.9, spp, 2, learned_model=model, fallbacks=fb)
        learned_pts.append({"cfl": round(0.9 * Lr.PERIOD / spp, 4), "relL2_vs_exact": err,
                            "seconds": secs, "fell_back_steps": fb[0], "steps": 2 * spp})
    lerr, lsecs = learned_pts[1]["relL2_vs_exact"], learned_pts[1]["seconds"]
    speed = Lr.equal_error_speedup([(e, t) for e, t, _ in plain + coarse], (lerr, lsecs))
    last = ev["per_step"][-1]
    out = {
        "workload": f"{size}^3 FP32, ABC velocity with amplitude sin(2 pi (m+1/2)/100), CFL 0.9 at peak; "
                    f"{fields} fields x {steps_per_field} steps x {cells} nodes per round, "
                    f"{rounds} rounds of pairs from the model's own rollouts: {pairs.m} training pairs",
        "pairs_seconds": pairs_s,
        "train_iters": iters * (rounds + 1), "train_batch": batch, "train_seconds": train_s,
        "loss_first": hist[0][1] if hist else None, "loss_last": hist[-1][1] if hist else None,
        "loss_per_round": [[h[0][1], h[-1][1]] for h in hists if h],
        "relL2_vs_third_order_after_200_steps": {"learned": last[1], "cir": last[2]},
        "relL2_vs_exact": ev["vs_exact"],
        "ms_per_step": ev["ms_per_step"],
        "fell_back": ev["fell_back"],
        "plain_error_vs_cost": [{"cfl": c, "relL2_vs_exact": e, "seconds": t} for e, t, c in plain],
        "plain_error_vs_resolution": [{"n": n, "relL2_vs_exact": e, "seconds": t} for e, t, n in coarse],
        "learned_error_vs_cost": learned_pts,
        "speedup_at_equal_L2": speed,
    }
    model.close()
    return out


def timed_steps(ctx, phi, u, dx, dt, steps, warmup, scheme=None):
    """Third-order steps (or ``scheme``'s) with the library's per-kernel
    timing; returns (wall seconds, per-kind (launches, ms))."""
    import torch
    from paper_1606_06117_amd import native
    scheme = native.CEC if scheme is None else scheme
    cmax = ctx.courant_max(u, dx, dt)
    for w in range(warmup):
        ctx.advect(phi, u, dx, dt, scheme, 1, step0=w, courant_max=cmax)
    ctx.check()
    torch.cuda.synchronize()
    ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advect(phi, u, dx, dt, scheme, steps, step0=warmup, courant_max=cmax)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = ctx.timing_read()
    ctx.timing(False)
    ctx.check()
    return wall, times, cmax


def cfl_section(ctx, size, cfls, steps, scheme=None, name="third order"):
    """The headline workload (8 Gaussians, ABC velocity) at other Courant
    numbers: reach 2 takes the fused x+y sweep and the z sweep (28 B per
    cell-update moved), reach 3 three sweeps (36 B); 20 B algorithmic.  With
    ``scheme`` = Strang splitting: x/2 y/2 in one kernel, z, y/2 x/2 (44 B)."""
    import numpy as np
    import torch
    from paper_1606_06117_amd import workloads as W
    shape = (size,) * 3
    dev = torch.device("cuda:0")
    phi = W.random_gaussians_torch(shape, 8, 2000, dev)
    u = W.abc_velocity_torch(shape, dev)
    dx = (2 * math.pi / size,) * 3
    rows = []
    for cfl in cfls:
        wall, times, cmax = timed_steps(ctx, phi, u, dx, W.abc_dt(shape, cfl), steps, 2, scheme)
        upd = size**3 * steps
        rows.append({"cfl": cfl, "courant_max": cmax, "value": upd / wall / 1e9, "unit": "Gcell-updates/s",
                     "ms_per_step": wall * 1e3 / steps,
                     "hbm_frac_step": 20 * upd / wall / (HBM_PEAK_GBS * 1e9),
                     "per_kind_ms": {k: round(v[1] / v[0], 4) for k, v in times.items()}})
    del phi, u
    torch.cuda.empty_cache()
    return {"workload": f"{name}, {size}^3, 8 Gaussians, ABC velocity, {steps} steps per CFL",
            "runs": rows}


def schemes_section(ctx, size, cfl, steps):
    """Every scheme on one workload (8 Gaussians, ABC velocity): the unsplit
    CIR, FEC and BEC steps, the third order, and the split options."""
    import numpy as np
    import torch
    from paper_1606_06117_amd import native
    from paper_1606_06117_amd import workloads as W
    shape = (size,) * 3
    dev = torch.device("cuda:0")
    phi = W.random_gaussians_torch(shape, 8, 2000, dev)
    u = W.abc_velocity_torch(shape, dev)
    dx = (2 * math.pi / size,) * 3
    rows = []
    for name in ("cir", "fec", "bec", "cec", "cec_strang", "fec_split", "bec_split"):
        wall, times, _ = timed_steps(ctx, phi, u, dx, W.abc_dt(shape, cfl), steps, 2, native.SCHEMES[name])
        upd = size**3 * steps
        rows.append({"scheme": name, "value": upd / wall / 1e9, "unit": "Gcell-updates/s",
                     "ms_per_step": wall * 1e3 / steps,
                     "hbm_frac_step": 20 * upd / wall / (HBM_PEAK_GBS * 1e9),
                     "per_kind_ms": {k: round(v[1] / v[0], 4) for k, v in times.items()}})
    del phi, u
    torch.cuda.empty_cache()
    return {"workload": f"every scheme, {size}^3, 8 Gaussians, ABC velocity, CFL {cfl}, {steps} steps each",
            "runs": rows}


def ec_section(ctx, size, cfl, steps):
    """Unsplit FEC and BEC on the headline workload: the one-pass z-march
    (the default, SLA_OPT_EC_KERNEL 3) against the chain of gather kernels
    (2), same inputs, same results bit for bit."""
    import numpy as np
    import torch
    from paper_1606_06117_amd import native
    from paper_1606_06117_amd import workloads as W
    shape = (size,) * 3
    dev = torch.device("cuda:0")
    phi0 = W.random_gaussians_torch(shape, 8, 2000, dev)
    u = W.abc_velocity_torch(shape, dev)
    dx = (2 * math.pi / size,) * 3
    dt = W.abc_dt(shape, cfl)
    rows = []
    for name in ("fec", "bec"):
        res, ms = {}, {}
        for ek in (3, 2):
            ctx.set_option(native.OPT_EC_KERNEL, ek)
            try:
                phi = phi0.clone()
                wall, _, _ = timed_steps(ctx, phi, u, dx, dt, steps, 2, native.SCHEMES[name])
            finally:
                ctx.set_option(native.OPT_EC_KERNEL, 3)
            res[ek] = phi
            ms[ek] = wall * 1e3 / steps
        rows.append({"scheme": name, "ms_per_step_march": ms[3], "ms_per_step_chain": ms[2],
                     "speedup": ms[2] / ms[3], "value_march": size**3 / ms[3] / 1e6,
                     "unit": "Gcell-updates/s", "same_bits": bool(torch.equal(res[2], res[3]))})
        del res
    del phi0, u
    torch.cuda.empty_cache()
    return {"workload": f"unsplit FEC and BEC, {size}^3, 8 Gaussians, ABC velocity, CFL {cfl}, "
                        f"{steps} steps each (after 2 warm-up steps)", "runs": rows}


def norms_section(ctx, size, reps):
    """The FP64 reductions (relative L2, max error, sums) of two FP32 fields
    of size^3: 8 B per element pair read; each call ends with the five
    results copied to the host."""
    import numpy as np
    import torch
    from paper_1606_06117_amd import workloads as W
    shape = (size,) * 3
    dev = torch.device("cuda:0")
    a = W.random_gaussians_torch(shape, 8, 2000, dev)
    b = a * 1.0001
    ctx.norms(a, b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.norms(a, b)
    wall = (time.perf_counter() - t0) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"workload": f"sla_norms on two FP32 {size}^3 fields, {reps} calls", "ms_per_call": wall * 1e3,
            "GB_per_s": 8 * size**3 / wall / 1e9, "hbm_frac": 8 * size**3 / wall / (HBM_PEAK_GBS * 1e9)}


def large_section(ctx, size, cfl, steps):
    """One large problem: a k^-5/3 field (|k| <= 64) on size^3 with the ABC
    velocity at CFL ``cfl``, built on the GPU."""
    import torch
    from paper_1606_06117_amd import workloads as W
    shape = (size,) * 3
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    phi = W.power_law_torch(shape, 5000, dev)
    u = W.abc_velocity_torch(shape, dev)
    torch.cuda.synchronize()
    build = time.perf_counter() - t0
    dx = (2 * math.pi / size,) * 3
    wall, times, cmax = timed_steps(ctx, phi, u, dx, W.abc_dt(shape, cfl), steps, 1)
    upd = size**3 * steps
    del phi, u
    torch.cuda.empty_cache()
    return {"workload": f"third order, {size}^3 FP32, k^-5/3 field (|k| <= 64), ABC velocity, CFL {cfl}, "
                        f"{steps} steps", "value": upd / wall / 1e9, "unit": "Gcell-updates/s",
            "ms_per_step": wall * 1e3 / steps, "courant_max": cmax,
            "hbm_frac_step": 20 * upd / wall / (HBM_PEAK_GBS * 1e9),
            "per_kind_ms": {k: round(v[1] / v[0], 4) for k, v in times.items()},
            "input_build_seconds": build,
            "learned_variant": "not run: the network reads the CIR field's 3x3x3 neighbourhood, "
                               "which holds the third-order stencil only at reach 1 (CFL < 1); "
                               "at CFL 2.0 (reach 3) the learned step falls back to the plain "
                               "third-order scheme by design, so its time would be this one"}


def batch_section(ctx, size, scalars, ngrids, steps):
    """Batched workload: ``scalars`` fields on a size^3 grid sharing one ABC
    velocity, plus ``ngrids`` cubic grids of uneven sizes 32^3..192^3 with
    their own uniform velocities, all at CFL 0.9, advanced by ``steps``
    third-order steps as one tuned plan (one graph launch)."""
    import torch
    from paper_1606_06117_amd import native
    from paper_1606_06117_amd import workloads as W
    dev = torch.device("cuda:0")
    shape = (size,) * 3
    dx = (2 * math.pi / size,) * 3
    dt = W.abc_dt(shape, 0.9)
    u = torch.from_numpy(W.abc_velocity(shape)).to(dev)
    probs = [(W.fourier_modes_torch(shape, 3000 + s, dev), u, dx, dt) for s in range(scalars)]
    sizes, vels = W.uneven_grids(count=ngrids)
    for gi, (n, v) in enumerate(zip(sizes, vels)):
        dxg = (2 * math.pi / n,) * 3
        dtg = 0.9 * dxg[0] / float(max(abs(v)))
        probs.append((W.fourier_modes_torch((n, n, n), 3200 + gi, dev), tuple(float(a) for a in v), dxg, dtg))
    cells_shared = scalars * size**3
    cells_uniform = sum(n**3 for n in sizes)
    t0 = time.perf_counter()
    plan = native.Plan(ctx, probs, steps, step0=0, courant_max=0.9, tune=True)
    setup = time.perf_counter() - t0
    plan.run()  # warm-up replay
    torch.cuda.synchronize()
    ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.run()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ctx.timing(False)
    ctx.check()
    updates = (cells_shared + cells_uniform) * steps
    # algorithmic bytes: shared fields read/write phi (8 B) and share one
    # read of the velocity (12 B per grid cell); uniform grids move phi only
    alg = steps * (cells_shared * 8 + size**3 * 12 + cells_uniform * 8)
    info = plan.info()
    plan.close()
    return {
        "workload": f"{scalars} scalars on {size}^3 sharing one ABC velocity + {ngrids} uniform-velocity "
                    f"grids of {min(sizes)}^3..{max(sizes)}^3 ({cells_uniform / 1e6:.0f} M cells), CFL 0.9, "
                    f"{steps} third-order steps in one graph launch",
        "value": updates / wall / 1e9,
        "unit": "Gcell-updates/s",
        "seconds": wall,
        "hbm_frac": alg / wall / (HBM_PEAK_GBS * 1e9),
        "algorithmic_bytes_per_cell_update": alg / updates,
        "plan": info,
        "plan_setup_seconds": setup,
    }


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--cfl", type=float, default=0.9)
    ap.add_argument("--scheme", default="cec", choices=["cir", "fec", "bec", "cec"])
    ap.add_argument("--cpu-edge", type=int, default=128, help="edge of the oracle's sample box")
    ap.add_argument("--cpu-steps", type=int, default=60, help="oracle steps on the sample box (about 13 s)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-workers", type=int, default=min(len(os.sched_getaffinity(0)), 16),
                    help="processes of the all-core oracle figure (0: skip it)")
    ap.add_argument("--cpu-all-steps", type=int, default=20,
                    help="oracle steps of the all-core figure on a --size x edge x edge box")
    ap.add_argument("--tune", choices=["on", "off"], default="on",
                    help="run the library's fused-step tuner on the workload before timing")
    ap.add_argument("--scheme-parity", choices=["on", "off"], default="on",
                    help="with the all-core oracle: every scheme's error against it on the whole "
                         "256^3 CFL 1.5 workload")
    ap.add_argument("--parity-steps", type=int, default=50)
    ap.add_argument("--path", choices=["auto", "sweeps"], default="auto",
                    help="auto: fused step where the library has one; sweeps: one kernel per axis")
    ap.add_argument("--other-cfl", choices=["on", "off"], default="on",
                    help="also time the headline workload at CFL 1.5 and 2.0 (10 steps each)")
    ap.add_argument("--large", choices=["on", "off"], default="on",
                    help="also time one 1024^3 problem at CFL 2.0 (10 steps)")
    ap.add_argument("--batch", choices=["on", "off"], default="on",
                    help="also run the batched workload (16 x 512^3 + 64 uneven grids)")
    ap.add_argument("--batch-scalars", type=int, default=16)
    ap.add_argument("--batch-grids", type=int, default=64)
    ap.add_argument("--learned", choices=["on", "off"], default="on",
                    help="also train and evaluate the learned correction (256^3)")
    ap.add_argument("--learned-size", type=int, default=256)
    ap.add_argument("--learned-fields", type=int, default=20)
    ap.add_argument("--learned-steps", type=int, default=100)
    ap.add_argument("--learned-cells", type=int, default=65536)
    ap.add_argument("--learned-iters", type=int, default=4000, help="Adam steps per training round")
    ap.add_argument("--learned-rounds", type=int, default=2,
                    help="rounds of pairs from the model's own rollouts after the first training")
    ap.add_argument("--probe", choices=["copy", "learned", "train"], default=None,
                    help="instead of the benchmark: copy, time a plain device copy of known size "
                         "(achievable bandwidth; calibrates HBM byte counters); learned, time the "
                         "learned step alone at --learned-size with random weights; train, time "
                         "training steps on 65 536 random feature rows")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(no sharding or collectives); run it with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if args.probe == "copy":
        return copy_probe(args.steps, args.warmup)
    if args.probe == "learned":
        return learned_probe(args.learned_size, args.steps, args.warmup)
    if args.probe == "train":
        return train_probe(65536, args.steps, args.warmup)

    sys.path.insert(0, ROOT)
    from paper_1606_06117_amd import native
    from paper_1606_06117_amd import workloads as W

    N = args.size
    shape = (N, N, N)
    print(f"[bench] building inputs {N}^3 ...", file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    phi_d = W.random_gaussians_torch(shape, 8, 2000, dev)  # random_gaussians' values
    # the host copy of the initial field feeds only the CPU oracle's sample
    phi0 = None if args.no_cpu_baseline else phi_d.cpu().numpy()
    u = W.abc_velocity(shape)
    dx = (2 * math.pi / N,) * 3
    dt = W.abc_dt(shape, args.cfl)
    scheme = native.SCHEMES[args.scheme]

    u_d = torch.from_numpy(u).to(dev)
    ctx = native.Context(0)
    cmax = ctx.courant_max(u_d, dx, dt)
    ctx.set_option(native.OPT_FUSED, 0 if args.path == "sweeps" else 1)
    tuned = None
    if args.scheme == "cec" and args.path == "auto" and cmax < 1.0 and args.tune == "on":
        # the library's tuner picks the fused-step implementation per parity
        print("[bench] tuning the fused step ...", file=sys.stderr, flush=True)
        tuned = ctx.tune(phi_d, u_d, dx, dt)

    for w in range(args.warmup):
        ctx.advect(phi_d, u_d, dx, dt, scheme, 1, step0=w, courant_max=cmax)
    ctx.check()
    torch.cuda.synchronize()

    print(f"[bench] timing {args.steps} steps ...", file=sys.stderr, flush=True)
    ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.advect(phi_d, u_d, dx, dt, scheme, args.steps, step0=args.warmup, courant_max=cmax)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    times = ctx.timing_read()
    ctx.timing(False)
    ctx.check()

    ncells = N**3
    value = ncells * args.steps / wall / 1e9
    ms_per_step = wall * 1e3 / args.steps
    step_bytes = algorithmic_bytes("cec3d", ncells, 3)  # per cell-update, whole step
    hbm_frac_step = step_bytes * args.steps / wall / (HBM_PEAK_GBS * 1e9)

    dom = max(times, key=lambda k: times[k][1])
    launches, total_ms = times[dom]
    avg_s = total_ms / launches / 1e3
    alg = algorithmic_bytes(dom, ncells, 3)
    achieved = alg / avg_s / 1e9
    workload = f"{args.scheme}-{N}^3-cfl{args.cfl}"
    traffic = measured_traffic(dom, workload)
    roofline = {
        "bound": "hbm",
        "kernel": dom,
        "achieved": achieved,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": achieved / HBM_PEAK_GBS,
        "traffic": traffic,
        "algorithmic_bytes_per_launch": alg,
        "avg_launch_ms": avg_s * 1e3,
        "launches": launches,
        "per_kind_ms": {k: round(v[1] / v[0], 4) for k, v in times.items()},
    }

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{'third-order (CEC)' if args.scheme == 'cec' else args.scheme.upper()} "
                        f"semi-Lagrangian advection, {N}^3 periodic FP32, 1 scalar (8 Gaussians), "
                        f"ABC(1,1,1) velocity, CFL {args.cfl}",
            "grid": [N, N, N],
            "scheme": args.scheme,
            "cfl": args.cfl,
            "scalars": 1,
            "path": args.path,
            "parallelism": "single GPU",
        },
        "hbm_frac_step": hbm_frac_step,
        "roofline": roofline,
        "tuned": tuned,
    }

    del phi_d, u_d
    torch.cuda.empty_cache()
    # secondary sections: a failure in one is recorded in its place (and its
    # traceback printed) so that the measured headline is still reported
    def section(key, msg, fn, *a):
        print(f"[bench] {msg} ...", file=sys.stderr, flush=True)
        try:
            out[key] = fn(*a)
        except Exception as exc:  # noqa: BLE001 - reported, not swallowed
            traceback.print_exc()
            out[key] = {"error": f"{type(exc).__name__}: {exc}"}

    if args.other_cfl == "on":
        section("other_cfl", "CFL 1.5 and 2.0", cfl_section, ctx, args.size, (1.5, 2.0), 10)
        section("strang", "Strang splitting at CFL 0.9 and 1.5", cfl_section, ctx, args.size,
                (0.9, 1.5), 10, native.CEC_STRANG, "third order with Strang splitting")
        section("schemes_256", "every scheme at 256^3, CFL 1.5", schemes_section, ctx, 256, 1.5, 10)
        section("ec_512", "unsplit FEC and BEC, march against chain", ec_section, ctx, args.size, 0.9, 10)
        section("norms_512", "FP64 reductions at 512^3", norms_section, ctx, 512, 20)
    if args.large == "on":
        section("large", "1024^3 at CFL 2.0", large_section, ctx, 1024, 2.0, 10)
    if args.batch == "on":
        section("batch", "batched workload", batch_section, ctx, args.size, args.batch_scalars,
                args.batch_grids, args.steps)
        torch.cuda.empty_cache()
    if args.learned == "on":
        section("learned", "learned correction: pairs, training, evaluation", learned_section, ctx,
                args.learned_size, args.learned_fields, args.learned_steps, args.learned_cells,
                args.learned_iters, 65536, 2e-3, args.learned_rounds)

    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle sample ...", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(phi0, u, dx, dt, scheme, args.cpu_edge, args.cpu_steps)
        if args.cpu_workers > 0:
            try:
                print(f"[bench] timing the CPU oracle on {args.cpu_workers} processes ...",
                      file=sys.stderr, flush=True)
                out["cpu_baseline"]["all_cores"] = cpu_all_cores(
                    phi0, u, dx, dt, scheme, args.cpu_edge, args.size, args.cpu_all_steps,
                    args.cpu_workers)
            except Exception as exc:  # noqa: BLE001 - reported, not swallowed
                traceback.print_exc()
                out["cpu_baseline"]["all_cores"] = {"error": f"{type(exc).__name__}: {exc}"}
        if args.cpu_workers > 0 and args.scheme_parity == "on":
            try:
                print(f"[bench] every scheme against the oracle at 256^3, CFL 1.5, "
                      f"{args.parity_steps} steps ...", file=sys.stderr, flush=True)
                out["cpu_baseline"]["scheme_parity_256"] = cpu_scheme_parity(
                    ctx, 256, 1.5, args.parity_steps, args.cpu_workers)
            except Exception as exc:  # noqa: BLE001 - reported, not swallowed
                traceback.print_exc()
                out["cpu_baseline"]["scheme_parity_256"] = {"error": f"{type(exc).__name__}: {exc}"}
    else:
        out["cpu_baseline"] = None

    print(json.dumps(out), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
