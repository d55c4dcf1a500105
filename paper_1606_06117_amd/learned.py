"""Learned correction driver: training pairs, training and evaluation.

Every step of the method runs in the library's kernels through
``native``; this module only sequences calls and keeps bookkeeping.

Workload.  Steady ABC flow (A = B = C = 1) on [0, 2 pi)^3 whose amplitude is
modulated in time by a_m = sin(2 pi (m + 1/2) / P) at step m (P = 100 steps
per period): step m advects with the same velocity field over the signed
time step a_m * dt.  Over a whole period the modulation sums to zero, so the
exact solution returns to the initial field after every period.

* ``generate_pairs``: for each initial field (8 random Gaussians) and each
  step, the CIR step and the third-order step of the current field; training
  pairs are sampled at random nodes (features of the CIR field, target the
  third-order correction).  The trajectory continues with the third-order
  field, or, given a model, with the learned step, so that the pairs cover
  the states the learned scheme itself visits.
* ``train``: Adam on minibatches of the pairs.
* ``train_rollout``: ``train``, then rounds of pairs from the current
  model's own trajectories added to the set and training continued
  (dataset aggregation: a network trained only on third-order trajectories
  meets states it never saw once its own small errors accumulate, and its
  rollout drifts).
* ``evaluate``: learned, third-order and CIR runs from the same field; per
  step the relative L2 distance of learned and CIR to the third-order run,
  the error against the exact field after whole periods, time per step.
"""

from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import native
from . import workloads as W

PERIOD = 100


def modulation(m: int, period: int = PERIOD) -> float:
    return math.sin(2.0 * math.pi * (m + 0.5) / period)


def init_params(seed: int) -> np.ndarray:
    """He-initialised weights (FP32 flat vector in the library's layout)."""
    rng = np.random.default_rng(seed)
    nf, nh = native.MLP_INPUTS, native.MLP_HIDDEN
    W1 = rng.normal(0.0, math.sqrt(2.0 / 30.0), (nf, nh))
    W1[30:] = 0.0  # the two padding inputs are always zero
    b1 = np.zeros(nh)
    W2 = rng.normal(0.0, math.sqrt(2.0 / nh), (nh, nh))
    b2 = np.zeros(nh)
    w3 = rng.normal(0.0, math.sqrt(1.0 / nh), nh) * 0.1
    b3 = np.zeros(1)
    return np.concatenate([W1.ravel(), b1, W2.ravel(), b2, w3, b3]).astype(np.float32)


@dataclass
class Pairs:
    feats: object   # torch int16 [m, 32] (BF16 bits)
    target: object  # torch float32 [m]
    sigma: object   # torch float32 [m]
    m: int
    seconds: float


def _hint(cfl: float, a: float) -> float:
    # bound on |c| for the modulated step (max |u_d| dt/dx = cfl at |a| = 1)
    return cfl * abs(a) * (1.0 + 1e-5) + 1e-12


def generate_pairs(ctx, shape, fields, steps_per_field, cells_per_snapshot, cfl, seed_cells,
                   period=PERIOD, model=None) -> Pairs:
    import torch
    N = shape[-1]
    dx = (2 * math.pi / N,) * 3
    dt = W.abc_dt(shape, cfl)
    u = torch.from_numpy(W.abc_velocity(shape)).cuda()
    total = len(fields) * steps_per_field * cells_per_snapshot
    feats = torch.empty((total, native.MLP_INPUTS), dtype=torch.int16, device="cuda")
    target = torch.empty(total, device="cuda")
    sigma = torch.empty(total, device="cuda")
    rng = np.random.default_rng(seed_cells)
    ncells = int(np.prod(shape))
    o = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for seed in fields:
        phi = W.random_gaussians_torch(shape, 8, seed, "cuda")
        for m in range(steps_per_field):
            a = modulation(m, period)
            phi1 = phi.clone()
            ctx.advect(phi1, u, dx, a * dt, native.CIR, 1, step0=m, courant_max=_hint(cfl, a))
            nxt = phi.clone()
            ctx.advect(nxt, u, dx, a * dt, native.CEC, 1, step0=m, courant_max=_hint(cfl, a))
            cells = torch.from_numpy(rng.integers(0, ncells, cells_per_snapshot).astype(np.int32)).cuda()
            k = cells_per_snapshot
            native.make_pairs(ctx, phi1, nxt, u, dx, a * dt, cells, feats[o:o + k], target[o:o + k],
                              sigma[o:o + k])
            o += k
            if model is None:
                phi = nxt
            else:
                native.advect_learned(ctx, model, phi, u, dx, a * dt, 1, step0=m,
                                      courant_max=_hint(cfl, a), allow_fallback=False)
    torch.cuda.synchronize()
    ctx.check()
    return Pairs(feats, target, sigma, total, time.perf_counter() - t0)


def concat(a: Pairs, b: Pairs) -> Pairs:
    import torch
    return Pairs(torch.cat([a.feats, b.feats]), torch.cat([a.target, b.target]),
                 torch.cat([a.sigma, b.sigma]), a.m + b.m, a.seconds + b.seconds)


def train(ctx, pairs: Pairs, iters: int, batch: int, lr: float, seed: int, cfl: float,
          log_every: int = 0, model=None):
    """Adam over shuffled minibatches; returns (model, loss history, seconds).
    A given model is trained further (its Adam state continues)."""
    import torch
    if model is None:
        model = native.Model(ctx)
        model.set_params(init_params(seed))
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    perm = torch.randperm(pairs.m, device="cuda", generator=gen)
    feats = pairs.feats[perm].contiguous()
    target = pairs.target[perm].contiguous()
    nb = max(1, pairs.m // batch)
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(iters):
        b = it % nb
        # cosine decay of the learning rate
        lr_it = lr * 0.5 * (1.0 + math.cos(math.pi * it / iters))
        want = log_every > 0 and (it % log_every == 0 or it == iters - 1)
        loss = model.train_step(feats[b * batch:(b + 1) * batch], target[b * batch:(b + 1) * batch],
                                lr_it, want_loss=want)
        if want:
            hist.append((it, loss))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    model.set_courant_range(cfl * (1.0 + 1e-4))
    return model, hist, secs


def train_rollout(ctx, shape, fields, steps_per_field, cells_per_snapshot, cfl, seed, rounds,
                  iters, batch, lr, log_every=0):
    """``train`` on third-order pairs, then ``rounds`` rounds that add pairs
    from the model's own trajectories (new initial fields each round) and
    continue training.  Returns (model, pairs, loss history per round,
    seconds spent making pairs, seconds spent training)."""
    pairs = generate_pairs(ctx, shape, fields, steps_per_field, cells_per_snapshot, cfl,
                           seed_cells=seed)
    model, hist, tsec = train(ctx, pairs, iters, batch, lr, seed + 1, cfl, log_every)
    hists = [hist]
    psec = pairs.seconds
    for r in range(rounds):
        new_fields = [f + 1000 * (r + 1) for f in fields]
        more = generate_pairs(ctx, shape, new_fields, steps_per_field, cells_per_snapshot, cfl,
                              seed_cells=seed + 10 * (r + 1), model=model)
        psec += more.seconds
        pairs = concat(pairs, more)
        model, hist, t = train(ctx, pairs, iters, batch, lr, seed + 2 + r, cfl, log_every, model=model)
        hists.append(hist)
        tsec += t
    return model, pairs, hists, psec, tsec


def evaluate(ctx, model, shape, seed, periods, cfl, period=PERIOD):
    """Learned vs third-order vs CIR over ``periods`` modulation periods."""
    import torch
    N = shape[-1]
    dx = (2 * math.pi / N,) * 3
    dt = W.abc_dt(shape, cfl)
    u = torch.from_numpy(W.abc_velocity(shape)).cuda()
    phi0 = W.random_gaussians_torch(shape, 8, seed, "cuda")
    runs = {"cec": phi0.clone(), "learned": phi0.clone(), "cir": phi0.clone()}
    times = {k: 0.0 for k in runs}
    per_step = []
    vs_exact = []
    fell_back = False
    steps = periods * period
    for m in range(steps):
        a = modulation(m, period)
        h = _hint(cfl, a)
        for name, phi in runs.items():
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if name == "learned":
                fell_back |= native.advect_learned(ctx, model, phi, u, dx, a * dt, 1, step0=m,
                                                   courant_max=h)
            else:
                ctx.advect(phi, u, dx, a * dt, native.CEC if name == "cec" else native.CIR, 1,
                           step0=m, courant_max=h)
            torch.cuda.synchronize()
            times[name] += time.perf_counter() - t0
        nl = ctx.norms(runs["learned"], runs["cec"])
        nc = ctx.norms(runs["cir"], runs["cec"])
        per_step.append((m + 1, math.sqrt(nl[0] / nl[1]), math.sqrt(nc[0] / nc[1])))
        if (m + 1) % period == 0:
            row = {"step": m + 1}
            for name, phi in runs.items():
                s = ctx.norms(phi, phi0)
                row[name] = math.sqrt(s[0] / s[1])
            vs_exact.append(row)
    ctx.check()
    return {
        "per_step": per_step,
        "vs_exact": vs_exact,
        "ms_per_step": {k: 1e3 * v / steps for k, v in times.items()},
        "fell_back": fell_back,
    }


def error_at_cfl(ctx, shape, seed, cfl, steps_per_period, periods, learned_model=None,
                 fallbacks=None):
    """Error vs the exact field after ``periods`` periods when a period takes
    ``steps_per_period`` steps (so the Courant number is cfl*100/steps_per_period).
    With a learned model, the number of steps that fell back to the plain
    scheme is appended to ``fallbacks`` (a list) when one is given."""
    import torch
    N = shape[-1]
    dx = (2 * math.pi / N,) * 3
    c = cfl * PERIOD / steps_per_period
    dt = W.abc_dt(shape, c)
    u = torch.from_numpy(W.abc_velocity(shape)).cuda()
    phi0 = W.random_gaussians_torch(shape, 8, seed, "cuda")
    phi = phi0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fell = 0
    for m in range(periods * steps_per_period):
        a = modulation(m, steps_per_period)
        if learned_model is not None:
            fell += native.advect_learned(ctx, learned_model, phi, u, dx, a * dt, 1, step0=m,
                                          courant_max=_hint(c, a))
        else:
            ctx.advect(phi, u, dx, a * dt, native.CEC, 1, step0=m, courant_max=_hint(c, a))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    if fallbacks is not None:
        fallbacks.append(fell)
    s = ctx.norms(phi, phi0)
    return math.sqrt(s[0] / s[1]), secs


def error_at_resolution(ctx, n, ref_n, seed, cfl, periods, period=PERIOD):
    """Plain third-order error against the exact field after ``periods``
    periods on an n^3 grid, with the physical time step of the ref_n^3 run at
    ``cfl`` at peak amplitude: the same physical problem (field, flow, time
    step) resolved with fewer or more cells.  Returns (error, seconds)."""
    import torch
    shape = (n, n, n)
    dx = (2 * math.pi / n,) * 3
    dt = W.abc_dt((ref_n,) * 3, cfl)
    c = cfl * n / ref_n  # the Courant number on this grid
    u = torch.from_numpy(W.abc_velocity(shape)).cuda()
    phi0 = W.random_gaussians_torch(shape, 8, seed, "cuda")
    phi = phi0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m in range(periods * period):
        a = modulation(m, period)
        ctx.advect(phi, u, dx, a * dt, native.CEC, 1, step0=m, courant_max=_hint(c, a))
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    s = ctx.norms(phi, phi0)
    return math.sqrt(s[0] / s[1]), secs


def equal_error_speedup(points_plain, point_learned):
    """Cost of the plain scheme at the learned error, by log-log interpolation
    of its (error, seconds) points; None when the learned error is outside
    the plain curve."""
    e_l, t_l = point_learned
    pts = sorted(points_plain)
    for (e0, t0), (e1, t1) in zip(pts, pts[1:]):
        if e0 <= e_l <= e1 and e0 > 0 and e1 > e0:
            w = (math.log(e_l) - math.log(e0)) / (math.log(e1) - math.log(e0))
            t = math.exp(math.log(t0) + w * (math.log(t1) - math.log(t0)))
            return t / t_l
    return None
