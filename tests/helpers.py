"""Shared test helpers: GPU round trips through the C ABI and oracle boxes."""

from __future__ import annotations

import math

import numpy as np

import oracle
from oracle import characteristics as ch
from paper_1606_06117_amd import workloads as W


def gpu_advect(ctx, phi, u, dx, dt, scheme, steps, step0=0, courant_max=0.0):
    """Copy FP32 inputs to the GPU, advance through the C ABI, return FP64 numpy."""
    import torch
    p = torch.from_numpy(np.ascontiguousarray(phi, dtype=np.float32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(u, dtype=np.float32)).cuda()
    ctx.advect(p, v, dx, dt, scheme, steps, step0, courant_max)
    torch.cuda.synchronize()
    return p.cpu().numpy().astype(np.float64)


def oracle_advect(phi, u, dx, dt, scheme, steps, step0=0):
    return oracle.advect(np.asarray(phi, np.float32).astype(np.float64),
                         np.asarray(u, np.float32), dx, dt, scheme, steps, step0)


def rel_l2(x, ref):
    return oracle.rel_l2(x, ref)


def periodic_box(arr, lo, size, axes_offset=0):
    """Periodic sub-box of ``arr``: for each axis, indices lo[a] .. lo[a]+size[a]-1 mod n."""
    out = arr
    for a, (l, s) in enumerate(zip(lo, size)):
        ax = a + axes_offset
        idx = np.arange(l, l + s) % arr.shape[ax]
        out = np.take(out, idx, axis=ax)
    return out


def box_parity(gpu_out, phi0, u, dx, dt, scheme, steps, halo, inner, rng, nboxes, step0=0):
    """Compare ``gpu_out`` with the oracle on ``nboxes`` random inner boxes.

    The oracle runs on the inner box grown by ``halo`` cells per side (taken
    periodically from the full inputs); cells farther than ``halo`` from the
    box edge cannot feel the box's own wrap-around, so there the oracle's
    result is the full-grid result.  Returns the worst relative L2 and L-inf
    (relative to max |phi0|) over the boxes.
    """
    shape = phi0.shape
    worst_l2, worst_inf = 0.0, 0.0
    scale = float(np.max(np.abs(phi0)))
    for _ in range(nboxes):
        lo = [int(rng.integers(0, n)) for n in shape]
        big = [min(n, i + 2 * halo) for n, i in zip(shape, inner)]
        lo_big = [l - (b - i) // 2 for l, b, i in zip(lo, big, inner)]
        sub_phi = periodic_box(phi0, lo_big, big)
        sub_u = periodic_box(u, lo_big, big, axes_offset=1)
        ref = oracle.advect(sub_phi.astype(np.float64), sub_u, dx, dt, scheme, steps, step0)
        cut = tuple(slice((b - i) // 2, (b - i) // 2 + i) for b, i in zip(big, inner))
        ref_in = ref[cut]
        got_in = periodic_box(gpu_out, lo, inner)
        worst_l2 = max(worst_l2, rel_l2(got_in, ref_in))
        worst_inf = max(worst_inf, float(np.max(np.abs(got_in - ref_in))) / scale)
    return worst_l2, worst_inf


def reach(cfl):
    return int(math.floor(cfl)) + 1


PATCH_LO, PATCH_HI, PATCH_T, SWIRL_UMAX = (0.15, 0.55), (0.40, 0.80), 200.0, 0.0038538656


def patch_case(N, cfl=0.75):
    """The 2D patch test: a unit square patch, the swirl flow, T = 200, CFL
    0.75 (u_max = 0.00385); the exact field at the nodes by characteristics."""
    shape = (N, N)
    phi = W.square_patch(shape, PATCH_LO, PATCH_HI)
    u = W.swirl_velocity_2d(shape)
    steps = int(math.ceil(PATCH_T / (cfl / N / SWIRL_UMAX)))
    feet = np.mod(ch.foot(ch.node_points(shape, 1.0), ch.swirl(), PATCH_T, 200), 1.0)
    exact = W.square_patch_at(feet, PATCH_LO, PATCH_HI).reshape(shape)
    return phi, u, (1.0 / N, 1.0 / N), PATCH_T / steps, steps, exact
