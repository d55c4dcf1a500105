"""Unsplit FEC and BEC: the z-march, the LDS-tile kernel and the chain of
gather kernels.

All implementations perform the same FP32 operations per node, so they must
agree bit for bit (SLA_OPT_EC_KERNEL 0, 1, 2 and the default 3, which at
reach 1 in 3D runs the z-march), in 1D, 2D and 3D, below and above CFL 1,
on ragged grids; the chain is also held to the oracle with the per-step
bound of the other parity tests.
"""

import numpy as np
import pytest

import oracle
from paper_1606_06117_amd import workloads as W

from helpers import gpu_advect, oracle_advect, rel_l2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_06117_amd import native
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = native.Context(0)
    yield c
    c.close()


def _case(ndim, cfl):
    if ndim == 3:
        shape = (20, 27, 70)
        u = W.abc_velocity(shape)
        div = 2.0
    elif ndim == 2:
        shape = (29, 37)
        u = W.cellular_velocity_2d(shape)
        div = 1.0
    else:
        shape = (45,)
        u = np.full((1, 45), 1.0, dtype=np.float32)
        div = 1.0
    phi = W.random_gaussians(shape, 5, seed=51).astype(np.float32)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    return phi, u, dx, cfl * min(dx) / div


@pytest.mark.parametrize("scheme", [oracle.FEC, oracle.BEC])
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("cfl", [0.9, 2.5])
def test_chain_matches_fused(ctx, scheme, ndim, cfl):
    from paper_1606_06117_amd import native
    phi, u, dx, dt = _case(ndim, cfl)
    outs = []
    for ek in (0, 1, 2, 3):
        ctx.set_option(native.OPT_EC_KERNEL, ek)
        try:
            outs.append(gpu_advect(ctx, phi, u, dx, dt, scheme, 3, step0=1))
        finally:
            ctx.set_option(native.OPT_EC_KERNEL, 3)
    for o in outs[1:]:
        assert np.array_equal(outs[0], o)
    ref = oracle_advect(phi, u, dx, dt, scheme, 3, step0=1)
    l2 = rel_l2(outs[1], ref)
    print(f"scheme {scheme} {ndim}D cfl={cfl}: relL2 vs oracle {l2:.2e}")
    assert l2 <= 1e-5 * 3


@pytest.mark.parametrize("scheme", [oracle.FEC, oracle.BEC])
@pytest.mark.parametrize("shape", [(40, 48, 72), (37, 45, 130), (13, 11, 250), (11, 13, 9),
                                   (150, 20, 64)])
@pytest.mark.parametrize("launch", [0, -16, 1])
def test_march_matches_chain(ctx, scheme, shape, launch):
    """The one-pass z-march (reach 1, 3D) against the chain, bit for bit:
    partial x windows and row groups, windows past the row's end, rows
    narrower than a window; persistent workgroups whose plane ranges cross
    from one group into the next (0, 1 per CU) and march chunks (-16)."""
    from paper_1606_06117_amd import native
    phi = W.random_gaussians(shape, 5, seed=52).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * min(dx) / 2.0
    outs = []
    for ek in (2, 3):
        ctx.set_option(native.OPT_EC_KERNEL, ek)
        ctx.set_option(native.OPT_EC_SHAPE, launch)
        try:
            outs.append(gpu_advect(ctx, phi, u, dx, dt, scheme, 2, step0=0))
        finally:
            ctx.set_option(native.OPT_EC_KERNEL, 3)
            ctx.set_option(native.OPT_EC_SHAPE, 0)
    assert np.array_equal(outs[0], outs[1])
