"""Unsplit FEC and BEC: the fused kernel and the chain of gather kernels.

Both implementations perform the same FP32 operations per node, so they must
agree bit for bit (SLA_OPT_EC_KERNEL 0, 1 and the default 2), in 1D, 2D and
3D, below and above CFL 1, on ragged grids; the chain is also held to the
oracle with the per-step bound of the other parity tests.
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
    for ek in (0, 1, 2):
        ctx.set_option(native.OPT_EC_KERNEL, ek)
        try:
            outs.append(gpu_advect(ctx, phi, u, dx, dt, scheme, 3, step0=1))
        finally:
            ctx.set_option(native.OPT_EC_KERNEL, 2)
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[1], outs[2])
    ref = oracle_advect(phi, u, dx, dt, scheme, 3, step0=1)
    l2 = rel_l2(outs[1], ref)
    print(f"scheme {scheme} {ndim}D cfl={cfl}: relL2 vs oracle {l2:.2e}")
    assert l2 <= 1e-5 * 3
