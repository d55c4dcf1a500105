"""sla_advect_noalloc: the work field in static device memory, nothing
allocated.  Its results equal sla_advect's bit for bit on two calls in a row
(the second on a smaller grid, so the array holds the first call's values
when it starts), for every scheme; a grid above the limit is refused before
any work; a captured call replays like the eager one."""

import warnings

import numpy as np
import pytest

from paper_1606_06117_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_06117_amd import native
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = native.Context(0)
    yield c
    c.close()


def case(shape, seed, cfl):
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = cfl * dx[0] / 2
    phi = W.random_gaussians(shape, 4, seed=seed).astype(np.float32)
    return phi, u, dx, dt


@pytest.mark.parametrize("scheme", range(8))
def test_noalloc_matches_advect_two_calls(ctx, scheme):
    import torch
    # the largest grid first (128 x 256 x 256 = 2^23 cells, the limit), then
    # smaller, ragged ones: odd nx (one node per lane) and even nx (the
    # two-node x+y kernel) at reach 2
    for shape, seed, cfl, steps, cm in [((128, 256, 256), 11, 0.9, 3, 0.9),
                                         ((20, 34, 45), 12, 1.7, 4, 0.0),
                                         ((20, 34, 46), 13, 1.7, 4, 0.0)]:
        phi, u, dx, dt = case(shape, seed, cfl)
        ud = torch.from_numpy(u).cuda()
        a = torch.from_numpy(phi).cuda()
        b = a.clone()
        ctx.advect(a, ud, dx, dt, scheme, steps, 1, cm)
        ctx.advect_noalloc(b, ud, dx, dt, scheme, steps, 1, cm)
        torch.cuda.synchronize()
        # the literal weights are NaN where |c| is whole (c = 0 at some nodes)
        assert torch.equal(torch.nan_to_num(a, nan=7.0), torch.nan_to_num(b, nan=7.0)), (scheme, shape)
        assert torch.equal(torch.isnan(a), torch.isnan(b)), (scheme, shape)
    ctx.check()


def test_noalloc_2d_and_limit(ctx):
    import torch
    from paper_1606_06117_amd import native
    shape = (40, 52)
    rng = np.random.default_rng(3)
    phi = rng.standard_normal(shape).astype(np.float32)
    u = torch.from_numpy(W.cellular_velocity_2d(shape)).cuda()
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    a = torch.from_numpy(phi).cuda()
    b = a.clone()
    ctx.advect(a, u, dx, 0.04, native.CEC, 5)
    ctx.advect_noalloc(b, u, dx, 0.04, native.CEC, 5)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    # one cell over the limit: refused, phi untouched
    big = (8, 8, native.NOALLOC_MAX_CELLS // 64 + 1)
    p = torch.full(big, 1.5, device="cuda")
    v = torch.zeros((3,) + big, device="cuda")
    with pytest.raises(native.SlaError) as ei:
        ctx.advect_noalloc(p, v, (0.1, 0.1, 0.1), 0.01, native.CEC, 1, 0, 0.5)
    assert ei.value.status == native.EINVAL
    assert bool((p == 1.5).all())
    ctx.check()


def test_noalloc_captured_replays(ctx):
    import torch
    from paper_1606_06117_amd import native
    phi, u, dx, dt = case((24, 40, 72), 13, 0.9)
    ud = torch.from_numpy(u).cuda()
    phi0 = torch.from_numpy(phi).cuda()
    static = phi0.clone()
    g = torch.cuda.CUDAGraph()
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        with torch.cuda.graph(g):
            ctx.advect_noalloc(static, ud, dx, dt, native.CEC, 3, 0, 0.9)
    torch.cuda.synchronize()
    assert torch.equal(static, phi0)
    expected = phi0.clone()
    for rep in range(3):
        g.replay()
        ctx.advect(expected, ud, dx, dt, native.CEC, 3, 0, 0.9)
        torch.cuda.synchronize()
        assert torch.equal(static, expected), rep
    ctx.check()
