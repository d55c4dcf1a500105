"""The convenience entry points: several fields sharing a velocity, a batch
of independent problems of any scheme, and a caller-owned workspace.  Every
result equals the standalone sla_advect run bit for bit."""

import warnings

import numpy as np
import pytest

import oracle
from paper_1606_06117_amd import workloads as W

from helpers import gpu_advect

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_06117_amd import native
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = native.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("cfl", [0.9, 1.5])
def test_multi_matches_single_fields(ctx, cfl):
    import torch
    from paper_1606_06117_amd import native
    shape = (24, 40, 72)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = cfl * dx[0] / 2
    fields = [W.random_gaussians(shape, 4, seed=60 + k).astype(np.float32) for k in range(3)]
    dev = [torch.from_numpy(f).cuda() for f in fields]
    ctx.advect_multi(dev, torch.from_numpy(u).cuda(), dx, dt, native.CEC, 3, step0=1)
    torch.cuda.synchronize()
    ctx.check()
    for f, d in zip(fields, dev):
        ref = gpu_advect(ctx, f, u, dx, dt, oracle.CEC, 3, step0=1)
        assert np.array_equal(d.cpu().numpy().astype(np.float64), ref)


@pytest.mark.parametrize("shape,nf,steps,step0", [((24, 40, 72), 7, 3, 0), ((37, 45, 130), 4, 2, 1),
                                                 ((11, 13, 9), 5, 3, 1), ((40, 48, 250), 2, 4, 0)])
def test_shared_velocity_groups_match_single_fields(ctx, shape, nf, steps, step0):
    """Third order at reach 1 runs the fields four (then two, then one) at a
    time through the fused kernel that loads the shared velocity once per
    tile; every field equals its standalone run bit for bit.  The shapes
    leave partial x windows, row groups and march chunks, rows narrower than
    a window, and windows past the row's end."""
    import torch
    from paper_1606_06117_amd import native
    u = torch.from_numpy(W.abc_velocity(shape)).cuda()
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    fields = [W.random_gaussians(shape, 3, seed=90 + k).astype(np.float32) for k in range(nf)]
    dev = [torch.from_numpy(f).cuda() for f in fields]
    ctx.advect_multi(dev, u, dx, dt, native.CEC, steps, step0=step0)
    torch.cuda.synchronize()
    ctx.check()
    for f, d in zip(fields, dev):
        p = torch.from_numpy(f).cuda()
        ctx.advect(p, u, dx, dt, native.CEC, steps, step0)
        torch.cuda.synchronize()
        assert torch.equal(d, p)


def test_shared_velocity_with_small_workspace(ctx):
    """A caller workspace of two fields runs the shared-velocity groups two
    at a time; one of one field, one at a time; same bits either way."""
    import torch
    from paper_1606_06117_amd import native
    shape = (20, 34, 70)
    u = torch.from_numpy(W.abc_velocity(shape)).cuda()
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.8 * dx[0] / 2
    fields = [W.random_gaussians(shape, 3, seed=120 + k).astype(np.float32) for k in range(5)]
    ref = []
    for f in fields:
        p = torch.from_numpy(f).cuda()
        ctx.advect(p, u, dx, dt, native.CEC, 3)
        ref.append(p)
    n = int(np.prod(shape))
    for nfield in (2, 1):
        buf = torch.empty(nfield * n, device="cuda")
        ctx.set_workspace(buf)
        try:
            dev = [torch.from_numpy(f).cuda() for f in fields]
            ctx.advect_multi(dev, u, dx, dt, native.CEC, 3)
            torch.cuda.synchronize()
        finally:
            ctx.set_workspace(None)
        for d, r in zip(dev, ref):
            assert torch.equal(d, r)
    ctx.check()


def batch_problems(seed, cfl):
    """Two 3D problems with velocity fields, a 3D and a 2D uniform one."""
    rng = np.random.default_rng(seed)
    out = []
    for shape in [(20, 24, 40), (16, 30, 33)]:
        u = W.abc_velocity(shape)
        dx = tuple(2 * np.pi / n for n in reversed(shape))
        out.append((rng.standard_normal(shape).astype(np.float32), u, dx, cfl * min(dx) / 2))
    for shape in [(12, 17, 19), (26, 35)]:
        vel = rng.uniform(-1.0, 1.0, len(shape)).astype(np.float32)
        dx = tuple(2 * np.pi / n for n in reversed(shape))
        out.append((rng.standard_normal(shape).astype(np.float32), tuple(float(v) for v in vel), dx,
                    cfl * min(dx) / float(np.max(np.abs(vel)))))
    return out


@pytest.mark.parametrize("scheme,cfl", [("cec", 0.9), ("cec", 1.5), ("fec", 0.9), ("bec", 1.3),
                                        ("cir", 2.2)])
def test_batch_matches_single_problems(ctx, scheme, cfl):
    """CEC below CFL 1 with only 3D problems runs a plan; the 2D problem
    here sends every case through the per-problem path, so the plan is also
    checked on the 3D problems alone."""
    import torch
    from paper_1606_06117_amd import native
    probs = batch_problems(5, cfl)
    sch = native.SCHEMES[scheme]
    for subset in (probs, [p for p in probs if p[0].ndim == 3]):
        dev = [(torch.from_numpy(f).cuda(), u if isinstance(u, tuple) else torch.from_numpy(u).cuda(), dx,
                dt) for f, u, dx, dt in subset]
        ctx.advect_batch(dev, sch, 3, step0=0)
        torch.cuda.synchronize()
        ctx.check()
        for (d, _, _, _), (f, u, dx, dt) in zip(dev, subset):
            uf = W.uniform_velocity(f.shape, np.array(u, np.float32)) if isinstance(u, tuple) else u
            ref = gpu_advect(ctx, f, uf, dx, dt, sch, 3, step0=0)
            assert np.array_equal(d.cpu().numpy().astype(np.float64), ref), (scheme, f.shape)


def test_caller_workspace(ctx):
    """A caller-owned workspace of exactly sla_workspace_size bytes gives the
    same bits; one float short is rejected; None returns to library memory."""
    import torch
    from paper_1606_06117_amd import native
    shape = (24, 40, 72)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 1.5 * dx[0] / 2
    f = W.random_gaussians(shape, 4, seed=70).astype(np.float32)
    ref = gpu_advect(ctx, f, u, dx, dt, oracle.CEC, 3)
    nbytes = ctx.workspace_size(shape, dx, native.CEC)
    assert nbytes == 4 * int(np.prod(shape))
    buf = torch.empty(nbytes // 4, device="cuda")
    ud = torch.from_numpy(u).cuda()
    try:
        ctx.set_workspace(buf)
        p = torch.from_numpy(f).cuda()
        ctx.advect(p, ud, dx, dt, native.CEC, 3)
        torch.cuda.synchronize()
        ctx.check()
        assert np.array_equal(p.cpu().numpy().astype(np.float64), ref)
        ctx.set_workspace(buf[:-1])
        with pytest.raises(native.SlaError) as ei:
            ctx.advect(torch.from_numpy(f).cuda(), ud, dx, dt, native.CEC, 1)
        assert ei.value.status == native.EINVAL
    finally:
        ctx.set_workspace(None)
    p = torch.from_numpy(f).cuda()
    ctx.advect(p, ud, dx, dt, native.CEC, 3)
    torch.cuda.synchronize()
    assert np.array_equal(p.cpu().numpy().astype(np.float64), ref)


def test_graph_capture_and_replays(ctx):
    """Two third-order steps (courant_max given, work memory already there)
    captured into a graph: every replay, with eager runs and synchronisations
    between replays, equals the eager result bitwise.  A call that would
    measure the Courant bound while the stream is captured is refused."""
    import torch
    from paper_1606_06117_amd import native
    shape = (24, 40, 72)
    u = torch.from_numpy(W.abc_velocity(shape)).cuda()
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    phi0 = torch.from_numpy(W.random_gaussians(shape, 4, seed=80).astype(np.float32)).cuda()
    warm = phi0.clone()
    ctx.advect(warm, u, dx, dt, native.CEC, 2, 0, 0.9)  # allocates the work memory
    torch.cuda.synchronize()
    static = phi0.clone()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.advect(static, u, dx, dt, native.CEC, 2, 0, 0.9)
    torch.cuda.synchronize()
    assert torch.equal(static, phi0)  # capturing ran nothing
    expected = phi0.clone()
    for rep in range(3):
        g.replay()
        ctx.advect(expected, u, dx, dt, native.CEC, 2, 0, 0.9)  # eager, between replays
        torch.cuda.synchronize()
        assert torch.equal(static, expected), rep
    g2 = torch.cuda.CUDAGraph()
    other = phi0.clone()
    with pytest.raises(native.SlaError) as ei, warnings.catch_warnings():
        warnings.simplefilter("ignore")  # the refused capture leaves an empty graph
        with torch.cuda.graph(g2):
            ctx.advect(other, u, dx, dt, native.CEC, 1)  # would measure the bound
    assert ei.value.status == native.ECAPTURE
    torch.cuda.synchronize()
    # the learned step would measure the bound; a plan allocates and synchronises
    model = native.Model(ctx)
    refused = [
        lambda: native.advect_learned(ctx, model, other, u, dx, dt, 1),
        lambda: native.Plan(ctx, [(other, u, dx, dt)], 1, tune=False),
    ]
    for call in refused:
        g3 = torch.cuda.CUDAGraph()
        with pytest.raises(native.SlaError) as ei, warnings.catch_warnings():
            warnings.simplefilter("ignore")
            with torch.cuda.graph(g3):
                call()
        assert ei.value.status == native.ECAPTURE
        torch.cuda.synchronize()
    model.close()
    assert torch.equal(other, phi0)
    ctx.check()


def test_empty_calls_are_no_ops(ctx):
    """Zero fields, zero problems and zero steps succeed without touching memory."""
    import ctypes
    import torch
    from paper_1606_06117_amd import native
    lib = native.load()
    shape = (16, 16, 16)
    g = native.make_grid(shape, (0.1, 0.1, 0.1))
    u = torch.zeros((3,) + shape, device="cuda")
    phi = torch.full(shape, 2.5, device="cuda")
    assert lib.sla_advect_multi(ctx.h, ctypes.byref(g), 0, None, ctypes.c_void_p(u.data_ptr()), 0.01,
                                native.CEC, 3, 0, 0.0) == native.OK
    assert lib.sla_advect_batch(ctx.h, 0, None, native.CEC, 3, 0, 0.0) == native.OK
    assert lib.sla_advect_batch(ctx.h, -1, None, native.CEC, 3, 0, 0.0) == native.EINVAL
    for scheme in range(7):
        ctx.advect(phi, u, (0.1, 0.1, 0.1), 0.01, scheme, 0)
    torch.cuda.synchronize()
    assert bool((phi == 2.5).all())
    ctx.check()
