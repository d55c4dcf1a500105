"""Batched plans: every problem of a batched, graph-replayed run equals its
standalone third-order run bit for bit (fields sharing a velocity and
uniform-velocity grids of uneven sizes together), and both match the
oracle."""

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


def make_batch(seed=0):
    """3 fields sharing one ABC velocity + 4 uneven grids with uniform velocity."""
    import torch
    shared_shape = (36, 40, 72)
    u = W.abc_velocity(shared_shape)
    dx_s = tuple(2 * np.pi / n for n in reversed(shared_shape))
    dt_s = 0.9 * dx_s[0] / 2
    probs, host = [], []
    ut = torch.from_numpy(u).cuda()
    for k in range(3):
        f = W.random_gaussians(shared_shape, 4, seed=seed + k).astype(np.float32)
        host.append((f, u, dx_s, dt_s))
        probs.append((torch.from_numpy(f).cuda(), ut, dx_s, dt_s))
    rng = np.random.default_rng(seed + 50)
    for shape in [(20, 24, 33), (9, 40, 17), (32, 32, 32), (13, 11, 70)]:
        vel = rng.uniform(-1.0, 1.0, 3).astype(np.float32)
        dx = tuple(2 * np.pi / n for n in reversed(shape))
        dt = 0.9 * min(dx) / float(np.max(np.abs(vel)))
        f = rng.standard_normal(shape).astype(np.float32)
        host.append((f, W.uniform_velocity(shape, vel), dx, dt))
        probs.append((torch.from_numpy(f).cuda(), tuple(float(v) for v in vel), dx, dt))
    return probs, host


@pytest.mark.parametrize("steps,tune", [(3, False), (2, True)])
def test_plan_matches_standalone_bitwise(ctx, steps, tune):
    import torch
    from paper_1606_06117_amd import native
    probs, host = make_batch()
    plan = native.Plan(ctx, probs, steps, step0=0, tune=tune)
    info = plan.info()
    print("plan", info)
    plan.run()
    torch.cuda.synchronize()
    ctx.check()
    for (phi_d, _, dx, dt), (f, u, _, _) in zip(probs, host):
        got = phi_d.cpu().numpy().astype(np.float64)
        ref = gpu_advect(ctx, f, u, dx, dt, oracle.CEC, steps, step0=0)
        assert np.array_equal(got, ref)
        o = oracle_advect(f, u, dx, dt, oracle.CEC, steps)
        assert rel_l2(got, o) < 1e-5 * steps
    plan.close()


def test_plan_replays(ctx):
    """Replays continue the run (even step count keeps the sweep parity);
    eager work between replays does not disturb them."""
    import torch
    from paper_1606_06117_amd import native
    probs, host = make_batch(seed=7)
    plan = native.Plan(ctx, probs, 2, step0=0, tune=False)
    for rep in range(1, 4):
        plan.run()
        ctx.norms(probs[0][0], probs[1][0])  # eager work between replays
        torch.cuda.synchronize()
        for (phi_d, _, dx, dt), (f, u, _, _) in zip(probs, host):
            ref = gpu_advect(ctx, f, u, dx, dt, oracle.CEC, 2 * rep, step0=0)
            assert np.array_equal(phi_d.cpu().numpy().astype(np.float64), ref), rep
    plan.close()


def test_plan_rejects_large_courant(ctx):
    import torch
    from paper_1606_06117_amd import native
    shape = (16, 16, 16)
    phi = torch.zeros(shape, device="cuda")
    with pytest.raises(native.SlaError) as ei:
        native.Plan(ctx, [(phi, (1.5, 0.0, 0.0), (1.0, 1.0, 1.0), 1.0)], 2)
    assert ei.value.status == native.ECOURANT


def test_plan_with_large_problems(ctx):
    """Problems of at least 2^24 cells with their own velocity run their own
    fused-step launches inside the plan's graph, next to the persistent
    kernel's tiles of the small ones; every result still equals its
    standalone run bit for bit (odd step count: the copy back included)."""
    import torch
    from paper_1606_06117_amd import native
    shape = (256, 256, 256)
    dev = torch.device("cuda:0")
    u = W.abc_velocity_torch(shape, dev)
    dx = (2 * np.pi / 256,) * 3
    dt = W.abc_dt(shape, 0.9)
    big = [W.fourier_modes_torch(shape, 40 + k, dev) for k in range(3)]
    probs, small = [], []
    for f in big:
        probs.append((f.clone(), u, dx, dt))
    rng = np.random.default_rng(3)
    for sh in [(20, 24, 33), (32, 32, 32)]:
        vel = rng.uniform(-1.0, 1.0, 3).astype(np.float32)
        dxs = tuple(2 * np.pi / n for n in reversed(sh))
        dts = 0.9 * min(dxs) / float(np.max(np.abs(vel)))
        f = rng.standard_normal(sh).astype(np.float32)
        small.append((f, W.uniform_velocity(sh, vel), dxs, dts))
        probs.append((torch.from_numpy(f).cuda(), tuple(float(v) for v in vel), dxs, dts))
    steps = 3
    plan = native.Plan(ctx, probs, steps, step0=0, tune=True)
    info = plan.info()
    print("plan", info)
    plan.run()
    torch.cuda.synchronize()
    ctx.check()
    for k, f in enumerate(big):
        ref = f.clone()
        ctx.advect(ref, u, dx, dt, native.CEC, steps, 0, 0.0)
        torch.cuda.synchronize()
        assert torch.equal(probs[k][0], ref), k
    for (phi_d, _, dxs, dts), (f, uu, _, _) in zip(probs[3:], small):
        ref = gpu_advect(ctx, f, uu, dxs, dts, oracle.CEC, steps, step0=0)
        assert np.array_equal(phi_d.cpu().numpy().astype(np.float64), ref)
    plan.close()


def test_plan_batch_workload_sample(ctx):
    """A sample of the batched workload at its full sizes: two of the 512^3
    fields sharing the ABC velocity (8 Fourier modes per axis, seeds 3000 and
    3001) and the first six of the 64 uneven uniform-velocity grids (sizes
    seed 3100, velocities seed 3101, fields seeds 3200..), CFL 0.9, three
    third-order steps in one graph.  Each problem equals its standalone run
    bit for bit; sampled boxes of the large fields match the oracle."""
    import torch
    from paper_1606_06117_amd import native
    from helpers import box_parity
    shape = (512, 512, 512)
    dev = torch.device("cuda:0")
    u = W.abc_velocity_torch(shape, dev)
    dx = (2 * np.pi / 512,) * 3
    dt = W.abc_dt(shape, 0.9)
    big = [W.fourier_modes_torch(shape, 3000 + k, dev) for k in range(2)]
    probs = [(f.clone(), u, dx, dt) for f in big]
    sizes, vels = W.uneven_grids()
    small = []
    for j in range(6):
        n = int(sizes[j])
        sh = (n, n, n)
        vel = vels[j].astype(np.float32)
        dxs = (2 * np.pi / n,) * 3
        dts = 0.9 * dxs[0] / float(np.max(np.abs(vel)))
        f = W.fourier_modes(sh, 3200 + j)
        small.append((f, W.uniform_velocity(sh, vel), dxs, dts))
        probs.append((torch.from_numpy(f).cuda(), tuple(float(v) for v in vel), dxs, dts))
    steps = 3
    plan = native.Plan(ctx, probs, steps, step0=0, tune=False)
    print("plan", plan.info())
    plan.run()
    torch.cuda.synchronize()
    ctx.check()
    for k, f in enumerate(big):
        ref = f.clone()
        ctx.advect(ref, u, dx, dt, native.CEC, steps, 0, 0.9)
        torch.cuda.synchronize()
        assert torch.equal(probs[k][0], ref), k
    for (phi_d, _, dxs, dts), (f, uu, _, _) in zip(probs[2:], small):
        ref = gpu_advect(ctx, f, uu, dxs, dts, oracle.CEC, steps, step0=0)
        assert np.array_equal(phi_d.cpu().numpy().astype(np.float64), ref)
    # the large fields against the oracle on two boxes each (exact halos)
    uh = u.cpu().numpy()
    for k, f in enumerate(big):
        l2, linf = box_parity(probs[k][0].cpu().numpy().astype(np.float64), f.cpu().numpy(), uh, dx,
                              dt, oracle.CEC, steps, steps * 3, (16, 16, 16),
                              np.random.default_rng(20 + k), 2)
        print(f"512^3 field {k} boxes relL2={l2:.3e} Linf={linf:.3e}")
        assert l2 <= 1e-5 * steps and linf <= 1e-5 * steps
    plan.close()
    del probs, big, u
    torch.cuda.empty_cache()
