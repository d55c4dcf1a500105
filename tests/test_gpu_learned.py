"""GPU tests of the learned correction: the matrix-core network against the
FP64 network oracle, the training pairs against the oracle's features, the
learned step, the fallback to the third-order scheme, and training.

Tolerances.  The GPU holds weights, features and hidden activations in
BF16 (8 significant bits, relative rounding up to 2^-9) and accumulates in
FP32; the oracle takes the same BF16 weights and features and computes in
FP64.  Two rounded activation layers leave a relative error of a few
2^-9 in y and in the gradients: the bound used is 3e-2 relative L2.
"""

import numpy as np
import pytest

import oracle
from oracle import mlp
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


def he_params(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = {
        "W1": rng.normal(0, scale * np.sqrt(2 / 30), (mlp.NF, mlp.NH)),
        "b1": rng.normal(0, 0.05, mlp.NH),
        "W2": rng.normal(0, scale * np.sqrt(2 / 64), (mlp.NH, mlp.NH)),
        "b2": rng.normal(0, 0.05, mlp.NH),
        "w3": rng.normal(0, scale * np.sqrt(1 / 64), mlp.NH),
        "b3": rng.normal(0, 0.05, 1),
    }
    p["W1"][30:] = 0.0
    return mlp.pack(p).astype(np.float32)


def bf16_bits(x):
    """FP32 array -> uint16 BF16 bit patterns (round to nearest even)."""
    r = mlp.bf16_round(x)
    return (r.view(np.uint32) >> 16).astype(np.uint16)


def rand_features(m, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(m, mlp.NF)).astype(np.float32)
    X[:, 27:30] = rng.uniform(-0.9, 0.9, (m, 3))
    X[:, 30:] = 0.0
    return mlp.bf16_round(X)


def rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def device(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.cuda()


def test_forward_matches_oracle(ctx):
    import torch
    from paper_1606_06117_amd import native
    model = native.Model(ctx)
    params = he_params(1)
    model.set_params(params)
    for m in (1000, 4096 + 17):
        X = rand_features(m, 2)
        y = torch.empty(m, device="cuda")
        model.forward(device(bf16_bits(X)), y)
        torch.cuda.synchronize()
        pr = mlp.unpack(mlp.bf16_round(params).astype(np.float64))
        ref, _ = mlp.forward(pr, X.astype(np.float64))
        err = rel(y.cpu().numpy().astype(np.float64), ref)
        print(f"forward m={m}: rel L2 {err:.3e}")
        assert err < 3e-2
    model.close()


def test_gradients_match_oracle(ctx):
    from paper_1606_06117_amd import native
    model = native.Model(ctx)
    params = he_params(3)
    model.set_params(params)
    m = 3000
    X = rand_features(m, 4)
    t = np.random.default_rng(5).normal(size=m).astype(np.float32)
    g, loss = model.grads(device(bf16_bits(X)), device(t))
    pr = mlp.unpack(mlp.bf16_round(params).astype(np.float64))
    y, cache = mlp.forward(pr, X.astype(np.float64))
    ref = mlp.backward(pr, cache, y, t.astype(np.float64))
    assert loss == pytest.approx(mlp.loss(y, t), rel=3e-2)
    gu = mlp.unpack(g.astype(np.float64))
    for name in ("W1", "b1", "W2", "b2", "w3", "b3"):
        if name == "W1":
            err = rel(gu[name][:30], ref[name][:30])
            assert np.all(gu[name][30:] == 0.0)  # zero inputs get zero gradient
        else:
            err = rel(gu[name], ref[name])
        print(f"grad {name}: rel L2 {err:.3e}")
        assert err < 3e-2, name
    # deterministic: the same call gives the same bits
    g2, loss2 = model.grads(device(bf16_bits(X)), device(t))
    assert np.array_equal(g, g2) and loss == loss2
    model.close()


def test_adam_step_matches_oracle(ctx):
    from paper_1606_06117_amd import native
    model = native.Model(ctx)
    params = he_params(6)
    model.set_params(params)
    m = 2048
    X = device(bf16_bits(rand_features(m, 7)))
    t = device(np.random.default_rng(8).normal(size=m).astype(np.float32))
    g, _ = model.grads(X, t)
    model.train_step(X, t, 1e-3)
    got = model.get_params().astype(np.float64)
    ref, _, _ = mlp.adam(params.astype(np.float64), g.astype(np.float64), np.zeros(g.size),
                         np.zeros(g.size), 1, 1e-3)
    assert np.max(np.abs(got - ref)) <= 1e-6 * (1 + np.max(np.abs(ref)))
    model.close()


def test_make_pairs_match_oracle_features(ctx):
    import torch
    from paper_1606_06117_amd import native
    shape = (20, 24, 40)
    phi = W.random_gaussians(shape, 5, seed=11).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    phi1 = gpu_advect(ctx, phi, u, dx, dt, oracle.CIR, 1).astype(np.float32)
    nxt = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 1).astype(np.float32)
    rng = np.random.default_rng(12)
    m = 777
    cells = rng.integers(0, phi.size, m).astype(np.int32)
    feats = torch.empty((m, mlp.NF), dtype=torch.int16, device="cuda")
    target = torch.empty(m, device="cuda")
    sigma = torch.empty(m, device="cuda")
    native.make_pairs(ctx, device(phi1), device(nxt), device(u), dx, dt, device(cells), feats,
                      target, sigma)
    torch.cuda.synchronize()
    fb = feats.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    got = fb.view(np.float32).astype(np.float64)
    z, y, x = np.unravel_index(cells, shape)
    c = oracle.courant(u, dt, dx)
    Xr, sr = mlp.features(phi1.astype(np.float64), c, (z, y, x))
    # within one BF16 rounding of the FP64 features
    assert np.all(np.abs(got - Xr) <= 2.0**-8 * np.abs(Xr) + 1e-6)
    assert np.allclose(sigma.cpu().numpy(), sr, rtol=1e-5)
    tr = (nxt.ravel()[cells] - phi1.ravel()[cells]) / sr
    assert np.allclose(target.cpu().numpy(), tr, rtol=1e-4, atol=1e-6 * np.max(np.abs(tr)))


@pytest.mark.parametrize("shape", [(16, 20, 36), (9, 11, 40), (12, 14, 100), (70, 13, 130),
                                   (33, 66, 64), (8, 8, 8)])
def test_learned_march_matches_gather(ctx, shape):
    """The z-march correction (staged neighbourhoods, one node per lane) and
    the per-node gather give the same bits: same FP32 operations per node.
    The shapes leave partial x windows and row groups, rows shorter than a
    window, march chunks that do not divide the planes, and axes of 8."""
    import torch
    from paper_1606_06117_amd import native
    phi = W.random_gaussians(shape, 4, seed=17).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    model = native.Model(ctx)
    model.set_params(he_params(15, scale=0.5))
    model.set_courant_range(1.0)
    res = []
    for kern in (0, 1):
        ctx.set_option(native.OPT_LEARNED_KERNEL, kern)
        p = device(phi)
        try:
            assert not native.advect_learned(ctx, model, p, device(u), dx, dt, 2)
        finally:
            ctx.set_option(native.OPT_LEARNED_KERNEL, 1)
        torch.cuda.synchronize()
        res.append(p.cpu().numpy())
    assert np.array_equal(res[0], res[1])
    model.close()


@pytest.mark.parametrize("shape", [(16, 20, 36), (9, 11, 40), (12, 14, 100)])
def test_learned_step_matches_oracle(ctx, shape):
    """(9, 11, 40) has 198 row tiles: the last group of four leaves idle
    waves.  (12, 14, 100) has interior row tiles (no neighbour wraps), which
    take the gather without periodic wrap."""
    import torch
    from paper_1606_06117_amd import native
    phi = W.random_gaussians(shape, 4, seed=13).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    params = he_params(14, scale=0.5)
    model = native.Model(ctx)
    model.set_params(params)
    model.set_courant_range(1.0)
    p = device(phi)
    fell = native.advect_learned(ctx, model, p, device(u), dx, dt, 1)
    assert not fell
    got = p.cpu().numpy().astype(np.float64)
    c = oracle.courant(u, dt, dx)
    ref = mlp.learned_step(phi.astype(np.float64), c, params)
    cir = oracle.cir(phi.astype(np.float64), c)
    err = rel(got - cir, ref - cir)
    print(f"learned step: correction rel L2 {err:.3e}, |corr|/|phi| {np.linalg.norm(ref - cir) / np.linalg.norm(phi):.3e}")
    assert err < 3e-2
    # the first and last node of every row (whose x neighbours wrap) are no
    # worse than the rest: a wrong neighbour there would stand out
    d = np.abs(got - ref)
    edge, inner = d[..., [0, -1]].max(), d[..., 1:-1].max()
    print(f"max |error| at the row ends {edge:.3e}, elsewhere {inner:.3e}")
    assert edge <= 4 * inner + 1e-7
    model.close()


def test_zero_model_is_cir_and_fallback(ctx):
    import torch
    from paper_1606_06117_amd import native
    shape = (16, 16, 32)
    phi = W.random_gaussians(shape, 3, seed=15).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    model = native.Model(ctx)  # zero weights, untrained
    # untrained: falls back to the third-order scheme, bit for bit
    p = device(phi)
    assert native.advect_learned(ctx, model, p, device(u), dx, dt, 2, step0=5)
    cec = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 2, step0=5)
    assert np.array_equal(p.cpu().numpy().astype(np.float64), cec)
    with pytest.raises(native.SlaError) as ei:
        native.advect_learned(ctx, model, device(phi), device(u), dx, dt, 1, allow_fallback=False)
    assert ei.value.status == native.ENOMODEL
    # zero weights with a range: the correction is sigma * 0, i.e. the CIR step
    model.set_courant_range(1.0)
    p = device(phi)
    assert not native.advect_learned(ctx, model, p, device(u), dx, dt, 1)
    cir = gpu_advect(ctx, phi, u, dx, dt, oracle.CIR, 1)
    assert np.array_equal(p.cpu().numpy().astype(np.float64), cir)
    # Courant number beyond the trained range
    model.set_courant_range(0.5)
    with pytest.raises(native.SlaError) as ei:
        native.advect_learned(ctx, model, device(phi), device(u), dx, dt, 1, allow_fallback=False)
    assert ei.value.status == native.ECOURANT
    assert native.advect_learned(ctx, model, device(phi), device(u), dx, dt, 1)
    model.close()


def test_training_reduces_loss(ctx):
    """A few hundred Adam steps on pairs from the GPU third-order scheme."""
    import torch
    from paper_1606_06117_amd import native
    from paper_1606_06117_amd import learned
    shape = (48, 48, 48)
    data = learned.generate_pairs(ctx, shape, fields=[21, 22], steps_per_field=6, cells_per_snapshot=4096,
                                  cfl=0.9, seed_cells=23)
    model = native.Model(ctx)
    model.set_params(learned.init_params(24))
    first = None
    for it in range(300):
        loss = model.train_step(data.feats, data.target, 2e-3, want_loss=(it % 50 == 0 or it == 299))
        if loss is not None:
            first = loss if first is None else first
            last = loss
    print(f"training loss {first:.4e} -> {last:.4e}")
    assert last < 0.5 * first
    model.close()


@pytest.mark.parametrize("b3", [1.0e3, -1.0e3])
def test_learned_step_limited_to_neighbourhood(ctx, b3):
    """A network with a huge output gives exactly the maximum (minimum) of the
    27 CIR values around each node: the limiter, checked on the GPU's own
    CIR field (a max/min of FP32 values is exact)."""
    from paper_1606_06117_amd import native
    shape = (12, 20, 40)
    phi = W.random_gaussians(shape, 4, seed=16).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    p = {name: np.zeros(s) for name, s in mlp.SHAPES}
    p["b3"][0] = b3
    model = native.Model(ctx)
    model.set_params(mlp.pack(p).astype(np.float32))
    model.set_courant_range(1.0)
    d = device(phi)
    assert not native.advect_learned(ctx, model, d, device(u), dx, dt, 1)
    got = d.cpu().numpy()
    phi1 = gpu_advect(ctx, phi, u, dx, dt, oracle.CIR, 1).astype(np.float32)
    lo, hi = mlp.neighbourhood_range(phi1)
    assert np.array_equal(got, (hi if b3 > 0 else lo).astype(np.float32))
    model.close()


def test_learned_steps_keep_the_maximum_norm(ctx):
    """Untrained random weights, 30 learned steps: max|phi| never grows."""
    import torch
    from paper_1606_06117_amd import native
    shape = (16, 24, 32)
    phi = W.random_gaussians(shape, 4, seed=17).astype(np.float32)
    phi += 0.05 * np.random.default_rng(18).normal(size=shape).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    model = native.Model(ctx)
    model.set_params(he_params(19, scale=3.0))
    model.set_courant_range(1.0)
    d = device(phi)
    m = float(np.max(np.abs(phi)))
    for step in range(30):
        native.advect_learned(ctx, model, d, device(u), dx, dt, 1, step0=step)
        mm = float(torch.max(torch.abs(d)).item())
        assert mm <= m
        m = mm
    model.close()


def test_trained_network_beats_cir_in_rollout(ctx):
    """What the network gains over the method without it: trained on the GPU
    third-order scheme (one extra round of pairs from its own rollouts), the
    learned scheme stays closer to the third-order run than plain CIR over
    100 steps of the time-modulated flow."""
    import math
    import torch
    from paper_1606_06117_amd import native
    from paper_1606_06117_amd import learned
    shape = (48, 48, 48)
    model, pairs, hists, _, _ = learned.train_rollout(
        ctx, shape, fields=[31, 32, 33, 34], steps_per_field=100, cells_per_snapshot=4096, cfl=0.9,
        seed=35, rounds=1, iters=1500, batch=16384, lr=2e-3, log_every=500)
    ev = learned.evaluate(ctx, model, shape, seed=36, periods=1, cfl=0.9)
    step, d_learned, d_cir = ev["per_step"][-1]
    print(f"after {step} steps: learned {d_learned:.3e}, CIR {d_cir:.3e} (relative L2 to third order); "
          f"losses {[(h[0][1], h[-1][1]) for h in hists]}")
    assert not ev["fell_back"]
    assert math.isfinite(d_learned) and d_learned < 0.5 * d_cir
    model.close()
