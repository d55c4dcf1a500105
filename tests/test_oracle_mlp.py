"""Pins of the network oracle: finite differences, Adam's first step,
BF16 rounding of known values, and the invariances the features are built
to have."""

import numpy as np
import pytest

import oracle
from oracle import mlp


def rand_params(rng, scale=0.3):
    return {name: rng.normal(0.0, scale, shape) for name, shape in mlp.SHAPES}


def test_backward_matches_finite_differences():
    rng = np.random.default_rng(1)
    params = rand_params(rng)
    X = rng.normal(size=(40, mlp.NF))
    t = rng.normal(size=40)
    y, cache = mlp.forward(params, X)
    g = mlp.backward(params, cache, y, t)
    flat = mlp.pack(params)
    gflat = mlp.pack(g)
    h = 1e-6
    worst = 0.0
    for idx in rng.choice(flat.size, 300, replace=False):
        p = flat.copy()
        p[idx] += h
        lp = mlp.loss(mlp.forward(mlp.unpack(p), X)[0], t)
        p[idx] -= 2 * h
        lm = mlp.loss(mlp.forward(mlp.unpack(p), X)[0], t)
        fd = (lp - lm) / (2 * h)
        worst = max(worst, abs(fd - gflat[idx]) / (1.0 + abs(fd)))
    assert worst < 1e-7


def test_backward_every_bias_and_last_layer():
    """Exhaustive central differences on b1, b2, w3, b3."""
    rng = np.random.default_rng(2)
    params = rand_params(rng)
    X = rng.normal(size=(25, mlp.NF))
    t = rng.normal(size=25)
    y, cache = mlp.forward(params, X)
    g = mlp.backward(params, cache, y, t)
    for name in ("b1", "b2", "w3", "b3"):
        for i in range(params[name].size):
            p = {k: v.copy() for k, v in params.items()}
            p[name].flat[i] += 1e-6
            lp = mlp.loss(mlp.forward(p, X)[0], t)
            p[name].flat[i] -= 2e-6
            lm = mlp.loss(mlp.forward(p, X)[0], t)
            assert g[name].flat[i] == pytest.approx((lp - lm) / 2e-6, rel=1e-5, abs=1e-9)


def test_adam_first_step_is_signed_lr():
    """After one step from zero moments, Adam moves each weight by
    lr * g / (|g| + eps), i.e. lr * sign(g) for |g| >> eps."""
    rng = np.random.default_rng(3)
    flat = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = mlp.adam(flat, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    assert np.allclose(new - flat, -1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_bf16_round_known_values():
    # 3e38 = 1.7632.. * 2^127; 8 significant bits keep 226/128
    x = np.array([1.0, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-9, 1.0 + 2.0**-7, -2.5, 0.0, 3.0e38],
                 dtype=np.float32)
    got = mlp.bf16_round(x)
    expect = np.array([1.0, 1.0, 1.0 + 2.0**-7, 1.0 + 2.0**-7, -2.5, 0.0, 226 / 128 * 2.0**127],
                      dtype=np.float32)
    assert np.array_equal(got, expect)


def test_feature_invariances():
    rng = np.random.default_rng(4)
    shape = (6, 7, 8)
    phi1 = rng.normal(size=shape)
    c = rng.uniform(-0.9, 0.9, (3,) + shape)
    cells = np.indices(shape).reshape(3, -1)
    X, s = mlp.features(phi1, c, cells)
    X2, s2 = mlp.features(phi1 + 4.0, c, cells)      # constant shift
    X3, s3 = mlp.features(-2.5 * phi1, c, cells)      # scaling
    assert np.allclose(X2, X, atol=1e-12) and np.allclose(s2, s)
    assert np.allclose(X3[:, :27], -X[:, :27], atol=1e-12) and np.allclose(s3, 2.5 * s)
    assert np.all(X[:, 13] == 0.0) and np.all(X[:, 30:] == 0.0)
    assert np.allclose(np.sum(X[:, :27] ** 2, axis=1), 27.0, rtol=1e-12)
    # the Courant inputs are the node's own
    assert np.array_equal(X[:, 27], c[0].ravel())


def test_feature_neighbour_order():
    """Offset k = 9 (dz+1) + 3 (dy+1) + (dx+1): a field linear in x gives
    d_k = dx, so only x-differences are non-zero."""
    shape = (5, 5, 9)
    x = np.arange(9, dtype=np.float64)
    phi1 = np.broadcast_to(0.5 * x, shape).copy()
    c = np.zeros((3,) + shape)
    X, s = mlp.features(phi1, c, (np.array([2]), np.array([2]), np.array([4])))
    d = X[0, :27] * s[0]
    for k, (dz, dy, dx) in enumerate(mlp.offsets27()):
        assert d[k] == pytest.approx(0.5 * dx)


def test_zero_network_is_cir():
    """With all weights zero the learned step is exactly the CIR step."""
    rng = np.random.default_rng(5)
    shape = (6, 6, 6)
    phi = rng.normal(size=shape)
    c = rng.uniform(-0.9, 0.9, (3,) + shape)
    out = mlp.learned_step(phi, c, np.zeros(mlp.NPARAMS))
    assert np.allclose(out, oracle.cir(phi, c), atol=1e-15)


def _range_brute(phi1, z, y, x):
    nz, ny, nx = phi1.shape
    vals = [phi1[(z + a) % nz, (y + b) % ny, (x + c) % nx]
            for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    return min(vals), max(vals)


@pytest.mark.parametrize("b3", [1.0e3, -1.0e3])
def test_learned_step_limited_to_neighbourhood(b3):
    """A network whose output is huge gives, at every node, the maximum
    (resp. minimum) of the 27 CIR values around it (checked by brute force)."""
    rng = np.random.default_rng(6)
    shape = (5, 6, 7)
    phi = rng.normal(size=shape)
    c = rng.uniform(-0.9, 0.9, (3,) + shape)
    p = {name: np.zeros(s) for name, s in mlp.SHAPES}
    p["b3"][0] = b3
    out = mlp.learned_step(phi, c, mlp.pack(p))
    phi1 = oracle.cir(phi, c)
    for z, y, x in np.ndindex(*shape):
        lo, hi = _range_brute(phi1, z, y, x)
        assert out[z, y, x] == (hi if b3 > 0 else lo)


def test_learned_steps_keep_the_maximum_norm():
    """Random (untrained) weights: repeated learned steps never raise max|phi|."""
    rng = np.random.default_rng(7)
    shape = (6, 6, 8)
    phi = rng.normal(size=shape)
    c = rng.uniform(-0.9, 0.9, (3,) + shape)
    flat = mlp.pack(rand_params(rng, scale=2.0))
    m = np.max(np.abs(phi))
    for _ in range(5):
        phi = mlp.learned_step(phi, c, flat)
        assert np.max(np.abs(phi)) <= m
        m = np.max(np.abs(phi))
