"""Pins of the oracle's literal reading of the large-CFL weights
(eq. intro:CECcoefSL: 3A = 2 - 1/(U % 1), B = 1 - A, applied to eq.
intro:FEC and eq. intro:BEC one axis at a time).

* Below U = 1 the weights are those of eq. intro:CECcoef, and A FEC + B BEC
  equals the division-free third-order sweep (an identity of the two
  formulas, checked here against the separately pinned ``cec_split``).
* For a uniform Courant number every step maps a Fourier mode to itself;
  its factor has the closed form A (h g + w) + B h g (1 + w), with
  h = exp(-i s n theta), g = (1 - f) + f exp(-i s theta) and
  w = (1 - |g|^2)/2 (CIR is h g, L_{-U} L_U is |g|^2, FEC's correction sits
  at the arrival node, BEC's is re-interpolated).  Split 2D steps multiply
  the per-axis factors.
* That factor's error against exp(-i c theta) falls as theta^3 once U > 1
  (second order), against theta^4 for the third-order sweep, and the
  formula divides by zero at an integer U.
"""
import numpy as np
import pytest

import oracle


def literal_factor(c, theta):
    s = 1.0 if c >= 0 else -1.0
    u = abs(c)
    n = np.floor(u)
    f = u - n
    h = np.exp(-1j * s * n * theta)
    g = (1.0 - f) + f * np.exp(-1j * s * theta)
    w = (1.0 - abs(g) ** 2) / 2.0
    a = (2.0 - 1.0 / f) / 3.0
    return a * (h * g + w) + (1.0 - a) * h * g * (1.0 + w)


def measured_factor_1d(step_fn, c, k, N):
    x = np.arange(N)
    theta = 2 * np.pi * k / N
    cc = np.full((1, N), c)
    re = step_fn(np.cos(theta * x), cc)
    im = step_fn(np.sin(theta * x), cc)
    z = (re + 1j * im) / np.exp(1j * theta * x)
    assert np.allclose(z, z[0], atol=1e-12)  # one mode in, the same mode out
    return z[0], theta


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_literal_equals_third_order_below_one(ndim):
    rng = np.random.default_rng(70 + ndim)
    shape = (7, 9, 11)[3 - ndim:]
    phi = rng.standard_normal(shape)
    c = rng.uniform(-0.95, 0.95, size=(ndim,) + shape)
    c[np.abs(c) < 1e-3] = 0.5  # 1/U: no zero Courant numbers
    for m in (0, 1):
        lit = oracle.cec_literal(phi, c, m)
        ref = oracle.cec_split(phi, c, m)
        assert np.max(np.abs(lit - ref)) < 1e-12


@pytest.mark.parametrize("c", [0.3, -0.6, 1.3, 2.3, -1.7, 3.75, -3.4])
def test_literal_fourier_factor(c):
    for k in (1, 3, 7):
        z, theta = measured_factor_1d(lambda p, cc: oracle.cec_literal(p, cc), c, k, 32)
        assert abs(z - literal_factor(c, theta)) < 1e-12


def test_literal_split_2d_multiplies_factors():
    ny, nx, ky, kx, cx, cy = 24, 20, 2, 3, 2.3, -1.6
    y, x = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    tx, ty = 2 * np.pi * kx / nx, 2 * np.pi * ky / ny
    c = np.stack([np.full((ny, nx), cx), np.full((ny, nx), cy)])
    mode = np.exp(1j * (tx * x + ty * y))
    out = oracle.cec_literal(mode.real, c) + 1j * oracle.cec_literal(mode.imag, c)
    want = literal_factor(cx, tx) * literal_factor(cy, ty) * mode
    assert np.max(np.abs(out - want)) < 1e-12


def test_literal_is_second_order_beyond_one():
    """Local error of one step on a resolved mode: theta^3 for the literal
    weights at U = 2.3 (ratio 8 when theta halves), theta^4 for the
    division-free third order (ratio 16), whose factor is measured too."""
    c = 2.3
    errs_lit, errs_cec = [], []
    for N in (64, 128, 256):
        z, theta = measured_factor_1d(lambda p, cc: oracle.cec_literal(p, cc), c, 1, N)
        errs_lit.append(abs(z - np.exp(-1j * c * theta)))
        z3, _ = measured_factor_1d(lambda p, cc: oracle.cec_split(p, cc), c, 1, N)
        errs_cec.append(abs(z3 - np.exp(-1j * c * theta)))
    r_lit = [errs_lit[i] / errs_lit[i + 1] for i in range(2)]
    r_cec = [errs_cec[i] / errs_cec[i + 1] for i in range(2)]
    assert all(7.0 < r < 9.0 for r in r_lit), r_lit
    assert all(14.0 < r < 18.0 for r in r_cec), r_cec


def test_literal_integer_courant_number_is_not_finite():
    phi = np.cos(2 * np.pi * np.arange(16) / 16)
    out = oracle.cec_literal(phi, np.full((1, 16), 2.0))
    assert not np.any(np.isfinite(out))
