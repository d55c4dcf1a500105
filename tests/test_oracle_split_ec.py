"""Pins of the oracle's FEC and BEC split per axis.

The split schemes apply the one-dimensional FEC or BEC along one axis at a
time (eqs. split:1-2 with eqs. intro:FEC and intro:BEC), the order
alternating between steps.  Pinned to: the product of the printed
one-dimensional symbols under a uniform velocity; the unsplit scheme in 1D;
exact shifts at whole-cell Courant numbers; second order under a variable
velocity; and a difference from the unsplit 2D scheme, whose symbol has
cross terms the split one lacks.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import characteristics as ch
from paper_1606_06117_amd import workloads as W

from test_oracle_pins import xi_bec, xi_fec


@pytest.mark.parametrize("name,xi", [("fec_split", xi_fec), ("bec_split", xi_bec)])
@pytest.mark.parametrize("c", [(0.7, 0.4, 0.9), (0.25, 0.8, 0.55)])
def test_uniform_velocity_symbol(name, xi, c):
    shape = (12, 10, 16)
    m = (3, 2, 1)
    th = [2 * np.pi * m[d] / shape[2 - d] for d in range(3)]
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    arg = th[0] * x + th[1] * y + th[2] * z
    cs = np.stack([np.full(shape, cd) for cd in c])
    sid = oracle.SCHEMES[name]
    re = oracle.step(np.cos(arg), cs, sid, 1)
    im = oracle.step(np.sin(arg), cs, sid, 1)
    g = (re + 1j * im) * np.exp(-1j * arg)
    assert np.max(np.abs(g - g.mean())) < 1e-12
    assert g.mean() == pytest.approx(xi(c[0], th[0]) * xi(c[1], th[1]) * xi(c[2], th[2]), abs=1e-13)


@pytest.mark.parametrize("split,plain", [("fec_split", "fec"), ("bec_split", "bec")])
def test_one_dimension_is_the_unsplit_scheme(split, plain):
    rng = np.random.default_rng(8)
    phi = rng.standard_normal(40)
    c = rng.uniform(-0.95, 0.95, (1, 40))
    a = oracle.step(phi, c, oracle.SCHEMES[split], 0)
    b = oracle.step(phi, c, oracle.SCHEMES[plain], 0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name", ["fec_split", "bec_split"])
def test_whole_cell_shifts(name):
    rng = np.random.default_rng(10)
    phi = rng.standard_normal((9, 10, 11))
    c = np.stack([np.full(phi.shape, v) for v in (1.0, -2.0, 3.0)])
    out = oracle.step(phi, c, oracle.SCHEMES[name], 0)
    assert np.array_equal(out, np.roll(np.roll(np.roll(phi, 1, axis=2), -2, axis=1), 3, axis=0))


@pytest.mark.parametrize("name", ["fec_split", "bec_split"])
def test_differs_from_unsplit_in_2d(name):
    rng = np.random.default_rng(12)
    phi = rng.standard_normal((16, 18))
    c = np.stack([np.full(phi.shape, 0.6), np.full(phi.shape, 0.3)])
    split = oracle.step(phi, c, oracle.SCHEMES[name], 0)
    unsplit = oracle.step(phi, c, oracle.SCHEMES[name.split("_")[0]], 0)
    assert np.max(np.abs(split - unsplit)) > 1e-3


@pytest.mark.parametrize("name", ["fec_split", "bec_split"])
def test_variable_velocity_order_two(name):
    L = 2 * math.pi
    errs = []
    for N in (32, 64, 128):
        shape = (N, N)
        phi = W.random_gaussians(shape, 4, seed=11)
        u = W.cellular_velocity_2d(shape)
        steps = int(round(1.0 / (0.8 * L / N)))
        out = oracle.advect(phi, u, (L / N, L / N), 1.0 / steps, name, steps)
        exact = W.random_gaussians_at(ch.foot(ch.node_points(shape, L), ch.cellular(), 1.0, 200),
                                      4, seed=11).reshape(shape)
        errs.append(oracle.rel_l2(out, exact))
    slope = math.log2(errs[1] / errs[2])
    print(name, errs, slope)
    assert errs[0] > errs[1] > errs[2]
    assert abs(slope - 2) < 0.25, (errs, slope)
