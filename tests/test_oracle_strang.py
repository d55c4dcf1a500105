"""Pins of the oracle's third-order step with Strang splitting.

Section 5 names Strang's symmetric splitting as the way a split scheme keeps
its order; the library's default alternates the sweep order between steps
instead.  The Strang step is x/2, y/2, z, y/2, x/2 (2D: x/2, y, x/2).  Pinned
here to: the product of the printed one-dimensional symbols under a uniform
velocity (the sweeps commute and each multiplies a Fourier mode by its
symbol); exact shifts when every sweep moves a whole number of cells; the
plain sweep in 1D; and its order under a variable velocity against the
characteristics reference.
"""

import math

import numpy as np
import pytest

import oracle
from oracle import characteristics as ch
from paper_1606_06117_amd import workloads as W

from test_oracle_pins import xi_bec, xi_fec


def xi_third(U, th):
    """Printed symbols combined as A xi_F + B xi_B (0 < U < 1); from 1 up the
    integer shift times the symbol of the fractional part."""
    n = math.floor(U)
    f = U - n
    A = (2 - 1 / f) / 3
    return np.exp(-1j * n * th) * (A * xi_fec(f, th) + (1 - A) * xi_bec(f, th))


@pytest.mark.parametrize("c", [(0.7, 0.4, 0.9), (0.35, 0.8, 1.6), (1.3, 0.6, 0.45)])
def test_uniform_velocity_symbol(c):
    shape = (12, 10, 16)  # z, y, x
    m = (3, 2, 1)         # wave numbers along x, y, z
    th = [2 * np.pi * m[d] / shape[2 - d] for d in range(3)]
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    arg = th[0] * x + th[1] * y + th[2] * z
    cs = np.stack([np.full(shape, cd) for cd in c])
    re = oracle.step(np.cos(arg), cs, oracle.CEC_STRANG)
    im = oracle.step(np.sin(arg), cs, oracle.CEC_STRANG)
    g = (re + 1j * im) * np.exp(-1j * arg)
    assert np.max(np.abs(g - g.mean())) < 1e-12
    want = xi_third(c[0] / 2, th[0]) ** 2 * xi_third(c[1] / 2, th[1]) ** 2 * xi_third(c[2], th[2])
    assert g.mean() == pytest.approx(want, abs=1e-13)
    # and it is not the alternating step, whose x and y sweeps take whole steps
    alt = oracle.step(np.cos(arg), cs, oracle.CEC, 0)
    assert np.max(np.abs(alt - re)) > 1e-6


def test_whole_cell_sweeps_are_exact_shifts():
    rng = np.random.default_rng(5)
    phi = rng.standard_normal((9, 10, 11))
    c = np.stack([np.full(phi.shape, v) for v in (2.0, -4.0, 3.0)])  # halves: 1, -2 (x, y)
    out = oracle.step(phi, c, oracle.CEC_STRANG)
    want = np.roll(np.roll(np.roll(phi, 2, axis=2), -4, axis=1), 3, axis=0)
    assert np.array_equal(out, want)


def test_one_dimension_is_the_plain_sweep():
    rng = np.random.default_rng(6)
    phi = rng.standard_normal(40)
    c = rng.uniform(-1.8, 1.8, (1, 40))
    assert np.array_equal(oracle.step(phi, c, oracle.CEC_STRANG), oracle.step(phi, c, oracle.CEC, 0))


def test_variable_velocity_order_two():
    """Cellular flow, T = 1, CFL 0.8: second order, like the alternating
    splitting (the one-step backtrace caps both at 2)."""
    L = 2 * math.pi
    errs = []
    for N in (32, 64, 128):
        shape = (N, N)
        phi = W.random_gaussians(shape, 4, seed=11)
        u = W.cellular_velocity_2d(shape)
        steps = int(round(1.0 / (0.8 * L / N)))
        out = oracle.advect(phi, u, (L / N, L / N), 1.0 / steps, "cec_strang", steps)
        exact = W.random_gaussians_at(ch.foot(ch.node_points(shape, L), ch.cellular(), 1.0, 200),
                                      4, seed=11).reshape(shape)
        errs.append(oracle.rel_l2(out, exact))
    slope = math.log2(errs[1] / errs[2])
    assert errs[0] > errs[1] > errs[2]
    assert abs(slope - 2) < 0.25, (errs, slope)
