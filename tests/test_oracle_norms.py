"""Pins of the oracle's error and mass reductions, and of the whole oracle on
the 64 x 64 Gaussian problem.

The paper rates its schemes by the norm of the difference to a reference
profile (section 4) and by their conservation of the integral (section 2,
uniform velocity).  `oracle.norms` gives those measures their plain
definitions; the tests below fix every output against values worked out by
hand on small arrays, exact rational sums, and sign conventions, so that a
dropped square, a swapped argument, a missing absolute value or a wrong
normalisation fails.
"""

import math
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import CIR, FEC, BEC, CEC

from test_oracle_pins import periodic_gaussian_2d


# ---------------------------------------------------------------------------
# reductions: all five outputs on arrays small enough to sum by hand
# ---------------------------------------------------------------------------

def test_reductions_hand_values():
    a = np.array([1.0, 2.0, 3.0, 4.0], dtype=np.float32)
    b = np.array([0.0, 2.0, 5.0, 1.0], dtype=np.float32)
    # a - b = (1, 0, -2, 3)
    s = oracle.reductions(a, b)
    assert s == (14.0, 30.0, 3.0, 10.0, 8.0)


def test_reductions_argument_order_and_sign():
    # the largest difference is negative: max |a - b| must take its magnitude
    a = np.array([0.0, 0.0, 1.0])
    b = np.array([5.0, -1.0, 1.0])
    s = oracle.reductions(a, b)
    assert s[2] == 5.0
    # sum b^2 is over the second argument only; the sums keep their order
    assert s[1] == 27.0 and s[3] == 1.0 and s[4] == 5.0
    t = oracle.reductions(b, a)
    assert t[1] == 1.0 and t[3] == 5.0 and t[4] == 1.0
    assert t[0] == s[0] == 26.0 and t[2] == s[2]


def test_reductions_are_correctly_rounded_sums():
    # a naive FP64 running sum of these returns 0; the exact sum is 1
    a = np.array([1e16, 1.0, -1e16])
    b = np.zeros(3)
    s = oracle.reductions(a, b)
    assert s[3] == 1.0
    assert s[4] == 0.0
    # sum of squares of FP32 inputs against exact rational arithmetic
    rng = np.random.default_rng(7)
    x = rng.standard_normal(257).astype(np.float32)
    y = rng.standard_normal(257).astype(np.float32)
    s = oracle.reductions(x, y)
    exact_sq = sum((Fraction(float(p)) - Fraction(float(q))) ** 2 for p, q in zip(x, y))
    exact_b2 = sum(Fraction(float(q)) ** 2 for q in y)
    exact_a = sum(Fraction(float(p)) for p in x)
    # each square is rounded once in FP64 before the exact sum
    assert abs(s[0] - float(exact_sq)) <= 257 * 2.0**-53 * float(exact_sq)
    assert abs(s[1] - float(exact_b2)) <= 257 * 2.0**-53 * float(exact_b2)
    # the plain sums of FP32 inputs are exact up to the final rounding
    assert s[3] == float(exact_a)
    brute_max = max(abs(float(p) - float(q)) for p, q in zip(x, y))
    assert s[2] == brute_max


def test_reductions_empty_and_single():
    assert oracle.reductions(np.zeros(0), np.zeros(0)) == (0.0, 0.0, 0.0, 0.0, 0.0)
    assert oracle.reductions(np.array([-2.5]), np.array([0.5])) == (9.0, 0.25, 3.0, -2.5, 0.5)


# ---------------------------------------------------------------------------
# rel_l2, linf, mass_error
# ---------------------------------------------------------------------------

def test_rel_l2_and_linf_hand_values():
    ref = np.array([3.0, 4.0])           # |ref| = 5
    x = ref + np.array([0.3, -0.4])      # |x - ref| = 0.5
    assert oracle.rel_l2(x, ref) == pytest.approx(0.1, rel=1e-15)
    assert oracle.linf(x, ref) == pytest.approx(0.4, rel=1e-15)
    # the normalisation is by the reference (second argument), not by x
    assert oracle.rel_l2(ref, x) == pytest.approx(0.5 / math.hypot(3.3, 3.6), rel=1e-15)
    # scale invariance of the relative norm, not of the absolute one
    assert oracle.rel_l2(7 * x, 7 * ref) == pytest.approx(0.1, rel=1e-14)
    assert oracle.linf(7 * x, 7 * ref) == pytest.approx(2.8, rel=1e-14)
    assert oracle.rel_l2(ref, ref) == 0.0 and oracle.linf(ref, ref) == 0.0


def test_mass_error_known_drift_and_sign():
    phi0 = np.array([1.0, -1.0, 2.0, 0.0])   # sum 2, sum |.| 4
    assert oracle.mass_error(phi0 + 0.5, phi0) == 0.5    # gained 2 of 4
    assert oracle.mass_error(phi0 - 0.25, phi0) == -0.25  # lost 1 of 4
    assert oracle.mass_error(phi0, phi0) == 0.0
    # normalised by sum |phi0| (not by |sum phi0| = 2, nor by sum |phi_m|)
    assert oracle.mass_error(np.array([1.0, -1.0, 2.0, 4.0]), phi0) == 1.0
    # a permutation (an exact shift) keeps the mass exactly
    rng = np.random.default_rng(3)
    f = rng.standard_normal(1000)
    assert oracle.mass_error(np.roll(f, 17), f) == 0.0


# ---------------------------------------------------------------------------
# the whole oracle on the 2D Gaussian problem (64 x 64, uniform velocity
# (1, 0.5), CFL 0.7, 100 steps): errors against the exactly translated
# Gaussian.  The reference values come from an independent computation made
# when the build was planned (with its own code, under the same readings of
# the paper); they are not the paper's numbers, which prints no such table.
# ---------------------------------------------------------------------------

C1_TABLE = {
    CIR: (2.711e-1, 3.484e-1),
    FEC: (5.175e-2, 5.809e-2),
    BEC: (1.069e-2, 1.411e-2),
    CEC: (4.450e-3, 7.000e-3),
}


@pytest.mark.parametrize("scheme", [CIR, FEC, BEC, CEC])
def test_gaussian_64_errors_table(scheme):
    N, steps = 64, 100
    c = np.stack([np.full((N, N), 0.7), np.full((N, N), 0.35)])
    phi0 = periodic_gaussian_2d(N, 0.5, 0.5, 0.1)
    out = oracle.run(phi0, c, scheme, steps)
    T = steps * 0.7 / N
    exact = periodic_gaussian_2d(N, (0.5 + T) % 1.0, (0.5 + 0.5 * T) % 1.0, 0.1)
    l2, li = C1_TABLE[scheme]
    assert float(f"{oracle.rel_l2(out, exact):.3e}") == l2
    assert float(f"{oracle.linf(out, exact):.3e}") == li
    # a uniform velocity conserves the integral up to FP64 rounding
    assert abs(oracle.mass_error(out, phi0)) <= 2.3e-16
