"""The midpoint backtrace (beyond the paper) and what it shows.

The paper takes the velocity at the arrival node and backtraces one
explicit step (its stencils use U_i at node i).  ``cec_split_midpoint``
departs instead from the second-order Runge-Kutta foot of each call's own
characteristic.  Pins: the midpoint Courant number is exact for a velocity
linear between nodes and equal to the node's for a uniform one, so the
scheme is the third-order split step there; the two directions use their
own characteristics.  The study: with a variable velocity the third-order
scheme converges at second order against the exact solution (characteristics
integrated with RK4), and the midpoint backtrace keeps it there: the order
lost to a variable velocity does not come back from the backtrace.
"""
import numpy as np
import pytest

import oracle
from oracle import characteristics as CH


def test_midpoint_courant_uniform_and_linear():
    c = np.full((1, 16), 0.7)
    assert np.max(np.abs(oracle.midpoint_courant(c[0], 0, 1.0) - c[0])) < 1e-15
    # a ramp c_i = a + b i, sampled away from the periodic wrap: the midpoint
    # x_i -+ c_i / 2 lies between nodes where c is linear, so it is exact
    n, a, b = 64, 0.3, 0.01
    ramp = a + b * np.arange(n)
    for sign in (1.0, -1.0):
        got = oracle.midpoint_courant(ramp, 0, sign)
        i = np.arange(8, n - 8)
        want = a + b * (i - sign * 0.5 * ramp[i])
        assert np.max(np.abs(got[i] - want)) < 1e-15


def test_midpoint_courant_follows_each_axis():
    rng = np.random.default_rng(5)
    c = rng.uniform(-1.2, 1.2, size=(5, 6, 7))  # (z, y, x)
    got = oracle.midpoint_courant(c, 1, 1.0)  # along y: NumPy axis 1
    for z in range(5):
        for x in range(7):
            col = c[z, :, x]
            want = oracle.midpoint_courant(col, 0, 1.0)
            assert np.allclose(got[z, :, x], want, atol=0, rtol=0)


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_midpoint_uniform_velocity_is_the_third_order(ndim):
    rng = np.random.default_rng(40 + ndim)
    shape = (6, 8, 10)[3 - ndim:]
    phi = rng.standard_normal(shape)
    c = np.stack([np.full(shape, v) for v in (1.3, -0.4, 2.2)[:ndim]])
    for m in (0, 1):  # the interpolated constant may differ from it in the last bit
        diff = oracle.cec_split_midpoint(phi, c, m) - oracle.cec_split(phi, c, m)
        assert np.max(np.abs(diff)) < 1e-13


def test_directions_use_their_own_characteristic():
    """With a velocity that varies, the reverse call's midpoint is taken
    downstream: swapping the two Courant fields changes the result."""
    n = 32
    x = 2 * np.pi * np.arange(n) / n
    c = 0.6 + 0.3 * np.sin(x)
    phi = np.exp(np.cos(x))
    cf = oracle.midpoint_courant(c, 0, 1.0)
    cb = oracle.midpoint_courant(c, 0, -1.0)
    assert np.max(np.abs(cf - cb)) > 1e-2
    right = oracle.cec_sweep_pair(phi, cf, cb, 0)
    assert np.array_equal(right, oracle.cec_split_midpoint(phi, c[None, :]))
    assert np.max(np.abs(right - oracle.cec_sweep_pair(phi, cb, cf, 0))) > 1e-4


def _orders(stepper):
    vel = lambda p, t: 1.0 + 0.5 * np.sin(p[:, :1])  # noqa: E731
    errs = []
    for n in (32, 64, 128, 256):
        dx = 2 * np.pi / n
        x = np.arange(n) * dx
        T = 2.0
        steps = int(round(T / (0.5 * dx / 1.5)))
        dt = T / steps
        c = ((1.0 + 0.5 * np.sin(x)) * dt / dx)[None, :]
        phi = np.exp(np.cos(x))
        for k in range(steps):
            phi = stepper(phi, c, k)
        foot = CH.foot(x[:, None], vel, T, 2000)
        errs.append(oracle.rel_l2(phi, np.exp(np.cos(foot[:, 0]))))
    return errs, [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]


def _rk3_stepper(p, c, k):
    """Departures from a third-order Runge-Kutta foot of the analytic
    velocity (no interpolation error in the velocity either)."""
    n = p.shape[-1]
    x = np.arange(n) * (2 * np.pi / n)
    scale = c[0] / (1.0 + 0.5 * np.sin(x))  # dt / dx
    u = lambda y: 1.0 + 0.5 * np.sin(y)  # noqa: E731
    h = scale * (2 * np.pi / n)  # dt, the same at every node

    def disp(sign):
        k1 = u(x)
        k2 = u(x - sign * 0.5 * h * k1)
        k3 = u(x - sign * h * (2.0 * k2 - k1))
        return scale * (k1 + 4.0 * k2 + k3) / 6.0

    return oracle.cec_sweep_pair(p, disp(1.0), disp(-1.0), 0)


def test_variable_velocity_order_stays_two():
    e_euler, o_euler = _orders(lambda p, c, k: oracle.cec_split(p, c, k))
    e_mid, o_mid = _orders(lambda p, c, k: oracle.cec_split_midpoint(p, c, k))
    e_rk3, o_rk3 = _orders(_rk3_stepper)
    print("arrival-node backtrace", ["%.2e" % e for e in e_euler], ["%.2f" % o for o in o_euler])
    print("midpoint backtrace    ", ["%.2e" % e for e in e_mid], ["%.2f" % o for o in o_mid])
    print("RK3, exact velocity   ", ["%.2e" % e for e in e_rk3], ["%.2f" % o for o in o_rk3])
    for o in o_euler[1:] + o_mid[1:] + o_rk3[1:]:
        assert 1.7 < o < 2.3
