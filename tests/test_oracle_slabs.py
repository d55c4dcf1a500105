"""The oracle over slabs in worker processes equals the oracle in one process.

The slab runner times the oracle on every host core; these tests hold it to
the one-process result bit for bit, for every scheme, in 2D and 3D, at
Courant numbers below and above 1 (where the halo grows with the integer
offset), with slabs thinner than their halo, and starting at an odd step
(so the third-order sweep order is carried over).
"""

import numpy as np
import pytest

import oracle
from oracle import slabs


def _case(shape, cmax, seed):
    rng = np.random.default_rng(seed)
    nd = len(shape)
    phi = rng.standard_normal(shape)
    dx = tuple(1.0 / n for n in shape[::-1])
    dt = 1.0 / max(shape)
    u = np.empty((nd,) + shape, dtype=np.float32)
    for d in range(nd):
        # |c_d| up to cmax, both signs, varying from cell to cell
        u[d] = rng.uniform(-cmax, cmax, shape) * dx[d] / dt
    return phi, u, dx, dt


@pytest.mark.parametrize("scheme", ["cir", "fec", "bec", "cec"])
@pytest.mark.parametrize("shape,cmax,workers,steps,step0", [
    ((18, 10, 12), 0.9, 3, 3, 0),
    ((10, 9, 11), 2.6, 4, 2, 1),   # slabs of 2-3 planes, halo 9
    ((21, 13), 1.7, 5, 3, 0),      # 2D: slabs along y
])
def test_slabs_equal_one_process(scheme, shape, cmax, workers, steps, step0):
    phi, u, dx, dt = _case(shape, cmax, 7)
    ref = oracle.advect(phi, u, dx, dt, scheme, steps, step0=step0)
    got = slabs.advect_slabs(phi, u, dx, dt, scheme, steps, workers, step0=step0)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


def test_step_halo():
    shape = (8, 8, 8)
    phi, u, dx, dt = _case(shape, 0.9, 1)
    assert slabs.step_halo(u, dx, dt) == 3
    u[2, 3, 4, 5] = 2.5 * dx[2] / dt      # one z Courant number of 2.5
    assert slabs.step_halo(u, dx, dt) == 9
