"""GPU parity of FEC and BEC split per axis (SLA_FEC_SPLIT, SLA_BEC_SPLIT).

One one-dimensional FEC or BEC sweep per axis in the tile sweep kernels,
the order alternating between steps like the third-order scheme's.  Held to
the oracle with the per-step bound of the other parity tests; whole-cell
Courant numbers must give exact shifts.
"""

import numpy as np
import pytest

import oracle
from paper_1606_06117_amd import workloads as W

from helpers import gpu_advect, oracle_advect, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5
SPLIT = [oracle.FEC_SPLIT, oracle.BEC_SPLIT]


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_06117_amd import native
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = native.Context(0)
    yield c
    c.close()


def check(got, ref, phi0, steps, label):
    l2 = rel_l2(got, ref)
    linf = float(np.max(np.abs(got - ref))) / float(np.max(np.abs(phi0)))
    print(f"{label}: relL2={l2:.2e} Linf={linf:.2e}")
    assert l2 <= TOL * steps and linf <= TOL * steps, label


@pytest.mark.parametrize("scheme", SPLIT)
@pytest.mark.parametrize("cfl", [0.9, 1.5, 2.5, 3.5])
def test_abc_3d(ctx, scheme, cfl):
    shape = (36, 40, 72)
    phi = W.random_gaussians(shape, 8, seed=2000).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = cfl * dx[0] / 2.0
    for steps in (1, 3):
        got = gpu_advect(ctx, phi, u, dx, dt, scheme, steps, step0=1)
        ref = oracle_advect(phi, u, dx, dt, scheme, steps, step0=1)
        check(got, ref, phi, steps, f"split {scheme} abc cfl={cfl} steps={steps}")


@pytest.mark.parametrize("scheme", SPLIT)
def test_cellular_2d_and_1d(ctx, scheme):
    shape = (29, 37)
    phi = np.random.default_rng(78).standard_normal(shape).astype(np.float32)
    u = W.cellular_velocity_2d(shape)
    dx = (2 * np.pi / 37, 2 * np.pi / 29)
    dt = 1.3 * min(dx)
    got = gpu_advect(ctx, phi, u, dx, dt, scheme, 5)
    ref = oracle_advect(phi, u, dx, dt, scheme, 5)
    check(got, ref, phi, 5, f"split {scheme} cellular2d")
    N = 30
    p1 = (-np.cos(2 * np.pi * np.arange(N) / N)).astype(np.float32)
    u1 = np.ones((1, N), dtype=np.float32)
    got = gpu_advect(ctx, p1, u1, (1.0 / N,), 0.75 / N, scheme, 40)
    ref = oracle_advect(p1, u1, (1.0 / N,), 0.75 / N, scheme, 40)
    check(got, ref, p1, 40, f"split {scheme} 1d")


@pytest.mark.parametrize("scheme", SPLIT)
def test_whole_cell_shifts(ctx, scheme):
    shape = (20, 24, 72)
    phi = np.random.default_rng(13).standard_normal(shape).astype(np.float32)
    u = W.uniform_velocity(shape, (1.0, -2.0, 3.0))
    got = gpu_advect(ctx, phi, u, (1.0, 1.0, 1.0), 1.0, scheme, 2)
    want = np.roll(np.roll(np.roll(phi.astype(np.float64), 2, axis=2), -4, axis=1), 6, axis=0)
    assert np.array_equal(got, want)
