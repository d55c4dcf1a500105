"""GPU parity of the literal large-CFL weights (SLA_CEC_LITERAL).

One sweep per axis in the tile sweep kernels, A FEC + B BEC with
3A = 2 - 1/(|c| mod 1) (eq. intro:CECcoefSL read literally).  Held to the
oracle with the per-step bound of the other parity tests on velocity fields
whose Courant numbers keep their fractional parts away from 0 (there the
weights grow like 1/(3 f) and so does FP32 rounding).  Below |c| = 1 the
scheme is the third order's: the GPU results agree with SLA_CEC's to
rounding.  The paper's 1D cosine at CFL 3.75 shows the second-order drift.
"""

import numpy as np
import pytest

import oracle
from paper_1606_06117_amd import workloads as W

from helpers import gpu_advect, oracle_advect, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5


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


def banded_velocity(shape, base, amp):
    """Per-axis velocity base_d + amp sin(...) of the other coordinates:
    with dt = dx = 1 its Courant numbers are the velocity itself, and their
    fractional parts stay within base_d mod 1 +- amp."""
    nd = len(shape)
    grids = np.meshgrid(*[2 * np.pi * np.arange(n) / n for n in shape], indexing="ij")
    u = np.empty((nd,) + tuple(shape), dtype=np.float32)
    for d in range(nd):
        ax = nd - 1 - d
        other = grids[(ax + 1) % nd] if nd > 1 else grids[0]
        u[d] = base[d] + amp * np.sin(other)
    return u


@pytest.mark.parametrize("shape,base", [
    ((20, 24, 40), (2.3, -1.6, 3.4)),
    ((20, 24, 40), (0.4, -0.7, 0.55)),
    ((30, 44), (-3.75, 2.4)),
])
def test_literal_matches_oracle(ctx, shape, base):
    phi = W.random_gaussians(shape, 5, seed=90).astype(np.float32)
    u = banded_velocity(shape, base, 0.15)
    dx = (1.0,) * len(shape)
    for steps, step0 in ((1, 0), (3, 1)):
        got = gpu_advect(ctx, phi, u, dx, 1.0, oracle.CEC_LITERAL, steps, step0=step0)
        ref = oracle_advect(phi, u, dx, 1.0, oracle.CEC_LITERAL, steps, step0=step0)
        check(got, ref, phi, steps, f"literal {shape} {base} steps={steps}")


def test_literal_below_one_is_the_third_order(ctx):
    shape = (20, 24, 40)
    phi = W.random_gaussians(shape, 5, seed=91).astype(np.float32)
    u = banded_velocity(shape, (0.4, -0.7, 0.55), 0.15)
    dx = (1.0, 1.0, 1.0)
    lit = gpu_advect(ctx, phi, u, dx, 1.0, oracle.CEC_LITERAL, 4)
    cec = gpu_advect(ctx, phi, u, dx, 1.0, oracle.CEC, 4)
    assert rel_l2(lit, cec) < 2e-6


def test_paper_cosine_at_cfl_375(ctx):
    """Section 4's cosine, N = 30, CFL 3.75, 10 periods (80 steps): the GPU
    follows the oracle, and the literal weights end farther from the exact
    profile than the third-order scheme."""
    N, steps = 30, 80
    x = np.arange(N) / N
    phi = np.cos(2 * np.pi * x).astype(np.float32)
    u = np.ones((1, N), dtype=np.float32)
    dx, dt = (1.0 / N,), 3.75 / N
    got = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC_LITERAL, steps)
    ref = oracle_advect(phi, u, dx, dt, oracle.CEC_LITERAL, steps)
    check(got, ref, phi, steps, "literal cosine cfl 3.75")
    exact = np.cos(2 * np.pi * x)
    third = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, steps)
    e_lit, e_cec = rel_l2(got, exact), rel_l2(third, exact)
    print(f"10 periods at CFL 3.75: literal {e_lit:.3e}, third order {e_cec:.3e}")
    assert e_lit > 2 * e_cec
