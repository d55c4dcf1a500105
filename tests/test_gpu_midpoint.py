"""GPU parity of the midpoint backtrace (SLA_OPT_BACKTRACE = 1; beyond the
paper).

Third-order steps with the option set run one tile sweep per axis whose
calls depart from the midpoint (second-order Runge-Kutta) feet of their
characteristics, the velocity interpolated between nodes.  Held to the
oracle's ``cec_split_midpoint`` with the per-step bound of the other parity
tests, at reach 1 to 4, in 1D, 2D and 3D; a uniform velocity gives the
default backtrace's results to rounding; batched plans refuse the option.
"""

import numpy as np
import pytest

import oracle
from paper_1606_06117_amd import workloads as W

from helpers import gpu_advect, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_06117_amd import native
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = native.Context(0)
    c.set_option(native.OPT_BACKTRACE, 1)
    yield c
    c.close()


def oracle_midpoint(phi, u, dx, dt, steps, step0=0):
    c = oracle.courant(np.asarray(u, np.float32), dt, dx)
    out = np.asarray(phi, np.float32).astype(np.float64)
    for k in range(steps):
        out = oracle.cec_split_midpoint(out, c, step0 + k)
    return out


def check(got, ref, phi0, steps, label):
    l2 = rel_l2(got, ref)
    linf = float(np.max(np.abs(got - ref))) / float(np.max(np.abs(phi0)))
    print(f"{label}: relL2={l2:.2e} Linf={linf:.2e}")
    assert l2 <= TOL * steps and linf <= TOL * steps, label


@pytest.mark.parametrize("cfl", [0.9, 1.5, 2.5, 3.5])
def test_midpoint_abc_3d(ctx, cfl):
    shape = (24, 28, 40)
    phi = W.random_gaussians(shape, 6, seed=95).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = cfl * dx[0] / 2.0
    for steps, step0 in ((1, 0), (3, 1)):
        got = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, steps, step0=step0)
        ref = oracle_midpoint(phi, u, dx, dt, steps, step0)
        check(got, ref, phi, steps, f"midpoint abc cfl={cfl} steps={steps}")


def test_midpoint_2d_and_1d(ctx):
    shape = (29, 37)
    phi = np.random.default_rng(96).standard_normal(shape).astype(np.float32)
    u = W.cellular_velocity_2d(shape)
    dx = (2 * np.pi / 37, 2 * np.pi / 29)
    dt = 1.3 * min(dx)
    got = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 5)
    check(got, oracle_midpoint(phi, u, dx, dt, 5), phi, 5, "midpoint cellular 2d")
    n = 64
    x = 2 * np.pi * np.arange(n) / n
    p1 = np.exp(np.cos(x)).astype(np.float32)
    u1 = (1.0 + 0.5 * np.sin(x))[None, :].astype(np.float32)
    dt1 = 2.2 * (2 * np.pi / n) / 1.5
    got = gpu_advect(ctx, p1, u1, (2 * np.pi / n,), dt1, oracle.CEC, 20)
    check(got, oracle_midpoint(p1, u1, (2 * np.pi / n,), dt1, 20), p1, 20, "midpoint 1d")


def test_midpoint_uniform_velocity_is_the_default(ctx):
    from paper_1606_06117_amd import native
    shape = (20, 24, 36)
    phi = W.random_gaussians(shape, 5, seed=97).astype(np.float32)
    u = W.uniform_velocity(shape, (0.37, -0.81, 0.55))
    dx = (1.0, 1.0, 1.0)
    mid = gpu_advect(ctx, phi, u, dx, 2.5, oracle.CEC, 3)
    ctx.set_option(native.OPT_BACKTRACE, 0)
    try:
        plain = gpu_advect(ctx, phi, u, dx, 2.5, oracle.CEC, 3)
    finally:
        ctx.set_option(native.OPT_BACKTRACE, 1)
    assert rel_l2(mid, plain) < 1e-6


def test_plans_refuse_the_midpoint_backtrace(ctx):
    import torch
    from paper_1606_06117_amd import native
    shape = (16, 16, 16)
    phi = torch.zeros(shape, device="cuda")
    with pytest.raises(native.SlaError) as ei:
        native.Plan(ctx, [(phi, (0.1, 0.2, 0.3), (1.0, 1.0, 1.0), 1.0)], 2)
    assert ei.value.status == native.EINVAL
    with pytest.raises(native.SlaError):
        ctx.set_option(native.OPT_BACKTRACE, 2)
