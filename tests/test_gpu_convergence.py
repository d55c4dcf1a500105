"""GPU convergence under a variable velocity, against the exact solution.

The exact solution is the initial field at the foot of each node's
characteristic, found by RK4 in FP64 (oracle/characteristics.py) and
evaluated with the same analytic formula the grids are sampled from.  The
errors are measured at nodes shared by every grid of a refinement series, so
each grid's result is compared at the same points.

Two series:

* ABC flow with 8 Gaussians (the 256^3 workload's recipe) on 64^3, 128^3 and
  256^3 at CFL 0.9, T = 16 steps of the coarsest grid, every scheme.  The
  expected orders are 1 for CIR and 2 for the others: the schemes' third
  order is for a uniform velocity (sections 3-4); with a variable one, the
  one-step backtrace from the arrival node and the splitting cap it at 2,
  as the oracle's own series on the cellular flow shows on the CPU.
* The large workload's field (k^-5/3, |k| <= 64) under the ABC flow at CFL
  2.0 on 256^3, 512^3 and 1024^3, with T = 10 steps of the coarsest grid
  (10, 20 and 40 steps), the third-order scheme, errors at the 256^3 nodes of
  the sub-box [0, 2 pi / 8)^3.  At 256^3 the modes of |k| = 64 have four
  nodes per wavelength, so this series is not yet asymptotic.
"""

import math

import numpy as np
import pytest

from oracle import characteristics as ch
from paper_1606_06117_amd import workloads as W

pytestmark = pytest.mark.gpu

L = 2 * math.pi


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_06117_amd import native
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = native.Context(0)
    yield c
    c.close()


def _sample_nodes(n_coarse, count, seed, box=None):
    """``count`` distinct nodes of the coarse grid, (P, 3) integer x, y, z."""
    rng = np.random.default_rng(seed)
    hi = n_coarse if box is None else box
    flat = rng.choice(hi ** 3, size=count, replace=False)
    return np.stack([flat % hi, (flat // hi) % hi, flat // (hi * hi)], axis=1)


def _gather(phi, nodes, stride):
    import torch
    idx = torch.from_numpy(nodes * stride).to(phi.device)
    return phi[idx[:, 2], idx[:, 1], idx[:, 0]].double().cpu().numpy()


@pytest.mark.parametrize("scheme,order", [("cir", 1), ("fec", 2), ("bec", 2), ("cec", 2)])
def test_abc_gaussians_orders(ctx, scheme, order):
    import torch
    from paper_1606_06117_amd import native
    dev = torch.device("cuda:0")
    sid = {"cir": native.CIR, "fec": native.FEC, "bec": native.BEC, "cec": native.CEC}[scheme]
    Ns, base = (64, 128, 256), 64
    nodes = _sample_nodes(base, 8192, 21)
    dt0 = W.abc_dt((base,) * 3, 0.9)
    T = 16 * dt0
    pts = nodes.astype(np.float64) * (L / base)
    exact = W.random_gaussians_at(ch.foot(pts, ch.abc(), T, 64), 8, seed=2000)
    errs = []
    for N in Ns:
        shape = (N,) * 3
        steps = 16 * N // base
        phi = torch.from_numpy(W.random_gaussians(shape, 8, seed=2000).astype(np.float32)).to(dev)
        u = W.abc_velocity_torch(shape, dev)
        ctx.advect(phi, u, (L / N,) * 3, T / steps, sid, steps, 0, 0.0)
        ctx.check()
        got = _gather(phi, nodes, N // base)
        errs.append(float(np.linalg.norm(got - exact) / np.linalg.norm(exact)))
        del phi, u
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print(f"ABC, 8 Gaussians, {scheme}: relL2 vs exact {['%.3e' % e for e in errs]}, "
          f"slopes {['%.2f' % s for s in slopes]}")
    assert errs[0] > errs[1] > errs[2]
    assert abs(slopes[-1] - order) < 0.3, (errs, slopes)


def test_large_field_refinement_cfl2(ctx):
    import torch
    from paper_1606_06117_amd import native
    dev = torch.device("cuda:0")
    base, box = 256, 32
    nodes = _sample_nodes(base, 4096, 22, box=box)
    pts = nodes.astype(np.float64) * (L / base)
    T = 10 * W.abc_dt((base,) * 3, 2.0)
    exact = W.power_law_at(ch.foot(pts, ch.abc(), T, 40), 5000)
    start = W.power_law_at(pts, 5000)
    errs = []
    for N in (256, 512, 1024):
        shape = (N,) * 3
        steps = 10 * N // base
        phi = W.power_law_torch(shape, 5000, dev)
        # the field the GPU starts from is the analytic one at the sampled nodes
        p0 = _gather(phi, nodes, N // base)
        assert np.max(np.abs(p0 - start)) <= 2.0 ** -22 * np.max(np.abs(start))
        u = W.abc_velocity_torch(shape, dev)
        ctx.advect(phi, u, (L / N,) * 3, T / steps, native.CEC, steps, 0, 0.0)
        ctx.check()
        got = _gather(phi, nodes, N // base)
        errs.append(float(np.linalg.norm(got - exact) / np.linalg.norm(exact)))
        del phi, u
        torch.cuda.empty_cache()
    slopes = [math.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    print(f"k^-5/3 field, ABC, CFL 2.0, third order, T = 10 steps of 256^3: relL2 vs exact "
          f"{['%.3e' % e for e in errs]}, slopes {['%.2f' % s for s in slopes]}")
    assert errs[0] > errs[1] > errs[2]
    assert slopes[-1] > 1.0
