"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerance.  The GPU interpolates in FP32; each output is a short chain of
FP32 lerps (at most ~20 roundings of relative size 2^-24 per call, three
calls per axis), so a step's FP32 error is a few 1e-7 of the field scale.
The bound used is the one the method's target states, 1e-5 relative L2 per
step, accumulated linearly over K steps (the schemes are L2-stable, so a
step does not amplify earlier rounding errors): relL2 <= 1e-5 K, and the
same bound on max |gpu - oracle| / max |phi0|.  Cases whose result is a
permutation of FP32 inputs (integer Courant numbers) or a constant must be
bit-exact.
"""

import numpy as np
import pytest

import oracle
from paper_1606_06117_amd import workloads as W

from helpers import box_parity, gpu_advect, oracle_advect, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-5
SCHEMES = [oracle.CIR, oracle.FEC, oracle.BEC, oracle.CEC]
NAMES = {0: "cir", 1: "fec", 2: "bec", 3: "cec"}


@pytest.fixture(scope="module")
def ctx():
    import torch
    from paper_1606_06117_amd import native
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    c = native.Context(0)
    yield c
    c.close()


def check(got, ref, phi0, steps, label=""):
    l2 = rel_l2(got, ref)
    linf = float(np.max(np.abs(got - ref))) / float(np.max(np.abs(phi0)))
    print(f"{label} relL2={l2:.3e} Linf={linf:.3e}")
    assert l2 <= TOL * steps, (label, l2)
    assert linf <= TOL * steps, (label, linf)


# ---------------------------------------------------------------------------
# small configurations: full-grid comparison
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", SCHEMES)
def test_gaussian_2d_uniform(ctx, scheme):
    """64x64 Gaussian, uniform U = (1, 0.5), CFL 0.7, 1 and 100 steps."""
    N = 64
    phi = W.gaussians((N, N), [(0.5, 0.5)], [0.1]).astype(np.float32)
    u = W.uniform_velocity((N, N), (1.0, 0.5))
    dx = (1.0 / N, 1.0 / N)
    dt = 0.7 / N
    for steps in (1, 100):
        got = gpu_advect(ctx, phi, u, dx, dt, scheme, steps)
        ref = oracle_advect(phi, u, dx, dt, scheme, steps)
        check(got, ref, phi, steps, f"2d {NAMES[scheme]} steps={steps}")


@pytest.mark.parametrize("cfl", [0.9, 1.5, 2.0, 3.5])
@pytest.mark.parametrize("scheme", SCHEMES)
def test_abc_3d(ctx, scheme, cfl):
    """ABC flow, 3D, several tiles with ragged tails, reach 1..4."""
    shape = (36, 40, 72)  # z, y, x: x spans 2 tiles of 64 (ragged), y 5 tiles of 8
    phi = W.random_gaussians(shape, 8, seed=2000).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = cfl * dx[0] / 2.0
    for steps in (1, 3):
        got = gpu_advect(ctx, phi, u, dx, dt, scheme, steps, step0=1)
        ref = oracle_advect(phi, u, dx, dt, scheme, steps, step0=1)
        check(got, ref, phi, steps, f"abc {NAMES[scheme]} cfl={cfl} steps={steps}")


@pytest.mark.parametrize("scheme", SCHEMES)
def test_cellular_2d_ragged(ctx, scheme):
    """2D cellular flow on a ragged 37 x 29 grid at CFL 1.3, variable signs."""
    shape = (29, 37)
    rng = np.random.default_rng(77)
    phi = rng.standard_normal(shape).astype(np.float32)
    u = W.cellular_velocity_2d(shape)
    dx = (2 * np.pi / 37, 2 * np.pi / 29)
    dt = 1.3 * dx[1]
    for steps in (1, 6):
        got = gpu_advect(ctx, phi, u, dx, dt, scheme, steps)
        ref = oracle_advect(phi, u, dx, dt, scheme, steps)
        check(got, ref, phi, steps, f"cell2d {NAMES[scheme]} steps={steps}")


@pytest.mark.parametrize("cfl,steps", [(0.75, 40), (3.75, 8)])
@pytest.mark.parametrize("scheme", SCHEMES)
def test_cosine_1d_paper(ctx, scheme, cfl, steps):
    """The paper's 1D cosine test: N = 30 at CFL 0.75 and 3.75 (section 4)."""
    N = 30
    x = np.arange(N) / N
    phi = (-np.cos(2 * np.pi * x)).astype(np.float32)
    u = np.ones((1, N), dtype=np.float32)
    dx = (1.0 / N,)
    dt = cfl / N
    got = gpu_advect(ctx, phi, u, dx, dt, scheme, steps)
    ref = oracle_advect(phi, u, dx, dt, scheme, steps)
    check(got, ref, phi, steps, f"1d {NAMES[scheme]} cfl={cfl}")


# ---------------------------------------------------------------------------
# exact cases
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", SCHEMES)
@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_integer_shift_bit_exact(ctx, scheme, ndim):
    shape = (20, 24, 72)[3 - ndim:]
    rng = np.random.default_rng(100 + ndim)
    phi = rng.standard_normal(shape).astype(np.float32)
    shifts = (1, -2, 3)[:ndim]
    dx = tuple(1.0 for _ in range(ndim))
    u = W.uniform_velocity(shape, shifts)
    got = gpu_advect(ctx, phi, u, dx, 1.0, scheme, 3, step0=0)
    expect = phi.astype(np.float64)
    for d, k in enumerate(shifts):
        expect = np.roll(expect, 3 * k, axis=ndim - 1 - d)
    assert np.array_equal(got, expect)
    ref = oracle_advect(phi, u, dx, 1.0, scheme, 3)
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("scheme", SCHEMES)
def test_constant_field_bit_exact(ctx, scheme):
    shape = (24, 20, 40)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    for val in (1.0, -2.5, 0.1):
        phi = np.full(shape, val, dtype=np.float32)
        got = gpu_advect(ctx, phi, u, dx, 1.7 * dx[0] / 2, scheme, 2)
        assert np.all(got == np.float64(np.float32(val)))


def test_linear_field_cir(ctx):
    """CIR reproduces a field linear in x away from the periodic seam (FP32)."""
    ny, nx = 16, 128
    x = np.arange(nx, dtype=np.float64)
    phi = np.broadcast_to(0.01 * x + 0.5, (ny, nx)).astype(np.float32)
    rng = np.random.default_rng(4)
    u = rng.uniform(-2.5, 2.5, (2, ny, nx)).astype(np.float32)
    got = gpu_advect(ctx, phi, u, (1.0, 1.0), 1.0, oracle.CIR, 1)
    c = oracle.courant(u, 1.0, (1.0, 1.0))
    expect = 0.01 * (x[None, :] - c[0]) + 0.5
    inner = np.broadcast_to((x - 3 >= 0) & (x + 3 < nx), (ny, nx))
    # inputs carry up to half an ulp of rounding, the lerp adds one rounding
    assert np.max(np.abs(got - expect)[inner]) < 4 * 2.0**-24 * 2.0


# ---------------------------------------------------------------------------
# state, determinism, resumption, Courant bound, errors
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", SCHEMES)
def test_deterministic_and_resumable(ctx, scheme):
    shape = (24, 32, 40)
    phi = W.random_gaussians(shape, 4, seed=9).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 1.2 * dx[0] / 2
    a = gpu_advect(ctx, phi, u, dx, dt, scheme, 5, step0=0)
    b = gpu_advect(ctx, phi, u, dx, dt, scheme, 5, step0=0)
    assert np.array_equal(a, b)
    first = gpu_advect(ctx, phi, u, dx, dt, scheme, 3, step0=0).astype(np.float32)
    rest = gpu_advect(ctx, first, u, dx, dt, scheme, 2, step0=3)
    assert np.array_equal(a, rest)


def test_courant_hint(ctx):
    import torch
    from paper_1606_06117_amd import native
    shape = (24, 24, 32)
    phi = W.random_gaussians(shape, 4, seed=10).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 1.5 * dx[0] / 2
    ut = torch.from_numpy(u).cuda()
    assert ctx.courant_max(ut, dx, dt) == pytest.approx(1.5, rel=1e-6)
    measured = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 2)
    hinted = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 2, courant_max=1.5)
    assert np.array_equal(measured, hinted)
    ctx.check()
    # a hint below the true bound: kernels clamp (in bounds) and report it
    gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 1, courant_max=0.5)
    with pytest.raises(native.SlaError) as ei:
        ctx.check()
    assert ei.value.status == native.ECOURANT
    ctx.check()  # the record was cleared


def test_errors(ctx):
    import torch
    from paper_1606_06117_amd import native
    shape = (16, 16, 16)
    phi = torch.zeros(shape, device="cuda")
    u = torch.zeros((3,) + shape, device="cuda")
    dx = (1.0, 1.0, 1.0)
    with pytest.raises(native.SlaError) as ei:
        ctx.advect(phi, u, dx, float("nan"), "cec", 1)
    assert ei.value.status == native.EINVAL
    with pytest.raises(native.SlaError) as ei:
        ctx.advect(phi, u, dx, 1.0, 8, 1)
    assert ei.value.status == native.EINVAL
    with pytest.raises(native.SlaError) as ei:
        ctx.advect(phi, u, dx, 1.0, "cec", -1)
    assert ei.value.status == native.EINVAL
    with pytest.raises(native.SlaError) as ei:
        ctx.advect(phi, u, (1.0, 0.0, 1.0), 1.0, "cec", 1)
    assert ei.value.status == native.EINVAL
    small = torch.zeros((4, 16, 16), device="cuda")
    with pytest.raises(native.SlaError) as ei:
        ctx.advect(small, torch.zeros((3, 4, 16, 16), device="cuda"), dx, 1.0, "cec", 1)
    assert ei.value.status == native.EINVAL
    # Courant number 4 is beyond the kernels' reach
    u.fill_(4.0)
    with pytest.raises(native.SlaError) as ei:
        ctx.advect(phi, u, dx, 1.0, "cec", 1)
    assert ei.value.status == native.ECOURANT
    u.fill_(float("nan"))
    with pytest.raises(native.SlaError) as ei:
        ctx.advect(phi, u, dx, 1.0, "cir", 1)
    assert ei.value.status == native.EINVAL
    # steps == 0 leaves phi untouched
    phi.fill_(3.0)
    ctx.advect(phi, u, dx, 1.0, "cec", 0)
    assert bool((phi == 3.0).all())


def test_norms(ctx):
    import torch
    rng = np.random.default_rng(5)
    for n in (1, 1000, 1 << 20, 3_000_001):
        a = rng.standard_normal(n).astype(np.float32)
        b = rng.standard_normal(n).astype(np.float32)
        got = ctx.norms(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
        ref = oracle.reductions(a, b)
        for k in (0, 1, 3, 4):
            assert got[k] == pytest.approx(ref[k], rel=1e-12, abs=1e-12 * n)
        assert got[2] == ref[2]
        again = ctx.norms(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda())
        assert again == got  # bitwise reproducible
        if n > 1:
            # fields that do not start on a 16-byte boundary take the scalar loads
            da, db = torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()
            got1 = ctx.norms(da[1:], db[1:])
            ref1 = oracle.reductions(a[1:], b[1:])
            for k in (0, 1, 3, 4):
                assert got1[k] == pytest.approx(ref1[k], rel=1e-12, abs=1e-12 * n)
            assert got1[2] == ref1[2]
            # the same values in aligned memory give the same bits
            assert ctx.norms(da[1:].clone(), db[1:].clone()) == got1


def test_cec_1d_reads_only_its_plane(ctx):
    """A 1D third-order step reads the one velocity plane it is given: NaN in
    the memory after it does not reach the result, which equals the one
    kernel per axis path bit for bit."""
    import torch
    from paper_1606_06117_amd import native
    n = 30
    x = np.arange(n) / n
    phi = (-np.cos(2 * np.pi * x)).astype(np.float32)
    big = torch.full((2 * n,), float("nan"), device="cuda")
    big[:n] = 1.0
    u = big[:n].view(1, n)
    dx = (1.0 / n,)
    dt = 0.75 * dx[0]
    p = torch.from_numpy(phi).cuda()
    ctx.advect(p, u, dx, dt, native.CEC, 4)
    torch.cuda.synchronize()
    got = p.cpu().numpy()
    assert np.isfinite(got).all()
    ctx.set_option(native.OPT_SWEEP_KERNEL, 1)
    try:
        q = torch.from_numpy(phi).cuda()
        ctx.advect(q, u, dx, dt, native.CEC, 4)
        torch.cuda.synchronize()
    finally:
        ctx.set_option(native.OPT_SWEEP_KERNEL, 3)
    assert np.array_equal(got, q.cpu().numpy())
    ref = oracle_advect(phi, u.cpu().numpy(), dx, dt, oracle.CEC, 4)
    check(got.astype(np.float64), ref, phi, 4, "1d cec, NaN after u")
    ctx.check()


# ---------------------------------------------------------------------------
# full-size configurations (the benchmark's launch shapes), sampled boxes
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("scheme", SCHEMES)
def test_abc_256_cfl15_boxes(ctx, scheme):
    """256^3, 8 Gaussians, ABC, CFL 1.5: oracle on sampled boxes (exact halos)."""
    shape = (256, 256, 256)
    phi = W.random_gaussians(shape, 8, seed=2000).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 1.5 * dx[0] / 2
    steps = 2
    got = gpu_advect(ctx, phi, u, dx, dt, scheme, steps)
    halo = steps * 3 * 2
    l2, linf = box_parity(got, phi, u, dx, dt, scheme, steps, halo, (24, 24, 24),
                          np.random.default_rng(1), 3)
    print(f"256^3 {NAMES[scheme]} boxes relL2={l2:.3e} Linf={linf:.3e}")
    assert l2 <= TOL * steps and linf <= TOL * steps


def test_abc_512_cfl09_cec_boxes(ctx):
    """The benchmark's workload: 512^3 one scalar, ABC, CFL 0.9, third order."""
    import torch
    shape = (512, 512, 512)
    phi = W.random_gaussians(shape, 8, seed=2000).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    steps = 2
    got = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, steps, courant_max=0.9)
    l2, linf = box_parity(got, phi, u, dx, dt, oracle.CEC, steps, steps * 3, (24, 24, 24),
                          np.random.default_rng(2), 4)
    print(f"512^3 cec boxes relL2={l2:.3e} Linf={linf:.3e}")
    assert l2 <= TOL * steps and linf <= TOL * steps
    torch.cuda.empty_cache()


@pytest.mark.parametrize("cfl", [1.5, 2.0])
def test_abc_512_reach23_sweeps(ctx, cfl):
    """The benchmark's 512^3 workload at CFL 1.5 and 2.0 (reach 2 and 3), in
    the launch shapes the benchmark times: the x+y kernel with two nodes per
    lane (five windows of 104 outputs per row, 128-row chunks) and the
    two-column z march.  Two steps from an odd step, so both orders run.
    The whole grid agrees bitwise with one kernel per axis (one node per
    lane, SLA_OPT_SWEEP_KERNEL 1), and four 24^3 boxes match the oracle."""
    import torch
    from paper_1606_06117_amd import native
    shape = (512, 512, 512)
    phi = W.random_gaussians(shape, 8, seed=2000).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = cfl * dx[0] / 2
    steps = 2
    got = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, steps, step0=1, courant_max=cfl)
    ctx.set_option(native.OPT_SWEEP_KERNEL, 1)
    try:
        per_axis = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, steps, step0=1, courant_max=cfl)
    finally:
        ctx.set_option(native.OPT_SWEEP_KERNEL, 3)
    assert np.array_equal(got, per_axis)
    del per_axis
    l2, linf = box_parity(got, phi, u, dx, dt, oracle.CEC, steps, steps * 3 * (int(cfl) + 1),
                          (24, 24, 24), np.random.default_rng(5), 4, step0=1)
    print(f"512^3 cfl={cfl} boxes relL2={l2:.3e} Linf={linf:.3e}")
    assert l2 <= TOL * steps and linf <= TOL * steps
    torch.cuda.empty_cache()


@pytest.mark.parametrize("variant,launch", [(1, 0), (2, 0), (4, 0), (5, 0), (6, 0), (7, 0), (7, 16),
                                            (8, 0), (8, -16), (8, 1),
                                            (9, -16), (10, 0), (11, -16), (12, 0), (13, 1),
                                            (14, 0), (14, -16)])
@pytest.mark.parametrize("step0", [0, 1])
@pytest.mark.parametrize("shape", [(40, 48, 72), (37, 45, 130), (13, 11, 250), (11, 13, 9)])
def test_fused_step_matches_sweeps(ctx, step0, variant, launch, shape):
    """At reach 1 the fused 3D step and the three sweep kernels evaluate the
    same FP32 operations per node, so their results agree bitwise.  The
    second shape leaves partial x windows, row segments and march chunks;
    the third has 5 x windows (a workgroup of 2 windows past the row's end)
    and fewer rows than one shared-halo workgroup holds; in the fourth a row
    is narrower than a window (its lanes wrap around the row).  Variant 8
    runs in 16-plane chunks and persistent (its workgroups' ranges then
    cross from one group of rows into the next).  Variant 14 (128-node
    windows of two nodes per lane) has one window narrower than the row in
    the first shape, a 2-node last window in the second, and falls back to
    variant 8 on the fourth's odd nx."""
    from paper_1606_06117_amd import native
    phi = W.random_gaussians(shape, 6, seed=31).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    ctx.set_option(native.OPT_CEC3D_KERNEL, variant)
    ctx.set_option(native.OPT_CEC3D_SHAPE, launch)
    try:
        fused = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 3, step0=step0)
    finally:
        ctx.set_option(native.OPT_CEC3D_KERNEL, native.CEC3D_DEFAULT)
        ctx.set_option(native.OPT_CEC3D_SHAPE, 0)
    ctx.set_option(native.OPT_FUSED, 0)
    try:
        sweeps = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 3, step0=step0)
    finally:
        ctx.set_option(native.OPT_FUSED, 1)
    assert np.array_equal(fused, sweeps)
    ref = oracle_advect(phi, u, dx, dt, oracle.CEC, 3, step0=step0)
    check(fused, ref, phi, 3, f"fused step0={step0}")


def test_tuner_choice_is_used_and_gives_the_same_bits(ctx, tmp_path):
    """sla_tune times every fused-step implementation on the grid, keeps the
    fastest per parity, writes its table; a fresh context that loads the
    table runs the same choice.  Results equal the three sweeps bitwise."""
    import torch
    from paper_1606_06117_amd import native
    shape = (48, 40, 72)
    phi = W.random_gaussians(shape, 6, seed=33).astype(np.float32)
    u = W.abc_velocity(shape)
    dx = tuple(2 * np.pi / n for n in reversed(shape))
    dt = 0.9 * dx[0] / 2
    path = str(tmp_path / "tune.txt")
    info = ctx.tune(torch.from_numpy(phi).cuda(), torch.from_numpy(u).cuda(), dx, dt, path)
    print("tuned", info)
    assert info is not None
    for par in ("even", "odd"):
        v, sh, ms = info[par]
        assert v in (1, 2, 4, 6, 7, 8, 9, 10, 11, 14) and ms > 0  # the tuner's candidates
    text = open(path).read()
    assert f"{shape[2]} {shape[1]} {shape[0]} " in text
    tuned = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 3, step0=1)
    ctx.set_option(native.OPT_FUSED, 0)
    try:
        sweeps = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, 3, step0=1)
    finally:
        ctx.set_option(native.OPT_FUSED, 1)
    assert np.array_equal(tuned, sweeps)
    other = native.Context(0)
    try:
        assert other.tune_info(shape) is None
        other.tune_load(path)
        loaded = other.tune_info(shape)
        for par in ("even", "odd"):  # the table keeps the times to 4 decimals
            assert loaded[par][:2] == info[par][:2]
            assert abs(loaded[par][2] - info[par][2]) < 1e-4
        again = gpu_advect(other, phi, u, dx, dt, oracle.CEC, 3, step0=1)
        assert np.array_equal(again, sweeps)
    finally:
        other.close()
    # a Courant number of 1 or more is refused
    with pytest.raises(native.SlaError) as ei:
        ctx.tune(torch.from_numpy(phi).cuda(), torch.from_numpy(u).cuda(), dx, 2.2 * dt)
    assert ei.value.status == native.ECOURANT
    with open(path, "a") as fh:
        fh.write("1 2 3 x\n")
    with pytest.raises(native.SlaError):
        ctx.tune_load(path)


@pytest.mark.parametrize("shape,cfl,steps", [
    ((40, 96, 24), 0.9, 2),    # reach 1, y axis chunked
    ((40, 96, 24), 1.5, 3),    # reach 2
    ((12, 33, 70), 1.8, 3),    # reach 2, ragged (x windows, y chunks)
    ((12, 33, 69), 1.8, 3),    # odd nx: no two-node windows
    ((8, 20, 250), 1.5, 2),    # three two-node windows of 84 outputs
    ((1, 50, 66), 1.5, 2),     # 2D, reach 2
    ((12, 33, 70), 2.5, 2),    # reach 3, ragged
    ((8, 9, 70), 3.5, 2),      # reach 4: halo 12 > axis length 8 and 9
    ((1, 50, 66), 3.5, 2),     # 2D
    ((64, 8, 16), 0.9, 2),     # z columns walked in 2 chunks
])
def test_marching_sweeps_match_tiles(ctx, shape, cfl, steps):
    """The four ways the sweeps run give the same bits (same FP32 operations
    per node): the fused x+y kernel with two nodes per lane (default; even
    nx, reach <= 3) and with one (reach <= 2), z walking columns, one kernel
    per axis with x in lane windows and y, z walking columns, and the
    LDS-tile sweeps.  Odd then even steps, so both orders of the x+y kernels
    run."""
    from paper_1606_06117_amd import native
    if shape[0] == 1:
        shp = shape[1:]
        phi = W.random_gaussians(shp, 5, seed=41).astype(np.float32)
        u = W.cellular_velocity_2d(shp)
    else:
        shp = shape
        phi = W.random_gaussians(shp, 5, seed=41).astype(np.float32)
        u = W.abc_velocity(shp)
    dx = tuple(2 * np.pi / n for n in reversed(shp))
    umax = float(np.max(np.abs(u)))
    dt = cfl * min(dx) / umax
    ctx.set_option(native.OPT_FUSED, 0)
    try:
        pairs = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, steps, step0=1)
        ctx.set_option(native.OPT_SWEEP_KERNEL, 2)
        fused_xy = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, steps, step0=1)
        ctx.set_option(native.OPT_SWEEP_KERNEL, 1)
        march = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, steps, step0=1)
        ctx.set_option(native.OPT_SWEEP_KERNEL, 0)
        tiles = gpu_advect(ctx, phi, u, dx, dt, oracle.CEC, steps, step0=1)
    finally:
        ctx.set_option(native.OPT_SWEEP_KERNEL, 3)
        ctx.set_option(native.OPT_FUSED, 1)
    assert np.array_equal(march, tiles)
    assert np.array_equal(fused_xy, tiles)
    assert np.array_equal(pairs, tiles)


@pytest.mark.parametrize("scheme", [oracle.FEC_SPLIT, oracle.BEC_SPLIT, oracle.CEC_LITERAL])
@pytest.mark.parametrize("shape,cfl", [
    ((40, 96, 24), 0.9),    # reach 1
    ((12, 33, 70), 1.8),    # reach 2, ragged
    ((12, 33, 69), 1.8),    # odd nx
    ((12, 33, 70), 2.5),    # reach 3: x and y in the two-node kernel
    ((8, 9, 70), 3.5),      # reach 4: one sweep per axis
    ((1, 50, 66), 1.5),     # 2D
])
def test_split_schemes_sweep_kernels_agree(ctx, scheme, shape, cfl):
    """FEC, BEC and the literal-weight third order split per axis run on the
    third order's sweep kernels (only the last stage of a sweep differs): the
    default (x and y in one kernel with two nodes per lane where nx is even),
    one node per lane, one kernel per axis, and the LDS tiles give the same
    bits.  Two steps from an odd step, so both sweep orders run."""
    from paper_1606_06117_amd import native
    if shape[0] == 1:
        shp = shape[1:]
        phi = W.random_gaussians(shp, 5, seed=43).astype(np.float32)
        u = W.cellular_velocity_2d(shp)
    else:
        shp = shape
        phi = W.random_gaussians(shp, 5, seed=43).astype(np.float32)
        u = W.abc_velocity(shp)
    dx = tuple(2 * np.pi / n for n in reversed(shp))
    dt = cfl * min(dx) / float(np.max(np.abs(u)))
    outs = []
    for kern in (3, 2, 1, 0):
        ctx.set_option(native.OPT_SWEEP_KERNEL, kern)
        try:
            outs.append(gpu_advect(ctx, phi, u, dx, dt, scheme, 2, step0=1))
        finally:
            ctx.set_option(native.OPT_SWEEP_KERNEL, 3)
    for o in outs[1:]:  # the literal weights are NaN where |c| is whole (c = 0 at some nodes)
        assert np.array_equal(outs[0], o, equal_nan=True)
    if scheme != oracle.CEC_LITERAL:  # the literal weights amplify rounding near whole |c|
        ref = oracle_advect(phi, u, dx, dt, scheme, 2, step0=1)
        assert rel_l2(outs[0], ref) < 1e-5


def test_fused_1024_matches_sweeps_and_last_cell(ctx):
    """2^30 cells, the largest grid the fused kernels take, at CFL 0.9 (the
    fused path, default implementation): two steps agree bitwise with the
    three sweeps over the whole grid, and 16^3 boxes, one wrapping around
    the grid's last cell and one inside, match the FP64 oracle.  A buffer
    descriptor's size tops out one byte short of 2^32, so a descriptor on
    the field's start would clip the last element of such a field; the
    kernels rebase theirs on each row or plane."""
    import torch
    from paper_1606_06117_amd import native
    N, steps, inner = 1024, 2, 16
    halo = 3 * steps  # three calls of reach 1 per axis and step
    shape = (N, N, N)
    dev = torch.device("cuda:0")
    phi0 = W.fourier_modes_torch(shape, 11, dev)
    u = W.abc_velocity_torch(shape, dev)
    dx = (2 * np.pi / N,) * 3
    dt = W.abc_dt(shape, 0.9)
    big = inner + 2 * halo
    boxes = {"last cell": (np.arange(big) + N - inner // 2 - halo) % N, "interior": np.arange(big) + 500}
    idx = {k: torch.from_numpy(v).to(dev) for k, v in boxes.items()}
    sub = lambda a, i: a[..., i[:, None, None], i[None, :, None], i[None, None, :]]
    inputs = {k: (sub(phi0, i).cpu().numpy(), torch.stack([sub(u[d], i) for d in range(3)]).cpu().numpy())
              for k, i in idx.items()}
    fused = phi0.clone()
    ctx.advect(fused, u, dx, dt, native.CEC, steps, 0, 0.0)
    ctx.set_option(native.OPT_FUSED, 0)
    try:
        sweeps = phi0.clone()
        ctx.advect(sweeps, u, dx, dt, native.CEC, steps, 0, 0.0)
    finally:
        ctx.set_option(native.OPT_FUSED, 1)
    torch.cuda.synchronize()
    diff = (fused != sweeps).reshape(-1)
    ndiff = int(diff.sum())
    first = torch.nonzero(diff)[:4].reshape(-1).tolist() if ndiff else []
    inner_sl = (slice(halo, halo + inner),) * 3
    got = {k: sub(fused, i).cpu().numpy()[inner_sl] for k, i in idx.items()}
    del phi0, u, fused, sweeps, diff
    torch.cuda.empty_cache()
    assert ndiff == 0, f"{ndiff} cells differ, first flat indices {first}"
    for k, (p0, u0) in inputs.items():
        ref = oracle.advect(p0.astype(np.float64), u0, dx, dt, oracle.CEC, steps, 0)[inner_sl]
        check(got[k].astype(np.float64), ref, p0, steps, f"1024^3 fused, {k} box")


def test_large_1024_cfl2_cec_box(ctx):
    """The large problem at its full size: 1024^3 (2^30 cells, the largest
    grid the 32-bit offsets of the fused and marching kernels take), a
    k^-5/3 field (|k| <= 64) built on the GPU, ABC velocity, CFL 2.0 (reach
    3, three-sweep path), 10 third-order steps.  The oracle runs on a 308^3
    block around a 128^3 box: each step moves information at most 9 cells
    per axis (three calls of reach 3), so after 10 steps the central 128^3
    of the block equals the full-grid result."""
    import torch
    from paper_1606_06117_amd import native
    N, steps, inner, halo = 1024, 10, 128, 90
    shape = (N, N, N)
    dev = torch.device("cuda:0")
    phi = W.power_law_torch(shape, 5000, dev)
    u = W.abc_velocity_torch(shape, dev)
    dx = (2 * np.pi / N,) * 3
    dt = W.abc_dt(shape, 2.0)
    lo = np.random.default_rng(7).integers(0, N, 3)
    big = inner + 2 * halo
    idx = [torch.from_numpy((np.arange(big) + int(l) - halo) % N).to(dev) for l in lo]
    sub = lambda a: a[..., idx[0][:, None, None], idx[1][None, :, None], idx[2][None, None, :]]
    sub_phi = sub(phi).cpu().numpy()
    sub_u = torch.stack([sub(u[d]) for d in range(3)]).cpu().numpy()
    ctx.advect(phi, u, dx, dt, native.CEC, steps, 0, 0.0)
    torch.cuda.synchronize()
    got = sub(phi).cpu().numpy()[halo:halo + inner, halo:halo + inner, halo:halo + inner]
    del phi, u
    torch.cuda.empty_cache()
    ref = oracle.advect(sub_phi.astype(np.float64), sub_u, dx, dt, oracle.CEC, steps, 0)
    ref = ref[halo:halo + inner, halo:halo + inner, halo:halo + inner]
    l2 = rel_l2(got.astype(np.float64), ref)
    linf = float(np.max(np.abs(got - ref))) / float(np.max(np.abs(sub_phi)))
    print(f"1024^3 cfl 2.0 cec, 128^3 box: relL2={l2:.3e} Linf={linf:.3e}")
    assert l2 <= TOL * steps and linf <= TOL * steps
