"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a formula
the paper prints in a different form from the oracle's composition of
interpolation calls, a textbook special case, an exact invariant, or a
measured convergence order.  A plausible slip in the oracle (a dropped
term, a wrong sign, a swapped index, a wrong sweep) breaks at least one.
"""

import math
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import CIR, FEC, BEC, CEC

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
NAMES = {"cir": CIR, "fec": FEC, "bec": BEC, "cec": CEC}


def impulse_response(scheme, c, N=16):
    """Coefficient of Phi[i + o] in output i, for constant Courant ``c`` (1D)."""
    i0 = N // 2
    coef = {}
    for j in range(N):
        phi = np.zeros(N)
        phi[j] = 1.0
        out = oracle.step(phi, np.full((1, N), c), scheme)
        o = (j - i0 + N // 2) % N - N // 2
        if out[i0] != 0.0:
            coef[o] = out[i0]
    return coef


# ---------------------------------------------------------------------------
# constant-velocity stencils (golden fixture, hand-evaluated paper formulas)
# ---------------------------------------------------------------------------

def load_golden():
    rows = []
    with open(os.path.join(GOLDEN, "const_u_stencils.txt")) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            name, U, off, val = line.split()
            rows.append((name, Fraction(U), int(off), Fraction(val)))
    return rows


def test_golden_stencils_match_impulse_response():
    rows = load_golden()
    assert len(rows) == 6 + 9 + 12 + 12
    by_key = {}
    for name, U, off, val in rows:
        by_key.setdefault((name, U), {})[off] = val
    for (name, U), expect in by_key.items():
        assert sum(expect.values()) == 1, (name, U)  # consistency of the fixture
        got = impulse_response(NAMES[name], float(U))
        assert set(got) == set(expect), (name, U, got)
        for off, val in expect.items():
            assert got[off] == pytest.approx(float(val), abs=1e-15), (name, U, off)


@pytest.mark.parametrize("U", [0.05, 0.3, 0.61, 0.9, 0.999])
def test_const_u_stencils_random_u(U):
    """eq. cstUHALO and eq. cstUBEC at arbitrary U, and A*FEC+B*BEC for CEC."""
    fec = {1: -0.5 * U * (1 - U), 0: 1 - U * U, -1: 0.5 * U * (1 + U)}
    bec = {1: -U / 2 * (1 - U) ** 2,
           0: (1 - U) / 2 * (3 - (1 - U) ** 2 - 2 * U * U),
           -1: U / 2 * (3 - 2 * (1 - U) ** 2 - U * U),
           -2: -U * U / 2 * (1 - U)}
    A = (2 - 1 / U) / 3
    B = 1 - A
    cec = {o: A * fec.get(o, 0.0) + B * bec.get(o, 0.0) for o in bec}
    for scheme, expect in ((FEC, fec), (BEC, bec), (CEC, cec)):
        got = impulse_response(scheme, U)
        for o in set(got) | set(expect):
            assert got.get(o, 0.0) == pytest.approx(expect.get(o, 0.0), abs=2e-14), (scheme, U, o)
    # mirrored velocity: the stencil mirrors
    for scheme, expect in ((FEC, fec), (BEC, bec), (CEC, cec)):
        got = impulse_response(scheme, -U)
        for o in expect:
            assert got.get(-o, 0.0) == pytest.approx(expect[o], abs=2e-14)


@pytest.mark.parametrize("U", [0.1, 0.37, 0.5, 0.83])
def test_cec_is_cubic_lagrange(U):
    """Textbook special case: the third-order constant-U scheme is the cubic
    Lagrange interpolant through nodes i+1, i, i-1, i-2 at x_i - U."""
    x = -U
    nodes = [1, 0, -1, -2]
    got = impulse_response(CEC, U)
    for k in nodes:
        L = 1.0
        for m in nodes:
            if m != k:
                L *= (x - m) / (k - m)
        assert got.get(k, 0.0) == pytest.approx(L, abs=2e-15)


def test_table1_cec_formula_sign_corrected():
    """Table 1's CEC row, with its second coefficient read as (2U-1)/(6U):
    L_U[Phi + (1+U)/(6U) e] + (2U-1)/(6U) e.  The printed (1-2U)/(6U) is off."""
    rng = np.random.default_rng(7)
    N = 40
    phi = rng.standard_normal(N)
    for U in (0.2, 0.45, 0.8):
        c = np.full((1, N), U)
        phi1 = oracle.interp(phi, c)
        e = phi - oracle.interp(phi1, -c)
        fixed = oracle.interp(phi + (1 + U) / (6 * U) * e, c) + (2 * U - 1) / (6 * U) * e
        printed = oracle.interp(phi + (1 + U) / (6 * U) * e, c) + (1 - 2 * U) / (6 * U) * e
        got = oracle.step(phi, c, CEC)
        assert np.max(np.abs(got - fixed)) < 1e-14
        assert np.max(np.abs(got - printed)) > 1e-3


# ---------------------------------------------------------------------------
# variable-velocity stencils (Appendix A)
# ---------------------------------------------------------------------------

def _var_u(N, seed, mixed=True):
    rng = np.random.default_rng(seed)
    U = rng.uniform(0.02, 0.98, N)
    s = rng.choice([-1, 1], N) if mixed else np.ones(N, dtype=int)
    return rng.standard_normal(N), U, s


@pytest.mark.parametrize("mixed", [False, True])
def test_appendix_fec_variable_u(mixed):
    """eq. exp:FEC with the velocity subscripts read as -U_i(1-U_{i+s_i}) on
    Phi_{i+s_i} and U_i(1+U_i) on Phi_{i-s_i}: the printed subscripts do not
    sum to 2 (a constant would not be preserved)."""
    N = 48
    phi, U, s = _var_u(N, 11, mixed)
    W = lambda k: U[k % N]  # noqa: E731
    S = lambda k: s[k % N]  # noqa: E731
    P = lambda k: phi[k % N]  # noqa: E731
    expect = np.empty(N)
    for i in range(N):
        si = S(i)
        two = (-W(i) * (1 - W(i + si)) * P(i + si)
               + (2 - W(i) * W(i)) * P(i)
               - W(i) * W(i + si) * P(i + si - S(i + si))
               + W(i) * (1 + W(i)) * P(i - si))
        expect[i] = 0.5 * two
    got = oracle.fec(phi, (s * U)[None, :])
    assert np.max(np.abs(got - expect)) < 1e-14


@pytest.mark.parametrize("mixed", [False, True])
def test_appendix_bec_variable_u(mixed):
    """eq. exp:bec, its seven coefficients f as printed.  The position of the
    sixth term is read as i - s_i + s_{i-s_i} - s_{i-s_i+s_{i-s_i}} (the print
    has s_{i+s_i} in the middle, which only differs when signs are mixed)."""
    N = 48
    phi, U, s = _var_u(N, 12, mixed)
    W = lambda k: U[k % N]  # noqa: E731
    S = lambda k: s[k % N]  # noqa: E731
    expect = np.zeros(N)
    for i in range(N):
        si = S(i)
        j = i - si
        terms = [
            (i + si, -(1 - W(i)) * W(i) * (1 - W(i + si))),
            (i, (1 - W(i)) * (3 - (1 - W(i)) ** 2)),
            (j + S(j), -W(i) * W(j) * (1 - W(j + S(j)))),
            (i + si - S(i + si), -(1 - W(i)) * W(i) * W(i + si)),
            (j, W(i) * (3 - (1 - W(j)) ** 2) - (1 - W(i)) * ((1 - W(i)) * W(i))),
            (j + S(j) - S(j + S(j)), -W(i) * W(j) * W(j + S(j))),
            (j - S(j), -W(i) * (1 - W(j)) * W(j)),
        ]
        assert sum(v for _, v in terms) == pytest.approx(2.0, abs=1e-14)
        expect[i] = 0.5 * sum(v * phi[p % N] for p, v in terms)
    got = oracle.bec(phi, (s * U)[None, :])
    assert np.max(np.abs(got - expect)) < 1e-14


def test_cir2d_printed_form():
    """eq. CIR2D: four weights, including the diagonal corner."""
    rng = np.random.default_rng(5)
    ny, nx = 12, 14
    phi = rng.standard_normal((ny, nx))
    Ux = rng.uniform(0, 0.99, (ny, nx))
    Uy = rng.uniform(0, 0.99, (ny, nx))
    sx = rng.choice([-1, 1], (ny, nx))
    sy = rng.choice([-1, 1], (ny, nx))
    expect = np.empty_like(phi)
    for j in range(ny):
        for i in range(nx):
            ux, uy, a, b = Ux[j, i], Uy[j, i], sx[j, i], sy[j, i]
            expect[j, i] = ((1 - ux) * (1 - uy) * phi[j, i]
                            + (1 - ux) * uy * phi[(j - b) % ny, i]
                            + ux * (1 - uy) * phi[j, (i - a) % nx]
                            + ux * uy * phi[(j - b) % ny, (i - a) % nx])
    c = np.stack([sx * Ux, sy * Uy])
    assert np.max(np.abs(oracle.cir(phi, c) - expect)) < 1e-14


def test_split_sweeps_match_split_upwind_form():
    """eqs. split:1 and split:2 are the CIR sweeps of a split step; the
    third-order sweep built from them reduces to them when its correction
    vanishes (e = 0 for an integer Courant number)."""
    rng = np.random.default_rng(6)
    ny, nx = 10, 12
    phi = rng.standard_normal((ny, nx))
    Ux = rng.uniform(0, 0.99, (ny, nx))
    sx = rng.choice([-1, 1], (ny, nx))
    star = np.empty_like(phi)
    for j in range(ny):
        for i in range(nx):
            star[j, i] = (1 - Ux[j, i]) * phi[j, i] + Ux[j, i] * phi[j, (i - sx[j, i]) % nx]
    c = np.stack([sx * Ux, np.zeros_like(Ux)])
    assert np.max(np.abs(oracle.interp(phi, c) - star)) < 1e-14


# ---------------------------------------------------------------------------
# amplification factors and modified equations (section 3, Table 1)
# ---------------------------------------------------------------------------

def symbol(scheme, c, N, m, ndim=1):
    """Measured amplification of the mode exp(i theta j) with theta = 2 pi m / N."""
    theta = 2 * np.pi * m / N
    j = np.arange(N)
    if ndim == 1:
        cs = np.full((1, N), c)
        re = oracle.step(np.cos(theta * j), cs, scheme)
        im = oracle.step(np.sin(theta * j), cs, scheme)
        z = (re + 1j * im) * np.exp(-1j * theta * j)
        assert np.max(np.abs(z - z.mean())) < 1e-12  # a Fourier mode is an eigenvector
        return z.mean()
    raise ValueError


def xi_fec(U, th):
    """Printed amplification factor of FEC (section 3)."""
    return 1 - U * U + U * U * np.cos(th) - 1j * U * np.sin(th)


def xi_bec(U, th):
    """Printed amplification factor of BEC (section 3)."""
    s = np.sin(th / 2)
    return 1 - 2j * U * s * (np.exp(-0.5j * th) * U * (1 + 2 * (1 - U) * s * s)
                             + np.cos(th / 2) * (1 - U))


@pytest.mark.parametrize("U", [0.15, 0.5, 0.72, 0.95])
@pytest.mark.parametrize("m", [1, 3, 7, 16])
def test_printed_amplification_factors(U, m):
    N = 32
    th = 2 * np.pi * m / N
    assert symbol(FEC, U, N, m) == pytest.approx(xi_fec(U, th), abs=1e-13)
    assert symbol(BEC, U, N, m) == pytest.approx(xi_bec(U, th), abs=1e-13)
    # CEC is linear in FEC and BEC (eq. intro:CEC), so its factor is A xi_F + B xi_B
    A = (2 - 1 / U) / 3
    assert symbol(CEC, U, N, m) == pytest.approx(A * xi_fec(U, th) + (1 - A) * xi_bec(U, th), abs=1e-13)
    # CIR: first equation of section 3
    assert symbol(CIR, U, N, m) == pytest.approx(1 - U + U * np.exp(-1j * th), abs=1e-13)


@pytest.mark.parametrize("U", [0.2, 0.45, 0.8])
def test_modified_equation_coefficients(U):
    """Table 1 error column.  With U = u dt/dx and theta = k dx, a term
    C_a d^a/dx^a of the modified equation contributes C_a (ik)^a dt to
    log(g); each coefficient is compared with the measured log-symbol of a
    well-resolved mode, where higher terms are down by O(theta)."""
    N, m = 1024, 2
    th = 2 * np.pi * m / N
    lead = -1j * U * th
    # CIR: D = (1-U)|u|dx/2 on d2/dx2 -> -U(1-U) theta^2 / 2
    g = np.log(symbol(CIR, U, N, m)) - lead
    assert g.real / th**2 == pytest.approx(-U * (1 - U) / 2, rel=2e-2)
    # FEC: -(1-U^2) u dx^2/3! d3 -> i U (1-U^2) theta^3/6 ; -3(1-U^2)u^2 dx^2 dt/4! d4
    g = np.log(symbol(FEC, U, N, m)) - lead
    assert g.imag / th**3 == pytest.approx(U * (1 - U * U) / 6, rel=2e-2)
    assert g.real / th**4 == pytest.approx(-3 * (1 - U * U) * U * U / 24, rel=2e-2)
    # BEC: -(1-U)(1-2U) u dx^2/3! d3 ; -9(1-U)^2 u^2 dx^2 dt/4! d4
    g = np.log(symbol(BEC, U, N, m)) - lead
    assert g.imag / th**3 == pytest.approx(U * (1 - U) * (1 - 2 * U) / 6, rel=2e-2, abs=1e-9)
    assert g.real / th**4 == pytest.approx(-9 * (1 - U) ** 2 * U * U / 24, rel=2e-2)
    # CEC: no third-derivative term; -(1+U)(1-U)(2-U)|u| dx^3/4! d4
    g = np.log(symbol(CEC, U, N, m)) - lead
    assert abs(g.imag / th**3) < 1e-2 * U
    assert g.real / th**4 == pytest.approx(-(1 + U) * (1 - U) * (2 - U) * U / 24, rel=2e-2)


# ---------------------------------------------------------------------------
# large Courant numbers (section 4, eq. intro:CECcoefSL)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("U", [1.0, 1.3, 2.0, 2.75, 3.5])
@pytest.mark.parametrize("sign", [1, -1])
def test_large_cfl_is_shift_of_fractional_scheme(U, sign):
    """Weights from U mod 1: the step at U = n + f is the shift by n of the
    step at f, for every scheme that uses them (CIR and the third order)."""
    rng = np.random.default_rng(3)
    N = 40
    phi = rng.standard_normal(N)
    n = int(math.floor(U))
    f = U - n
    for scheme in (CIR, CEC):
        big = oracle.step(phi, np.full((1, N), sign * U), scheme)
        small = oracle.step(phi, np.full((1, N), sign * f), scheme)
        assert np.array_equal(big, np.roll(small, sign * n)), scheme


def test_stability_nonlocal():
    """|g| <= 1 for the non-local stencils at Courant numbers up to 4 (the
    paper's large-CFL claim, section 4), for every scheme."""
    N = 64
    for scheme in (CIR, FEC, BEC, CEC):
        worst = 0.0
        for U in np.linspace(0.05, 3.95, 40):
            for m in range(1, N // 2 + 1, 3):
                worst = max(worst, abs(symbol(scheme, U, N, m)))
        assert worst <= 1 + 1e-12, scheme


# ---------------------------------------------------------------------------
# exact invariants
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("scheme", [CIR, FEC, BEC, CEC])
def test_integer_courant_is_exact_shift(ndim, scheme):
    rng = np.random.default_rng(ndim)
    shape = (9, 10, 11)[3 - ndim:]
    phi32 = rng.standard_normal(shape).astype(np.float32)
    shifts = (1, -2, 0)[:ndim]
    c = np.stack([np.full(shape, float(k)) for k in shifts])
    out = oracle.step(phi32.astype(np.float64), c, scheme, m=1)
    expect = phi32.astype(np.float64)
    for d, k in enumerate(shifts):
        expect = np.roll(expect, k, axis=ndim - 1 - d)
    assert np.array_equal(out, expect)
    # the FP32 result is exact too (the values are FP32 inputs moved around)
    assert np.array_equal(out.astype(np.float32).astype(np.float64), out)


@pytest.mark.parametrize("scheme", [CIR, FEC, BEC, CEC])
def test_constants_exact(scheme):
    rng = np.random.default_rng(9)
    shape = (6, 7, 8)
    c = rng.uniform(-2.9, 2.9, (3,) + shape)
    for val in (0.0, 1.0, -3.25, 0.1):
        out = oracle.step(np.full(shape, val), c, scheme, m=0)
        assert np.all(out == val)


def test_linear_field_cir_variable_u():
    """CIR reproduces a field linear in x exactly away from the periodic seam."""
    rng = np.random.default_rng(10)
    ny, nx = 8, 64
    alpha, beta = 0.37, -1.2
    x = np.arange(nx, dtype=np.float64)
    phi = np.broadcast_to(alpha * x + beta, (ny, nx)).copy()
    cx = rng.uniform(-2.5, 2.5, (ny, nx))
    cy = rng.uniform(-2.5, 2.5, (ny, nx))
    out = oracle.cir(phi, np.stack([cx, cy]))
    expect = alpha * (x[None, :] - cx) + beta
    inner = (x[None, :] - np.abs(cx) >= 1) & (x[None, :] + np.abs(cx) <= nx - 2)
    assert inner.sum() > 300
    assert np.max(np.abs(out - expect)[inner]) < 1e-13 * 30


@pytest.mark.parametrize("scheme", [CIR, FEC, BEC, CEC])
def test_mass_conserved_uniform_u(scheme):
    rng = np.random.default_rng(13)
    shape = (10, 12, 14)
    phi = rng.uniform(0, 1, shape)
    c = np.stack([np.full(shape, v) for v in (0.63, -1.41, 2.2)])
    out = oracle.run(phi, c, scheme, 5)
    assert abs(oracle.mass_error(out, phi)) < 1e-14


def test_split_uniform_u_is_tensor_product():
    """Uniform U: the sweeps commute, so the sweep order does not matter and
    the 2D factor is the product of the 1D factors."""
    ny, nx = 16, 16
    cx, cy = 0.3, -0.55
    c = np.stack([np.full((ny, nx), cx), np.full((ny, nx), cy)])
    j, i = np.mgrid[0:ny, 0:nx]
    for mx, my in ((1, 2), (3, 5)):
        tx, ty = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
        mode_r = np.cos(tx * i + ty * j)
        mode_i = np.sin(tx * i + ty * j)
        for m in (0, 1):
            z = oracle.cec_split(mode_r, c, m) + 1j * oracle.cec_split(mode_i, c, m)
            g = (z * np.exp(-1j * (tx * i + ty * j))).mean()
            gx = symbol(CEC, cx, nx, mx)
            gy = symbol(CEC, cy, ny, my)
            assert g == pytest.approx(gx * gy, abs=1e-13)


def test_unsplit_fec_bec_symbols_2d():
    """Definitions of FEC and BEC applied to a 2D mode with uniform U: with
    g the bilinear CIR factor, FEC -> g + (1-|g|^2)/2, BEC -> g (1 + (1-|g|^2)/2)."""
    ny, nx = 16, 16
    cx, cy = 0.7, 0.35
    c = np.stack([np.full((ny, nx), cx), np.full((ny, nx), cy)])
    j, i = np.mgrid[0:ny, 0:nx]
    mx, my = 2, 3
    tx, ty = 2 * np.pi * mx / nx, 2 * np.pi * my / ny
    g = (1 - cx + cx * np.exp(-1j * tx)) * (1 - cy + cy * np.exp(-1j * ty))
    w = (1 - abs(g) ** 2) / 2
    for scheme, expect in ((CIR, g), (FEC, g + w), (BEC, g * (1 + w))):
        z = oracle.step(np.cos(tx * i + ty * j), c, scheme) + 1j * oracle.step(np.sin(tx * i + ty * j), c, scheme)
        got = (z * np.exp(-1j * (tx * i + ty * j))).mean()
        assert got == pytest.approx(expect, abs=1e-13)


def test_sweep_order_alternates():
    assert oracle.sweep_order(0, 3) == (0, 1, 2)
    assert oracle.sweep_order(1, 3) == (2, 1, 0)
    assert oracle.sweep_order(6, 2) == (0, 1)
    assert oracle.sweep_order(7, 2) == (1, 0)


def test_variable_u_sweep_order_matters_and_is_used():
    """With a variable velocity the sweeps do not commute; step m uses x,y,z
    for even m and z,y,x for odd m."""
    rng = np.random.default_rng(21)
    shape = (8, 9, 10)
    phi = rng.standard_normal(shape)
    c = rng.uniform(-0.9, 0.9, (3,) + shape)
    xyz = oracle.cec_sweep(oracle.cec_sweep(oracle.cec_sweep(phi, c[0], 0), c[1], 1), c[2], 2)
    zyx = oracle.cec_sweep(oracle.cec_sweep(oracle.cec_sweep(phi, c[2], 2), c[1], 1), c[0], 0)
    assert np.max(np.abs(xyz - zyx)) > 1e-3
    assert np.array_equal(oracle.cec_split(phi, c, 4), xyz)
    assert np.array_equal(oracle.cec_split(phi, c, 5), zyx)


# ---------------------------------------------------------------------------
# convergence orders (Table 1 errors; C_alpha ~ N^(1-alpha), Appendix B)
# ---------------------------------------------------------------------------

def periodic_gaussian_2d(N, cx, cy, sigma):
    x = (np.arange(N) + 0.0) / N
    out = np.zeros((N, N))
    for ox in (-1, 0, 1):
        for oy in (-1, 0, 1):
            gx = np.exp(-((x - cx + ox) ** 2) / (2 * sigma**2))
            gy = np.exp(-((x - cy + oy) ** 2) / (2 * sigma**2))
            out += gy[:, None] * gx[None, :]
    return out


def conv_errors(scheme, Ns, steps64=100):
    errs = []
    for N in Ns:
        steps = steps64 * N // 64
        cx, cy = 0.7, 0.35  # u = (1, 0.5), CFL 0.7
        c = np.stack([np.full((N, N), cx), np.full((N, N), cy)])
        phi0 = periodic_gaussian_2d(N, 0.5, 0.5, 0.1)
        out = oracle.run(phi0, c, scheme, steps)
        T = steps * 0.7 / N
        exact = periodic_gaussian_2d(N, (0.5 + T * 1.0) % 1.0, (0.5 + T * 0.5) % 1.0, 0.1)
        errs.append(oracle.rel_l2(out, exact))
    return errs


@pytest.mark.parametrize("scheme,order", [(CIR, 1), (FEC, 2), (BEC, 2), (CEC, 3)])
def test_convergence_orders(scheme, order):
    Ns = (32, 64, 128) if scheme != CEC else (32, 64, 128)
    errs = conv_errors(scheme, Ns, steps64=50)
    slope = math.log(errs[-2] / errs[-1], 2)
    tol = 0.2 if order > 1 else 0.25
    assert abs(slope - order) < tol, (scheme, errs, slope)
