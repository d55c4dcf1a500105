"""FP64 oracle of the advection step (test infrastructure only).

Arrays follow NumPy C order with x fastest: a 3D field is ``phi[z, y, x]``,
a 2D field ``phi[y, x]``, a 1D field ``phi[x]``.  Physical axis ``d``
(0 = x, 1 = y, 2 = z) is NumPy axis ``ndim - 1 - d``.  Velocities and
Courant numbers are stacked per physical axis: ``c[d]`` has the field's shape.

What is computed, and where the paper defines it:

* The advection problem and the interpolation operator
  ``L_U[Phi](x) = Phi~(x - U dt)`` are set up in section 2 ("Multi-stage
  approaches", eq. intro:adv and the definition of L_U after it).
* The one-dimensional CIR step, the sign ``s_i = sgn(u_i)`` and the reduced
  velocity ``U_i = |u_i| dt/dx`` are those of section 3 ("One-dimensional
  algorithms", first equation).  With a non-local stencil (section 4,
  large-CFL paragraph before eq. intro:CECcoefSL) the departure point may
  lie ``n = floor(U)`` cells away; the two nodes bracketing it are used.
* The multi-dimensional CIR step is the tensor-product (multilinear)
  interpolation of section 5 ("Multi-dimensional problems", eq. CIR2D),
  extended to 3D in the same way.
* FEC and BEC are eq. intro:FEC and eq. intro:BEC (Table 1 rows 2-3),
  applied unsplit in 2D/3D.
* The third-order scheme ("CEC") is eq. intro:CEC with the weights of
  eq. intro:CECcoef; in 2D/3D it is applied one axis at a time
  (section 5, eqs. split:1 and split:2), alternating the sweep order
  between consecutive steps so that pairs of steps are symmetric (section 5
  asks for a Strang-type splitting for more than first order).

Readings taken where the paper is ambiguous (each one is listed with its
justification in the design notes):

* Per-axis third-order sweep, division-free form:
  ``Phi' = Phi1 + 1/2 [e_a + (1+f)/3 (e_b - e_a)]`` with
  ``Phi1 = L_U Phi``, ``e = Phi - L_{-U} L_U Phi``, ``a``/``b`` the anchor
  and far nodes of the departure interval and ``f`` the fractional
  Courant number.  For U < 1 it equals ``A FEC + B BEC`` with
  ``3A = 2 - 1/U``, ``B = 1 - A`` exactly; for U >= 1 it is the integer
  shift composed with the fractional-U scheme of eq. intro:CECcoefSL.
* Table 1's CEC formula has a sign slip in its second term; the form that
  equals ``A FEC + B BEC`` carries ``(2U-1)/(6U)``.
* The Courant number ``c = u dt/dx`` decides the integer part of the
  departure offset.  That decision is taken in FP32, as the GPU takes it:
  ``c = fl32(u * fl32(dt/dx))``.  Everything after the decision is FP64.
* ``c = 0`` (and ``-0.0``) counts as ``s = +1``; then ``f = 0`` and the
  result does not depend on ``s``.
* Linear interpolation is written ``p + f (q - p)`` with ``p`` the node
  nearer the arrival point, so integer shifts and constants come out
  exact in any precision.
"""

from __future__ import annotations

import itertools

import numpy as np

CIR, FEC, BEC, CEC, CEC_STRANG, FEC_SPLIT, BEC_SPLIT, CEC_LITERAL = 0, 1, 2, 3, 4, 5, 6, 7
SCHEMES = {"cir": CIR, "fec": FEC, "bec": BEC, "cec": CEC, "cec_strang": CEC_STRANG,
           "fec_split": FEC_SPLIT, "bec_split": BEC_SPLIT, "cec_literal": CEC_LITERAL}


# ---------------------------------------------------------------------------
# departure decomposition (section 3, definitions of s_i and U_i; section 4,
# non-local stencil for CFL > 1)
# ---------------------------------------------------------------------------

def courant(u, dt, dx):
    """Courant numbers ``c[d] = u[d] * dt / dx[d]`` decided in FP32.

    ``u`` is an array of shape ``(ndim, *grid)`` (any float dtype; it is
    rounded to FP32 first, as the GPU receives it).  ``dx`` is a sequence of
    ``ndim`` cell sizes (x first).  ``dt / dx`` is formed in FP64 and
    rounded to FP32 once; the product with ``u`` is one FP32 multiply.
    The result is returned promoted to FP64.
    """
    u = np.asarray(u)
    ndim = u.shape[0]
    if len(dx) != ndim:
        raise ValueError("need one cell size per axis")
    out = np.empty(u.shape, dtype=np.float64)
    for d in range(ndim):
        lam = np.float32(float(dt) / float(dx[d]))
        out[d] = (u[d].astype(np.float32) * lam).astype(np.float64)
    return out


def departure(c):
    """Split Courant numbers into sign, integer offset and fraction.

    Returns ``(s, n, f)`` with ``s = +1`` where ``c >= 0`` else ``-1``,
    ``n = floor(|c|)`` and ``f = |c| - n`` in ``[0, 1)``.  The departure
    point ``x_i - c`` lies between the anchor node ``i - s n`` and the far
    node ``i - s (n + 1)``.
    """
    c = np.asarray(c, dtype=np.float64)
    s = np.where(c >= 0.0, 1, -1).astype(np.int64)
    mag = np.abs(c)
    n = np.floor(mag)
    f = mag - n
    return s, n.astype(np.int64), f


def _lerp(p, q, f):
    return p + f * (q - p)


def _nodes(shape, axis, s, n):
    """Anchor and far indices (positive modulo) along one NumPy axis."""
    N = shape[axis]
    view = [1] * len(shape)
    view[axis] = N
    i = np.arange(N, dtype=np.int64).reshape(view)
    a = np.mod(i - s * n, N)
    b = np.mod(i - s * (n + 1), N)
    return a, b


# ---------------------------------------------------------------------------
# interpolation operator L_U (section 2; CIR: section 3 and eq. CIR2D)
# ---------------------------------------------------------------------------

def interp(phi, c):
    """``L_U[phi]``: multilinear interpolation at every node's departure point.

    ``phi`` has ``ndim`` axes and ``c`` shape ``(ndim, *phi.shape)``.  The
    ``2**ndim`` bracketing nodes are combined by nested 1D interpolations,
    first along x, then y, then z.  ``L_{-U}`` is ``interp(phi, -c)``.
    """
    phi = np.asarray(phi, dtype=np.float64)
    nd = phi.ndim
    if c.shape[0] != nd:
        raise ValueError("need one Courant array per axis")
    nodes, frac = [], []
    for d in range(nd):
        s, n, f = departure(c[d])
        a, b = _nodes(phi.shape, nd - 1 - d, s, n)
        nodes.append((np.broadcast_to(a, phi.shape), np.broadcast_to(b, phi.shape)))
        frac.append(f)
    # field values at every node of the departure cell
    vals = {}
    for choice in itertools.product((0, 1), repeat=nd):  # choice[d]: 0 anchor, 1 far
        sel = []
        for ax in range(nd):
            d = nd - 1 - ax
            sel.append(nodes[d][choice[d]])
        vals[choice] = phi[tuple(sel)]
    # reduce axes in order x, y, z
    for d in range(nd):
        nxt = {}
        for rest in itertools.product((0, 1), repeat=nd - d - 1):
            nxt[rest] = _lerp(vals[(0,) + rest], vals[(1,) + rest], frac[d])
        vals = nxt
    return vals[()]


def cir(phi, c):
    """CIR step: one call of L_U (section 3; eq. CIR2D in 2D)."""
    return interp(phi, c)


def fec(phi, c):
    """Forward error correction, eq. intro:FEC (two calls).

    ``phibar = L_{-U}[L_U[phi]]`` and ``FEC = L_U[phi] + (phi - phibar)/2``.
    """
    phi = np.asarray(phi, dtype=np.float64)
    phi1 = interp(phi, c)
    phibar = interp(phi1, -c)
    return phi1 + 0.5 * (phi - phibar)


def bec(phi, c):
    """Backward error correction, eq. intro:BEC (three calls).

    ``BEC = L_U[phi + (phi - phibar)/2]`` with ``phibar`` as in FEC.
    """
    phi = np.asarray(phi, dtype=np.float64)
    phi1 = interp(phi, c)
    phibar = interp(phi1, -c)
    return interp(phi + 0.5 * (phi - phibar), c)


# ---------------------------------------------------------------------------
# third-order combination, one axis at a time (eqs. intro:CEC, intro:CECcoef,
# intro:CECcoefSL; section 5 for the splitting)
# ---------------------------------------------------------------------------

def _take(arr, idx, axis):
    return np.take_along_axis(arr, np.broadcast_to(idx, arr.shape), axis=axis)


def cec_sweep(phi, cd, d):
    """One third-order sweep along physical axis ``d`` with Courant ``cd``.

    Steps, in the paper's order: ``Phi1 = L_U Phi`` (first call),
    ``phibar = L_{-U} Phi1`` (second call), ``e = Phi - phibar``, then the
    combination ``A FEC + B BEC`` whose BEC part re-interpolates ``e`` at
    the departure point (third call), written division-free as
    ``Phi1 + 1/2 [e_a + (1+f)/3 (e_b - e_a)]``.
    """
    phi = np.asarray(phi, dtype=np.float64)
    nd = phi.ndim
    ax = nd - 1 - d
    s, n, f = departure(cd)
    a, b = _nodes(phi.shape, ax, s, n)
    phi1 = _lerp(_take(phi, a, ax), _take(phi, b, ax), f)
    sr, nr, fr = departure(-cd)
    ar, br = _nodes(phi.shape, ax, sr, nr)
    phibar = _lerp(_take(phi1, ar, ax), _take(phi1, br, ax), fr)
    e = phi - phibar
    ea = _take(e, a, ax)
    eb = _take(e, b, ax)
    w = (1.0 + f) / 3.0
    return phi1 + 0.5 * (ea + w * (eb - ea))


def sweep_order(m, ndim):
    """Axes swept at global step ``m``: x, y[, z] when even, reversed when odd."""
    axes = tuple(range(ndim))
    return axes if m % 2 == 0 else axes[::-1]


def cec_split(phi, c, m=0):
    """Third-order step at global step index ``m``: one sweep per axis."""
    out = np.asarray(phi, dtype=np.float64)
    for d in sweep_order(m, out.ndim):
        out = cec_sweep(out, c[d], d)
    return out


def cec_strang(phi, c):
    """Third-order step with Strang's symmetric splitting (section 5 names it
    as the way to keep a split scheme's order): half a step along every axis
    but the last, a whole step along the last, then the half steps again in
    reverse order.  In 3D: x/2, y/2, z, y/2, x/2; in 2D: x/2, y, x/2; in 1D
    one whole sweep.  A half step is the same sweep with the Courant number
    halved (exact in binary floating point)."""
    out = np.asarray(phi, dtype=np.float64)
    nd = out.ndim
    for d in range(nd - 1):
        out = cec_sweep(out, c[d] / 2.0, d)
    out = cec_sweep(out, c[nd - 1], nd - 1)
    for d in reversed(range(nd - 1)):
        out = cec_sweep(out, c[d] / 2.0, d)
    return out


def ec_split(phi, c, scheme, m=0):
    """FEC or BEC split per axis (eqs. split:1-2 applied to eqs. intro:FEC
    and intro:BEC): the scheme applied along one axis at a time, with the
    Courant numbers of the other axes set to zero (L_U then moves nothing
    along them), in the order of ``sweep_order``."""
    out = np.asarray(phi, dtype=np.float64)
    one = fec if scheme == FEC else bec
    for d in sweep_order(m, out.ndim):
        cd = np.zeros_like(c)
        cd[d] = c[d]
        out = one(out, cd)
    return out


def midpoint_courant(cd, d, sign):
    """Courant number of a midpoint (second-order Runge-Kutta) backtrace
    along physical axis ``d``: ``cd`` taken at ``x - sign cd(x)/2`` (in
    cells), linearly interpolated between the two nodes around that point
    (periodic).  ``sign = +1`` traces the characteristic of ``L_U``, ``-1``
    that of ``L_{-U}``.  Beyond the paper, which samples the velocity at the
    arrival node only."""
    cd = np.asarray(cd, dtype=np.float64)
    ax = cd.ndim - 1 - d
    n = cd.shape[ax]
    shape = [1] * cd.ndim
    shape[ax] = n
    pos = np.arange(n, dtype=np.float64).reshape(shape) - sign * 0.5 * cd
    i0 = np.floor(pos)
    fr = pos - i0
    i0 = i0.astype(np.int64) % n
    return (1.0 - fr) * _take(cd, i0, ax) + fr * _take(cd, (i0 + 1) % n, ax)


def cec_sweep_pair(phi, cf, cb, d):
    """``cec_sweep`` with separate Courant numbers for the two directions:
    ``cf`` for the calls of ``L_U`` (the first call and the re-interpolation
    of ``e``), ``cb`` for the call of ``L_{-U}``.  With ``cf = cb`` it is
    ``cec_sweep``."""
    phi = np.asarray(phi, dtype=np.float64)
    ax = phi.ndim - 1 - d
    s, n, f = departure(cf)
    a, b = _nodes(phi.shape, ax, s, n)
    phi1 = _lerp(_take(phi, a, ax), _take(phi, b, ax), f)
    sr, nr, fr = departure(-np.asarray(cb))
    ar, br = _nodes(phi.shape, ax, sr, nr)
    phibar = _lerp(_take(phi1, ar, ax), _take(phi1, br, ax), fr)
    e = phi - phibar
    ea = _take(e, a, ax)
    eb = _take(e, b, ax)
    w = (1.0 + f) / 3.0
    return phi1 + 0.5 * (ea + w * (eb - ea))


def cec_split_midpoint(phi, c, m=0):
    """The third-order split step with a midpoint backtrace (beyond the
    paper): along each axis the calls of ``L_U`` depart from
    ``x - c(x - c/2)`` and the call of ``L_{-U}`` from ``x + c(x + c/2)``,
    each the second-order Runge-Kutta foot of its own characteristic.  Used
    to measure whether the order lost to a variable velocity comes back."""
    out = np.asarray(phi, dtype=np.float64)
    for d in sweep_order(m, out.ndim):
        cf = midpoint_courant(c[d], d, 1.0)
        cb = midpoint_courant(c[d], d, -1.0)
        out = cec_sweep_pair(out, cf, cb, d)
    return out


def cec_literal(phi, c, m=0):
    """The weights of eq. intro:CECcoefSL read literally, one axis at a time
    (a second-order comparison, not the third-order scheme).

    Along axis ``d`` (Courant numbers of the other axes set to zero, in the
    order of ``sweep_order``) the step is ``A FEC + B BEC``: FEC as in eq.
    intro:FEC, its correction ``(phi - phibar)/2`` added at the arrival
    node, BEC as in eq. intro:BEC, the correction re-interpolated at the
    departure point, and ``3A = 2 - 1/(U % 1)``, ``B = 1 - A`` with
    ``U = |c|``.  For ``U < 1`` this is eq. intro:CECcoef and equals
    ``cec_split``; for ``U > 1`` the arrival-node correction no longer
    matches the shifted interpolation and the scheme is second order.  An
    integer ``U`` divides by zero: the result there is not finite, as the
    formula is.
    """
    out = np.asarray(phi, dtype=np.float64)
    for d in sweep_order(m, out.ndim):
        cd = np.zeros_like(c)
        cd[d] = c[d]
        frac = np.abs(np.asarray(c[d], dtype=np.float64)) % 1.0
        with np.errstate(divide="ignore", invalid="ignore"):
            a = (2.0 - 1.0 / frac) / 3.0
            out = a * fec(out, cd) + (1.0 - a) * bec(out, cd)
    return out


def step(phi, c, scheme, m=0):
    """One time step of ``scheme`` (CIR, FEC, BEC, CEC, CEC_STRANG, FEC_SPLIT,
    BEC_SPLIT or CEC_LITERAL) at global step ``m``."""
    if scheme == CIR:
        return cir(phi, c)
    if scheme == FEC:
        return fec(phi, c)
    if scheme == BEC:
        return bec(phi, c)
    if scheme == CEC:
        return cec_split(phi, c, m)
    if scheme == CEC_STRANG:
        return cec_strang(phi, c)
    if scheme == FEC_SPLIT:
        return ec_split(phi, c, FEC, m)
    if scheme == BEC_SPLIT:
        return ec_split(phi, c, BEC, m)
    if scheme == CEC_LITERAL:
        return cec_literal(phi, c, m)
    raise ValueError(f"unknown scheme {scheme!r}")


def run(phi, c, scheme, steps, step0=0):
    """``steps`` steps with fixed Courant numbers ``c`` (FP64)."""
    out = np.asarray(phi, dtype=np.float64)
    for k in range(steps):
        out = step(out, c, scheme, step0 + k)
    return out


def advect(phi, u, dx, dt, scheme, steps, step0=0):
    """Advance ``phi`` by ``steps`` steps of ``scheme`` with velocity ``u``.

    ``u`` has shape ``(ndim, *phi.shape)`` (physical velocity, x first),
    ``dx`` the cell sizes (x first), ``dt`` the time step.  The velocity is
    held fixed over the call; a time-dependent velocity is advanced one
    call per step.  Returns the FP64 result.
    """
    if isinstance(scheme, str):
        scheme = SCHEMES[scheme]
    c = courant(u, dt, dx)
    return run(phi, c, scheme, steps, step0)
