"""Seeded synthetic inputs (fields and velocities) for tests and benchmarks.

This module only builds inputs: periodic scalar fields and divergence-free
velocities on Cartesian grids.  It holds none of the advection arithmetic and
imports neither the oracle nor the HIP binding, so both can be fed from it.
Arrays are NumPy, C order with x fastest (``[z, y, x]``), FP64 unless stated;
callers round to FP32 where the GPU takes FP32.

Recipes (each seeded through ``numpy.random.default_rng``):

* ``gaussians``: a sum of Gaussian blobs on a periodic box, each periodised
  over the 3**d neighbouring images so the field is smooth across the seam.
* ``abc_velocity``: the Arnold-Beltrami-Childress flow
  ``u = A sin z + C cos y, v = B sin x + A cos z, w = C sin y + B cos x`` on
  ``[0, 2 pi)^3``, divergence free, ``max |u_d| = 2`` for A = B = C = 1.
* ``fourier_modes``: ``sum_k g_k / (1 + |k|^2) cos(k.x + phi_k)`` over the
  wave vectors ``k in {0..7}^3 \\ {0}`` (8 modes per axis), Gaussian ``g_k``,
  uniform phases, rescaled to unit RMS.
* ``power_law``: an isotropic random field with energy spectrum ``k^-5/3``
  for ``1 <= |k| <= kmax`` (amplitude ``|k|^-11/6`` per mode in 3D), random
  phases, unit RMS.
"""

from __future__ import annotations

import math

import numpy as np

TWO_PI = 2.0 * math.pi


def node_coords(n: int, length: float) -> np.ndarray:
    """Node positions ``i * length / n`` of a periodic axis."""
    return np.arange(n, dtype=np.float64) * (length / n)


def _periodic_gauss_1d(x, centre, sigma, length):
    out = np.zeros_like(x)
    for img in (-1, 0, 1):
        out += np.exp(-((x - centre + img * length) ** 2) / (2.0 * sigma * sigma))
    return out


def gaussians(shape, centres, sigmas, length=1.0, amplitude=1.0):
    """Sum of periodised Gaussians; ``centres[j]`` is x first."""
    ndim = len(shape)
    out = np.zeros(shape, dtype=np.float64)
    for c, s in zip(centres, sigmas):
        prod = None
        for d in range(ndim):
            n = shape[ndim - 1 - d]
            g = _periodic_gauss_1d(node_coords(n, length), c[d], s, length)
            view = [1] * ndim
            view[ndim - 1 - d] = n
            g = g.reshape(view)
            prod = g if prod is None else prod * g
        out += amplitude * prod
    return out


def random_gaussians(shape, count, seed, length=TWO_PI, smin=0.05, smax=0.15):
    """``count`` Gaussians, centres uniform in the box, sigma = length * U[smin, smax]."""
    rng = np.random.default_rng(seed)
    ndim = len(shape)
    centres = rng.uniform(0.0, length, (count, ndim))
    sigmas = length * rng.uniform(smin, smax, count)
    return gaussians(shape, centres, sigmas, length)


def random_gaussians_torch(shape, count, seed, device, length=TWO_PI, smin=0.05, smax=0.15):
    """``random_gaussians`` built on ``device``: the same seeded centres and
    widths and the same 1D factors (NumPy), whose products and sum torch
    forms in FP64 in the same order, so the FP64 field is the same bit for
    bit; returned as an FP32 torch tensor.  A 512^3 field takes seconds on
    the host this way instead of tens of them."""
    import torch
    rng = np.random.default_rng(seed)
    ndim = len(shape)
    centres = rng.uniform(0.0, length, (count, ndim))
    sigmas = length * rng.uniform(smin, smax, count)
    out = torch.zeros(tuple(shape), dtype=torch.float64, device=device)
    for c, s in zip(centres, sigmas):
        prod = None
        for d in range(ndim):
            n = shape[ndim - 1 - d]
            g = torch.from_numpy(_periodic_gauss_1d(node_coords(n, length), c[d], s, length)).to(device)
            view = [1] * ndim
            view[ndim - 1 - d] = n
            g = g.reshape(view)
            prod = g if prod is None else prod * g
        out += prod  # amplitude 1: 1.0 * prod is prod
        del prod
    return out.to(torch.float32)


def gaussians_at(points, centres, sigmas, length=1.0, amplitude=1.0):
    """``gaussians`` evaluated at arbitrary ``points`` (rows, x first), FP64.

    Points are wrapped into the box first, so the value is that of the
    periodic field ``gaussians`` samples at the nodes.
    """
    p = np.mod(np.asarray(points, dtype=np.float64), length)
    out = np.zeros(p.shape[0], dtype=np.float64)
    for c, s in zip(centres, sigmas):
        prod = np.ones(p.shape[0], dtype=np.float64)
        for d in range(p.shape[1]):
            prod *= _periodic_gauss_1d(p[:, d], c[d], s, length)
        out += amplitude * prod
    return out


def random_gaussians_at(points, count, seed, length=TWO_PI, smin=0.05, smax=0.15):
    """The field of ``random_gaussians`` (same seed) at arbitrary ``points``."""
    rng = np.random.default_rng(seed)
    ndim = np.asarray(points).shape[1]
    centres = rng.uniform(0.0, length, (count, ndim))
    sigmas = length * rng.uniform(smin, smax, count)
    return gaussians_at(points, centres, sigmas, length)


def abc_velocity(shape, A=1.0, B=1.0, C=1.0, dtype=np.float32):
    """ABC flow on ``[0, 2 pi)^3`` sampled at the nodes; returns (3, nz, ny, nx)."""
    nz, ny, nx = shape
    x = node_coords(nx, TWO_PI)
    y = node_coords(ny, TWO_PI)
    z = node_coords(nz, TWO_PI)
    u = np.empty((3, nz, ny, nx), dtype=dtype)
    u[0] = (A * np.sin(z)[:, None, None] + C * np.cos(y)[None, :, None]).astype(dtype)
    u[1] = (B * np.sin(x)[None, None, :] + A * np.cos(z)[:, None, None]).astype(dtype)
    u[2] = (C * np.sin(y)[None, :, None] + B * np.cos(x)[None, None, :]).astype(dtype)
    return u


def uniform_velocity(shape, vel, dtype=np.float32):
    """Constant velocity ``vel`` (x first) on every node; (ndim, *shape)."""
    ndim = len(shape)
    u = np.empty((ndim,) + tuple(shape), dtype=dtype)
    for d in range(ndim):
        u[d] = vel[d]
    return u


def cellular_velocity_2d(shape, amp=1.0, dtype=np.float32):
    """Divergence-free cellular flow ``u = sin x cos y, v = -cos x sin y`` on [0, 2 pi)^2."""
    ny, nx = shape
    x = node_coords(nx, TWO_PI)[None, :]
    y = node_coords(ny, TWO_PI)[:, None]
    u = np.empty((2, ny, nx), dtype=dtype)
    u[0] = (amp * np.sin(x) * np.cos(y)).astype(dtype)
    u[1] = (-amp * np.cos(x) * np.sin(y)).astype(dtype)
    return u


def _swirl_profile(eta):
    """``eta (1 - eta) (1/2 - eta) [cos(2 pi eta (1 - eta)) + 1] / (2 pi^2)``."""
    s = eta * (1.0 - eta)
    return s * (0.5 - eta) * (np.cos(TWO_PI * s) + 1.0) / (2.0 * math.pi ** 2)


def swirl_velocity_2d(shape, length=1.0, dtype=np.float32):
    """The swirling flow of the paper's 2D patch test (section 5) on
    ``[0, length)^2``: ``u = P(y / length)``, ``v = -P(x / length)`` with
    ``P(eta) = eta (1 - eta) (1/2 - eta) [cos(2 pi eta (1 - eta)) + 1] / (2 pi^2)``.
    Zero on the box edges, divergence free; (2, ny, nx)."""
    ny, nx = shape
    x = node_coords(nx, length) / length
    y = node_coords(ny, length) / length
    u = np.empty((2, ny, nx), dtype=dtype)
    u[0] = np.broadcast_to(_swirl_profile(y)[:, None], shape).astype(dtype)
    u[1] = np.broadcast_to(-_swirl_profile(x)[None, :], shape).astype(dtype)
    return u


def square_patch_at(points, lo, hi):
    """1 inside the square ``[lo, hi)`` (per axis, x first), 0 outside."""
    p = np.asarray(points, dtype=np.float64)
    inside = np.all((p >= np.asarray(lo)) & (p < np.asarray(hi)), axis=1)
    return inside.astype(np.float64)


def square_patch(shape, lo, hi, length=1.0):
    """``square_patch_at`` at the nodes of a periodic 2D grid."""
    ny, nx = shape
    X, Y = np.meshgrid(node_coords(nx, length), node_coords(ny, length))
    return square_patch_at(np.stack([X.ravel(), Y.ravel()], axis=1), lo, hi).reshape(shape)


def _fourier_parts(shape, seed, kmax):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    ks = np.arange(kmax)
    kz, ky, kx = np.meshgrid(ks, ks, ks, indexing="ij")
    g = rng.standard_normal((kmax, kmax, kmax))
    ph = rng.uniform(0.0, TWO_PI, (kmax, kmax, kmax))
    amp = g / (1.0 + kx**2 + ky**2 + kz**2)
    amp[0, 0, 0] = 0.0
    a = amp * np.exp(1j * ph)
    ex = np.exp(1j * np.outer(ks, node_coords(nx, TWO_PI)))
    ey = np.exp(1j * np.outer(ks, node_coords(ny, TWO_PI)))
    ez = np.exp(1j * np.outer(node_coords(nz, TWO_PI), ks))
    A = np.einsum("zyk,kx->zyx", a, ex)
    B = np.einsum("zkx,ky->zyx", A, ey)
    return ez, B.reshape(kmax, ny * nx)


def fourier_modes_torch(shape, seed, device, kmax=8):
    """``fourier_modes`` with its final mode sum done in FP64 by torch on
    ``device``; returns an FP32 torch tensor (same recipe and seed)."""
    import torch
    nz, ny, nx = shape
    ez, Bf = _fourier_parts(shape, seed, kmax)
    er = torch.from_numpy(np.ascontiguousarray(ez.real)).to(device)
    ei = torch.from_numpy(np.ascontiguousarray(ez.imag)).to(device)
    br = torch.from_numpy(np.ascontiguousarray(Bf.real)).to(device)
    bi = torch.from_numpy(np.ascontiguousarray(Bf.imag)).to(device)
    out = (er @ br - ei @ bi).reshape(nz, ny, nx)
    out /= torch.sqrt(torch.mean(out * out))
    return out.to(torch.float32).contiguous()


def fourier_modes(shape, seed, kmax=8, dtype=np.float32):
    """Smooth random field with ``kmax`` modes per axis (3D), unit RMS."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    ks = np.arange(kmax)
    kz, ky, kx = np.meshgrid(ks, ks, ks, indexing="ij")
    g = rng.standard_normal((kmax, kmax, kmax))
    ph = rng.uniform(0.0, TWO_PI, (kmax, kmax, kmax))
    amp = g / (1.0 + kx**2 + ky**2 + kz**2)
    amp[0, 0, 0] = 0.0
    a = amp * np.exp(1j * ph)  # field = Re sum_k a_k e^{i k.x}
    ex = np.exp(1j * np.outer(ks, node_coords(nx, TWO_PI)))  # (kmax, nx)
    ey = np.exp(1j * np.outer(ks, node_coords(ny, TWO_PI)))
    ez = np.exp(1j * np.outer(node_coords(nz, TWO_PI), ks))  # (nz, kmax)
    A = np.einsum("zyk,kx->zyx", a, ex)  # A[kz, ky, x] = sum_kx a e^{i kx x}
    B = np.einsum("zkx,ky->zyx", A, ey)  # B[kz, y, x] = sum_ky A e^{i ky y}
    out = np.empty((nz, ny, nx), dtype=np.float64)
    Bf = B.reshape(kmax, ny * nx)
    for z0 in range(0, nz, 64):
        z1 = min(nz, z0 + 64)
        out[z0:z1] = np.real(ez[z0:z1] @ Bf).reshape(z1 - z0, ny, nx)
    out /= math.sqrt(np.mean(out * out))
    return out.astype(dtype)


def power_law(shape, seed, kmax=64, dtype=np.float32):
    """Isotropic random field, E(k) ~ k^-5/3 for 1 <= |k| <= kmax, unit RMS."""
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    kz = np.fft.fftfreq(nz, 1.0 / nz)[:, None, None]
    ky = np.fft.fftfreq(ny, 1.0 / ny)[None, :, None]
    kx = np.fft.rfftfreq(nx, 1.0 / nx)[None, None, :]
    kk = np.sqrt(kx * kx + ky * ky + kz * kz)
    with np.errstate(divide="ignore"):
        amp = np.where((kk >= 1.0) & (kk <= kmax), kk ** (-11.0 / 6.0), 0.0)
    ph = rng.uniform(0.0, TWO_PI, amp.shape)
    spec = amp * np.exp(1j * ph)
    out = np.fft.irfftn(spec, s=(nz, ny, nx))
    out /= math.sqrt(np.mean(out * out))
    return out.astype(dtype)


def abc_velocity_torch(shape, device, A=1.0, B=1.0, C=1.0):
    """``abc_velocity`` evaluated in FP64 by torch on ``device`` (for grids
    too large to build on the host); FP32 (3, nz, ny, nx) tensor."""
    import torch
    nz, ny, nx = shape
    f64 = dict(dtype=torch.float64, device=device)
    x = torch.arange(nx, **f64) * (TWO_PI / nx)
    y = torch.arange(ny, **f64) * (TWO_PI / ny)
    z = torch.arange(nz, **f64) * (TWO_PI / nz)
    u = torch.empty((3, nz, ny, nx), dtype=torch.float32, device=device)
    u[0] = (A * torch.sin(z)[:, None, None] + C * torch.cos(y)[None, :, None]).float()
    u[1] = (B * torch.sin(x)[None, None, :] + A * torch.cos(z)[:, None, None]).float()
    u[2] = (C * torch.sin(y)[None, :, None] + B * torch.cos(x)[None, None, :]).float()
    return u


def power_law_torch(shape, seed, device, kmax=64):
    """Isotropic random field with E(k) ~ k^-5/3 for 1 <= |k| <= kmax at unit
    RMS, like ``power_law``, but with phases drawn (seeded) only for the
    modes inside the box |k_d| <= kmax and the inverse FFT done by torch on
    ``device`` in FP64; FP32 tensor."""
    import torch
    nz, ny, nx = shape
    kb, _, coef = _power_law_block(seed, kmax)
    block = torch.from_numpy(coef).to(device)
    spec = torch.zeros((nz, ny, nx // 2 + 1), dtype=torch.complex128, device=device)
    iz = torch.from_numpy(kb % nz).to(device)
    iy = torch.from_numpy(kb % ny).to(device)
    spec[iz[:, None, None], iy[None, :, None], torch.arange(kmax + 1, device=device)[None, None, :]] = block
    out = torch.fft.irfftn(spec, s=(nz, ny, nx))
    del spec
    out /= torch.sqrt(torch.mean(out * out))
    return out.float().contiguous()


def _power_law_block(seed, kmax):
    """The seeded spectral block of ``power_law_torch``: (kz, ky, kx) with
    ``|kz|, |ky| <= kmax`` and ``0 <= kx <= kmax``; the wave numbers and the
    complex coefficients."""
    rng = np.random.default_rng(seed)
    kb = np.arange(-kmax, kmax + 1)
    kxb = np.arange(0, kmax + 1)
    KZ, KY, KX = np.meshgrid(kb, kb, kxb, indexing="ij")
    kk = np.sqrt(KX * KX + KY * KY + KZ * KZ)
    with np.errstate(divide="ignore"):
        amp = np.where((kk >= 1.0) & (kk <= kmax), kk ** (-11.0 / 6.0), 0.0)
    ph = rng.uniform(0.0, TWO_PI, amp.shape)
    return kb, kxb, amp * np.exp(1j * ph)


def power_law_at(points, seed, kmax=64, chunk=256):
    """The field of ``power_law_torch`` (same seed) at arbitrary ``points``
    (rows x, y, z on [0, 2 pi)^3), FP64.

    The inverse real FFT of the block is, on any grid finer than 2 kmax + 1
    nodes per axis, the samples of one trigonometric polynomial: each
    coefficient of the kx = 0 plane contributes the real part of its wave,
    each of kx > 0 twice that (the conjugate half of the spectrum).  Its mean
    square follows from Parseval's identity, so the unit-RMS field does not
    depend on the grid.
    """
    kb, kxb, c = _power_law_block(seed, kmax)
    w = np.where(kxb == 0, 1.0, 2.0)
    cw = (c * w[None, None, :]).reshape(-1, kxb.size)
    # mean square: Hermitian-completed coefficients G_k, sum of |G_k|^2
    n = 2 * kmax + 1
    G = np.zeros((n, n, n), dtype=np.complex128)
    iz = (kb % n)[:, None, None]
    iy = (kb % n)[None, :, None]
    ix = kxb[None, None, :]
    half = np.where(kxb == 0, 0.5, 1.0)[None, None, :]
    np.add.at(G, (iz, iy, ix % n), c * half)
    np.add.at(G, (((-kb) % n)[:, None, None], ((-kb) % n)[None, :, None], (-kxb) % n),
              np.conj(c) * half)
    rms = math.sqrt(float(np.sum(np.abs(G) ** 2)))
    p = np.asarray(points, dtype=np.float64)
    out = np.empty(p.shape[0], dtype=np.float64)
    for s in range(0, p.shape[0], chunk):
        q = p[s:s + chunk]
        ex = np.exp(1j * q[:, 0:1] * kxb[None, :])        # (P, Kx)
        ey = np.exp(1j * q[:, 1:2] * kb[None, :])         # (P, K)
        ez = np.exp(1j * q[:, 2:3] * kb[None, :])
        t1 = (cw @ ex.T).reshape(kb.size, kb.size, -1)    # (Kz, Ky, P)
        t2 = np.einsum("zyp,py->zp", t1, ey)
        out[s:s + chunk] = np.einsum("zp,pz->p", t2, ez).real
    return out / rms


def abc_dt(shape, cfl, length=TWO_PI, umax=2.0):
    """Time step giving ``max |u_d| dt / dx = cfl`` on a cubic periodic box."""
    dx = length / shape[-1]
    return cfl * dx / umax


def uneven_grids(count=64, seed_sizes=3100, seed_vel=3101, nmin=32, nmax=192):
    """Sizes ``N_g ~ U{nmin..nmax}`` and uniform velocities ``U[-1, 1]^3``."""
    sizes = np.random.default_rng(seed_sizes).integers(nmin, nmax + 1, count)
    vels = np.random.default_rng(seed_vel).uniform(-1.0, 1.0, (count, 3))
    return [int(s) for s in sizes], vels
