"""FP64 oracle of the learned per-cell correction (test infrastructure only).

Not in the paper: the network is this library's.  A small MLP reads the CIR
output's 3x3x3 neighbourhood around a node and the node's Courant numbers
and predicts the correction that takes the CIR step to the third-order step
(section 2, eq. intro:CEC, applied per axis as in section 5).

Features of node i (30 used, padded to 32):
    d_k = Phi1[i + o_k] - Phi1[i]     for the 27 offsets o_k in {-1,0,1}^3,
                                       z outermost, x innermost (d_13 = 0)
    sigma = sqrt(sum_k d_k^2 / 27 + 1e-30)
    x_k = d_k / sigma (k < 27),  x_27..29 = c_x, c_y, c_z,  x_30 = x_31 = 0
The network predicts y; the corrected value is Phi1[i] + sigma * y, limited
to [min, max] of the 27 values Phi1[i + o_k] (so a step never leaves the
range of the CIR field around the node, and the maximum norm of the field
cannot grow whatever the network outputs).  The training target is
(Phi_third_order[i] - Phi1[i]) / sigma (not limited).  Differences make
the prediction invariant to adding a constant to Phi, and the sigma scaling
makes it linear in the scale of Phi, as the true correction is.

Network: h1 = relu(x W1 + b1), h2 = relu(h1 W2 + b2), y = h2 w3 + b3 with
W1 32x64, W2 64x64, w3 64; loss = mean((y - t)^2).  The GPU runs it with
BF16 weights and activations on the matrix cores (FP32 accumulation); this
oracle takes BF16-rounded weights and features and computes in FP64.
"""

from __future__ import annotations

import numpy as np

from .schemes import interp

NF = 32        # padded input width
NH = 64        # hidden width
NUSED = 30     # used inputs
SIGMA_FLOOR = 1e-30

# flat parameter vector layout (FP32 on the GPU): W1 (row-major k x n), b1,
# W2 (row-major k x n), b2, w3, b3
SHAPES = [("W1", (NF, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)),
          ("w3", (NH,)), ("b3", (1,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def pack(params):
    return np.concatenate([np.asarray(params[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def bf16_round(a):
    """Round FP32 values to the nearest BF16 (ties to even), returned as FP32."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def offsets27():
    """The 27 neighbour offsets (dz, dy, dx), z outermost, x innermost."""
    return [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


def features(phi1, c, cells):
    """Features and sigma of the nodes ``cells`` = (z, y, x) index arrays (3D)."""
    phi1 = np.asarray(phi1, dtype=np.float64)
    nz, ny, nx = phi1.shape
    z, y, x = (np.asarray(v, dtype=np.int64) for v in cells)
    centre = phi1[z, y, x]
    d = np.empty((z.size, 27))
    for k, (dz, dy, dx) in enumerate(offsets27()):
        d[:, k] = phi1[(z + dz) % nz, (y + dy) % ny, (x + dx) % nx] - centre
    sigma = np.sqrt(np.sum(d * d, axis=1) / 27.0 + SIGMA_FLOOR)
    X = np.zeros((z.size, NF))
    X[:, :27] = d / sigma[:, None]
    X[:, 27] = c[0][z, y, x]
    X[:, 28] = c[1][z, y, x]
    X[:, 29] = c[2][z, y, x]
    return X, sigma


def forward(params, X):
    """``y`` and the activations the backward pass needs."""
    a1 = X @ params["W1"] + params["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ params["W2"] + params["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ params["w3"] + params["b3"][0]
    return y, (X, a1, h1, a2, h2)


def loss(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t):
    """Gradients of ``mean((y - t)^2)`` with respect to every parameter."""
    X, a1, h1, a2, h2 = cache
    M = y.shape[0]
    dy = 2.0 * (y - t) / M
    g = {}
    g["w3"] = h2.T @ dy
    g["b3"] = np.array([dy.sum()])
    dh2 = np.outer(dy, params["w3"]) * (a2 > 0)
    g["W2"] = h1.T @ dh2
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ params["W2"].T) * (a1 > 0)
    g["W1"] = X.T @ dh1
    g["b1"] = dh1.sum(axis=0)
    return g


def adam(flat, grad, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba) of the flat parameter vector; step >= 1."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1**step)
    vhat = v / (1.0 - beta2**step)
    return flat - lr * mhat / (np.sqrt(vhat) + eps), m, v


def learned_step(phi, c, flat_params):
    """One learned step on a 3D field: CIR, features, network, correction.

    Weights are rounded to BF16 as the GPU holds them; features are rounded
    to BF16 as the GPU feeds them to the matrix cores.
    """
    params = unpack(bf16_round(np.asarray(flat_params, dtype=np.float32)).astype(np.float64))
    phi1 = interp(np.asarray(phi, dtype=np.float64), c)
    nz, ny, nx = phi1.shape
    cells = np.indices(phi1.shape).reshape(3, -1)
    X, sigma = features(phi1, c, cells)
    X = bf16_round(X.astype(np.float32)).astype(np.float64)
    y, _ = forward(params, X)
    lo, hi = neighbourhood_range(phi1)
    return np.clip(phi1.ravel() + sigma * y, lo.ravel(), hi.ravel()).reshape(phi1.shape)


def neighbourhood_range(phi1):
    """Minimum and maximum of the 27 values around every node (periodic)."""
    lo = np.asarray(phi1, dtype=np.float64).copy()
    hi = lo.copy()
    for dz, dy, dx in offsets27():
        v = np.roll(phi1, (-dz, -dy, -dx), axis=(0, 1, 2))
        lo = np.minimum(lo, v)
        hi = np.maximum(hi, v)
    return lo, hi
