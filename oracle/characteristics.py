"""Exact solutions of the advection equation along characteristics.

TEST INFRASTRUCTURE ONLY.  A passive scalar carried by a velocity ``u(x, t)``
keeps its value along the characteristics ``dX/dt = u(X, t)``, so the exact
field at time ``T`` is ``Phi(x, T) = Phi0(X(0; x, T))``: the initial field at
the foot, at ``t = 0``, of the characteristic that reaches ``x`` at ``T``
(section 2, the advection problem; section 6 compares the schemes with such
a fully Lagrangian solution computed with a much finer time step).

The foot is found by integrating the characteristic backwards in time with
the classical fourth-order Runge-Kutta method in FP64, with sub-steps much
finer than the schemes' time step, so its error is far below theirs.  The
velocities are the analytic formulas the grids are sampled from.

Points are arrays of shape ``(P, ndim)``, x first.
"""

from __future__ import annotations

import numpy as np


def abc(A=1.0, B=1.0, C=1.0):
    """ABC flow ``u = A sin z + C cos y, v = B sin x + A cos z, w = C sin y + B cos x``."""
    def vel(p, t):
        x, y, z = p[:, 0], p[:, 1], p[:, 2]
        return np.stack([A * np.sin(z) + C * np.cos(y),
                         B * np.sin(x) + A * np.cos(z),
                         C * np.sin(y) + B * np.cos(x)], axis=1)
    return vel


def cellular(amp=1.0):
    """2D cellular flow ``u = sin x cos y, v = -cos x sin y`` (stream function sin x sin y)."""
    def vel(p, t):
        x, y = p[:, 0], p[:, 1]
        return amp * np.stack([np.sin(x) * np.cos(y), -np.cos(x) * np.sin(y)], axis=1)
    return vel


def swirl(length=1.0):
    """The 2D patch test's flow (section 5): ``u = P(y/l)``, ``v = -P(x/l)``,
    ``P(e) = e (1 - e) (1/2 - e) [cos(2 pi e (1 - e)) + 1] / (2 pi^2)``."""
    def prof(e):
        s = e * (1.0 - e)
        return s * (0.5 - e) * (np.cos(2.0 * np.pi * s) + 1.0) / (2.0 * np.pi ** 2)

    def vel(p, t):
        q = np.mod(p, length) / length
        return np.stack([prof(q[:, 1]), -prof(q[:, 0])], axis=1)
    return vel


def uniform(u):
    """Constant velocity ``u`` (x first)."""
    u = np.asarray(u, dtype=np.float64)

    def vel(p, t):
        return np.broadcast_to(u, p.shape)
    return vel


def foot(points, vel, T, substeps):
    """``X(0; x, T)`` for every row ``x`` of ``points``: ``substeps`` RK4 steps
    of ``dX/ds = -u(X, T - s)`` from ``s = 0`` to ``s = T``."""
    X = np.array(points, dtype=np.float64)
    h = T / substeps
    for k in range(substeps):
        t = T - k * h
        k1 = vel(X, t)
        k2 = vel(X - 0.5 * h * k1, t - 0.5 * h)
        k3 = vel(X - 0.5 * h * k2, t - 0.5 * h)
        k4 = vel(X - h * k3, t - h)
        X = X - (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
    return X


def node_points(shape, length):
    """Every node of a periodic grid of ``shape`` (NumPy order) as points, in C order."""
    axes = [np.arange(n, dtype=np.float64) * (length / n) for n in shape]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel() for g in grids[::-1]], axis=1)
