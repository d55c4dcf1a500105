"""The oracle run over slabs of the outermost axis in worker processes.

TEST INFRASTRUCTURE ONLY (timing of the oracle on every host core).  The
arithmetic is that of ``schemes.advect``, unchanged: each time step, every
worker advances one slab of the outermost NumPy axis (z in 3D, y in 2D) plus
``halo`` planes on either side, taken periodically from the whole field,
and hands back the slab's own planes.

Why the result is the whole-field result bit for bit: one step of any scheme
reads, along an axis, only nodes within ``floor(|c|) + 1`` cells of the
arrival node per call of the interpolation operator L_U (section 3, the
two nodes that bracket the departure point; section 4 for |c| > 1), and a
step makes at most three nested calls along one axis (FEC and BEC,
eqs. intro:FEC and intro:BEC; the split third-order scheme, eq. intro:CEC,
sweeps each axis once per step).  A slab with ``halo >= 3 (floor(c_max) + 1)``
planes therefore computes its own planes from exactly the same values, in
the same order, as the whole field does; the wrong values that the slab's
own periodic wrap puts into its halo never reach them.

The velocity and two copies of the field (read one, write the other, swap
every step) live in POSIX shared memory, so a pool started with ``spawn``
(fresh interpreters, nothing inherited from the parent) passes no array
through a pipe.
"""

from __future__ import annotations

import math
from concurrent.futures import ProcessPoolExecutor
from multiprocessing import get_context, shared_memory

import numpy as np

from .schemes import advect, courant

_U = None
_PHI = None
_SHM = ()
_ARGS = None
_USLAB = {}


def step_halo(u, dx, dt) -> int:
    """Planes of the outermost axis that one step of any scheme can read."""
    c = courant(u, dt, dx)[-1]
    return 3 * (int(math.floor(float(np.max(np.abs(c))))) + 1)


def _init(names, shape, dtype, args):
    global _U, _PHI, _SHM, _ARGS
    _SHM = tuple(shared_memory.SharedMemory(name=nm) for nm in names)
    _U = np.ndarray(shape, dtype=np.dtype(dtype), buffer=_SHM[0].buf)
    _PHI = tuple(np.ndarray(shape[1:], dtype=np.float64, buffer=b.buf) for b in _SHM[1:])
    _ARGS = args
    _USLAB.clear()


def _ready(_):
    return _U is not None


def _slab_step(job):
    lo, hi, halo, m, src = job
    idx = np.arange(lo - halo, hi + halo) % _U.shape[1]
    key = (lo, hi, halo)
    us = _USLAB.get(key)
    if us is None:
        us = _USLAB[key] = np.ascontiguousarray(_U[:, idx])
    dx, dt, scheme = _ARGS
    out = advect(_PHI[src][idx], us, dx, dt, scheme, 1, step0=m)
    _PHI[1 - src][lo:hi] = out[halo:halo + hi - lo]
    return True


class SlabPool:
    """A pool of ``workers`` processes advancing slabs of one problem.

    ``u``, ``dx``, ``dt`` and ``scheme`` are those of ``schemes.advect``.
    ``start`` is the multiprocessing start method.  Use as a context manager;
    the shared memory is released on exit.  A worker that dies raises
    ``BrokenProcessPool`` in the caller instead of stalling it.
    """

    def __init__(self, u, dx, dt, scheme, workers, start="spawn"):
        u = np.ascontiguousarray(u)
        self.n = u.shape[1]
        self.workers = max(1, min(int(workers), self.n))
        self.halo = step_halo(u, dx, dt)
        self.bounds = np.linspace(0, self.n, self.workers + 1).astype(int)
        phi_bytes = max(1, int(np.prod(u.shape[1:])) * 8)
        self._shm = []
        self._pool = None
        try:
            # the velocity, then the field twice (read one, write the other)
            for size in (max(1, u.nbytes), phi_bytes, phi_bytes):
                self._shm.append(shared_memory.SharedMemory(create=True, size=size))
            np.ndarray(u.shape, dtype=u.dtype, buffer=self._shm[0].buf)[...] = u
            self._phi = [np.ndarray(u.shape[1:], dtype=np.float64, buffer=b.buf) for b in self._shm[1:]]
            self._pool = ProcessPoolExecutor(
                self.workers, mp_context=get_context(start), initializer=_init,
                initargs=(tuple(b.name for b in self._shm), u.shape, u.dtype.str, (dx, dt, scheme)))
            # workers started and attached before anything is timed
            assert all(self._pool.map(_ready, range(self.workers)))
        except BaseException:
            self.close(ok=False)
            raise

    def advect(self, phi, steps, step0=0):
        """``steps`` steps from global step ``step0``; returns the FP64 field."""
        phi = np.asarray(phi, dtype=np.float64)
        if phi.shape != self._phi[0].shape:
            raise ValueError("field and velocity differ in shape")
        self._phi[0][...] = phi
        h = self.halo
        for k in range(steps):
            jobs = [(lo, hi, h, step0 + k, k % 2) for lo, hi in zip(self.bounds[:-1], self.bounds[1:])]
            assert all(self._pool.map(_slab_step, jobs))
        return self._phi[steps % 2].copy()

    def close(self, ok=True):
        if self._pool is not None:
            # joins the workers: their CPU time is then in RUSAGE_CHILDREN
            self._pool.shutdown(wait=True, cancel_futures=not ok)
            self._pool = None
        self._phi = None
        for b in self._shm:
            b.close()
            b.unlink()
        self._shm = []

    def __enter__(self):
        return self

    def __exit__(self, exc_type, exc, tb):
        self.close(ok=exc_type is None)
        return False


def advect_slabs(phi, u, dx, dt, scheme, steps, workers, step0=0, start="spawn"):
    """``schemes.advect`` over ``workers`` slabs in a process pool."""
    with SlabPool(u, dx, dt, scheme, workers, start) as pool:
        return pool.advect(phi, steps, step0)
