"""ctypes binding of ``libsla.so`` (argument marshalling only).

Every function here converts torch tensors to device pointers, calls the C
ABI declared in ``include/sla.h`` and turns a negative status into an
exception.  No arithmetic of the method happens in Python; if the library is
missing, loading fails loudly instead of falling back to anything else.
"""

from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libsla.so")

CIR, FEC, BEC, CEC, CEC_STRANG, FEC_SPLIT, BEC_SPLIT, CEC_LITERAL = 0, 1, 2, 3, 4, 5, 6, 7
SCHEMES = {"cir": CIR, "fec": FEC, "bec": BEC, "cec": CEC, "cec_strang": CEC_STRANG,
           "fec_split": FEC_SPLIT, "bec_split": BEC_SPLIT, "cec_literal": CEC_LITERAL}
MAX_REACH = 4
NOALLOC_MAX_CELLS = 1 << 23

OK, EINVAL, ECOURANT, EHIP, ENOMEM, ENOMODEL, ECAPTURE = 0, -1, -2, -3, -4, -5, -6
OPT_FUSED = 0
OPT_CEC3D_KERNEL = 1
CEC3D_DEFAULT = 5  # the library's default fused-step implementation
OPT_SWEEP_KERNEL = 2
OPT_EC_KERNEL = 3
OPT_CEC3D_SHAPE = 4
OPT_LEARNED_KERNEL = 5
OPT_SHARED_VELOCITY = 6
OPT_EC_SHAPE = 7
OPT_BACKTRACE = 8

# every symbol include/sla.h declares, with (restype, argtypes)
_c = ctypes
_vp = _c.c_void_p
SIGNATURES = {
    "sla_create": (_c.c_int, [_c.POINTER(_vp), _c.c_int, _vp]),
    "sla_destroy": (None, [_vp]),
    "sla_set_stream": (_c.c_int, [_vp, _vp]),
    "sla_strerror": (_c.c_char_p, [_c.c_int]),
    "sla_last_error": (_c.c_char_p, [_vp]),
    "sla_courant_max": (_c.c_int, [_vp, _vp, _vp, _c.c_double, _c.POINTER(_c.c_double)]),
    "sla_advect": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_double, _c.c_int32, _c.c_int32,
                              _c.c_int64, _c.c_double]),
    "sla_advect_noalloc": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_double, _c.c_int32, _c.c_int32,
                                      _c.c_int64, _c.c_double]),
    "sla_advect_multi": (_c.c_int, [_vp, _vp, _c.c_int32, _vp, _vp, _c.c_double, _c.c_int32,
                                    _c.c_int32, _c.c_int64, _c.c_double]),
    "sla_workspace_size": (_c.c_size_t, [_vp, _c.c_int32, _c.c_int32]),
    "sla_set_workspace": (_c.c_int, [_vp, _vp, _c.c_size_t]),
    "sla_advect_batch": (_c.c_int, [_vp, _c.c_int32, _vp, _c.c_int32, _c.c_int32, _c.c_int64,
                                    _c.c_double]),
    "sla_check": (_c.c_int, [_vp]),
    "sla_norms": (_c.c_int, [_vp, _c.c_int64, _vp, _vp, _c.POINTER(_c.c_double)]),
    "sla_set_option": (_c.c_int, [_vp, _c.c_int, _c.c_int64]),
    "sla_plan_create": (_c.c_int, [_vp, _c.POINTER(_vp), _c.c_int32, _vp, _c.c_int32, _c.c_int64,
                                   _c.c_double, _c.c_int32]),
    "sla_plan_run": (_c.c_int, [_vp, _vp]),
    "sla_plan_info": (_c.c_int, [_vp, _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32),
                                 _c.POINTER(_c.c_int32), _c.POINTER(_c.c_double)]),
    "sla_plan_destroy": (None, [_vp]),
    "sla_model_create": (_c.c_int, [_vp, _c.POINTER(_vp)]),
    "sla_model_destroy": (None, [_vp]),
    "sla_model_set_params": (_c.c_int, [_vp, _vp, _vp, _c.c_int64]),
    "sla_model_get_params": (_c.c_int, [_vp, _vp, _vp, _c.c_int64]),
    "sla_model_load": (_c.c_int, [_vp, _vp, _vp, _c.c_int64]),
    "sla_model_save": (_c.c_int, [_vp, _vp, _vp, _c.c_int64]),
    "sla_model_set_courant_range": (_c.c_int, [_vp, _c.c_double]),
    "sla_make_pairs": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_double, _vp, _c.c_int64, _vp,
                                  _vp, _vp]),
    "sla_model_forward": (_c.c_int, [_vp, _vp, _vp, _c.c_int64, _vp]),
    "sla_model_grads": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_int64, _vp, _c.POINTER(_c.c_double)]),
    "sla_model_train_step": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_int64, _c.c_double,
                                        _c.POINTER(_c.c_double)]),
    "sla_advect_learned": (_c.c_int, [_vp, _vp, _vp, _vp, _vp, _c.c_double, _c.c_int32,
                                      _c.c_int64, _c.c_double, _c.POINTER(_c.c_int32)]),
    "sla_tune": (_c.c_int, [_vp, _vp, _vp, _vp, _c.c_double, _c.c_char_p]),
    "sla_tune_load": (_c.c_int, [_vp, _c.c_char_p]),
    "sla_tune_info": (_c.c_int, [_vp, _vp, _c.POINTER(_c.c_int32), _c.POINTER(_c.c_int32),
                                 _c.POINTER(_c.c_double)]),
    "sla_timing": (_c.c_int, [_vp, _c.c_int]),
    "sla_timing_read": (_c.c_int, [_vp, _c.POINTER(_c.c_int64), _c.POINTER(_c.c_double)]),
}

KERNEL_KINDS = ["cir", "fec", "bec", "sweep_x", "sweep_y", "sweep_z", "cec3d", "copy", "learned",
                "sweep_xy"]
MLP_INPUTS, MLP_HIDDEN, MLP_PARAMS = 32, 64, 6337


class SlaError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__(f"sla status {status}: {detail}")


class Grid(ctypes.Structure):
    """Mirror of ``sla_grid``."""
    _fields_ = [("ndim", ctypes.c_int32), ("n", ctypes.c_int32 * 3), ("dx", ctypes.c_double * 3)]


class Problem(ctypes.Structure):
    """Mirror of ``sla_problem``."""
    _fields_ = [("grid", Grid), ("phi", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("u_uniform", ctypes.c_float * 3), ("dt", ctypes.c_double)]


_LIB = None


def load(path: str = LIB_PATH):
    """Load the library once and attach the ABI signatures."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(path):
        raise ImportError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def make_grid(shape, dx=None) -> Grid:
    """``shape`` in NumPy order (z, y, x) / (y, x) / (x,); ``dx`` x first."""
    ndim = len(shape)
    n = list(reversed([int(v) for v in shape])) + [1] * (3 - ndim)
    if dx is None:
        dx = [1.0 / v for v in n[:ndim]]
    dx = list(dx) + [1.0] * (3 - ndim)
    g = Grid()
    g.ndim = ndim
    for d in range(3):
        g.n[d] = n[d]
        g.dx[d] = float(dx[d])
    return g


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _check_field(t, name):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) torch tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """One library context bound to a device; calls go to torch's current stream."""

    def __init__(self, device: int = 0):
        self.lib = load()
        self.device = device
        h = ctypes.c_void_p()
        st = self.lib.sla_create(ctypes.byref(h), device, None)
        if st != OK:
            raise SlaError(st, self.lib.sla_strerror(st).decode())
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.sla_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        import torch
        self.lib.sla_set_stream(self.h, ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream))

    def _raise(self, st):
        if st != OK:
            raise SlaError(st, self.lib.sla_last_error(self.h).decode() or self.lib.sla_strerror(st).decode())

    def courant_max(self, u, dx, dt) -> float:
        _check_field(u, "u")
        g = make_grid(u.shape[1:], dx)
        out = ctypes.c_double()
        self._stream()
        self._raise(self.lib.sla_courant_max(self.h, ctypes.byref(g), _ptr(u), float(dt), ctypes.byref(out)))
        return out.value

    def advect(self, phi, u, dx, dt, scheme, steps, step0=0, courant_max=0.0):
        """Advance ``phi`` (float32, (z, y, x)) in place; ``u`` is (ndim, *phi.shape)."""
        if isinstance(scheme, str):
            scheme = SCHEMES[scheme]
        _check_field(phi, "phi")
        _check_field(u, "u")
        if tuple(u.shape) != (phi.dim(),) + tuple(phi.shape):
            raise ValueError(f"u must have shape {(phi.dim(),) + tuple(phi.shape)}, got {tuple(u.shape)}")
        g = make_grid(phi.shape, dx)
        self._stream()
        self._raise(self.lib.sla_advect(self.h, ctypes.byref(g), _ptr(phi), _ptr(u), float(dt),
                                        int(scheme), int(steps), int(step0), float(courant_max)))
        return phi

    def advect_noalloc(self, phi, u, dx, dt, scheme, steps, step0=0, courant_max=0.0):
        """``advect`` through ``sla_advect_noalloc`` (static work memory, no allocation)."""
        if isinstance(scheme, str):
            scheme = SCHEMES[scheme]
        _check_field(phi, "phi")
        _check_field(u, "u")
        if tuple(u.shape) != (phi.dim(),) + tuple(phi.shape):
            raise ValueError(f"u must have shape {(phi.dim(),) + tuple(phi.shape)}, got {tuple(u.shape)}")
        g = make_grid(phi.shape, dx)
        self._stream()
        self._raise(self.lib.sla_advect_noalloc(self.h, ctypes.byref(g), _ptr(phi), _ptr(u), float(dt),
                                                int(scheme), int(steps), int(step0), float(courant_max)))
        return phi

    def advect_multi(self, phis, u, dx, dt, scheme, steps, step0=0, courant_max=0.0):
        """Advance every field of ``phis`` (same shape) in place; they share ``u``."""
        if isinstance(scheme, str):
            scheme = SCHEMES[scheme]
        for f in phis:
            _check_field(f, "phi")
            if f.shape != phis[0].shape:
                raise ValueError("the fields must have one shape")
        _check_field(u, "u")
        if phis and tuple(u.shape) != (phis[0].dim(),) + tuple(phis[0].shape):
            raise ValueError("u must have shape (ndim, *phi.shape)")
        g = make_grid(phis[0].shape if phis else u.shape[1:], dx)
        arr = (ctypes.c_void_p * max(1, len(phis)))(*[f.data_ptr() for f in phis])
        self._stream()
        self._raise(self.lib.sla_advect_multi(self.h, ctypes.byref(g), len(phis), arr, _ptr(u),
                                              float(dt), int(scheme), int(steps), int(step0),
                                              float(courant_max)))

    def advect_batch(self, problems, scheme, steps, step0=0, courant_max=0.0):
        """Advance independent problems in place: a list of ``(phi, u, dx, dt)``
        with ``u`` a (ndim, *phi.shape) tensor or an ndim-tuple uniform velocity."""
        if isinstance(scheme, str):
            scheme = SCHEMES[scheme]
        arr, keep = problem_array(problems)
        self._stream()
        self._raise(self.lib.sla_advect_batch(self.h, len(problems), arr, int(scheme), int(steps),
                                              int(step0), float(courant_max)))
        del keep

    def workspace_size(self, shape, dx, scheme, nscalars=1):
        """Device bytes of work memory ``advect`` needs on a grid of ``shape``."""
        if isinstance(scheme, str):
            scheme = SCHEMES[scheme]
        g = make_grid(shape, dx)
        return int(self.lib.sla_workspace_size(ctypes.byref(g), int(scheme), int(nscalars)))

    def set_workspace(self, buf):
        """Use the device tensor ``buf`` as the work memory (None: back to the
        library's own).  The caller keeps ``buf`` alive while it is set."""
        if buf is None:
            self._raise(self.lib.sla_set_workspace(self.h, None, 0))
        else:
            if not buf.is_cuda or not buf.is_contiguous():
                raise TypeError("the workspace must be a contiguous device tensor")
            self._raise(self.lib.sla_set_workspace(self.h, _ptr(buf),
                                                   buf.numel() * buf.element_size()))

    def set_option(self, option: int, value: int):
        self._raise(self.lib.sla_set_option(self.h, int(option), int(value)))

    def check(self):
        self._stream()
        self._raise(self.lib.sla_check(self.h))

    def norms(self, a, b):
        """FP64 ``(sum (a-b)^2, sum b^2, max|a-b|, sum a, sum b)`` computed on the GPU."""
        _check_field(a, "a")
        _check_field(b, "b")
        if a.numel() != b.numel():
            raise ValueError("a and b must have the same number of elements")
        out = (ctypes.c_double * 5)()
        self._stream()
        self._raise(self.lib.sla_norms(self.h, a.numel(), _ptr(a), _ptr(b), out))
        return tuple(out)

    def tune(self, phi, u, dx, dt, path=None):
        """Time the fused-step implementations on this grid (sla_tune); the
        context then uses the fastest per parity.  Returns ``tune_info``."""
        _check_field(phi, "phi")
        _check_field(u, "u")
        g = make_grid(phi.shape, dx)
        self._stream()
        self._raise(self.lib.sla_tune(self.h, ctypes.byref(g), _ptr(phi), _ptr(u), float(dt),
                                      path.encode() if path else None))
        return self.tune_info(phi.shape)

    def tune_load(self, path):
        self._raise(self.lib.sla_tune_load(self.h, path.encode()))

    def tune_info(self, shape):
        """``{"even": (variant, shape, ms), "odd": (...)}`` or None."""
        g = make_grid(shape)
        v, sh, ms = (ctypes.c_int32 * 2)(), (ctypes.c_int32 * 2)(), (ctypes.c_double * 2)()
        if self.lib.sla_tune_info(self.h, ctypes.byref(g), v, sh, ms) != OK:
            return None
        return {"even": (v[0], sh[0], ms[0]), "odd": (v[1], sh[1], ms[1])}

    def timing(self, enable: bool):
        """Start (clearing totals) or stop per-kernel event timing."""
        self._stream()
        self._raise(self.lib.sla_timing(self.h, 1 if enable else 0))

    def timing_read(self):
        """``{kind: (launches, total_ms)}`` for kinds with at least one launch."""
        n = len(KERNEL_KINDS)
        launches = (ctypes.c_int64 * n)()
        ms = (ctypes.c_double * n)()
        self._stream()
        self._raise(self.lib.sla_timing_read(self.h, launches, ms))
        return {KERNEL_KINDS[k]: (launches[k], ms[k]) for k in range(n) if launches[k]}


class Model:
    """A learned-correction network living on a context's device."""

    def __init__(self, ctx: Context):
        self.ctx = ctx
        self.lib = ctx.lib
        h = ctypes.c_void_p()
        ctx._stream()
        ctx._raise(self.lib.sla_model_create(ctx.h, ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.sla_model_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, params):
        import numpy as np
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != MLP_PARAMS:
            raise ValueError(f"need {MLP_PARAMS} parameters")
        self.ctx._stream()
        self.ctx._raise(self.lib.sla_model_set_params(self.ctx.h, self.h, p.ctypes.data_as(ctypes.c_void_p),
                                                      p.size))

    def get_params(self):
        import numpy as np
        p = np.empty(MLP_PARAMS, dtype=np.float32)
        self.ctx._stream()
        self.ctx._raise(self.lib.sla_model_get_params(self.ctx.h, self.h, p.ctypes.data_as(ctypes.c_void_p),
                                                      p.size))
        return p

    def set_courant_range(self, r: float):
        if self.lib.sla_model_set_courant_range(self.h, float(r)) != OK:
            raise SlaError(EINVAL, "bad Courant range")

    def forward(self, feats, y):
        self.ctx._stream()
        self.ctx._raise(self.lib.sla_model_forward(self.ctx.h, self.h, _ptr(feats), feats.shape[0], _ptr(y)))

    def grads(self, feats, target):
        import numpy as np
        g = np.empty(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_double()
        self.ctx._stream()
        self.ctx._raise(self.lib.sla_model_grads(self.ctx.h, self.h, _ptr(feats), _ptr(target),
                                                 feats.shape[0], g.ctypes.data_as(ctypes.c_void_p),
                                                 ctypes.byref(loss)))
        return g, loss.value

    def train_step(self, feats, target, lr, want_loss=False, m=None):
        loss = ctypes.c_double()
        rows = feats.shape[0] if m is None else int(m)
        self.ctx._stream()
        self.ctx._raise(self.lib.sla_model_train_step(self.ctx.h, self.h, _ptr(feats), _ptr(target), rows,
                                                      float(lr), ctypes.byref(loss) if want_loss else None))
        return loss.value if want_loss else None


def make_pairs(ctx: Context, phi1, phi_next, u, dx, dt, cells, feats, target, sigma):
    """Features/targets of the nodes ``cells`` (int32 linear indices, device)."""
    g = make_grid(phi1.shape, dx)
    ctx._stream()
    ctx._raise(ctx.lib.sla_make_pairs(ctx.h, ctypes.byref(g), _ptr(phi1), _ptr(phi_next), _ptr(u),
                                      float(dt), _ptr(cells), cells.numel(), _ptr(feats), _ptr(target),
                                      _ptr(sigma)))


def advect_learned(ctx: Context, model: Model, phi, u, dx, dt, steps, step0=0, courant_max=0.0,
                   allow_fallback=True):
    """Learned steps in place; returns True if the call fell back to the plain scheme."""
    _check_field(phi, "phi")
    _check_field(u, "u")
    g = make_grid(phi.shape, dx)
    fb = ctypes.c_int32(0)
    ctx._stream()
    ctx._raise(ctx.lib.sla_advect_learned(ctx.h, model.h, ctypes.byref(g), _ptr(phi), _ptr(u), float(dt),
                                          int(steps), int(step0), float(courant_max),
                                          ctypes.byref(fb) if allow_fallback else None))
    return bool(fb.value)


def problem_array(problems):
    """``sla_problem`` array of ``(phi, u, dx, dt)`` problems, ``u`` a
    (ndim, *phi.shape) tensor or an ndim-tuple uniform velocity; returns the
    array and the objects it points into."""
    arr = (Problem * max(1, len(problems)))()
    keep = []
    for i, (phi, u, dx, dt) in enumerate(problems):
        _check_field(phi, "phi")
        arr[i].grid = make_grid(phi.shape, dx)
        arr[i].phi = phi.data_ptr()
        if isinstance(u, (tuple, list)):
            if len(u) != phi.dim():
                raise ValueError("a uniform velocity has one component per axis")
            arr[i].u = None
            for d in range(len(u)):
                arr[i].u_uniform[d] = float(u[d])
        else:
            _check_field(u, "u")
            if tuple(u.shape) != (phi.dim(),) + tuple(phi.shape):
                raise ValueError("u must have shape (ndim, *phi.shape)")
            arr[i].u = u.data_ptr()
        arr[i].dt = float(dt)
        keep.append((phi, u))
    return arr, keep


class Plan:
    """Batched third-order steps of many 3D problems, replayed as one graph.

    ``problems``: list of ``(phi, u, dx, dt)`` with ``phi`` a float32 (z, y, x)
    tensor and ``u`` either a (3, z, y, x) tensor (shared when the same tensor
    is passed for several problems) or a 3-tuple uniform velocity (x, y, z).
    """

    def __init__(self, ctx: Context, problems, steps, step0=0, courant_max=0.0, tune=True):
        self.ctx = ctx
        self.lib = ctx.lib
        if any(phi.dim() != 3 for phi, _, _, _ in problems):
            raise ValueError("plans take 3D fields")
        arr, self._keep = problem_array(problems)
        h = ctypes.c_void_p()
        ctx._stream()
        ctx._raise(self.lib.sla_plan_create(ctx.h, ctypes.byref(h), len(problems), arr, int(steps),
                                            int(step0), float(courant_max), 1 if tune else 0))
        self.h = h

    def run(self):
        self.ctx._stream()
        self.ctx._raise(self.lib.sla_plan_run(self.ctx.h, self.h))

    def info(self):
        y, b, n = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        ms = ctypes.c_double()
        self.lib.sla_plan_info(self.h, ctypes.byref(y), ctypes.byref(b), ctypes.byref(n), ctypes.byref(ms))
        return {"ychunk": y.value, "blocks": b.value, "items": n.value, "tuned_step_ms": ms.value}

    def close(self):
        if getattr(self, "h", None):
            self.lib.sla_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
