"""FP64 error and mass reductions (test infrastructure only).

The paper rates a scheme by the norm of its difference to a reference
profile (section 4, cosine test); the library reports the relative L2
error, the maximum error and the mass drift.  These are their plain
definitions.
"""

from __future__ import annotations

import math

import numpy as np


def reductions(a, b):
    """The five sums the GPU reduction returns, in FP64.

    ``(sum (a-b)^2, sum b^2, max |a-b|, sum a, sum b)`` over all elements,
    with ``a`` and ``b`` promoted to FP64 first.  ``math.fsum`` gives the
    correctly rounded sum, so the result does not depend on any order.
    """
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    d = a - b
    return (
        math.fsum(d * d),
        math.fsum(b * b),
        float(np.max(np.abs(d))) if d.size else 0.0,
        math.fsum(a),
        math.fsum(b),
    )


def rel_l2(x, ref):
    """``||x - ref||_2 / ||ref||_2``."""
    s = reductions(x, ref)
    return math.sqrt(s[0] / s[1])


def linf(x, ref):
    """``max |x - ref|``."""
    return reductions(x, ref)[2]


def mass_error(phi_m, phi_0):
    """``(sum phi_m - sum phi_0) / sum |phi_0|``."""
    phi_0 = np.asarray(phi_0, dtype=np.float64)
    return (math.fsum(np.asarray(phi_m, dtype=np.float64).ravel())
            - math.fsum(phi_0.ravel())) / math.fsum(np.abs(phi_0).ravel())
