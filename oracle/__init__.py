"""FP64 CPU oracle for multi-stage semi-Lagrangian advection.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
NumPy implementation of what the GPU library computes.  Only the test suite,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it.  It shares no code with the HIP path and imports nothing from it.

Modules
-------
schemes  departure decomposition, interpolation operator L_U, CIR, FEC, BEC and
         the directionally split third-order CEC (Cameron, Raynaud & Dormy,
         "Multi-stage high order semi-Lagrangian schemes for incompressible
         flows in Cartesian geometries", sections 2-5, Table 1).
norms    FP64 error and mass reductions.
mlp      FP64 forward/backward of the learned per-cell correction network
         (not in the paper; the network shape is the library's).
slabs    the same advection run over slabs in worker processes, bit for bit
         the one-process result (for timing the oracle on every core).
characteristics
         exact solutions under a variable velocity: the initial field at the
         foot of each node's characteristic (RK4 in FP64), the fully
         Lagrangian reference of section 6.

Every function is pinned by CPU tests against closed forms the paper prints
(constant-velocity stencils, amplification factors, modified equations),
exact invariants (integer shifts, constants, linear fields, mass) and
measured convergence orders.
"""

from .schemes import (  # noqa: F401
    CIR, FEC, BEC, CEC, CEC_STRANG, FEC_SPLIT, BEC_SPLIT, CEC_LITERAL, SCHEMES,
    courant, departure, interp, cir, fec, bec, cec_sweep, cec_split, cec_strang, ec_split,
    cec_literal, midpoint_courant, cec_sweep_pair, cec_split_midpoint,
    step, run, advect, sweep_order,
)
from .norms import reductions, rel_l2, linf, mass_error  # noqa: F401
