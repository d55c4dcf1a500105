"""Multi-stage semi-Lagrangian advection on MI355X (gfx950).

``paper_1606_06117_amd.native`` binds the C ABI of ``libsla.so`` (the HIP
kernels); ``paper_1606_06117_amd.workloads`` builds seeded synthetic inputs.
Importing the package loads nothing: the library is loaded on first use of
``native.Context`` and fails loudly if it has not been built.
"""

__all__ = ["native", "workloads"]
