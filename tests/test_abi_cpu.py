"""The C-ABI library loads and exports every declared symbol (no GPU needed)."""

import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "sla.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sla_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("sla_create", "sla_destroy", "sla_advect", "sla_norms", "sla_check",
                 "sla_courant_max", "sla_strerror", "sla_last_error", "sla_set_stream"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1606_06117_amd import native
    lib = native.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    # the binding covers the same set
    assert set(native.SIGNATURES) == set(declared_functions())


def test_strerror_and_null_handling():
    from paper_1606_06117_amd import native
    lib = native.load()
    assert lib.sla_strerror(0) == b"success"
    assert lib.sla_strerror(-2).startswith(b"Courant")
    assert lib.sla_strerror(12345) == b"unknown status"
    assert b"captured" in lib.sla_strerror(native.ECAPTURE)
    assert lib.sla_last_error(None) == b""
    assert lib.sla_advect(None, None, None, None, 0.0, 0, 0, 0, 0.0) == native.EINVAL
    assert lib.sla_norms(None, 0, None, None, None) == native.EINVAL
    assert lib.sla_check(None) == native.EINVAL
    assert lib.sla_advect_multi(None, None, 0, None, None, 0.0, 0, 0, 0, 0.0) == native.EINVAL
    assert lib.sla_advect_batch(None, 0, None, 0, 0, 0, 0.0) == native.EINVAL
    assert lib.sla_set_workspace(None, None, 0) == native.EINVAL
    assert lib.sla_workspace_size(None, 3, 1) == 0
    lib.sla_destroy(None)


def test_workspace_size():
    """One FP32 field of the grid, and for third order in 3D one per field up
    to four (shared-velocity groups); 0 for an invalid grid or scheme."""
    import ctypes
    from paper_1606_06117_amd import native
    lib = native.load()
    g = native.make_grid((12, 34, 56), (0.1, 0.1, 0.1))
    field = 4 * 12 * 34 * 56
    for scheme in range(8):
        for ns in (1, 2, 3, 16):
            want = field * (min(ns, 4) if scheme == native.CEC else 1)
            assert lib.sla_workspace_size(ctypes.byref(g), scheme, ns) == want
    g2 = native.make_grid((34, 56), (0.1, 0.1))
    assert lib.sla_workspace_size(ctypes.byref(g2), native.CEC, 16) == 4 * 34 * 56
    assert lib.sla_workspace_size(ctypes.byref(g), 8, 1) == 0
    assert lib.sla_workspace_size(ctypes.byref(g), 3, -1) == 0
    # grids of 2^31 cells or more, including extents whose product would
    # wrap a 64-bit integer, are invalid
    for shape in [(1 << 21,) * 3, (2**31 - 1,) * 3, (8, 1 << 15, 1 << 16), (1 << 10, 1 << 11, 1 << 10)]:
        big = native.make_grid(shape, (0.1, 0.1, 0.1))
        assert lib.sla_workspace_size(ctypes.byref(big), 3, 1) == 0, shape
    ok = native.make_grid((8, 1 << 12, 1 << 15), (0.1, 0.1, 0.1))  # 2^30 cells
    assert lib.sla_workspace_size(ctypes.byref(ok), 3, 1) == 4 << 30


def test_create_without_device_is_an_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    import ctypes
    from paper_1606_06117_amd import native
    lib = native.load()
    h = ctypes.c_void_p()
    assert lib.sla_create(ctypes.byref(h), 0, None) == native.EINVAL
    assert not h.value
