"""The C ABI's host code under AddressSanitizer and UBSan (no GPU needed).

The library's host side (argument checks, error strings, workspace sizes,
context creation without a device) is rebuilt with the host sanitisers on
(the device code is compiled as usual), linked with the other objects of the
library and driven by tests/asan/abi_driver.c through every entry point.
Any sanitiser report, or a failed check, fails the test.
"""

import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1606_06117_amd")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert res.returncode == 0, f"{' '.join(cmd)}\n{res.stdout}\n{res.stderr}"
    return res


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm compilers")
def test_abi_host_paths_under_sanitizers(tmp_path):
    from paper_1606_06117_amd import build
    objs = {os.path.basename(o): o for o in glob.glob(os.path.join(build.OBJDIR, "*.hip.o"))}
    srcs = sorted(glob.glob(os.path.join(build.CSRC, "*.hip")))
    if len(objs) < len(srcs):
        build.build()
        objs = {os.path.basename(o): o for o in glob.glob(os.path.join(build.OBJDIR, "*.hip.o"))}
    inc = ["-I", os.path.join(ROOT, "include"), "-I", build.CSRC]
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    api = str(tmp_path / "api.o")
    _run([HIPCC, f"--offload-arch={build.ARCH}", "-O1", "-g", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san, *inc,
          "-c", os.path.join(build.CSRC, "api.hip"), "-o", api])
    drv = str(tmp_path / "driver.o")
    _run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
          "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "asan", "abi_driver.c"),
          "-o", drv])
    others = [o for name, o in sorted(objs.items()) if name != "api.hip.o"]
    exe = str(tmp_path / "abi_driver")
    _run([HIPCC, f"--offload-arch={build.ARCH}", "-fsanitize=address", "-fsanitize=undefined",
          "-fno-gpu-sanitize", drv, api, *others, "-o", exe])
    import torch
    args = [exe] + ([] if torch.cuda.is_available() else ["--no-device"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run(args, capture_output=True, text=True, timeout=300, env=env)
    assert res.returncode == 0 and "abi driver: ok" in res.stdout, res.stdout + res.stderr
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr
