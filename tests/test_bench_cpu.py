"""bench.py's command line, without a GPU: the options parse, several GPUs
are refused with a message (the library has one-GPU kernels only), and the
byte model the roofline divides by is the one the kernels are sized for."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_help_lists_the_contract_options():
    res = _bench("--help")
    assert res.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup"):
        assert opt in res.stdout


def test_several_gpus_are_refused_with_a_message():
    res = _bench("--gpus", "2", "--steps", "3", "--warmup", "1")
    assert res.returncode == 2
    assert "one GPU only" in res.stderr
    assert res.stdout == ""   # no JSON line: nothing was measured


def test_algorithmic_bytes():
    sys.path.insert(0, ROOT)
    import bench
    n = 512 ** 3
    # a whole 3D step reads phi and three velocity planes and writes phi
    assert bench.algorithmic_bytes("cec3d", n, 3) == 20 * n
    assert bench.algorithmic_bytes("cir", n, 3) == 20 * n
    assert bench.algorithmic_bytes("cir", n, 2) == 16 * n
    # one sweep reads phi and one plane and writes phi; the x+y kernel two planes
    assert bench.algorithmic_bytes("sweep_z", n, 3) == 12 * n
    assert bench.algorithmic_bytes("sweep_xy", n, 3) == 16 * n
    assert bench.algorithmic_bytes("copy", n, 3) == 8 * n
