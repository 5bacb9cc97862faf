"""Cell keys (CPU): the library's key arithmetic, compiled for the host from
the same header the kernels use -- exact division against native 64-bit
division, and pack / unpack round trips of bit-packed and mixed-radix keys
(including a 65-bit Amazon-shaped layout and corner cells)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not found")
def test_key_layout_host_check(tmp_path):
    exe = tmp_path / "key_layout_check"
    src = os.path.join(HERE, "native", "key_layout_check.hip")
    r = subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"), src, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-2000:]
    assert "0 wrong" in r.stdout
