"""CPU check of the LDS placement of the NPR path matrices: the host build of ppos (sp_npr_layout.h), compiled by
hipcc for the host only from tests/npr_layout_check.cpp, is a one-to-one map whose access patterns fall in
distinct LDS bank slots, as that file describes."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not installed")
def test_npr_path_placement(tmp_path):
    exe = tmp_path / "npr_layout_check"
    hipcc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    r = subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O1", "-std=c++17",
                        os.path.join(HERE, "npr_layout_check.cpp"), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    print(r.stdout)
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout + r.stderr
