"""CPU check of the library's checkerboard index arithmetic: the host build of divq, site_of, nbr, eta_sign
(sp_device.h) and remap_block (sp_kernels.h), compiled by hipcc for the host only from tests/geom_check.cpp,
against plain lexicographic arithmetic (exhaustive or boundary-complete, as that file describes)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC) and shutil.which("hipcc") is None, reason="hipcc not installed")
def test_index_arithmetic_matches_lexicographic(tmp_path):
    exe = tmp_path / "geom_check"
    hipcc = HIPCC if os.path.exists(HIPCC) else shutil.which("hipcc")
    r = subprocess.run([hipcc, "-x", "hip", "--cuda-host-only", "-O2", "-std=c++17",
                        os.path.join(HERE, "geom_check.cpp"), "-o", str(exe)], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    print(r.stdout)
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout + r.stderr
