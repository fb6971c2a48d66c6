"""CPU builds with AddressSanitizer and UndefinedBehaviorSanitizer of the oracle (gcc) and of the library's
host-side ABI glue (hipcc, sanitizers on the host code only), each driven through every entry point that runs
without a GPU (tests/oracle_sanitize.c, tests/abi_sanitize.cpp). A sanitizer report aborts the test program."""
import glob
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = tmp_path / "oracle_san"
    r = subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-fno-sanitize-recover=undefined", os.path.join(ROOT, "oracle", "oracle.c"),
                        os.path.join(HERE, "oracle_sanitize.c"), "-o", str(exe), "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout + r.stderr


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)), reason="ROCm compilers not installed")
def test_abi_glue_under_address_and_undefined_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from paper_1511_00088_amd import build as B

    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
           "-fno-omit-frame-pointer"]
    flags = [f for f in B.CFLAGS if f != "-O3"] + ["-O1"]
    objs = []
    procs = []
    for src in B.SOURCES:
        obj = str(tmp_path / src.replace(".hip", ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([HIPCC, *flags, *san, "-c", os.path.join(B.CSRC, src), "-o", obj],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate()
        assert p.returncode == 0, err[-3000:]
    lib = str(tmp_path / "libstagcg_san.so")
    r = subprocess.run([HIPCC, "-shared", "-fPIC", f"--offload-arch={B.ARCH}", *objs, "-Xarch_host", "-fsanitize=address",
                        "-Xarch_host", "-fsanitize=undefined", "-shared-libasan", "-o", lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    exe = str(tmp_path / "abi_san")
    r = subprocess.run([CLANGXX, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                        "-shared-libasan", os.path.join(HERE, "abi_sanitize.cpp"), f"-L{tmp_path}", "-lstagcg_san",
                        f"-Wl,-rpath,{tmp_path}", "-o", exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux")
    env = dict(ENV, LD_LIBRARY_PATH=":".join(rt + [str(tmp_path), os.environ.get("LD_LIBRARY_PATH", "")]))
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and "ALL OK" in r.stdout, r.stdout + r.stderr[-3000:]
