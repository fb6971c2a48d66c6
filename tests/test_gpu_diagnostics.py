"""The library's host log (SP_LOG) in a child process: one line per solved system with its status, iterations,
reliable updates and true residual, and (SP_LOG=2) one per chunk poll; the solve's result is unchanged."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
pytestmark = pytest.mark.gpu

CODE = r"""
import sys
sys.path.insert(0, %r)
import torch
import lattice_inputs as li
import paper_1511_00088_amd as sp
dims = (8, 8, 8, 8)
G = sp.Gauge(sp.Lattice(dims), torch.from_numpy(li.near_identity_links(dims, 0.3, 701)).cuda(), lo_prec="f32", recon=12)
x, st = sp.cg_solve(G, 0.05, torch.from_numpy(li.gaussian_even_source(dims, 702)).cuda(), tol=1e-8, poll_chunk=5)
print("RESULT", st.iters, st.reliable_updates, st.converged, flush=True)
""" % ROOT


@pytest.mark.parametrize("level", ["1", "2"])
def test_host_log_lines(level):
    env = dict(os.environ, SP_LOG=level)
    r = subprocess.run([sys.executable, "-c", CODE], capture_output=True, text=True, timeout=240, env=env)
    assert r.returncode == 0, r.stderr[-2000:]
    res = [l for l in r.stdout.splitlines() if l.startswith("RESULT")][0].split()
    iters, rus = int(res[1]), int(res[2])
    lines = [l for l in r.stderr.splitlines() if l.startswith("[libstagcg]")]
    solve = [l for l in lines if "system 0 of 1" in l]
    assert len(solve) == 1 and "sp_cg_solve 8x8x8x8" in solve[0] and "status 0" in solve[0]
    assert f"{iters} iterations" in solve[0] and f"{rus} reliable updates" in solve[0]
    polls = [l for l in lines if l.startswith("[libstagcg] poll after chunk")]
    assert (len(polls) > 0) == (level == "2")
