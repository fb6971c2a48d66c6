"""Write the FP64 oracle's solution of the 20^3x64 workload at sampled sites (golden fixture).

Inputs: near-identity links (eps 0.3, seed 21), m = 0.01, Gaussian even source (seed 22). The oracle's
CG is driven to a true relative residual of 1e-12; the solution is recorded at 512 random checkerboard
sites (seed 23) plus the first and last 32 sites. Runs on the CPU only (about ten minutes) and calls
nothing but the oracle and the seeded input generators:

    python tests/golden/make_cfg1_samples.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lattice_inputs as li  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cfg1_solution_samples.txt")


def sample_sites(Vh):
    rng = np.random.default_rng(23)
    return np.unique(np.concatenate([rng.integers(0, Vh, 512), np.arange(32), np.arange(Vh - 32, Vh)]))


def main():
    c = li.cfg1()
    dims = c["dims"]
    Vh = li.volume(dims) // 2
    t0 = time.time()
    x, status, iters, res = oracle.cg_solve(dims, c["links"], c["mass"], c["source"], tol=1e-12, max_iter=20000)
    secs = time.time() - t0
    assert status == 0, status
    cbs = sample_sites(Vh)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle solution of (m^2 - D_eo D_oe) x = b on 20^3x64, near-identity links eps=0.3 seed 21,\n")
        f.write("# m=0.01, Gaussian even source seed 22, oracle CG to true relative residual 1e-12.\n")
        f.write("# Written by tests/golden/make_cfg1_samples.py (oracle only).\n")
        f.write(f"# iters {iters} true_rel_resid {res:.6e} norm_x {np.linalg.norm(x):.17e} seconds {secs:.1f}\n")
        f.write("# columns: cb re0 im0 re1 im1 re2 im2\n")
        for cb in cbs:
            v = x[cb]
            f.write(f"{cb} " + " ".join(f"{a:.17e} {b:.17e}" for a, b in zip(v.real, v.imag)) + "\n")
    print(f"wrote {OUT}: iters={iters} resid={res:.3e} {secs:.0f}s")


if __name__ == "__main__":
    main()
