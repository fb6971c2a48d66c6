"""Write the FP64 oracle's HYP-smeared links of the 20^3x64 workload field at sampled links (golden fixture).

Input: the near-identity links of the 20^3x64 workload (eps 0.3, seed 21), smeared with the standard weights
(a1, a2, a3) = (0.75, 0.6, 0.3). The smeared link is recorded for 128 random (direction, site) pairs
(seed 24) plus the first and last 8 sites in every direction. Runs on the CPU only (a few minutes) and
calls nothing but the oracle and the seeded input generators:

    python tests/golden/make_hyp_samples.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import lattice_inputs as li  # noqa: E402
from oracle import hyp  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "hyp_cfg1_samples.txt")


def sample_links(V):
    rng = np.random.default_rng(24)
    pairs = {(int(m), int(s)) for m, s in zip(rng.integers(0, 4, 128), rng.integers(0, V, 128))}
    for m in range(4):
        for s in list(range(8)) + list(range(V - 8, V)):
            pairs.add((m, s))
    return sorted(pairs)


def main():
    c = li.cfg1()
    dims = c["dims"]
    V = li.volume(dims)
    t0 = time.time()
    Vs = hyp.hyp_smear(dims, c["links"], hyp.HYP_ALPHA)
    secs = time.time() - t0
    with open(OUT, "w") as f:
        f.write("# FP64 oracle HYP smearing of the 20^3x64 near-identity field (eps=0.3, seed 21), alpha = "
                "(0.75, 0.6, 0.3)\n")
        f.write(f"# written by tests/golden/make_hyp_samples.py; oracle time {secs:.0f} s\n")
        f.write("# mu lex then the 3x3 matrix row by row as re im pairs (18 numbers)\n")
        for m, s in sample_links(V):
            vals = " ".join(f"{x:.17e}" for z in Vs[m, s].ravel() for x in (z.real, z.imag))
            f.write(f"{m} {s} {vals}\n")


if __name__ == "__main__":
    main()
