"""Shared helpers of the GPU parity tests (device transfer, tolerances)."""
import os

import numpy as np
import torch

import paper_1511_00088_amd as sp

DEV = "cuda:0"

# Operator tolerances, infinity-norm relative error max|y - y_ref| / max|y_ref| against the FP64 oracle.
# FP32 and FP16 are the targets of the method; BF16 (8-bit mantissa, unit roundoff 2^-8) cannot meet 5e-3,
# its gate is 3e-2. FP64 differs from the oracle by summation order only.
DSLASH_TOL = {"f64": 1e-13, "f32": 1e-6, "f16": 5e-3, "bf16": 3e-2}


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def gauge(dims, links: np.ndarray, prec="f32", recon=18, bc_t=0):
    lat = sp.Lattice(dims, bc_t)
    return sp.Gauge(lat, to_dev(links), lo_prec=prec, recon=recon)


def announce(msg: str):
    print(msg, flush=True)


def cfg1_golden():
    """Site indices and values of the 20^3x64 workload's solution sampled from the oracle's 1e-12 solve
    (written by tests/golden/make_cfg1_samples.py, which calls only the oracle)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "cfg1_solution_samples.txt")
    rows = np.loadtxt(path)
    cbs = rows[:, 0].astype(np.int64)
    vals = rows[:, 1::2] + 1j * rows[:, 2::2]
    return cbs, vals


def tune_file():
    return os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1511_00088_amd", "tune_mi355x.json")
