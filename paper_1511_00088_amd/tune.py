"""Tune the half-Dslash launch (block size, XCD-aware block order, link-load policy) for a set of lattice shapes
and storage precisions on the current GPU and write the table that sp_tune_load reads.

    python -m paper_1511_00088_amd.tune OUT.json [--dims X Y Z T ...]
"""
from __future__ import annotations

import argparse

import torch

from . import api

# the workload, the batched sizes, the 16^3x32 gradient lattice, the 32^3x64 control, the 28^3x96 production
# lattice and one GPU's share of the workload cut in time across 8 GPUs
DEFAULT_DIMS = [(20, 20, 20, 64), (8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32), (32, 32, 32, 64),
                (28, 28, 28, 96), (20, 20, 20, 8)]
# (vector precision, recon, link precision): each storage precision alone, and 16-bit links with FP32 vectors
COMBOS = [("f64", 18, "f64"), ("f32", 18, "f32"), ("f32", 12, "f32"), ("f16", 18, "f16"), ("f16", 12, "f16"),
          ("bf16", 18, "bf16"), ("bf16", 12, "bf16"), ("f32", 12, "f16"), ("f32", 18, "f16"), ("f32", 12, "bf16"),
          ("f32", 18, "bf16"), ("f32", 12, "i16"), ("f32", 18, "i16")]


def tune_all(dims_list, combos=COMBOS, device="cuda:0"):
    out = []
    for dims in dims_list:
        lat = api.Lattice(dims)
        # the launch shape does not depend on the link values: identity links suffice
        links = torch.zeros((4, lat.V, 3, 3), dtype=torch.complex128, device=device)
        links[..., 0, 0] = links[..., 1, 1] = links[..., 2, 2] = 1.0
        for prec, recon, lp in combos:
            g = api.Gauge(lat, links, lo_prec=lp, recon=recon)
            ms = api.tune_dslash(g, prec)
            out.append((dims, prec, recon, lp, ms))
            print(f"{dims} {prec} r{recon} links {lp}: {ms * 1e3:.2f} us", flush=True)
            del g
        del links
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--dims", type=int, nargs="+", default=None, help="groups of 4 extents")
    a = ap.parse_args()
    dims_list = DEFAULT_DIMS
    if a.dims:
        if len(a.dims) % 4:
            raise SystemExit("--dims takes groups of 4 extents")
        dims_list = [tuple(a.dims[i:i + 4]) for i in range(0, len(a.dims), 4)]
    tune_all(dims_list)
    api.tune_save(a.out)


if __name__ == "__main__":
    main()
