"""Tune the half-Dslash launch (block size, XCD-aware block order, link-load policy) for a set of lattice shapes
and storage precisions on the current GPU and write the table that sp_tune_load reads.

    python -m paper_1511_00088_amd.tune OUT.json [--dims X Y Z T ...] [--recon R ...] [--base TABLE.json]

--recon keeps the combinations of those link packings only; --base loads an existing table first, so that
OUT.json holds its entries with the newly tuned ones replacing or joining them.
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
COMBOS = [("f64", 18, "f64"), ("f32", 18, "f32"), ("f32", 12, "f32"), ("f32", 8, "f32"), ("f16", 18, "f16"),
          ("f16", 12, "f16"),
          ("bf16", 18, "bf16"), ("bf16", 12, "bf16"), ("f32", 12, "f16"), ("f32", 18, "f16"), ("f32", 12, "bf16"),
          ("f32", 18, "bf16"), ("f32", 12, "i16"), ("f32", 18, "i16")]


def tune_all(dims_list, combos=COMBOS, device="cuda:0"):
    out = []
    for dims in dims_list:
        lat = api.Lattice(dims)
        # the launch shape does not depend on the link values: identity links suffice, and for recon 8 (which
        # cannot store a first row (1, 0, 0)) a rotation by pi/4 in the (0, 1) plane
        links = torch.zeros((4, lat.V, 3, 3), dtype=torch.complex128, device=device)
        links[..., 0, 0] = links[..., 1, 1] = links[..., 2, 2] = 1.0
        rot = None
        for prec, recon, lp in combos:
            if recon == 8 and rot is None:
                c = 0.5 ** 0.5
                rot = torch.zeros_like(links)
                rot[..., 0, 0] = rot[..., 1, 1] = rot[..., 0, 1] = c
                rot[..., 1, 0] = -c
                rot[..., 2, 2] = 1.0
            g = api.Gauge(lat, rot if recon == 8 else links, lo_prec=lp, recon=recon)
            ms = api.tune_dslash(g, prec)
            out.append((dims, prec, recon, lp, ms))
            print(f"{dims} {prec} r{recon} links {lp}: {ms * 1e3:.2f} us", flush=True)
            del g
        del links, rot
    return out


PREC_CODE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "i16": 4}
# single-solve combinations whose iteration is tuned on the solver's own launches: (inner, recon, link precision)
SOLVE_COMBOS = [("f32", 12, "f32"), ("f32", 18, "f32"), ("f32", 8, "f32"), ("f64", 18, "f64"), ("f32", 12, "i16"),
                ("f32", 12, "f16"), ("f16", 12, "f16"), ("bf16", 12, "bf16")]


def _table(entries):
    """Tuning-table text in the form sp_tune_save writes (one entry per line)."""
    lines = [f'  "{k}": {{"nt": {c["nt"]}, "remap": {c["remap"]}, "stream": {c["stream"]}}}' for k, c in entries.items()]
    return "{\n" + ",\n".join(lines) + "\n}\n"


def _load_entries(entries):
    import os
    import tempfile

    with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as f:
        f.write(_table(entries))
        path = f.name
    try:
        api.tune_load(path)
    finally:
        os.unlink(path)


def _key(dims, lp, recon, vp):
    return f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]}/l{PREC_CODE[lp]}/r{recon}/v{PREC_CODE[vp]}"


def _links(dims, device, seed=5):
    """Near-identity SU(3)-like links exp(i 0.3 H) on the device (the iteration's cost does not depend on the values,
    but a solve needs a well-posed system that does not converge within the timed iterations)."""
    V = dims[0] * dims[1] * dims[2] * dims[3]
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    out = torch.empty(4, V, 3, 3, dtype=torch.complex128, device=device)
    chunk = 1 << 20
    for mu in range(4):
        for s0 in range(0, V, chunk):
            n = min(chunk, V - s0)
            h = torch.randn(n, 3, 3, dtype=torch.complex128, device=device, generator=gen)
            out[mu, s0:s0 + n] = torch.linalg.matrix_exp(0.15j * (h + h.conj().transpose(-1, -2)))
    return out


def tune_solves(dims_list, combos=SOLVE_COMBOS, device="cuda:0", iters=75, reps=3):
    """Block order and link-load policy of the single-system solve, timed on the solve itself: a solve of `iters`
    iterations (m = 0.01, tol far below reach) per configuration, 256-thread blocks (what the fused iteration
    takes), the fastest per iteration kept as the "/solve" entry."""
    import time

    chosen = {}
    for dims in dims_list:
        lat = api.Lattice(dims)
        links = _links(dims, device)
        gen = torch.Generator(device=device)
        gen.manual_seed(6)
        b = torch.randn(lat.Vh, 3, dtype=torch.complex128, device=device, generator=gen)
        ws = api.Workspace()
        for inner, recon, lp in combos:
            g = api.Gauge(lat, links, lo_prec=lp, recon=recon)
            key = _key(dims, lp if inner != "f64" else "f64", recon if inner != "f64" else 18, inner) + "/solve"
            best = None
            for stream in (0, 1):
                for remap in (0, 1):
                    cfg = {"nt": 256, "remap": remap, "stream": stream}
                    _load_entries({key: cfg})
                    api.cg_solve(g, 0.01, b, tol=1e-14, inner=inner, max_iter=iters, workspace=ws)
                    ts = []
                    for _ in range(reps):
                        torch.cuda.synchronize()
                        t0 = time.perf_counter()
                        _, st = api.cg_solve(g, 0.01, b, tol=1e-14, inner=inner, max_iter=iters, workspace=ws)
                        torch.cuda.synchronize()
                        ts.append((time.perf_counter() - t0) / max(st.iters, 1))
                    t = sorted(ts)[len(ts) // 2]
                    if best is None or t < best[0]:
                        best = (t, cfg)
            chosen[key] = best[1]
            print(f"{dims} solve {inner} r{recon} links {lp}: {best[0] * 1e6:.2f} us/iteration with {best[1]}", flush=True)
            del g
        del links, b, ws
    _load_entries(chosen)  # leave the chosen entries in the process's table
    return chosen


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("out")
    ap.add_argument("--dims", type=int, nargs="+", default=None, help="groups of 4 extents")
    ap.add_argument("--recon", type=int, nargs="+", default=None, help="tune only these link packings")
    ap.add_argument("--base", default=None, help="a table to load first and keep the other entries of")
    a = ap.parse_args()
    dims_list = DEFAULT_DIMS
    if a.dims:
        if len(a.dims) % 4:
            raise SystemExit("--dims takes groups of 4 extents")
        dims_list = [tuple(a.dims[i:i + 4]) for i in range(0, len(a.dims), 4)]
    if a.base:
        api.tune_load(a.base)
    keep = (lambda c: c[1] in a.recon) if a.recon else (lambda c: True)
    tune_all(dims_list, [c for c in COMBOS if keep(c)])
    tune_solves([d for d in dims_list if d[0] * d[1] * d[2] * d[3] >= 4096], [c for c in SOLVE_COMBOS if keep(c)])
    api.tune_save(a.out)


if __name__ == "__main__":
    main()
