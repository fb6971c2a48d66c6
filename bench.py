"""Benchmark: CG time-to-1e-8 residual, mixed vs FP64; Dslash GFLOP/s and fraction of peak HBM.

Workload (the paper's single-GPU CG job shape, Sec. 3, Fig. 1 / Table 2): a 20^3x64 lattice with
near-identity SU(3) links exp(i 0.3 H) standing in for the HYP-smeared MILC asqtad coarse ensemble,
m = 0.01, one Gaussian even-site source. One step = one mixed-precision solve (FP32 iterations, FP64
reliable updates) of (m^2 - D_eo D_oe) x = b from x = 0 to an FP64 true relative residual of 1e-8, with
links packed and source resident in HBM before the timed region. Beside it, in the same run:
  * the plain FP64 GPU CG to the same residual (the comparator),
  * the half-Dslash kernel timed with HIP events on the stream it runs on (roofline),
  * the FP64 CPU oracle timed on a bounded sample (FP64 CG iterations on the same lattice).
  * the packing of links and vectors, done once per gauge field or source and reported apart.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CG time-to-1e-8 residual, mixed vs FP64; Dslash GFLOP/s + % peak HBM"
HBM_PEAK_GBS = 8000.0
FLOP_PER_SITE = 570  # one half-Dslash output site: 8 SU(3) mat-vecs (66) + 7 colour-vector adds (6)
# algorithmic bytes per output site of one half-Dslash: 8 links + 1 input vector (perfect neighbour
# reuse) + 1 output vector
LINK_BYTES = {("f64", 18): 144, ("f32", 18): 72, ("f32", 12): 48, ("f32", 8): 32, ("f16", 18): 36, ("f16", 12): 24,
              ("bf16", 18): 36, ("bf16", 12): 24, ("i16", 18): 36, ("i16", 12): 24}
VEC_BYTES = {"f64": 48, "f32": 24, "f16": 16, "bf16": 12}


def dslash_bytes_per_site(prec, recon):
    return 8 * LINK_BYTES[(prec, recon)] + 2 * VEC_BYTES[prec]


def iteration_bytes_per_site(prec, recon, link_prec=None):
    """Algorithmic bytes per even site of one mixed-precision CG iteration. FP32 (and FP64) iterations take two
    launches: t = D_oe r + beta t with p = r + beta p (links, r, t read and written, p read and written) and
    x += alpha p, r -= alpha (m^2 p - D_eo t) (links, t, p, x and r read and written); x is FP32 for every
    inner precision (FP64 for plain FP64 CG). 16-bit vector storage takes three: t = D_oe p, the same update,
    p = r + beta p. link_prec: the links' storage precision when it differs from the vectors' (16-bit links,
    FP32 vectors)."""
    links, v = 8 * LINK_BYTES[(link_prec or prec, recon)], VEC_BYTES[prec]
    x = VEC_BYTES["f64"] if prec == "f64" else VEC_BYTES["f32"]
    if prec in ("f32", "f64"):
        return (links + v + 2 * v + 2 * v) + (links + v + v + 2 * x + 2 * v)
    return (links + 2 * v) + (links + 2 * v + 2 * x + 2 * v) + 3 * v


def golden_err(x, dims, mass):
    """Relative error of a 20^3x64 workload solution (m = 0.01) at the sites sampled from the oracle's 1e-12 solve:
    a committed text file written by the oracle alone (tests/golden/cfg1_solution_samples.txt); no oracle code
    runs here. None for any other workload."""
    path = os.path.join(ROOT, "tests", "golden", "cfg1_solution_samples.txt")
    if tuple(dims) != (20, 20, 20, 64) or mass != 0.01 or not os.path.exists(path):
        return None
    import numpy as np
    import torch

    rows = np.loadtxt(path)
    cbs = torch.from_numpy(rows[:, 0].astype(np.int64)).to(x.device)
    ref = rows[:, 1::2] + 1j * rows[:, 2::2]
    xs = x[cbs].cpu().numpy()
    return float(np.linalg.norm(xs - ref) / np.linalg.norm(ref))


def mean_stderr(ts):
    """Mean and standard error of the mean of a list of times."""
    n = len(ts)
    m = sum(ts) / n
    if n < 2:
        return m, None
    return m, (sum((t - m) ** 2 for t in ts) / (n - 1) / n) ** 0.5


def timed_solves(torch, fn, n):
    """Wall time of each of n calls (each solve returns after its stream reaches the end)."""
    ts, out = [], None
    for _ in range(n):
        t0 = time.perf_counter()
        out = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return ts, out


# flop per lattice site (both parities) of one CG iteration: two half-Dslash (570 per output site each, on
# half the sites), m^2 p (12 per even site) and five vector updates or dots (12 per even site each)
CG_FLOP_PER_SITE = 606


def control_links(dims, eps, seed, dev, torch):
    """Near-identity SU(3) links exp(i eps H), H = sum_a h_a lambda_a / 2, generated on the GPU with a
    seeded torch generator: the control lattice only measures bandwidth and is too large for the host
    generator to be quick. [4][V][3][3] complex128."""
    import lattice_inputs as li

    V = dims[0] * dims[1] * dims[2] * dims[3]
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    lam = torch.from_numpy((li.gell_mann() / 2.0).reshape(8, 9)).to(dev)
    out = torch.empty(4, V, 3, 3, dtype=torch.complex128, device=dev)
    chunk = 1 << 20
    for mu in range(4):
        for s in range(0, V, chunk):
            n = min(chunk, V - s)
            h = torch.randn(n, 8, generator=gen, device=dev, dtype=torch.float64).to(torch.complex128)
            out[mu, s:s + n] = torch.linalg.matrix_exp((1j * eps) * (h @ lam).reshape(n, 3, 3))
    return out


def time_dslash(sp, torch, G, prec, inp, out, reps, stream):
    """Mean duration of one half-Dslash launch over `reps` back-to-back launches (HIP events on the launch
    stream). Between launches the links stay in the Infinity Cache when they fit in it (the warm figure)."""
    for _ in range(10):
        sp.dslash_packed(G, prec, inp, 1, out)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        sp.dslash_packed(G, prec, inp, 1, out)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


class Flush:
    """Evicts the Infinity Cache: the library's streaming read kernel over 768 MiB (three times the cache; read,
    not written, so the cache is left holding no dirty lines whose write-back a following launch would pay)."""

    def __init__(self, sp, torch, dev, nbytes=768 << 20):
        self.sp = sp
        self.buf = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        self.out = torch.empty(self.buf.numel(), dtype=torch.float32, device=dev)

    def __call__(self):
        self.sp.stream_probe("read", 1, self.buf, self.out)


def time_flushed(torch, fn, flush, stream, reps=200, trials=5):
    """Net duration of one launch of fn when the Infinity Cache has been flushed just before it, so that every
    byte comes from HBM: (reps pairs of flush + launch) minus (reps flushes alone), both timed with HIP events
    on the launch stream, per launch; median over trials, the two timings interleaved. Differencing removes the
    flush and the events' own cost; the launch's start after the flush stays in."""
    for _ in range(3):
        flush()
        fn()
    res = []
    for _ in range(trials):
        f0, f1, e0, e1 = (torch.cuda.Event(enable_timing=True) for _ in range(4))
        f0.record(stream)
        for _ in range(reps):
            flush()
        f1.record(stream)
        e0.record(stream)
        for _ in range(reps):
            flush()
            fn()
        e1.record(stream)
        e1.synchronize()
        res.append((e0.elapsed_time(e1) - f0.elapsed_time(f1)) / 1e3 / reps)
    res.sort()
    return res[len(res) // 2]


PREC_CODE = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3, "i16": 4}


def tune_key(dims, lp, recon, vp):
    return f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]}/l{PREC_CODE[lp]}/r{recon}/v{PREC_CODE[vp]}"


def pin_launch(sp, key, cfg):
    """Make the library use launch configuration cfg ({"nt", "remap", "stream"}) for one tuning key, through a
    temporary table file (sp_tune_load merges it into the process's table)."""
    import tempfile

    with tempfile.NamedTemporaryFile("w", suffix=".json", delete=False) as f:
        f.write("{\n  \"%s\": {\"nt\": %d, \"remap\": %d, \"stream\": %d}\n}\n"
                % (key, cfg["nt"], cfg["remap"], cfg.get("stream", 0)))
        path = f.name
    try:
        sp.tune_load(path)
    finally:
        os.unlink(path)


def tuned_entry(path, key):
    """The tuned launch of key in a table file, or the library's default."""
    try:
        with open(path) as f:
            return {"nt": 256, "remap": 1, "stream": 0, **json.load(f)[key]}
    except (OSError, KeyError, ValueError):
        return {"nt": 256, "remap": 1, "stream": 0}


def stream_ceiling(sp, torch, dev, stream, flush, log, nbytes=2 << 30, small_bytes=None):
    """The library's own streaming kernels (sp_stream_probe: read, copy, triad, 16-byte words per lane, 1, 2, 4
    or 8 words per lane) over nbytes per buffer, back to back: the attainable HBM rates. With small_bytes, also
    the read probe over a buffer of that size after an Infinity Cache flush (net, as time_flushed): what a
    cold read of the half-Dslash's size attains."""
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    c = torch.ones_like(a)
    out = {}
    for kind, per in (("read", 16), ("copy", 32), ("triad", 48)):
        best = None
        for k in (1, 2, 4, 8):
            fn = lambda: sp.stream_probe(kind, k, a, b, c if kind == "triad" else None)
            for _ in range(2):
                fn()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(10):
                fn()
            e1.record(stream)
            e1.synchronize()
            gbs = per * (nbytes // 16) / (e0.elapsed_time(e1) / 1e3 / 10) / 1e9
            if best is None or gbs > best[0]:
                best = (gbs, k)
        out[kind] = {"GBs": best[0], "words_per_lane": best[1], "bytes_per_buffer": nbytes,
                     "hbm_frac": best[0] / HBM_PEAK_GBS}
    del a, b, c
    if small_bytes:
        n = small_bytes // 4
        a = torch.ones(n, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        best = None
        for k in (1, 2, 4, 8):
            t = time_flushed(torch, lambda: sp.stream_probe("read", k, a, b), flush, stream, reps=100, trials=3)
            gbs = small_bytes / t / 1e9
            if best is None or gbs > best[0]:
                best = (gbs, k, t)
        out["read_cold_small"] = {"GBs": best[0], "words_per_lane": best[1], "us": best[2] * 1e6,
                                  "bytes": small_bytes, "hbm_frac": best[0] / HBM_PEAK_GBS}
        del a, b
    log("stream probe: " + ", ".join(f"{k} {v['GBs']:.0f} GB/s" for k, v in out.items()))
    return out


KERNEL_SOURCES = ["paper_1511_00088_amd/csrc/sp_device.h", "paper_1511_00088_amd/csrc/sp_kernels.h",
                  "paper_1511_00088_amd/csrc/sp_launch_dslash.hip"]
TUNE_TABLE = os.path.join(ROOT, "paper_1511_00088_amd", "tune_mi355x.json")


def traffic_file(prec, recon, dims, policy="cached"):
    return os.path.join(ROOT, "profiles",
                        f"dslash_{prec}_r{recon}_{policy}_{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]}_traffic.md")


def kernel_source_digest(prec, recon, dims, policy):
    """Hash of the half-Dslash's sources and of the launch shape the counters see (block size and block order
    of the tuned entry, and the link-load policy): the counter summary holds while this is unchanged."""
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    e = tuned_entry(TUNE_TABLE, tune_key(dims, prec, recon, prec))
    h.update(f"nt={e['nt']} remap={e['remap']} policy={policy}".encode())
    return h.hexdigest()[:16]


def measured_traffic(prec, recon, dims, policy="cached"):
    """HBM bytes per half-Dslash launch (link loads of the given policy) from the committed counter summary, or
    None when there is none or the kernel sources or the counted launch shape changed since the counters were
    taken."""
    try:
        vals = {}
        with open(traffic_file(prec, recon, dims, policy)) as f:
            for line in f:
                if "=" in line and line.strip().split("=")[0].strip() in ("traffic_bytes_per_launch",
                                                                          "kernel_source_digest"):
                    k, v = (x.strip() for x in line.split("=", 1))
                    vals[k] = v
        if vals.get("kernel_source_digest") != kernel_source_digest(prec, recon, dims, policy):
            return None
        return float(vals["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def bench_batched(sp, li, torch, dev, log):
    """The batched workload: 8 right-hand sides on the 20^3x64 field plus 24 systems on 8^4, 12^3x24 and
    16^3x32 (masses uniform in [0.01, 0.1]), FP32 on recon-12 links + FP64 reliable updates, solved
    together and one by one."""
    gauges, systems = li.uneven_batch()
    G = []
    for dims, U in gauges:
        G.append(sp.Gauge(sp.Lattice(dims), torch.from_numpy(U).to(dev), lo_prec="f32", recon=12))
    sysl = [(G[s.gauge_index], s.mass, torch.from_numpy(s.source).to(dev)) for s in systems]
    ws = sp.Workspace()
    sp.cg_solve_batched(sysl, tol=1e-8, inner="f32", workspace=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, st = sp.cg_solve_batched(sysl, tol=1e-8, inner="f32", workspace=ws)
    torch.cuda.synchronize()
    t_b = time.perf_counter() - t0
    t0 = time.perf_counter()
    err = 0.0
    for (g, m, bb), xb in zip(sysl, xs):
        x1, _ = sp.cg_solve(g, m, bb, tol=1e-8, inner="f32", workspace=ws)
        err = max(err, float(torch.linalg.norm(x1 - xb) / torch.linalg.norm(x1)))
    torch.cuda.synchronize()
    t_s = time.perf_counter() - t0
    ok = all(s.converged for s in st)
    # algorithmic bytes of one batched iteration: per group of up to four systems sharing a gauge field, the links
    # of two half operators (t = D_oe p for all of them, then the update) and per system 264 B/site (t = D_oe p:
    # p in, t out; update: t, p, x and r with x and r read and written; p = r + beta p: r, p in, p out); every
    # system stays in its group's launches until the batch ends
    groups = {}
    for s_ in systems:
        groups[s_.gauge_index] = groups.get(s_.gauge_index, 0) + 1
    it_bytes = 0
    for gi, nsys in groups.items():
        vh = li.volume(gauges[gi][0]) // 2
        full, rest = divmod(nsys, 4)
        for nr in [4] * full + ([rest] if rest else []):
            it_bytes += vh * (2 * 8 * LINK_BYTES[("f32", 12)] + nr * 264)
    max_it = max(s.iters for s in st)
    log(f"batched 32 systems: {t_b * 1e3:.1f} ms together, {t_s * 1e3:.1f} ms one by one, all converged={ok}")
    return {"systems": len(sysl), "recon": 12, "s": t_b, "one_by_one_s": t_s, "speedup": t_s / t_b, "all_converged": ok,
            "max_iters": max_it, "max_rel_diff_vs_single": err, "iteration_bytes": it_bytes,
            "iteration_us": t_b / max_it * 1e6, "iteration_hbm_frac": it_bytes * max_it / t_b / 1e9 / HBM_PEAK_GBS,
            "note": "iteration figures over the whole batched solve (set-up, reliable updates, polling included)"}


# HYP smearing, algorithmic bytes per lattice site: level 1 reads the 4 input links and writes 12 fields,
# level 2 reads the 4 input links and the 12 level-1 fields and writes 12 fields, level 3 reads the 4 input
# links and the 12 level-2 fields and writes 4 links; 144 B per FP64 link.
HYP_BYTES_PER_SITE = 144 * ((4 + 12) + (4 + 12 + 12) + (4 + 12 + 4))


def bench_hyp(sp, torch, lat, links, stream, log):
    """HYP smearing of the workload's link field (the step before the solve), HIP events."""
    out = torch.empty_like(links)
    ws = sp.Workspace()
    sp.hyp_smear(lat, links, out=out, workspace=ws)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n = 5
    e0.record(stream)
    for _ in range(n):
        sp.hyp_smear(lat, links, out=out, workspace=ws)
    e1.record(stream)
    e1.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / n
    gbs = HYP_BYTES_PER_SITE * lat.V / t / 1e9
    log(f"HYP smearing {lat.dims}: {t * 1e3:.2f} ms ({gbs:.0f} GB/s of algorithmic bytes)")
    return {"dims": list(lat.dims), "ms": t * 1e3, "alpha": list(sp.HYP_ALPHA),
            "bytes_per_site": HYP_BYTES_PER_SITE, "achieved_GBs": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
            "note": "three FP64 levels with SU(3) projections (the closed-form maximiser, else a Newton polar factor and series, else SU(2)-subgroup sweeps); "
                    "bound by FP64 arithmetic, not bytes"}


# NPR contraction: flop per (field set, hypercube): 256 terms, each two bilinears chib^T U chi (U chi: 9
# complex multiply-adds = 66 flop, the dot with chib: 22 flop), their product (6) and the signed sum (4)
NPR_FLOP_PER_Z = 256 * (2 * (66 + 22) + 10)
NPR_SETS = 4  # field sets per contraction launch


def bench_npr(sp, torch, lat, links, stream, log):
    """The NPR one-colour-trace contraction on the workload lattice: path links once, then a contraction of
    NPR_SETS Gaussian field sets (labels gamma_5 x xi_5 for both bilinears), HIP events."""
    gen = torch.Generator(device=links.device)
    gen.manual_seed(61)
    f = [torch.randn(NPR_SETS, lat.V, 3, dtype=torch.complex128, device=links.device, generator=gen)
         for _ in range(4)]
    labels = (15, 15, 15, 15)
    uad = sp.npr_path_links(lat, links)
    sp.npr_contract(lat, uad, *f, labels)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    n = 10
    e0.record(stream)
    for _ in range(n):
        sp.npr_path_links(lat, links)
    e1.record(stream)
    e1.synchronize()
    t_p = e0.elapsed_time(e1) / 1e3 / n
    e0.record(stream)
    for _ in range(n):
        sp.npr_contract(lat, uad, *f, labels)
    e1.record(stream)
    e1.synchronize()
    t_c = e0.elapsed_time(e1) / 1e3 / n
    # fused: the path links built per hypercube on chip inside the contraction
    sp.npr_contract_links(lat, links, *f, labels)
    e0.record(stream)
    for _ in range(n):
        sp.npr_contract_links(lat, links, *f, labels)
    e1.record(stream)
    e1.synchronize()
    t_f = e0.elapsed_time(e1) / 1e3 / n
    nz = lat.V // 16
    bytes_c = nz * (256 * 144 + NPR_SETS * (4 * 16 * 48 + 16))
    res = {"dims": list(lat.dims), "sets": NPR_SETS, "labels": list(labels), "paths_ms": t_p * 1e3,
           "contract_ms": t_c * 1e3, "contract_gflops": NPR_FLOP_PER_Z * NPR_SETS * nz / t_c / 1e9,
           "contract_bytes": bytes_c, "contract_GBs": bytes_c / t_c / 1e9,
           "contract_hbm_frac": bytes_c / t_c / 1e9 / HBM_PEAK_GBS,
           "paths_bytes": lat.V * 4 * 144 + nz * 256 * 144,
           "paths_GBs": (lat.V * 4 * 144 + nz * 256 * 144) / t_p / 1e9,
           "fused_ms": t_f * 1e3, "fused_bytes": lat.V * 4 * 144 + nz * NPR_SETS * (4 * 16 * 48 + 16),
           "fused_GBs": (lat.V * 4 * 144 + nz * NPR_SETS * (4 * 16 * 48 + 16)) / t_f / 1e9,
           "fused_speedup_vs_two_launches": (t_p + t_c) / t_f}
    log(f"NPR: path links {t_p * 1e3:.3f} ms, contraction of {NPR_SETS} sets {t_c * 1e3:.3f} ms, fused {t_f * 1e3:.3f} ms "
        f"({res['contract_gflops']:.0f} GFLOP/s, {res['contract_GBs']:.0f} GB/s)")
    return res


def bench_gradient(sp, li, torch, dev, log):
    """16^3x32, m = 0.05: loss Re phi^dag A^-1 phi, forward solve + adjoint solve + force kernels."""
    c = li.cfg4()
    lat = sp.Lattice(c["dims"])
    U = torch.from_numpy(c["links"]).to(dev).requires_grad_(True)
    phi = torch.from_numpy(c["source"]).to(dev).requires_grad_(True)
    m = torch.tensor(c["mass"], dtype=torch.float64, device=dev, requires_grad=True)

    def step():
        x = sp.staggered_solve(U, m, phi, lat, inner="f32", tol=1e-10)
        loss = torch.vdot(phi.flatten(), x.flatten()).real
        loss.backward()
        return loss

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        U.grad = None
        step()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / 3
    log(f"gradient 16^3x32: {t * 1e3:.1f} ms forward + backward")
    return {"dims": list(c["dims"]), "s": t, "note": "forward solve + adjoint solve to 1e-10 + force kernels"}



def bench_large_lattices(sp, torch, dev, tune_file, log, ws):
    """Mixed FP32 recon-12 solves (m = 0.01, Gaussian source, tol 1e-8) on the 32^3x64 control lattice and the
    paper's 28^3x96 production lattice (Sec. 4), whose link fields exceed the Infinity Cache: time per iteration
    against the workload's, and the iteration's fraction of HBM peak at its algorithmic bytes; then the same
    systems on recon-8 links ("recon8")."""
    out = {}
    ib = iteration_bytes_per_site("f32", 12)
    for dims, seed in (((32, 32, 32, 64), 71), ((28, 28, 28, 96), 72)):
        lat = sp.Lattice(dims)
        links = control_links(dims, 0.3, seed, dev, torch)
        gen = torch.Generator(device=dev)
        gen.manual_seed(seed + 100)
        bsrc = torch.randn(lat.Vh, 3, dtype=torch.complex128, device=dev, generator=gen)
        G = sp.Gauge(lat, links, lo_prec="f32", recon=12)
        G8 = sp.Gauge(lat, links, lo_prec="f32", recon=8)
        del links
        key = f"{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]}"
        for g, rc in ((G, 12), (G8, 8)):
            sp.cg_solve(g, 0.01, bsrc, tol=1e-8, inner="f32", workspace=ws)
            torch.cuda.synchronize()
            ts, (_, st) = timed_solves(torch, lambda: sp.cg_solve(g, 0.01, bsrc, tol=1e-8, inner="f32", workspace=ws),
                                       2)
            t = min(ts)
            t_it = t / max(st.iters, 1)
            ibr = iteration_bytes_per_site("f32", rc)
            res = {"s": t, "iters": st.iters, "reliable_updates": st.reliable_updates, "converged": st.converged,
                   "true_rel_resid": st.true_rel_resid, "us_per_iteration": t_it * 1e6,
                   "iteration_hbm_frac": ibr * lat.Vh / t_it / 1e9 / HBM_PEAK_GBS}
            if rc == 12:
                out[key] = res
            else:  # the same system on recon-8 links
                res["speedup_vs_recon12"] = out[key]["s"] / t
                out[key]["recon8"] = res
            log(f"large lattice {dims} r{rc}: {t * 1e3:.1f} ms, {st.iters} iterations, {t_it * 1e6:.1f} us/iteration "
                f"({ibr * lat.Vh / t_it / 1e9 / HBM_PEAK_GBS:.3f} of peak)")
        del G, G8, bsrc
    return out


def bench_shard_share(sp, torch, dims, links, b, prec, recon, stream, log, ngpu=8):
    """One GPU's share of the workload cut in time across ngpu GPUs (20^3x8 of 20^3x64), through the shard path
    the multi-GPU solve would use: pack the two boundary faces, copy each (a device-to-device copy standing in
    for the transfer to the neighbour), unpack them into the ghost slices, then the half operator on the interior
    slices and on the boundary slices. HIP events over back-to-back repetitions of each part."""
    X, Y, Z, T = dims
    Tl = T // ngpu
    t0 = (ngpu // 2) * Tl
    XYZ = X * Y * Z
    F = XYZ // 2
    sh = sp.Shard((X, Y, Z, Tl), t0, T)
    G = sp.Gauge(sh.lat, links[:, t0 * XYZ:(t0 + Tl) * XYZ].contiguous(), lo_prec=prec, recon=recon)
    ghost = sh.ghost_pack(links[3, (t0 - 1) * XYZ:t0 * XYZ].contiguous(), prec, recon)
    ext = sh.pack_vec(b[t0 * F:(t0 + Tl) * F].contiguous(), prec)
    faces = [sh.face_pack(prec, ext, side) for side in (0, 1)]
    recv = [torch.empty_like(f) for f in faces]
    out = torch.empty(sh.lat.vec_bytes(prec), dtype=torch.uint8, device=b.device)

    def exchange():
        for side in (0, 1):
            sh.face_pack(prec, ext, side, faces[side])
            recv[side].copy_(faces[side])
            # the lowest slice becomes the ghost above of the neighbour below, the highest the ghost below of the one
            # above; here the shard's own faces stand in for its neighbours'
            sh.face_unpack(prec, recv[side], 1 - side, ext)

    parts = {"exchange": exchange,
             "interior": lambda: sh.dslash(G, ghost, prec, ext, 1, part=1, out=out),
             "boundary": lambda: sh.dslash(G, ghost, prec, ext, 1, part=2, out=out),
             "operator": lambda: sh.dslash(G, ghost, prec, ext, 1, part=0, out=out)}
    parts["step"] = lambda: (exchange(), parts["interior"](), parts["boundary"]())
    parts["step"]()
    torch.cuda.synchronize()
    eager = out.clone()
    res = {}
    # each part is captured REPS times back to back in one graph and the graph replayed, so that neither the rate
    # of the host's calls (several small launches of a few microseconds each) nor a graph launch's own latency
    # sets the time
    REPS, REPLAYS = 50, 10
    for name, fn in parts.items():
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            fn()
        torch.cuda.current_stream().wait_stream(side)
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for _ in range(REPS):
                fn()
        for _ in range(2):
            graph.replay()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(REPLAYS):
            graph.replay()
        e1.record(stream)
        e1.synchronize()
        res[name + "_us"] = e0.elapsed_time(e1) * 1e3 / (REPS * REPLAYS)
        if name == "step":
            res["graph_output_equals_eager"] = bool(torch.equal(out, eager))
        del graph
    bps = dslash_bytes_per_site(prec, recon)
    res.update(dims=[X, Y, Z, Tl], t0=t0, face_bytes=sh.face_bytes(prec),
               operator_hbm_frac=bps * sh.lat.Vh / (res["operator_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS,
               note=f"one GPU's share of {X}^3x{T} cut in t across {ngpu} GPUs: faces packed, copied on the device "
                    "(standing in for the transfer) and unpacked; interior and boundary launches")
    log(f"shard share {res['dims']}: operator {res['operator_us']:.2f} us, exchange {res['exchange_us']:.2f} us, "
        f"step {res['step_us']:.2f} us")
    return res

def bench_packing(sp, torch, lat, links, b, inner, recon, stream, log):
    """Packing, done once per gauge field (links) or per source and solution (vectors) and not part of the
    time-to-solution: natural complex128 links to the FP64 recon-18 layout and to the inner precision's
    layout, a source to the packed layout and back. HIP events over back-to-back calls on the stream they
    run on; bytes are what one call reads plus what it writes."""
    nat_links = 4 * lat.V * 9 * 16
    nat_vec = lat.Vh * 3 * 16
    packed = sp.pack_vec(lat, b, inner)
    cases = [("links_f64_r18", lambda: sp.pack_gauge(lat, links, "f64", 18), nat_links + lat.gauge_bytes("f64", 18)),
             (f"links_{inner}_r{recon}", lambda: sp.pack_gauge(lat, links, inner, recon),
              nat_links + lat.gauge_bytes(inner, recon)),
             (f"vec_pack_{inner}", lambda: sp.pack_vec(lat, b, inner), nat_vec + lat.vec_bytes(inner)),
             (f"vec_unpack_{inner}", lambda: sp.unpack_vec(lat, packed, inner), lat.vec_bytes(inner) + nat_vec)]
    out = {}
    for name, fn, nbytes in cases:
        fn()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        n = 10
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        e1.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / n
        out[name] = {"us": t * 1e6, "bytes": nbytes, "hbm_frac": nbytes / t / 1e9 / HBM_PEAK_GBS}
    log("packing: " + ", ".join(f"{k} {v['us']:.1f} us" for k, v in out.items()))
    out["note"] = ("natural complex128 input already in HBM; the recon-12 and recon-8 packings read whole links "
                   "(the dropped entries share their cache lines); the vector calls are short enough that the rate "
                   "of the Python calls, not the kernel, sets their time")
    return out


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--inner", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--recon", type=int, default=12, choices=[18, 12, 8],
                    help="link storage: 12 = first two rows, third rebuilt as conj(row0 x row1) (exact for SU(3)); "
                         "8 = U01, U02, U10 and two phases, the rest rebuilt from unitarity (FP32 links only, "
                         "entries good to about 1e-5)")
    ap.add_argument("--links", default=None, choices=["f16", "bf16", "i16"],
                    help="store the links of the timed solve in 16 bits (FP32 vectors; --inner f32 only)")
    ap.add_argument("--dims", type=int, nargs=4, default=[20, 20, 20, 64])
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparator solves")
    ap.add_argument("--dslash-reps", type=int, default=200)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 16-bit storage solves, the batched workload and the gradient timing")
    ap.add_argument("--tune-file", default=os.path.join(ROOT, "paper_1511_00088_amd", "tune_mi355x.json"),
                    help="tuned launch table to load (tunes in-process when the file is missing)")
    ap.add_argument("--policy", default="tuned", choices=["tuned", "cached", "streaming"],
                    help="traffic mode: link loads of the half-Dslash launches (the tuned one, or forced)")
    ap.add_argument("--mode", default="bench", choices=["bench", "traffic", "hyp", "npr", "large", "batched", "gradient"],
                    help="traffic: only a 1 GiB device copy (counter calibration) and the half-Dslash "
                         "launches, for hardware-counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the solver has no multi-GPU path",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import lattice_inputs as li
    import paper_1511_00088_amd as sp

    def log(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    dev = "cuda:0"
    dims = tuple(args.dims)
    log(f"generating 20^3x64-style inputs dims={dims}")
    c = li.cfg1(dims)
    mass, tol = c["mass"], c["tol"]
    lat = sp.Lattice(dims)
    links = torch.from_numpy(c["links"]).to(dev)
    b = torch.from_numpy(c["source"]).to(dev)
    if args.links and args.inner != "f32":
        raise SystemExit("--links needs --inner f32")
    G = sp.Gauge(lat, links, lo_prec=args.links or args.inner, recon=args.recon)
    G64 = sp.Gauge(lat, links, lo_prec="f64")
    links_cache = [links]

    def G64_links():
        return links_cache[0]
    if os.path.exists(args.tune_file):
        log(f"loading tuned launches from {args.tune_file}")
        sp.tune_load(args.tune_file)
    else:
        log("tuning the half-Dslash launch")
        sp.tune_dslash(G, args.inner)
        sp.tune_dslash(G64, "f64")
    ws = sp.Workspace()
    stream = torch.cuda.current_stream()

    if args.mode == "traffic":
        # calibration: a device-to-device copy of known size, then the dominant kernel alone
        n = 1 << 30
        src = torch.ones(n, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        inp = sp.pack_vec(lat, b, args.inner)
        out = torch.empty_like(inp)
        key = tune_key(dims, args.inner, args.recon, args.inner)
        cfg = tuned_entry(args.tune_file, key)
        if args.policy != "tuned":
            cfg = dict(cfg, stream=1 if args.policy == "streaming" else 0)
            pin_launch(sp, key, cfg)
        for _ in range(20):
            sp.dslash_packed(G, args.inner, inp, 1, out)
        torch.cuda.synchronize()
        pol = "streaming" if cfg.get("stream", 0) else "cached"
        print(json.dumps({"mode": "traffic", "copy_bytes": n, "dslash_launches": 20, "launch": cfg,
                          "dslash_algorithmic_bytes": dslash_bytes_per_site(args.inner, args.recon) * lat.Vh,
                          "kernel_source_digest": kernel_source_digest(args.inner, args.recon, dims, pol)}))
        return

    if args.mode == "npr":
        # the NPR contraction alone (for a kernel trace of its two launches)
        print(json.dumps({"mode": "npr", **bench_npr(sp, torch, lat, G64_links(), stream, log)}))
        return

    if args.mode == "batched":
        # the 32-system batched workload alone (for a kernel trace of its launches)
        print(json.dumps({"mode": "batched", **bench_batched(sp, li, torch, dev, log)}))
        return

    if args.mode == "gradient":
        # the 16^3x32 forward + adjoint solve + force alone (for a kernel trace)
        print(json.dumps({"mode": "gradient", **bench_gradient(sp, li, torch, dev, log)}))
        return

    if args.mode == "large":
        # the 32^3x64 and 28^3x96 solves alone (for a kernel trace of their iterations)
        print(json.dumps({"mode": "large", **bench_large_lattices(sp, torch, dev, args.tune_file, log, ws)}))
        return

    if args.mode == "hyp":
        # the HYP smearing of the workload field alone (for a kernel trace of its three launches)
        print(json.dumps({"mode": "hyp", **bench_hyp(sp, torch, lat, G64_links(), stream, log)}))
        return

    def solve_mixed():
        return sp.cg_solve(G, mass, b, tol=tol, inner=args.inner, workspace=ws)

    def solve_fp64(t=tol):
        return sp.cg_solve(G64, mass, b, tol=t, inner="f64", workspace=ws)

    log(f"warmup {args.warmup}")
    for _ in range(args.warmup):
        x, st = solve_mixed()
    torch.cuda.synchronize()
    log(f"timing {args.steps} mixed-precision solves")
    per, (x, st) = timed_solves(torch, solve_mixed, max(args.steps, 1))
    t_mixed, t_mixed_se = mean_stderr(per)
    assert st.converged, f"mixed solve did not converge: {st}"
    err_oracle = golden_err(x, dims, mass)
    log(f"mixed: {t_mixed * 1e3:.2f} ms/solve iters={st.iters} ru={st.reliable_updates} "
        f"resid={st.true_rel_resid:.3e} err vs oracle samples {err_oracle}")

    extra = {"err_vs_oracle_samples": err_oracle}
    if not args.no_fp64:
        x64, st64 = solve_fp64()
        torch.cuda.synchronize()
        per64, (x64, st64) = timed_solves(torch, solve_fp64, max(1, args.steps))
        t_fp64, t_fp64_se = mean_stderr(per64)
        xref, stref = solve_fp64(1e-12)
        err = float(torch.linalg.norm(x - xref) / torch.linalg.norm(xref))
        err64 = float(torch.linalg.norm(x64 - xref) / torch.linalg.norm(xref))
        log(f"fp64: {t_fp64 * 1e3:.2f} ms/solve iters={st64.iters}; mixed err vs 1e-12 FP64 solve {err:.3e}")
        extra.update(fp64_cg_s=t_fp64, fp64_cg_s_stderr=t_fp64_se, fp64_solves=len(per64),
                     fp64_cg_gflops=CG_FLOP_PER_SITE * lat.V * st64.iters / t_fp64 / 1e9,
                     fp64_iters=st64.iters, speedup_vs_fp64=t_fp64 / t_mixed,
                     err_mixed_vs_fp64_1e12=err, err_fp64_vs_fp64_1e12=err64, ref_iters_1e12=stref.iters,
                     fp64_true_rel_resid=st64.true_rel_resid, fp64_err_vs_oracle_samples=golden_err(x64, dims, mass))

    # --- dominant kernel: half-Dslash in the inner precision, HIP events on the launch stream ---
    inp = sp.pack_vec(lat, b, args.inner)
    out = torch.empty_like(inp)
    lprec = args.links or args.inner
    bps = 8 * LINK_BYTES[(lprec, args.recon)] + 2 * VEC_BYTES[args.inner]
    alg_bytes = bps * lat.Vh
    flush = Flush(sp, torch, dev)
    # both link-load policies of the tuned launch: warm (back-to-back; the 20^3x64 links, 66-98 MB in FP32
    # recon-8 or recon-12, stay in the Infinity Cache, the solver's situation) and cold (each launch after a 1 GiB read
    # that flushes the Infinity Cache, net of the flush: every byte from HBM, the roofline figure)
    key = tune_key(dims, lprec, args.recon, args.inner)
    tuned = tuned_entry(args.tune_file, key)
    policies = {}
    for pol, name in ((0, "cached"), (1, "streaming")):
        pin_launch(sp, key, dict(tuned, stream=pol))
        tw = time_dslash(sp, torch, G, args.inner, inp, out, args.dslash_reps, stream)
        tf = time_flushed(torch, lambda: sp.dslash_packed(G, args.inner, inp, 1, out), flush, stream)
        policies[name] = {"warm_us": tw * 1e6, "flushed_us": tf * 1e6, "warm_hbm_frac": alg_bytes / tw / 1e9 / HBM_PEAK_GBS,
                          "flushed_hbm_frac": alg_bytes / tf / 1e9 / HBM_PEAK_GBS,
                          "solver_uses": pol == tuned.get("stream", 0)}
    pin_launch(sp, key, tuned)
    solver_pol = "streaming" if tuned.get("stream", 0) else "cached"
    best_pol = min(policies, key=lambda k: policies[k]["flushed_us"])
    t_d = policies[solver_pol]["warm_us"] / 1e6
    t_df = policies[best_pol]["flushed_us"] / 1e6
    achieved = alg_bytes / t_df / 1e9
    gflops = FLOP_PER_SITE * lat.Vh / t_df / 1e9
    # FP64 half-Dslash as well (the reliable-update and plain-FP64 kernel)
    inp64 = sp.pack_vec(lat, b, "f64")
    out64 = torch.empty_like(inp64)
    t_d64 = time_dslash(sp, torch, G64, "f64", inp64, out64, args.dslash_reps // 2, stream)
    log(f"dslash {args.inner} r{args.recon}: flushed {t_df * 1e6:.2f} us ({achieved:.0f} GB/s), warm "
        f"{t_d * 1e6:.2f} us ({alg_bytes / t_d / 1e9:.0f} GB/s); f64 warm {t_d64 * 1e6:.2f} us")
    probe = stream_ceiling(sp, torch, dev, stream, flush, log, small_bytes=alg_bytes)
    dslash_extra = {"flushed_us": t_df * 1e6, "flushed_hbm_frac": achieved / HBM_PEAK_GBS, "policies": policies,
                    "tuned_launch": tuned,
                    "warm_us": t_d * 1e6, "warm_GBs": alg_bytes / t_d / 1e9, "warm_hbm_frac": alg_bytes / t_d / 1e9 / HBM_PEAK_GBS,
                    "warm_gflops": FLOP_PER_SITE * lat.Vh / t_d / 1e9}
    control = None
    if not args.no_extras:
        # control lattice 32^3x64: links of every packing are more than the 256 MB Infinity Cache
        cd = (32, 32, 32, 64)
        clat = sp.Lattice(cd)
        clinks = control_links(cd, 0.3, 51, dev, torch)
        cv = torch.randn(clat.Vh, 3, dtype=torch.complex128, device=dev)
        ctl = {}
        for rc in (18, 12) + ((8,) if args.inner == "f32" else ()):
            Gc = sp.Gauge(clat, clinks, lo_prec=args.inner, recon=rc)
            ci = sp.pack_vec(clat, cv, args.inner)
            co = torch.empty_like(ci)
            cb = dslash_bytes_per_site(args.inner, rc)
            tc = time_dslash(sp, torch, Gc, args.inner, ci, co, 100, stream)
            tcf = time_flushed(torch, lambda: sp.dslash_packed(Gc, args.inner, ci, 1, co), flush, stream, reps=50)
            ctl[f"{args.inner}_r{rc}"] = {"us": tc * 1e6, "hbm_frac": cb * clat.Vh / tc / 1e9 / HBM_PEAK_GBS,
                                          "flushed_us": tcf * 1e6,
                                          "flushed_hbm_frac": cb * clat.Vh / tcf / 1e9 / HBM_PEAK_GBS}
            log(f"control 32^3x64 {args.inner} r{rc}: {tc * 1e6:.1f} us, flushed {tcf * 1e6:.1f} us")
            del Gc, ci, co
        del clinks
        dslash_extra["control_32x32x32x64"] = ctl
        control = ctl.get(f"{args.inner}_r{args.recon}")
        # every packing at the workload shape, back-to-back (tuned launch of each)
        allc = {}
        for prec, rc in LINK_BYTES:
            if prec == "i16":  # a link storage only; its operator runs with FP32 vectors (links_16bit_vectors_f32)
                continue
            Ga = G64 if prec == "f64" else sp.Gauge(lat, G64_links(), lo_prec=prec, recon=rc)
            ai = sp.pack_vec(lat, b, prec)
            ao = torch.empty_like(ai)
            ta = time_dslash(sp, torch, Ga, prec, ai, ao, 100, stream)
            ab = dslash_bytes_per_site(prec, rc)
            allc[f"{prec}_r{rc}"] = {"us": ta * 1e6, "bytes_per_site": ab, "gflops": FLOP_PER_SITE * lat.Vh / ta / 1e9,
                                     "hbm_frac": ab * lat.Vh / ta / 1e9 / HBM_PEAK_GBS}
            del Ga, ai, ao
        dslash_extra["all_packings"] = allc
        log("all packings: " + ", ".join(f"{kk} {vv['us']:.1f} us" for kk, vv in allc.items()))
        # the halo-fed operator of the same packing (FP64 links are stored whole)
        extra_shard = bench_shard_share(sp, torch, dims, G64_links(), b, args.inner,
                                        18 if args.inner == "f64" else args.recon, stream, log)
        dslash_extra["shard_share"] = extra_shard
    del flush

    traffic = measured_traffic(args.inner, args.recon, dims, best_pol)

    t_r12 = t_mixed if (args.inner, args.recon, args.links) == ("f32", 12, None) else None
    if not args.no_extras and "err_mixed_vs_fp64_1e12" in extra:
        # FP32 iterations on the other link packings, same workload (recon 8: a third fewer link bytes, entries
        # rebuilt to about 1e-5, which the reliable updates absorb)
        f32c = {}
        if args.inner == "f32" and not args.links:
            for rc in (8, 12, 18):
                if rc == args.recon:
                    continue
                Gr = sp.Gauge(lat, G64_links(), lo_prec="f32", recon=rc)
                sp.cg_solve(Gr, mass, b, tol=tol, inner="f32", workspace=ws)
                torch.cuda.synchronize()
                pr, (xr_, str_) = timed_solves(
                    torch, lambda: sp.cg_solve(Gr, mass, b, tol=tol, inner="f32", workspace=ws), max(1, args.steps))
                tr, tr_se = mean_stderr(pr)
                ib = iteration_bytes_per_site("f32", rc)
                f32c[f"f32_r{rc}"] = {"s": tr, "s_stderr": tr_se, "solves": len(pr), "iters": str_.iters,
                                      "reliable_updates": str_.reliable_updates, "true_rel_resid": str_.true_rel_resid,
                                      "err_vs_fp64_1e12": float(torch.linalg.norm(xr_ - xref) / torch.linalg.norm(xref)),
                                      "err_vs_oracle_samples": golden_err(xr_, dims, mass),
                                      "speedup_vs_headline": t_mixed / tr, "iteration_bytes_per_site": ib,
                                      "iteration_hbm_frac": ib * lat.Vh * str_.iters / tr / 1e9 / HBM_PEAK_GBS}
                log(f"f32 r{rc}: {tr * 1e3:.2f} ms/solve iters={str_.iters}")
                if rc == 12:
                    t_r12 = tr
                del Gr
            extra["f32_other_recon"] = f32c
        # 16-bit storage of links and vectors with FP32 arithmetic, same workload
        low = {}
        for prec in ("f16", "bf16"):
            for rc in (18, 12):
                Gl = sp.Gauge(lat, G64_links(), lo_prec=prec, recon=rc)
                sp.cg_solve(Gl, mass, b, tol=tol, inner=prec, workspace=ws)
                torch.cuda.synchronize()
                pl, (xl, stl) = timed_solves(
                    torch, lambda: sp.cg_solve(Gl, mass, b, tol=tol, inner=prec, workspace=ws), max(1, args.steps))
                tl, tl_se = mean_stderr(pl)
                el = float(torch.linalg.norm(xl - xref) / torch.linalg.norm(xref))
                ib = iteration_bytes_per_site(prec, rc)
                low[f"{prec}_r{rc}"] = {"s": tl, "s_stderr": tl_se, "solves": len(pl), "iters": stl.iters,
                                        "reliable_updates": stl.reliable_updates,
                                        "true_rel_resid": stl.true_rel_resid, "err_vs_fp64_1e12": el,
                                        "err_vs_oracle_samples": golden_err(xl, dims, mass),
                                        "speedup_vs_inner": t_mixed / tl,
                                        "speedup_vs_f32_r12": t_r12 / tl if t_r12 else None,
                                        "iteration_bytes_per_site": ib,
                                        "iteration_hbm_frac": ib * lat.Vh * stl.iters / tl / 1e9 / HBM_PEAK_GBS}
                log(f"{prec} r{rc}: {tl * 1e3:.2f} ms/solve iters={stl.iters} err={el:.2e}")
                del Gl
        extra["storage_16bit"] = low
        # 16-bit links with FP32 vectors and arithmetic (the links are most of each iteration's bytes)
        l16 = {}
        for lp in ("i16", "f16", "bf16"):
            for rc in (12, 18):
                Gl = sp.Gauge(lat, G64_links(), lo_prec=lp, recon=rc)
                sp.cg_solve(Gl, mass, b, tol=tol, inner="f32", workspace=ws)
                torch.cuda.synchronize()
                pl, (xl, stl) = timed_solves(
                    torch, lambda: sp.cg_solve(Gl, mass, b, tol=tol, inner="f32", workspace=ws), max(1, args.steps))
                tl, tl_se = mean_stderr(pl)
                el = float(torch.linalg.norm(xl - xref) / torch.linalg.norm(xref))
                ib = iteration_bytes_per_site("f32", rc, lp)
                l16[f"links_{lp}_r{rc}"] = {"s": tl, "s_stderr": tl_se, "solves": len(pl), "iters": stl.iters,
                                            "reliable_updates": stl.reliable_updates,
                                            "true_rel_resid": stl.true_rel_resid, "err_vs_fp64_1e12": el,
                                            "err_vs_oracle_samples": golden_err(xl, dims, mass),
                                            "speedup_vs_inner": t_mixed / tl,
                                            "speedup_vs_f32_r12": t_r12 / tl if t_r12 else None,
                                            "iteration_bytes_per_site": ib,
                                            "iteration_hbm_frac": ib * lat.Vh / (tl / max(stl.iters, 1)) / 1e9 / HBM_PEAK_GBS}
                log(f"links {lp} r{rc} + f32 vectors: {tl * 1e3:.2f} ms/solve iters={stl.iters} err={el:.2e}")
                del Gl
        extra["links_16bit_vectors_f32"] = l16
        extra["hyp"] = bench_hyp(sp, torch, lat, G64_links(), stream, log)
        extra["npr"] = bench_npr(sp, torch, lat, G64_links(), stream, log)
        extra["batched"] = bench_batched(sp, li, torch, dev, log)
        extra["gradient"] = bench_gradient(sp, li, torch, dev, log)
        extra["large_lattices"] = bench_large_lattices(sp, torch, dev, args.tune_file, log, ws)
        extra["packing"] = bench_packing(sp, torch, lat, G64_links(), b, args.inner, args.recon, stream, log)

    cpu = None
    if not args.no_cpu:
        import oracle

        oracle.build(force=False)
        bh = c["source"]
        # the whole FP64 solve of the same system to the same 1e-8 true residual, single-threaded
        log(f"CPU oracle: FP64 CG on {dims} to {tol} (one core)")
        t0 = time.perf_counter()
        _, status, it_cpu, res_cpu = oracle.cg_solve(dims, c["links"], mass, bh, tol=tol)
        t_cpu = time.perf_counter() - t0
        # cross-check: 40 iterations, scaled per iteration
        n_it = 40
        t0 = time.perf_counter()
        oracle.cg_solve(dims, c["links"], mass, bh, tol=1e-30, max_iter=n_it)
        t_cpu40 = time.perf_counter() - t0
        t0 = time.perf_counter()
        oracle.dslash_eo(dims, c["links"], bh, 1)
        t_cpu_d = time.perf_counter() - t0
        cpu = {"value": t_cpu, "unit": "s", "cores": 1, "kind": "oracle",
               "sample": f"the whole single-threaded FP64 oracle CG solve of the same {dims[0]}^3x{dims[3]} system from "
                         f"x = 0 to a true relative residual of {tol} ({it_cpu} iterations, residual {res_cpu:.3e}, "
                         f"status {status}); host {cpu_model()}, {os.cpu_count()} logical CPUs, one used",
               "iters": it_cpu, "true_rel_resid": res_cpu, "status": status, "host": cpu_model(),
               "host_logical_cpus": os.cpu_count(),
               "per_iteration_s": t_cpu / max(it_cpu + 2, 1),
               "per_iteration_s_40_iteration_sample": t_cpu40 / (n_it + 2),
               "dslash_s": t_cpu_d, "dslash_gflops": FLOP_PER_SITE * lat.Vh / t_cpu_d / 1e9,
               "gpu_speedup_mixed": t_cpu / t_mixed}
        log(f"CPU oracle: {t_cpu:.1f} s, {it_cpu} iterations, residual {res_cpu:.2e}")

    ibps = iteration_bytes_per_site(args.inner, args.recon, args.links)
    t_it = t_mixed / max(st.iters, 1)
    line = {
        "metric": METRIC,
        "value": t_mixed,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_mixed * 1e3,
        "value_stderr": t_mixed_se,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.inner,
        "data": "synthetic",
        "config": {"workload": f"even-odd mixed-precision staggered CG, {dims[0]}^3x{dims[3]}, near-identity "
                               f"SU(3) links eps=0.3, m={mass}, Gaussian source, tol={tol}",
                   "dims": list(dims), "mass": mass, "tol": tol, "inner": args.inner, "recon": args.recon,
                   "links": args.links or args.inner,
                   "reliable_update": ("FP64 true residual every 75 iterations or on |r| < 0.1 |r_ru|"
                                       if args.links == "i16" else
                                       "FP64 true residual every 100 iterations or on |r| < 0.1 |r_ru|"),
                   "parallelism": "single GPU"},
        "iters": st.iters,
        "reliable_updates": st.reliable_updates,
        "true_rel_resid": st.true_rel_resid,
        "solve_s_min": min(per) if per else None,
        "cg_gflops": CG_FLOP_PER_SITE * lat.V * st.iters / t_mixed / 1e9,
        "dslash": {"prec": args.inner, "recon": args.recon, "us": t_df * 1e6, "gflops": gflops,
                   "bytes_per_site": bps, "hbm_frac": achieved / HBM_PEAK_GBS, "f64_us": t_d64 * 1e6,
                   "f64_gflops": FLOP_PER_SITE * lat.Vh / t_d64 / 1e9, **dslash_extra},
        "iteration": {"bytes_per_site": ibps, "us": t_it * 1e6, "achieved_GBs": ibps * lat.Vh / t_it / 1e9,
                      "hbm_frac": ibps * lat.Vh / t_it / 1e9 / HBM_PEAK_GBS,
                      "note": "whole solve time / iterations (reliable updates, set-up and polling included)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"half-Dslash {args.inner} vectors, {lprec} recon-{args.recon} links, {dims[0]}^3x{dims[3]}, "
                               f"{lat.Vh} output sites, "
                               f"{bps} algorithmic B/site",
                     "measured": "each launch after an Infinity Cache flush, net of the flush (HIP events, differencing)",
                     "link_loads": best_pol,
                     "solver_link_loads": solver_pol,
                     "solver_config_flushed_frac": policies[solver_pol]["flushed_hbm_frac"],
                     "warm_frac": alg_bytes / t_d / 1e9 / HBM_PEAK_GBS,
                     "control_32x32x32x64_flushed_frac": control["flushed_hbm_frac"] if control else None,
                     "attainable_read_GBs": probe["read"]["GBs"],
                     "attainable_cold_read_same_bytes_GBs": probe["read_cold_small"]["GBs"],
                     "attainable_copy_GBs": probe["copy"]["GBs"],
                     "frac_of_attainable_read": achieved / probe["read"]["GBs"],
                     "frac_of_attainable_copy": achieved / probe["copy"]["GBs"],
                     "frac_of_attainable_cold_read_same_bytes": achieved / probe["read_cold_small"]["GBs"]},
        "stream_probe": probe,
        "cpu_baseline": cpu,
    }
    line.update(extra)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
