"""GPU parity of the even-odd CG solvers (sp_cg_solve through the C-ABI) against the FP64 oracle.

The solution of A x = b is unique (A is Hermitian positive definite), so the GPU result is compared with
the oracle's CG solution driven to 1e-12: within 1e-6 relative for a 1e-8 residual. The true residual
is recomputed by the oracle's operator on the GPU solution.
"""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1511_00088_amd as sp
from conftest import rel_err_2
from gpu_common import announce, cfg1_golden, gauge, to_dev, to_host

pytestmark = pytest.mark.gpu


def _true_resid(dims, U, m, b, x, bc_t=0):
    r = b - oracle.apply_A(dims, U, m, x, bc_t=bc_t)
    return np.linalg.norm(r) / np.linalg.norm(b)


@pytest.mark.parametrize("use_graph", [0, 1])
def test_cfg0_fp64(use_graph):
    c = li.cfg0()
    dims, U, m, b = c["dims"], c["links"], c["mass"], c["source"]
    announce(f"cfg0 fp64 graph={use_graph}")
    G = gauge(dims, U, "f64")
    x, st = sp.cg_solve(G, m, to_dev(b), tol=1e-10, inner="f64", use_graph=bool(use_graph))
    x = to_host(x)
    xr, s0, _, _ = oracle.cg_solve(dims, U, m, b, tol=1e-12)
    announce(f"  iters={st.iters} resid={st.true_rel_resid:.3e} err={rel_err_2(x, xr):.3e}")
    assert st.converged and st.status == 0 and st.true_rel_resid <= 1e-10
    assert _true_resid(dims, U, m, b, x) <= 1.01e-10
    assert rel_err_2(x, xr) <= 1e-8


# the last two have a direction of extent 2, where both hops of that direction reach the same neighbour
# (with the antiperiodic sign applied from each side in t), and (2, 4, 6, 8) has one site per checkerboard row
SMALL = [((8, 8, 8, 8), 0), ((6, 8, 4, 12), 1), ((2, 4, 6, 8), 1), ((4, 4, 2, 2), 1)]


@pytest.mark.parametrize("inner,recon", [("f64", 18), ("f32", 18), ("f32", 12), ("f32", 8), ("f16", 18), ("f16", 12),
                                         ("bf16", 18), ("bf16", 12)])
@pytest.mark.parametrize("dims,bc_t", SMALL)
def test_mixed_precision_small(inner, recon, dims, bc_t):
    announce(f"cg {inner} r{recon} dims={dims} bc_t={bc_t}")
    U = li.near_identity_links(dims, 0.3, 201)
    b = li.gaussian_even_source(dims, 202)
    m = 0.02
    G = gauge(dims, U, inner, recon, bc_t)
    x, st = sp.cg_solve(G, m, to_dev(b), tol=1e-8, inner=inner)
    x = to_host(x)
    xr, s0, it0, _ = oracle.cg_solve(dims, U, m, b, tol=1e-12, bc_t=bc_t)
    err = rel_err_2(x, xr)
    res = _true_resid(dims, U, m, b, x, bc_t)
    announce(f"  iters={st.iters} (oracle {it0}) ru={st.reliable_updates} resid={st.true_rel_resid:.3e} "
             f"oracle-resid={res:.3e} err={err:.3e}")
    assert st.converged and st.status == 0
    assert st.true_rel_resid <= 1e-8 and res <= 1.01e-8
    assert err <= 1e-6


def test_graph_and_eager_bitwise_equal():
    dims = (8, 8, 8, 8)
    U = li.near_identity_links(dims, 0.3, 203)
    b = to_dev(li.gaussian_even_source(dims, 204))
    G = gauge(dims, U, "f32")
    x1, s1 = sp.cg_solve(G, 0.05, b, tol=1e-8, inner="f32", use_graph=True)
    x2, s2 = sp.cg_solve(G, 0.05, b, tol=1e-8, inner="f32", use_graph=False)
    x3, s3 = sp.cg_solve(G, 0.05, b, tol=1e-8, inner="f32", use_graph=True)
    assert s1.iters == s2.iters == s3.iters
    assert torch.equal(x1, x2) and torch.equal(x1, x3)


def test_tail_chunks_graph_and_eager_bitwise_equal():
    """A single solve of 2^16 even sites takes 100-iteration chunks, and 25-iteration ones once the host
    expects convergence within the chunk in flight and the next: graph replay and eager launches take the same
    chunk lengths and agree bit for bit, and the solve matches the one with 25-iteration chunks throughout."""
    dims = (16, 16, 16, 32)
    U = li.near_identity_links(dims, 0.3, 207)
    b = to_dev(li.gaussian_even_source(dims, 208))
    G = gauge(dims, U, "f32", 12)
    x1, s1 = sp.cg_solve(G, 0.05, b, tol=1e-10, inner="f32", use_graph=True)
    x2, s2 = sp.cg_solve(G, 0.05, b, tol=1e-10, inner="f32", use_graph=False)
    x3, s3 = sp.cg_solve(G, 0.05, b, tol=1e-10, inner="f32", poll_chunk=25)
    announce(f"tail chunks: iters {s1.iters} / {s2.iters} (25 throughout: {s3.iters}), ru {s1.reliable_updates}")
    assert s1.converged and s1.iters == s2.iters and torch.equal(x1, x2)
    assert s3.converged and rel_err_2(to_host(x1), to_host(x3)) <= 1e-6


def test_graph_cache_trimmed_between_solves():
    """More distinct solve set-ups than the graph cache holds (each workspace at its own address makes its graphs
    distinct): the cache is emptied before a solve takes its graphs, never between the graphs of one solve, and
    every solve still equals the eager one bit for bit."""
    dims = (4, 4, 4, 8)
    U = li.near_identity_links(dims, 0.3, 209)
    b = to_dev(li.gaussian_even_source(dims, 210))
    G = gauge(dims, U, "f32", 12)
    xr, sr = sp.cg_solve(G, 0.1, b, tol=1e-8, inner="f32", use_graph=False, workspace=sp.Workspace())
    keep = []
    for k in range(45):
        ws = sp.Workspace()
        keep.append(ws)
        x, st = sp.cg_solve(G, 0.1, b, tol=1e-8, inner="f32", workspace=ws)
        assert st.converged and st.iters == sr.iters and torch.equal(x, xr), k
    announce(f"graph cache: 45 set-ups, {sr.iters} iterations each")


def test_warm_start():
    dims = (8, 8, 8, 8)
    U = li.near_identity_links(dims, 0.3, 205)
    b = li.gaussian_even_source(dims, 206)
    G = gauge(dims, U, "f32")
    x1, s1 = sp.cg_solve(G, 0.05, to_dev(b), tol=1e-4, inner="f32")
    x2, s2 = sp.cg_solve(G, 0.05, to_dev(b), tol=1e-10, inner="f32", x0=x1)
    xr, _, _, _ = oracle.cg_solve(dims, U, 0.05, b, tol=1e-12)
    assert s1.converged and s2.converged
    assert rel_err_2(to_host(x2), xr) <= 1e-8
    # a start that already meets the tolerance stops at the first residual check and is returned unchanged
    x3, s3 = sp.cg_solve(G, 0.05, to_dev(b), tol=1e-8, inner="f32", x0=x2)
    assert s3.converged and s3.iters == 0 and bool((x3 == x2).all())


def test_not_converged_and_breakdown():
    dims = (4, 4, 4, 4)
    U = li.haar_links(dims, 207)
    b = li.gaussian_even_source(dims, 208)
    G = gauge(dims, U, "f32")
    x, st = sp.cg_solve(G, 0.01, to_dev(b), tol=1e-10, inner="f32", max_iter=3)
    assert st.status == 1 and not st.converged and st.iters == 3
    # the autograd glue asks for this, so that an unconverged solve never yields a gradient silently
    with pytest.raises(sp.StagError) as e:
        sp.cg_solve(G, 0.01, to_dev(b), tol=1e-10, inner="f32", max_iter=3, raise_on_not_converged=True)
    assert e.value.code == 1
    bn = b.copy()
    bn[3, 1] = np.nan
    with pytest.raises(sp.StagError) as e:
        sp.cg_solve(G, 0.01, to_dev(bn), tol=1e-10, inner="f32")
    assert e.value.code == -6


def test_zero_source():
    dims = (4, 4, 4, 4)
    G = gauge(dims, li.haar_links(dims, 209), "f32")
    x, st = sp.cg_solve(G, 0.1, torch.zeros((128, 3), dtype=torch.complex128, device="cuda:0"), tol=1e-8)
    assert st.converged and st.iters == 0 and float(x.abs().max()) == 0.0


def test_solves_from_two_host_threads_match_sequential():
    """Two host threads, each with its own torch stream and workspace, solve different systems three times
    at once (ctypes releases the interpreter lock, so the calls overlap on the host). The library serialises
    the solves, and every result equals the same solve run alone, bit for bit."""
    import threading

    dims = (8, 8, 8, 8)
    U = li.near_identity_links(dims, 0.3, 410)
    G = gauge(dims, U, "f32", 12)
    bs = [to_dev(li.gaussian_even_source(dims, 411 + i)) for i in range(2)]
    ms = [0.02, 0.05]
    ref = [sp.cg_solve(G, m, b, tol=1e-9, inner="f32")[0] for m, b in zip(ms, bs)]
    torch.cuda.synchronize()
    out, err = [[], []], []

    def run(i):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                ws = sp.Workspace()
                for _ in range(3):
                    out[i].append(sp.cg_solve(G, ms[i], bs[i], tol=1e-9, inner="f32", workspace=ws))
            s.synchronize()
        except Exception as e:  # reported below, in the main thread
            err.append(e)

    th = [threading.Thread(target=run, args=(i,)) for i in range(2)]
    for t in th:
        t.start()
    for t in th:
        t.join(timeout=120)
    assert not err and not any(t.is_alive() for t in th), err
    for i in range(2):
        assert len(out[i]) == 3
        for x, st in out[i]:
            assert st.converged and bool((x == ref[i]).all())


def test_out_buffer_checked():
    """A caller's output buffer of the wrong shape is refused before the solve writes through its pointer; one
    of the right shape receives the solution and is returned."""
    dims = (4, 4, 4, 4)
    G = gauge(dims, li.haar_links(dims, 420), "f32")
    b = to_dev(li.gaussian_even_source(dims, 421))
    with pytest.raises(ValueError):
        sp.cg_solve(G, 0.1, b, tol=1e-8, out=torch.empty((10, 3), dtype=torch.complex128, device="cuda:0"))
    out = torch.empty_like(b)
    x, st = sp.cg_solve(G, 0.1, b, tol=1e-8, out=out)
    assert x is out and st.converged


def test_light_mass_limits_of_16bit_storage():
    """m = 1e-3 on 8^4 (condition number ~1.6e7): FP32 iterations with FP64 reliable updates still reach the FP64
    solve's answer. 16-bit storage stalls in this regime; whatever it does, its report is truthful: converged
    and status agree with the true residual of the solution it returns, recomputed by the oracle, and the
    reported residual is that one."""
    dims = (8, 8, 8, 8)
    U = li.near_identity_links(dims, 0.3, 231)
    b = li.gaussian_even_source(dims, 232)
    m = 1e-3
    x64, s64 = sp.cg_solve(gauge(dims, U, "f64"), m, to_dev(b), tol=1e-8, inner="f64")
    x32, s32 = sp.cg_solve(gauge(dims, U, "f32", 12), m, to_dev(b), tol=1e-8, inner="f32")
    announce(f"m=1e-3: FP64 {s64.iters} iterations, FP32 {s32.iters} ({s32.reliable_updates} updates)")
    assert s64.converged and s32.converged
    assert rel_err_2(to_host(x32), to_host(x64)) <= 1e-6
    for inner in ("f16", "bf16"):
        x, st = sp.cg_solve(gauge(dims, U, inner, 12), m, to_dev(b), tol=1e-8, inner=inner, max_iter=20000)
        res = _true_resid(dims, U, m, b, to_host(x))
        announce(f"  {inner}: iters={st.iters} status={st.status} reported {st.true_rel_resid:.3e} oracle {res:.3e}")
        assert abs(res - st.true_rel_resid) <= 1e-6 * res
        if st.converged:
            assert st.status == 0 and res <= 1.01e-8
        else:
            assert st.status == 1 and res > 1e-8


_CFG1 = {}


def _cfg1():
    if not _CFG1:
        _CFG1.update(li.cfg1())
    return _CFG1


@pytest.mark.parametrize("inner,recon", [("f32", 18), ("f64", 18), ("f32", 12), ("f32", 8), ("f16", 18), ("bf16", 18),
                                         ("f16", 12), ("bf16", 12)])
def test_cfg1_full_size_vs_oracle_samples(inner, recon):
    """20^3x64, m = 0.01, to 1e-8 with the tuned launch the benchmark uses: the solution at the sampled sites
    against the oracle's 1e-12 solution (golden file written by the oracle alone), and the true residual of
    the whole GPU solution recomputed by the oracle's operator."""
    import os

    c = _cfg1()
    dims, U, m, b = c["dims"], c["links"], c["mass"], c["source"]
    sp.tune_load(os.path.join(os.path.dirname(os.path.dirname(__file__)), "paper_1511_00088_amd",
                              "tune_mi355x.json"))
    announce(f"cfg1 full size {inner} r{recon}")
    G = gauge(dims, U, inner, recon)
    x, st = sp.cg_solve(G, m, to_dev(b), tol=1e-8, inner=inner)
    x = to_host(x)
    cbs, ref = cfg1_golden()
    err = np.linalg.norm(x[cbs] - ref) / np.linalg.norm(ref)
    res = _true_resid(dims, U, m, b, x)
    announce(f"  iters={st.iters} ru={st.reliable_updates} resid={st.true_rel_resid:.3e} oracle-resid={res:.3e} "
             f"sampled err={err:.3e}")
    assert st.converged and st.true_rel_resid <= 1e-8
    assert res <= 1.01e-8
    assert err <= 1e-6


@pytest.mark.parametrize("dims,bc_t,inner,links", [((4, 4, 4, 4), 0, "f64", "haar"), ((8, 6, 4, 10), 1, "f32", "near"),
                                                   ((8, 8, 8, 8), 0, "f16", "near"), ((6, 4, 4, 8), 0, "bf16", "haar")])
def test_full_system_solve(dims, bc_t, inner, links):
    """(m + D) psi = src on the whole lattice: source preparation, even solve and odd reconstruction on the
    GPU against the oracle's full solve (pinned by dense solves), plus the full residual via the oracle's D."""
    announce(f"full solve dims={dims} bc_t={bc_t} {inner}")
    V = li.volume(dims)
    U = li.haar_links(dims, 501) if links == "haar" else li.near_identity_links(dims, 0.3, 501)
    src = li.gaussian_vector(V, 502)
    m = 0.1
    G = gauge(dims, U, inner, 18, bc_t)
    psi, st = sp.full_solve(G, m, to_dev(src), tol=1e-10, inner=inner)
    psi = to_host(psi)
    ref, s0, _ = oracle.full_solve(dims, U, m, src, tol=1e-12, bc_t=bc_t)
    res = np.linalg.norm(src - m * psi - oracle.dslash(dims, U, psi, bc_t=bc_t)) / np.linalg.norm(src)
    err = rel_err_2(psi, ref)
    announce(f"  iters={st.iters} err={err:.3e} full residual={res:.3e}")
    assert st.converged and s0 == 0
    assert err <= 1e-8
    assert res <= 1e-9


def test_full_system_solve_workload_size():
    """(m + D) psi = src on 20^3x64 (m = 0.01) with the benchmark's FP32 recon-12 launch, checked through the FP64
    half operator entry point: the odd half satisfies its rows to rounding (psi_o = (src_o - D_oe psi_e) / m),
    and the even rows' residual is the even solve's, (b_e - A psi_e) / m with b_e = m src_e - D_eo src_o, so
    its norm is the reported relative residual times |b_e| / m and at most tol |b_e| / m."""
    c = _cfg1()
    dims, m = c["dims"], c["mass"]
    lat = sp.Lattice(dims)
    G = sp.Gauge(lat, to_dev(c["links"]), lo_prec="f32", recon=12)
    src = li.gaussian_vector(lat.V, 510)
    announce(f"full solve at the workload size {dims}")
    psi, st = sp.full_solve(G, m, to_dev(src), tol=1e-8, inner="f32")
    X, Y, Z, _ = dims
    lex = np.arange(lat.V)
    par = (lex % X + (lex // X) % Y + (lex // (X * Y)) % Z + lex // (X * Y * Z)) & 1
    idx = [np.empty(lat.Vh, dtype=np.int64) for _ in range(2)]
    for q in (0, 1):
        idx[q][lex[par == q] >> 1] = lex[par == q]
    ph = to_host(psi)
    se, so, pe, po = (to_dev(a) for a in (src[idx[0]], src[idx[1]], ph[idx[0]], ph[idx[1]]))
    r_o = so - m * po - sp.dslash(G, pe, 1, "f64")
    r_e = se - m * pe - sp.dslash(G, po, 0, "f64")
    b_e = m * se - sp.dslash(G, so, 0, "f64")
    nb = torch.linalg.norm(b_e).item()
    ro = (torch.linalg.norm(r_o) / torch.linalg.norm(so)).item()
    re = torch.linalg.norm(r_e).item() * m / nb
    announce(f"  iters={st.iters} even residual {re:.3e} (reported {st.true_rel_resid:.3e}), odd rows {ro:.1e}")
    assert st.converged
    assert ro <= 1e-12
    assert re <= 1.01e-8 and abs(re - st.true_rel_resid) <= 1e-3 * re


def test_full_system_solve_rejects_zero_mass():
    dims = (4, 4, 4, 4)
    G = gauge(dims, li.haar_links(dims, 503), "f32")
    with pytest.raises(sp.StagError) as e:
        sp.full_solve(G, 0.0, to_dev(li.gaussian_vector(256, 504)))
    assert e.value.code == -1


@pytest.mark.parametrize("inner,recon", [("f32", 12), ("f32", 8), ("f16", 12)])
def test_control_lattice_true_residual_through_the_operator(inner, recon):
    """32^3x64 (beyond the Infinity Cache; 4,096 blocks, whose fused launches sum 16 block partials per thread
    before the operator), solved to 1e-8; the true residual |b - A x| / |b| is recomputed with the FP64 half
    operator entry point, independently of the solver's own reliable-update residual."""
    dims = (32, 32, 32, 64)
    announce(f"control lattice {dims} {inner} r{recon}")
    lat = sp.Lattice(dims)
    links, b = _gpu_links_and_source(lat, 71)
    _solve_and_check_operator_residual(lat, links, b, inner, recon)


@pytest.mark.parametrize("dims", [(32, 32, 16, 32), (32, 32, 16, 34)])
def test_partial_sums_either_side_of_the_early_load_limit(dims):
    """The fused launches load a thread's block partials before the operator's gathers when there are at most
    four per thread (1,024 blocks of 256 threads: 32x32x16x32) and sum them all first beyond that (1,088 blocks:
    32x32x16x34). Both solve to 1e-8 with the residual recomputed by the FP64 operator, and graph replay equals
    eager launches bit for bit."""
    lat = sp.Lattice(dims)
    announce(f"partial-sum paths {dims}: {lat.Vh // 256} blocks")
    links, b = _gpu_links_and_source(lat, 73)
    G = _solve_and_check_operator_residual(lat, links, b, "f32", 12)
    x1, s1 = sp.cg_solve(G, 0.01, b, tol=1e-8, inner="f32", use_graph=True)
    x2, s2 = sp.cg_solve(G, 0.01, b, tol=1e-8, inner="f32", use_graph=False)
    assert s1.iters == s2.iters and torch.equal(x1, x2)


def _gpu_links_and_source(lat, seed):
    """Near-identity links exp(i 0.3 H) and a Gaussian even source drawn on the GPU (seeded torch generator):
    these lattices are too large for the host generator to be quick."""
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(seed)
    V = lat.V
    lam = torch.from_numpy((li.gell_mann() / 2.0).reshape(8, 9)).to("cuda:0")
    links = torch.empty(4, V, 3, 3, dtype=torch.complex128, device="cuda:0")
    for mu in range(4):
        h = torch.randn(V, 8, generator=gen, device="cuda:0", dtype=torch.float64).to(torch.complex128)
        links[mu] = torch.linalg.matrix_exp((0.3j) * (h @ lam).reshape(V, 3, 3))
    b = torch.randn(lat.Vh, 3, dtype=torch.complex128, device="cuda:0", generator=gen)
    return links, b


def _solve_and_check_operator_residual(lat, links, b, inner, recon, m=0.01):
    G = sp.Gauge(lat, links, lo_prec=inner, recon=recon)
    x, st = sp.cg_solve(G, m, b, tol=1e-8, inner=inner)
    assert st.converged, st
    t = sp.dslash(G, x, 1, "f64")       # D_oe x
    Ax = m * m * x - sp.dslash(G, t, 0, "f64")  # m^2 x - D_eo D_oe x
    res = (torch.linalg.norm(b - Ax) / torch.linalg.norm(b)).item()
    announce(f"  iters={st.iters} ru={st.reliable_updates} solver resid={st.true_rel_resid:.3e} operator resid={res:.3e}")
    assert res <= 1.01e-8 and abs(res - st.true_rel_resid) <= 1e-3 * res
    return G


def test_production_lattice_28x28x28x96():
    """The paper's other production lattice (28^3x96, Sec. 4): the FP32 recon-12 half operator at sampled sites
    against the oracle, then a mixed solve whose true residual is recomputed with the FP64 operator."""
    dims = (28, 28, 28, 96)
    announce(f"production lattice {dims}")
    lat = sp.Lattice(dims)
    links, b = _gpu_links_and_source(lat, 72)
    G = _solve_and_check_operator_residual(lat, links, b, "f32", 12)
    U = to_host(links)
    xin = li.gaussian_vector(lat.Vh, 106)
    rng = np.random.default_rng(107)
    cbs = np.unique(np.concatenate([rng.integers(0, lat.Vh, 2000), np.arange(lat.Vh - 200, lat.Vh),
                                    np.arange(0, 200)]))
    for p in (0, 1):
        y = to_host(sp.dslash(G, to_dev(xin), p, "f32"))[cbs]
        ref = oracle.dslash_eo_sites(dims, U, xin, p, cbs)
        err = float(np.max(np.abs(y - ref)) / np.max(np.abs(ref)))
        announce(f"  parity {p}: sampled max rel err {err:.3e}")
        assert err <= 1e-6


@pytest.mark.parametrize("inner,recon", [("f32", 12), ("f64", 18), ("f16", 12)])
def test_schedules_reach_the_same_solution(inner, recon):
    # chunk length 1 never uses the t recurrence (every chunk starts from t = D_oe p), odd lengths end with a
    # state copy, and a short ru_every or a large delta put reliable updates at many positions; every
    # schedule must reach the oracle's solution, and the recurrence must not cost iterations
    dims = (8, 8, 8, 8)
    U = li.near_identity_links(dims, 0.3, 203)
    b = li.gaussian_even_source(dims, 204)
    m = 0.02
    G = gauge(dims, U, inner, recon)
    xr, _, _, _ = oracle.cg_solve(dims, U, m, b, tol=1e-12)
    iters = {}
    for chunk, every, delta in ((1, 0, 0.1), (7, 0, 0.1), (25, 0, 0.1), (64, 0, 0.1), (7, 10, 0.5), (25, 0, 0.0)):
        announce(f"cg {inner} r{recon} chunk={chunk} ru_every={every} delta={delta}")
        x, st = sp.cg_solve(G, m, to_dev(b), tol=1e-8, inner=inner, poll_chunk=chunk, ru_every=every,
                            delta=delta)
        x = to_host(x)
        err = rel_err_2(x, xr)
        announce(f"  iters={st.iters} ru={st.reliable_updates} resid={st.true_rel_resid:.3e} err={err:.3e}")
        assert st.converged and st.status == 0 and st.true_rel_resid <= 1e-8
        assert _true_resid(dims, U, m, b, x) <= 1.01e-8
        assert err <= 1e-6
        if inner == "f64":
            # plain FP64 CG: the true residual is recomputed only when the iterated one reaches tol
            assert st.reliable_updates <= 2
        iters[(chunk, every, delta)] = st.iters
    if inner != "f16":
        # the same reliable-update positions (delta and ru_every checked at chunk ends of length 1 vs 25 differ,
        # so compare the recurrence-free schedule with the default one loosely)
        assert iters[(25, 0, 0.1)] <= 1.05 * iters[(1, 0, 0.1)] + 2


@pytest.mark.parametrize("inner,recon", [("f64", 18), ("f32", 12), ("f16", 12), ("bf16", 12)])
def test_solution_scales_with_the_source(inner, recon):
    # A x = b is linear: sources scaled by 1e-30 and 1e30 must give the scaled solution. At 1e-30 the last
    # residuals reach the bottom of the FP32 range (~1e-38), where the FP16 site norm must not overflow
    # its reciprocal
    dims = (8, 8, 8, 8)
    U = li.near_identity_links(dims, 0.3, 211)
    b = to_dev(li.gaussian_even_source(dims, 212))
    G = gauge(dims, U, inner, recon)
    x1, st1 = sp.cg_solve(G, 0.02, b, tol=1e-8, inner=inner)
    assert st1.converged
    for s in (1e-30, 1e30):
        announce(f"cg {inner} r{recon} source scale {s:g}")
        xs, st = sp.cg_solve(G, 0.02, b * s, tol=1e-8, inner=inner, raise_on_not_converged=True)
        diff = (torch.linalg.norm(xs / s - x1) / torch.linalg.norm(x1)).item()
        announce(f"  iters={st.iters} (unscaled {st1.iters}) resid={st.true_rel_resid:.2e} diff={diff:.2e}")
        assert st.converged and st.true_rel_resid <= 1e-8
        assert diff <= 1e-6


@pytest.mark.parametrize("inner", ["f32", "f16", "bf16"])
def test_fast_converging_systems(inner):
    # heavy masses (up to m = 30, where A is 900 + [0, 16]) and a 2^4 lattice converge by many decades within
    # one 25-iteration chunk; the recursive residual must not be left to run far below the true one until the
    # chunk end (that once cost ~800 iterations at m = 1 and lost convergence with delta = 0): every case
    # converges to the oracle's solution in a bounded number of iterations, with and without the delta trigger
    for dims, kind, m, cap in (((8, 8, 8, 8), "near", 30.0, 40), ((8, 8, 8, 8), "near", 1.0, 60),
                               ((8, 8, 8, 8), "near", 0.3, 120),
                               ((2, 2, 2, 2), "haar", 0.1, 250), ((2, 2, 2, 2), "near", 0.1, 200)):
        U = li.haar_links(dims, 221) if kind == "haar" else li.near_identity_links(dims, 0.3, 221)
        b = li.gaussian_even_source(dims, 222)
        xr, _, _, _ = oracle.cg_solve(dims, U, m, b, tol=1e-12)
        G = gauge(dims, U, inner, 12)
        for delta in (0.1, 0.0):
            announce(f"cg {inner} {dims} {kind} m={m} delta={delta}")
            x, st = sp.cg_solve(G, m, to_dev(b), tol=1e-8, inner=inner, delta=delta, max_iter=3000)
            err = rel_err_2(to_host(x), xr)
            announce(f"  iters={st.iters} ru={st.reliable_updates} err={err:.2e}")
            assert st.converged and st.iters <= cap and err <= 1e-6
