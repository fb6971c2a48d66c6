"""GPU parity of sp_cg_solve_batched: systems grouped by gauge field share each link load, groups of
different volumes advance in the same launches, converged systems stop while the others continue.
Every system is compared with the oracle's solution and with the same system solved alone."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1511_00088_amd as sp
from conftest import rel_err_2
from gpu_common import announce, cfg1_golden, gauge, to_dev, to_host, tune_file

pytestmark = pytest.mark.gpu


def _batch(inner, recon=18):
    specs = [((8, 8, 8, 8), 301, [0.02, 0.05, 0.1]), ((6, 8, 4, 12), 302, [0.03, 0.08]), ((4, 4, 4, 4), 303, [0.1])]
    systems, host = [], []
    k = 0
    for dims, seed, masses in specs:
        U = li.near_identity_links(dims, 0.3, seed)
        G = gauge(dims, U, inner, recon)
        for m in masses:
            b = li.gaussian_even_source(dims, 310 + k)
            k += 1
            systems.append((G, m, to_dev(b)))
            host.append((dims, U, m, b))
    return systems, host


@pytest.mark.parametrize("inner,recon", [("f32", 18), ("f32", 12), ("f32", 8), ("f16", 18), ("bf16", 12), ("f64", 18)])
def test_batched_matches_oracle_and_single(inner, recon):
    announce(f"batched {inner} r{recon}")
    systems, host = _batch(inner, recon)
    xs, stats = sp.cg_solve_batched(systems, tol=1e-8, inner=inner)
    for i, ((G, m, b), (dims, U, _, bh), x, st) in enumerate(zip(systems, host, xs, stats)):
        xr, _, it0, _ = oracle.cg_solve(dims, U, m, bh, tol=1e-12)
        xs1, st1 = sp.cg_solve(G, m, b, tol=1e-8, inner=inner)
        err = rel_err_2(to_host(x), xr)
        announce(f"  sys {i} dims={dims} m={m}: iters={st.iters} (alone {st1.iters}, oracle {it0}) "
                 f"resid={st.true_rel_resid:.2e} err={err:.2e}")
        assert st.converged and st.true_rel_resid <= 1e-8
        assert err <= 1e-6
        assert rel_err_2(to_host(x), to_host(xs1)) <= 1e-6


def test_batched_more_than_eight_per_gauge():
    dims = (4, 4, 4, 8)
    U = li.near_identity_links(dims, 0.3, 320)
    G = gauge(dims, U, "f32")
    rng = np.random.default_rng(321)
    masses = rng.uniform(0.01, 0.1, 11)
    bs = [li.gaussian_even_source(dims, 330 + i) for i in range(11)]
    xs, stats = sp.cg_solve_batched([(G, m, to_dev(b)) for m, b in zip(masses, bs)], tol=1e-9, inner="f32")
    for m, b, x, st in zip(masses, bs, xs, stats):
        xr, _, _, _ = oracle.cg_solve(dims, U, m, b, tol=1e-12)
        assert st.converged and rel_err_2(to_host(x), xr) <= 1e-7


@pytest.mark.parametrize("inner,recon", [("f32", 12), ("f16", 18), ("bf16", 12), ("f64", 18)])
def test_batched_masses_two_decades_apart(inner, recon):
    """One gauge group whose masses span 0.01 to 2: the heavy systems converge in about a dozen
    iterations, their recursive residual falls decades below the last true one long before the
    light systems are done, and each must still end at the oracle's solution while the group keeps
    stepping the others."""
    announce(f"batched masses two decades apart {inner} r{recon}")
    dims = (8, 8, 8, 8)
    U = li.near_identity_links(dims, 0.3, 231)
    G = gauge(dims, U, inner, recon)
    masses = [1.0, 0.01, 0.5, 0.05, 2.0, 0.02]
    bs = [li.gaussian_even_source(dims, 240 + i) for i in range(len(masses))]
    xs, stats = sp.cg_solve_batched([(G, m, to_dev(b)) for m, b in zip(masses, bs)], tol=1e-8, inner=inner)
    for m, b, x, st in zip(masses, bs, xs, stats):
        xr, _, it0, _ = oracle.cg_solve(dims, U, m, b, tol=1e-12)
        err = rel_err_2(to_host(x), xr)
        announce(f"  m={m}: iters={st.iters} (oracle to 1e-12: {it0}) resid={st.true_rel_resid:.2e} err={err:.2e}")
        assert st.converged and st.true_rel_resid <= 1e-8
        assert err <= 1e-6


@pytest.mark.parametrize("inner,recon", [("f32", 12), ("f16", 18), ("bf16", 12), ("f64", 18)])
def test_batched_antiperiodic_groups_beside_periodic(inner, recon):
    """Groups whose time boundary differs in the same launches: one link field on 6x8x4x12 packed with
    antiperiodic and with periodic time, an antiperiodic 4^4 field and an antiperiodic 2x4x6x2 field (extent 2
    in x and t). Every system against the oracle's
    solution with its own boundary condition, and its true residual recomputed by the oracle."""
    announce(f"batched antiperiodic and periodic groups {inner} r{recon}")
    specs = [((6, 8, 4, 12), 1, 350, [0.03, 0.08]), ((6, 8, 4, 12), 0, 350, [0.05]), ((4, 4, 4, 4), 1, 351, [0.1, 0.02]),
             ((2, 4, 6, 2), 1, 352, [0.04])]
    systems, host = [], []
    k = 0
    for dims, bc, seed, masses in specs:
        U = li.near_identity_links(dims, 0.3, seed)
        G = gauge(dims, U, inner, recon, bc)
        for m in masses:
            b = li.gaussian_even_source(dims, 360 + k)
            k += 1
            systems.append((G, m, to_dev(b)))
            host.append((dims, bc, U, m, b))
    xs, stats = sp.cg_solve_batched(systems, tol=1e-8, inner=inner)
    for (dims, bc, U, m, b), x, st in zip(host, xs, stats):
        xr, _, it0, _ = oracle.cg_solve(dims, U, m, b, tol=1e-12, bc_t=bc)
        xh = to_host(x)
        err = rel_err_2(xh, xr)
        res = float(np.linalg.norm(b - oracle.apply_A(dims, U, m, xh, bc_t=bc)) / np.linalg.norm(b))
        announce(f"  dims={dims} bc_t={bc} m={m}: iters={st.iters} (oracle {it0}) resid={res:.2e} err={err:.2e}")
        assert st.converged and res <= 1.5e-8
        assert err <= 1e-6


def test_batched_zero_source_beside_others():
    """A zero right-hand side in a group with two others: it stops at the initial residual check with x = 0,
    while the group's other systems run on to the oracle's solution."""
    dims = (8, 4, 4, 8)
    U = li.near_identity_links(dims, 0.3, 370)
    G = gauge(dims, U, "f32", 12)
    b1 = li.gaussian_even_source(dims, 371)
    b3 = li.gaussian_even_source(dims, 372)
    zero = np.zeros_like(b1)
    xs, stats = sp.cg_solve_batched([(G, 0.05, to_dev(b1)), (G, 0.05, to_dev(zero)), (G, 0.02, to_dev(b3))],
                                    tol=1e-9, inner="f32")
    assert stats[1].converged and stats[1].iters == 0 and float(xs[1].abs().max()) == 0.0
    for i, (m, b) in ((0, (0.05, b1)), (2, (0.02, b3))):
        xr, _, _, _ = oracle.cg_solve(dims, U, m, b, tol=1e-12)
        assert stats[i].converged and stats[i].iters > 0
        assert rel_err_2(to_host(xs[i]), xr) <= 1e-7


def test_batched_iteration_cap():
    """max_iter cuts every system of a batch at the same count: each reports not converged (status 1) after
    exactly max_iter iterations, and its reported true residual is that of the x it returns, recomputed by
    the oracle."""
    dims = (4, 4, 4, 8)
    U = li.near_identity_links(dims, 0.3, 380)
    G = gauge(dims, U, "f32", 12)
    bs = [li.gaussian_even_source(dims, 381 + i) for i in range(3)]
    masses = [0.01, 0.02, 0.05]
    xs, stats = sp.cg_solve_batched([(G, m, to_dev(b)) for m, b in zip(masses, bs)], tol=1e-10, inner="f32",
                                    max_iter=7)
    for m, b, x, st in zip(masses, bs, xs, stats):
        res = float(np.linalg.norm(b - oracle.apply_A(dims, U, m, to_host(x))) / np.linalg.norm(b))
        assert st.status == 1 and not st.converged and st.iters == 7
        assert 1e-10 < res < 1.0
        assert abs(res - st.true_rel_resid) <= 1e-6 * res


def test_batched_full_size_workload_vs_oracle_samples():
    """The 20^3x64 workload inside a batch, in the launch configuration the benchmark times (FP32 iterations on
    recon-12 links, the tuned four-right-hand-side operator): the workload's own system (m = 0.01) and three
    more sources and masses on its field form one group, and four systems on a 16^3x32 field run in the same
    launches. The workload's solution at the sampled sites against the oracle's 1e-12 solution (golden file
    written by the oracle alone); every system's true residual recomputed with the FP64 half operator entry
    point, independently of the solver's reliable updates."""
    sp.tune_load(tune_file())
    c = li.cfg1()
    c4 = li.cfg4()
    G1 = gauge(c["dims"], c["links"], "f32", 12)
    G4 = gauge(c4["dims"], c4["links"], "f32", 12)
    systems = [(G1, c["mass"], to_dev(c["source"]))]
    systems += [(G1, m, to_dev(li.gaussian_even_source(c["dims"], 390 + i))) for i, m in enumerate([0.02, 0.05, 0.1])]
    systems += [(G4, m, to_dev(li.gaussian_even_source(c4["dims"], 395 + i))) for i, m in enumerate([0.01, 0.03, 0.05, 0.08])]
    announce("batched full size: 4 systems on 20^3x64 + 4 on 16^3x32, f32 r12")
    xs, stats = sp.cg_solve_batched(systems, tol=1e-8, inner="f32")
    for (G, m, b), x, st in zip(systems, xs, stats):
        t = sp.dslash(G, x, 1, "f64")
        ax = m * m * x - sp.dslash(G, t, 0, "f64")
        res = (torch.linalg.norm(b - ax) / torch.linalg.norm(b)).item()
        announce(f"  {G.lat.dims} m={m}: iters={st.iters} ru={st.reliable_updates} solver resid={st.true_rel_resid:.3e} "
                 f"operator resid={res:.3e}")
        assert st.converged and res <= 1.01e-8 and abs(res - st.true_rel_resid) <= 1e-3 * res
    cbs, ref = cfg1_golden()
    err = np.linalg.norm(to_host(xs[0])[cbs] - ref) / np.linalg.norm(ref)
    announce(f"  workload system: sampled err vs oracle {err:.3e}")
    assert err <= 1e-6


def test_batched_more_than_64_groups():
    """67 systems, each on its own 4^4 gauge field, so 67 groups: a block finds its group with one ballot per
    64 groups, and this crosses into the second one; every system against the oracle."""
    dims = (4, 4, 4, 4)
    systems, host = [], []
    for i in range(67):
        U = li.near_identity_links(dims, 0.3, 500 + i)
        b = li.gaussian_even_source(dims, 600 + i)
        m = 0.05 + 0.001 * i
        systems.append((gauge(dims, U, "f32", 12), m, to_dev(b)))
        host.append((U, m, b))
    xs, stats = sp.cg_solve_batched(systems, tol=1e-9, inner="f32")
    worst = 0.0
    for (U, m, b), x, st in zip(host, xs, stats):
        xr, _, _, _ = oracle.cg_solve(dims, U, m, b, tol=1e-12)
        assert st.converged
        worst = max(worst, rel_err_2(to_host(x), xr))
    announce(f"67 groups: worst error against the oracle {worst:.2e}")
    assert worst <= 1e-7


def test_batched_breakdown_of_one_system_leaves_the_others_solved():
    """A NaN in one source breaks that system down. The call returns SP_ERR_BREAKDOWN, and through the C-ABI
    the per-system statistics name that system while the two others of its group are solved to the oracle's
    answer: reductions and states are per system, so nothing leaks between them."""
    import ctypes

    from paper_1511_00088_amd import _lib as L

    dims = (4, 4, 4, 8)
    U = li.near_identity_links(dims, 0.3, 430)
    G = gauge(dims, U, "f32", 12)
    bs = [li.gaussian_even_source(dims, 431 + i) for i in range(3)]
    bs[1] = bs[1].copy()
    bs[1][5, 2] = np.nan
    ms = [0.05, 0.05, 0.02]
    bd = [to_dev(b) for b in bs]
    xs = [torch.empty_like(b) for b in bd]
    arr = (L.sp_system * 3)()
    for i in range(3):
        arr[i] = L.sp_system(ctypes.pointer(G.lat.geom), ctypes.pointer(G.struct), ms[i], bd[i].data_ptr(),
                             xs[i].data_ptr())
    prm = L.sp_cg_params(1e-9, 100000, L.SP_F32, 0.1, 0, 0, 0, 1)
    lib = L.load()
    nbytes = lib.sp_cg_workspace_bytes(3, arr, ctypes.byref(prm))
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    st = (L.sp_cg_stats * 3)()
    rc = lib.sp_cg_solve_batched(3, arr, ctypes.byref(prm), st, ctypes.c_void_p(ws.data_ptr()),
                                 ctypes.c_size_t(nbytes), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == L.SP_ERR_BREAKDOWN
    assert [st[i].status for i in range(3)] == [0, L.SP_ERR_BREAKDOWN, 0]
    for i in (0, 2):
        xr, _, _, _ = oracle.cg_solve(dims, U, ms[i], bs[i], tol=1e-12)
        assert st[i].converged and rel_err_2(to_host(xs[i]), xr) <= 1e-7
    # the binding: raises by default, returns every system's result on request
    sysl = [(G, m, b) for m, b in zip(ms, bd)]
    with pytest.raises(sp.StagError) as e:
        sp.cg_solve_batched(sysl, tol=1e-9, inner="f32")
    assert e.value.code == L.SP_ERR_BREAKDOWN
    xp, sp_st = sp.cg_solve_batched(sysl, tol=1e-9, inner="f32", raise_on_breakdown=False)
    assert [q.status for q in sp_st] == [0, L.SP_ERR_BREAKDOWN, 0]
    for i in (0, 2):
        assert bool((xp[i] == xs[i]).all())


def test_batched_deterministic():
    systems, _ = _batch("f32")
    xa, sa = sp.cg_solve_batched(systems, tol=1e-8, inner="f32")
    xb, sb = sp.cg_solve_batched(systems, tol=1e-8, inner="f32", use_graph=False)
    for a, b, s1, s2 in zip(xa, xb, sa, sb):
        assert s1.iters == s2.iters
        assert bool((a == b).all())


def test_batched_mixed_packings_rejected():
    dims = (4, 4, 4, 4)
    U = li.haar_links(dims, 340)
    G18 = gauge(dims, U, "f32", 18)
    G12 = gauge(dims, U, "f32", 12)
    b = to_dev(li.gaussian_even_source(dims, 341))
    with pytest.raises(sp.StagError) as e:
        sp.cg_solve_batched([(G18, 0.1, b), (G12, 0.1, b)], tol=1e-8, inner="f32")
    assert e.value.code == -3


def test_batched_workload_32_systems_vs_oracle():
    """The benchmark's batched workload itself (lattice_inputs.uneven_batch: 8 right-hand sides on the 20^3x64
    field at m = 0.01, and 8 systems each on 8^4, 12^3x24 and 16^3x32 with masses in [0.01, 0.1]) in the launch the
    benchmark times (FP32 iterations on recon-12 links, tuned table): every system's true residual recomputed by
    the oracle's FP64 operator, and each of the 24 smaller systems against the oracle's own 1e-12 solve (run in
    threads: each is single-threaded and releases the interpreter)."""
    from concurrent.futures import ThreadPoolExecutor

    sp.tune_load(tune_file())
    gauges, systems = li.uneven_batch()
    G = [gauge(dims, U, "f32", 12) for dims, U in gauges]
    sysl = [(G[s.gauge_index], s.mass, to_dev(s.source)) for s in systems]
    announce(f"batched workload: {len(sysl)} systems, f32 r12")
    xs, stats = sp.cg_solve_batched(sysl, tol=1e-8, inner="f32")
    xh = [to_host(x) for x in xs]

    def check(i):
        s = systems[i]
        dims, U = gauges[s.gauge_index]
        res = _true_resid_oracle(dims, U, s.mass, s.source, xh[i])
        err = None
        if li.volume(dims) < li.volume((20, 20, 20, 64)):
            xr, st0, _, _ = oracle.cg_solve(dims, U, s.mass, s.source, tol=1e-12)
            assert st0 == 0
            err = rel_err_2(xh[i], xr)
        return res, err

    with ThreadPoolExecutor(8) as ex:
        out = list(ex.map(check, range(len(systems))))
    for i, (s, st, (res, err)) in enumerate(zip(systems, stats, out)):
        announce(f"  sys {i} dims={s.dims} m={s.mass:.4f}: iters={st.iters} ru={st.reliable_updates} "
                 f"resid={st.true_rel_resid:.2e} oracle-resid={res:.2e} err={err if err is None else f'{err:.2e}'}")
        assert st.converged and st.status == 0 and st.true_rel_resid <= 1e-8
        assert res <= 1.01e-8
        if err is not None:
            assert err <= 1e-6
    assert sum(e is not None for _, e in out) == 24


def _true_resid_oracle(dims, U, m, b, x):
    r = b - oracle.apply_A(dims, U, m, x)
    return float(np.linalg.norm(r) / np.linalg.norm(b))
