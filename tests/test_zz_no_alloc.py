"""sp_cg_force_noalloc (the gradient with its scratch in the library's fixed device array) against sp_cg_force
(the same kernels with a caller workspace), called through the C-ABI: two calls in a row on one GPU, the second
on a smaller lattice, each output bit for bit equal to sp_cg_force's; the small case also against the oracle."""
import ctypes

import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1511_00088_amd as sp
from conftest import rel_err_2
from gpu_common import DEV, announce, gauge, to_dev, to_host
from paper_1511_00088_amd import _lib

pytestmark = pytest.mark.gpu


def _noalloc(G, m, x, lam, want_force=True, want_mass=True):
    lat = G.lat
    gamma = torch.full((4, lat.V, 3, 3), float("nan"), dtype=torch.complex128, device=DEV)
    force = torch.full_like(gamma, float("nan")) if want_force else None
    dm = torch.full((), float("nan"), dtype=torch.float64, device=DEV) if want_mass else None
    lib = _lib.load()
    rc = lib.sp_cg_force_noalloc(ctypes.byref(lat.geom), ctypes.byref(G.struct), float(m), ctypes.c_void_p(x.data_ptr()),
                                 ctypes.c_void_p(lam.data_ptr()), ctypes.c_void_p(gamma.data_ptr()),
                                 ctypes.c_void_p(force.data_ptr()) if force is not None else None,
                                 ctypes.c_void_p(dm.data_ptr()) if dm is not None else None,
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == _lib.SP_OK, lib.sp_last_error()
    torch.cuda.current_stream().synchronize()
    return gamma, force, dm


def test_noalloc_force_matches_workspace_force_on_two_calls():
    # the 16^3x32 gradient lattice first, then a smaller antiperiodic one: the second call reuses the array that
    # still holds the first call's contents
    cases = [((16, 16, 16, 32), 0, 0.05, 411), ((4, 6, 2, 8), 1, 0.07, 421)]
    for dims, bc_t, m, seed in cases:
        announce(f"noalloc force dims={dims} bc_t={bc_t}")
        U = li.near_identity_links(dims, 0.3, seed)
        V = li.volume(dims)
        xh = li.gaussian_vector(V // 2, seed + 1)
        lh = li.gaussian_vector(V // 2, seed + 2)
        G = gauge(dims, U, "f64", 18, bc_t)
        x, lam = to_dev(xh), to_dev(lh)
        g_ref, f_ref, dm_ref = sp.cg_force(G, m, x, lam)
        torch.cuda.synchronize()
        gamma, force, dm = _noalloc(G, m, x, lam)
        assert torch.equal(gamma, g_ref)
        assert torch.equal(force, f_ref)
        assert torch.equal(dm, dm_ref)
        if V <= 4096:
            g_or, f_or, dm_or = oracle.grad(dims, U, m, xh, lh, bc_t=bc_t)
            assert rel_err_2(to_host(gamma), g_or) <= 1e-13
            assert rel_err_2(to_host(force), f_or) <= 1e-13
            assert abs(float(dm) - dm_or) <= 1e-12 * abs(dm_or)
    # nullable outputs: gamma alone
    gamma, force, dm = _noalloc(G, m, x, lam, want_force=False, want_mass=False)
    assert torch.equal(gamma, g_ref) and force is None and dm is None


def test_noalloc_force_at_the_workload_size():
    # 20^3x64 (V/2 = 256,000: 49 MB of the 64 MiB array), bit for bit against sp_cg_force
    dims = (20, 20, 20, 64)
    announce(f"noalloc force dims={dims}")
    gen = torch.Generator(device=DEV)
    gen.manual_seed(431)
    V = li.volume(dims)
    H = torch.randn(4, V, 3, 3, dtype=torch.complex128, device=DEV, generator=gen)
    U = torch.linalg.matrix_exp(1j * 0.3 * (H + H.conj().transpose(-1, -2)) / 2)
    del H
    x = torch.randn(V // 2, 3, dtype=torch.complex128, device=DEV, generator=gen)
    lam = torch.randn(V // 2, 3, dtype=torch.complex128, device=DEV, generator=gen)
    G = sp.Gauge(sp.Lattice(dims), U.contiguous(), lo_prec="f64")
    g_ref, f_ref, dm_ref = sp.cg_force(G, 0.01, x, lam)
    torch.cuda.synchronize()
    gamma, force, dm = _noalloc(G, 0.01, x, lam)
    assert torch.equal(gamma, g_ref) and torch.equal(force, f_ref) and torch.equal(dm, dm_ref)
