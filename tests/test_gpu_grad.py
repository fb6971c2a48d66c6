"""GPU adjoint gradient (sp_cg_force and the autograd Function) against the oracle's gradient and against
FP64 finite differences of the GPU's own loss l = Re phi^dag A^-1 phi."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1511_00088_amd as sp
from conftest import rel_err_2
from gpu_common import DEV, announce, gauge, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dims,bc_t", [((4, 4, 4, 4), 0), ((6, 4, 8, 4), 1), ((4, 2, 6, 2), 1)])
def test_force_kernel_matches_oracle(dims, bc_t):
    announce(f"force dims={dims} bc_t={bc_t}")
    U = li.near_identity_links(dims, 0.3, 401)
    V = li.volume(dims)
    x = li.gaussian_vector(V // 2, 402)
    lam = li.gaussian_vector(V // 2, 403)
    m = 0.07
    G = gauge(dims, U, "f64", 18, bc_t)
    gamma, force, dm = sp.cg_force(G, m, to_dev(x), to_dev(lam))
    g_ref, f_ref, dm_ref = oracle.grad(dims, U, m, x, lam, bc_t=bc_t)
    assert rel_err_2(to_host(gamma), g_ref) <= 1e-13
    assert rel_err_2(to_host(force), f_ref) <= 1e-13
    assert abs(float(dm) - dm_ref) <= 1e-12 * abs(dm_ref)


def _loss_gpu(lat, U, m, phi, inner="f64"):
    x = sp.staggered_solve(U, m, phi, lat, inner=inner, tol=1e-13)
    return torch.vdot(phi.flatten(), x.flatten()).real


def test_autograd_vs_finite_differences():
    dims = (4, 4, 4, 4)
    announce("autograd FD 4^4")
    lat = sp.Lattice(dims)
    Uh = li.near_identity_links(dims, 0.3, 43)
    phih = li.gaussian_even_source(dims, 44)
    m0 = 0.05
    U = to_dev(Uh).requires_grad_(True)
    phi = to_dev(phih).requires_grad_(True)
    m = torch.tensor(m0, dtype=torch.float64, device=DEV, requires_grad=True)
    L = _loss_gpu(lat, U, m, phi)
    L.backward()
    gU, gm, gphi = U.grad, m.grad, phi.grad
    x = sp.staggered_solve(U.detach(), m0, phi.detach(), lat, inner="f64", tol=1e-13)
    # closed forms: dL/dphi = 2 x, dL/dm = -2 m |x|^2
    assert rel_err_2(to_host(gphi), 2 * to_host(x)) <= 1e-10
    assert abs(float(gm) + 2 * m0 * float(torch.vdot(x.flatten(), x.flatten()).real)) <= 1e-10 * abs(float(gm))
    # finite differences (4th order) of the GPU loss along random complex link directions
    rng = np.random.default_rng(45)
    h = 1e-4
    for trial in range(3):
        E = rng.standard_normal(Uh.shape) + 1j * rng.standard_normal(Uh.shape)
        Ed = to_dev(E)
        f = lambda t: float(_loss_gpu(lat, U.detach() + t * Ed, m0, phi.detach()))
        fd = (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)
        an = float((torch.conj(gU) * Ed).sum().real)
        announce(f"  direction {trial}: fd={fd:.12e} analytic={an:.12e}")
        assert abs(fd - an) <= 1e-6 * abs(an)
    fdm = (-float(_loss_gpu(lat, U.detach(), m0 + 2 * h, phi.detach())) + 8 * float(_loss_gpu(lat, U.detach(), m0 + h, phi.detach()))
           - 8 * float(_loss_gpu(lat, U.detach(), m0 - h, phi.detach())) + float(_loss_gpu(lat, U.detach(), m0 - 2 * h, phi.detach()))) / (12 * h)
    assert abs(fdm - float(gm)) <= 1e-6 * abs(float(gm))


def test_autograd_cfg4_vs_oracle_gradient():
    """16^3x32 near-identity links, m = 0.05: GPU backward (mixed-precision adjoint solve) vs oracle."""
    c = li.cfg4()
    dims, Uh, m0, phih = c["dims"], c["links"], c["mass"], c["source"]
    announce("autograd 16^3x32 vs oracle")
    lat = sp.Lattice(dims)
    U = to_dev(Uh).requires_grad_(True)
    phi = to_dev(phih).requires_grad_(True)
    m = torch.tensor(m0, dtype=torch.float64, device=DEV, requires_grad=True)
    x = sp.staggered_solve(U, m, phi, lat, inner="f32", tol=1e-10)
    L = torch.vdot(phi.flatten(), x.flatten()).real
    L.backward()
    xr, st, _, _ = oracle.cg_solve(dims, Uh, m0, phih, tol=1e-12)
    g_ref, _, dm_ref = oracle.grad(dims, Uh, m0, xr, xr, want_force=False)
    eg = rel_err_2(to_host(U.grad), g_ref)
    announce(f"  |dU - ref|/|ref| = {eg:.3e}, dm {float(m.grad):.10e} vs {dm_ref:.10e}")
    assert eg <= 1e-6
    assert abs(float(m.grad) - dm_ref) <= 1e-6 * abs(dm_ref)
    assert rel_err_2(to_host(phi.grad), 2 * xr) <= 1e-6


def _loss_gpu_mixed(lat, U, m, psi, phi, inner="f64"):
    x = sp.staggered_solve(U, m, phi, lat, inner=inner, tol=1e-13)
    return torch.vdot(psi.flatten(), x.flatten()).real


@pytest.mark.parametrize("bc_t", [0, 1])
def test_autograd_vs_finite_differences_lambda_ne_x(bc_t):
    """l = Re psi^dag A^-1 phi with psi != phi: the backward's adjoint solve gives lambda = A^-1 psi != x, so
    the mixed terms of the link gradient (lambda with D_oe x, x with D_oe lambda) are exercised apart."""
    dims = (4, 4, 4, 4)
    announce(f"autograd FD 4^4 lambda != x bc_t={bc_t}")
    lat = sp.Lattice(dims, bc_t)
    Uh = li.near_identity_links(dims, 0.3, 43)
    phih = li.gaussian_even_source(dims, 44)
    psih = li.gaussian_even_source(dims, 46)
    m0 = 0.05
    U = to_dev(Uh).requires_grad_(True)
    phi = to_dev(phih).requires_grad_(True)
    psi = to_dev(psih)
    m = torch.tensor(m0, dtype=torch.float64, device=DEV, requires_grad=True)
    L = _loss_gpu_mixed(lat, U, m, psi, phi)
    L.backward()
    gU, gm, gphi = U.grad, m.grad, phi.grad
    # the oracle's lambda = A^-1 psi: dl/dphi = lambda, and the oracle's gradient for the same x, lambda
    xr, _, _, _ = oracle.cg_solve(dims, Uh, m0, phih, tol=1e-13, bc_t=bc_t)
    lr, _, _, _ = oracle.cg_solve(dims, Uh, m0, psih, tol=1e-13, bc_t=bc_t)
    assert rel_err_2(to_host(gphi), lr) <= 1e-10
    g_ref, _, dm_ref = oracle.grad(dims, Uh, m0, xr, lr, bc_t=bc_t, want_force=False)
    assert rel_err_2(to_host(gU), g_ref) <= 1e-10
    assert abs(float(gm) - dm_ref) <= 1e-10 * abs(dm_ref)
    rng = np.random.default_rng(47 + bc_t)
    h = 1e-4

    def fd_of(f):
        return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)

    V = li.volume(dims)
    for trial in range(3):
        E = rng.standard_normal(Uh.shape) + 1j * rng.standard_normal(Uh.shape)
        if trial == 0:  # a single t-link on the last time slice (carries the antiperiodic sign)
            E = np.zeros_like(Uh)
            E[3, 3 * V // 4 + 5] = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        Ed = to_dev(E)
        fd = fd_of(lambda t: float(_loss_gpu_mixed(lat, U.detach() + t * Ed, m0, psi, phi.detach())))
        an = float((torch.conj(gU) * Ed).sum().real)
        announce(f"  direction {trial}: fd={fd:.12e} analytic={an:.12e}")
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3)
    fdm = fd_of(lambda t: float(_loss_gpu_mixed(lat, U.detach(), m0 + t, psi, phi.detach())))
    assert abs(fdm - float(gm)) <= 1e-6 * abs(float(gm))
    E = to_dev(rng.standard_normal(phih.shape) + 1j * rng.standard_normal(phih.shape))
    fdp = fd_of(lambda t: float(_loss_gpu_mixed(lat, U.detach(), m0, psi, phi.detach() + t * E)))
    anp = float((torch.conj(gphi) * E).sum().real)
    assert abs(fdp - anp) <= 1e-6 * abs(anp)
