"""Pins of the FP64 oracle's adjoint gradient against finite differences and closed forms.

Loss l = Re phi^dag A^-1 phi (even sites, A = m^2 - D_eo D_oe), so x = A^-1 phi, dl/dx = phi and
lambda = A^-1 phi = x. Checked:
* dl/dU (gamma) against 4th-order central differences along random complex directions (A stays HPD for
  non-unitary U, so these are legitimate);
* the su(3)-projected force F = TA(U gamma^dag) against differences along U -> exp(i t T^a) U;
* dl/dm = -2 m |x|^2 against differences in m; dl/dphi = 2 x against differences in phi;
* F traceless anti-Hermitian, and covariant F -> G(n) F G(n)^dag under gauge transforms.
"""
import numpy as np
import pytest

import lattice_inputs as li
from helpers import gauge_transform_links, gauge_transform_vec, half_rows

DIMS = (4, 4, 4, 4)


def _loss(oracle_lib, U, m, phi, bc_t=0):
    x, st, _, _ = oracle_lib.cg_solve(DIMS, U, m, phi, tol=1e-13, max_iter=3000, bc_t=bc_t)
    assert st in (0, 1)
    return np.vdot(phi, x).real


def _fd(f, h):
    return (-f(2 * h) + 8 * f(h) - 8 * f(-h) + f(-2 * h)) / (12 * h)


@pytest.fixture(scope="module")
def setup(oracle_lib):
    U = li.near_identity_links(DIMS, 0.3, 43)
    phi = li.gaussian_even_source(DIMS, 44)
    m = 0.3
    x, st, _, _ = oracle_lib.cg_solve(DIMS, U, m, phi, tol=1e-13)
    assert st == 0
    gamma, force, dm = oracle_lib.grad(DIMS, U, m, x, x)
    return U, phi, m, x, gamma, force, dm


@pytest.mark.parametrize("bc_t", [0, 1])
def test_gamma_vs_finite_differences(oracle_lib, setup, bc_t):
    U, phi, m, _, _, _, _ = setup
    x, st, _, _ = oracle_lib.cg_solve(DIMS, U, m, phi, tol=1e-13, bc_t=bc_t)
    gamma, _, _ = oracle_lib.grad(DIMS, U, m, x, x, bc_t=bc_t, want_force=False)
    rng = np.random.default_rng(7)
    for trial in range(3):
        E = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
        if trial == 0:  # one localised direction: a single link
            E = np.zeros_like(U)
            E[3, 200] = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        fd = _fd(lambda h: _loss(oracle_lib, U + h * E, m, phi, bc_t), 1e-4)
        an = np.sum(np.conj(gamma) * E).real
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (fd, an)


def test_force_vs_su3_differences(oracle_lib, setup):
    U, phi, m, _, gamma, force, _ = setup
    T = li.gell_mann() / 2
    rng = np.random.default_rng(8)
    links = [(int(rng.integers(4)), int(rng.integers(li.volume(DIMS)))) for _ in range(6)]
    for mu, s in links:
        for a in range(8):
            w, v = np.linalg.eigh(T[a])

            def f(t):
                Ut = U.copy()
                Ut[mu, s] = (v * np.exp(1j * t * w)) @ v.conj().T @ U[mu, s]
                return _loss(oracle_lib, Ut, m, phi)

            fd = _fd(f, 1e-4)
            an = (1j * np.trace(force[mu, s] @ T[a])).real
            assert abs(fd - an) <= 1e-6 * max(np.abs(force).max(), 1e-3), (mu, s, a, fd, an)


def test_mass_and_source_gradients(oracle_lib, setup):
    U, phi, m, x, _, _, dm = setup
    assert abs(dm - (-2 * m * np.vdot(x, x).real)) < 1e-12 * abs(dm)
    fd = _fd(lambda h: _loss(oracle_lib, U, m + h, phi), 1e-4)
    assert abs(fd - dm) <= 1e-6 * abs(dm)
    rng = np.random.default_rng(9)
    for _ in range(3):
        E = rng.standard_normal(phi.shape) + 1j * rng.standard_normal(phi.shape)
        fd = _fd(lambda h: _loss(oracle_lib, U, m, phi + h * E), 1e-4)
        an = np.sum(np.conj(2 * x) * E).real
        assert abs(fd - an) <= 1e-6 * abs(an)


def test_force_algebra_and_covariance(oracle_lib, setup):
    U, phi, m, x, gamma, force, _ = setup
    Fd = np.conj(np.swapaxes(force, -1, -2))
    np.testing.assert_allclose(force, -Fd, atol=1e-13)
    np.testing.assert_allclose(np.trace(force, axis1=-2, axis2=-1), 0, atol=1e-13)
    G = li.random_gauge_transform(DIMS, 10)
    Ug = gauge_transform_links(DIMS, U, G)
    phig = gauge_transform_vec(half_rows(DIMS, G, 0), phi)
    xg, st, _, _ = oracle_lib.cg_solve(DIMS, Ug, m, phig, tol=1e-13)
    _, fg, dmg = oracle_lib.grad(DIMS, Ug, m, xg, xg)
    expect = G[None] @ force @ np.conj(np.swapaxes(G, -1, -2))[None]
    np.testing.assert_allclose(fg, expect, atol=1e-9 * np.abs(force).max())


# ---------------------------------------------------------------------------------------------------------
# lambda != x: the loss l = Re psi^dag A^-1 phi with psi != phi has dl/dx = psi, so lambda = A^-1 psi differs
# from x = A^-1 phi and the two mixed terms of gamma (lambda with y_x, x with y_lambda) are no longer
# interchangeable. Swapping them, or taking lambda for x in either, changes gamma here while every pin with
# lambda = x above would still pass. Closed forms: dl/dphi = lambda, dl/dm = -2 m Re<lambda, x>.
# ---------------------------------------------------------------------------------------------------------
def _loss_mixed(oracle_lib, U, m, psi, phi, bc_t=0):
    x, st, _, _ = oracle_lib.cg_solve(DIMS, U, m, phi, tol=1e-13, max_iter=3000, bc_t=bc_t)
    assert st in (0, 1)
    return np.vdot(psi, x).real


def _mixed_setup(oracle_lib, bc_t):
    U = li.near_identity_links(DIMS, 0.3, 43)
    phi = li.gaussian_even_source(DIMS, 44)
    psi = li.gaussian_even_source(DIMS, 46)
    m = 0.3
    x, st, _, _ = oracle_lib.cg_solve(DIMS, U, m, phi, tol=1e-13, bc_t=bc_t)
    lam, st2, _, _ = oracle_lib.cg_solve(DIMS, U, m, psi, tol=1e-13, bc_t=bc_t)
    assert st == 0 and st2 == 0
    # lambda and x are far apart, so a term that mixes them up shows
    assert np.linalg.norm(lam - x) > 0.5 * np.linalg.norm(x)
    gamma, force, dm = oracle_lib.grad(DIMS, U, m, x, lam, bc_t=bc_t)
    return U, phi, psi, m, x, lam, gamma, force, dm


@pytest.mark.parametrize("bc_t", [0, 1])
def test_gamma_vs_finite_differences_lambda_ne_x(oracle_lib, bc_t):
    U, phi, psi, m, x, lam, gamma, _, _ = _mixed_setup(oracle_lib, bc_t)
    rng = np.random.default_rng(17 + bc_t)
    V = li.volume(DIMS)
    # the last time slice carries the antiperiodic sign: take the single link there (t = 3) for bc_t = 1
    single = 3 * V // 4 + 5 if bc_t else 200
    for trial in range(4):
        E = rng.standard_normal(U.shape) + 1j * rng.standard_normal(U.shape)
        if trial == 0:  # one localised direction: a single t-link
            E = np.zeros_like(U)
            E[3, single] = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        if trial == 1:  # a single x-link on an odd site (the second formula of gamma)
            E = np.zeros_like(U)
            E[0, 1] = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
        fd = _fd(lambda h: _loss_mixed(oracle_lib, U + h * E, m, psi, phi, bc_t), 1e-4)
        an = np.sum(np.conj(gamma) * E).real
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-3), (trial, fd, an)


@pytest.mark.parametrize("bc_t", [0, 1])
def test_force_vs_su3_differences_lambda_ne_x(oracle_lib, bc_t):
    U, phi, psi, m, x, lam, gamma, force, _ = _mixed_setup(oracle_lib, bc_t)
    T = li.gell_mann() / 2
    rng = np.random.default_rng(18 + bc_t)
    V = li.volume(DIMS)
    # an even and an odd site in each case, one of them a t-link on the last slice
    links = [(3, 3 * V // 4 + 2), (3, 3 * V // 4 + 1)] + [(int(rng.integers(4)), int(rng.integers(V))) for _ in range(2)]
    for mu, s in links:
        for a in range(8):
            w, v = np.linalg.eigh(T[a])

            def f(t):
                Ut = U.copy()
                Ut[mu, s] = (v * np.exp(1j * t * w)) @ v.conj().T @ U[mu, s]
                return _loss_mixed(oracle_lib, Ut, m, psi, phi, bc_t)

            fd = _fd(f, 1e-4)
            an = (1j * np.trace(force[mu, s] @ T[a])).real
            assert abs(fd - an) <= 1e-6 * max(np.abs(force).max(), 1e-3), (mu, s, a, fd, an)


@pytest.mark.parametrize("bc_t", [0, 1])
def test_mass_and_source_gradients_lambda_ne_x(oracle_lib, bc_t):
    U, phi, psi, m, x, lam, _, _, dm = _mixed_setup(oracle_lib, bc_t)
    fd = _fd(lambda h: _loss_mixed(oracle_lib, U, m + h, psi, phi, bc_t), 1e-4)
    assert abs(fd - dm) <= 1e-6 * abs(dm), (fd, dm)
    rng = np.random.default_rng(19)
    for _ in range(2):
        E = rng.standard_normal(phi.shape) + 1j * rng.standard_normal(phi.shape)
        fd = _fd(lambda h: _loss_mixed(oracle_lib, U, m, psi, phi + h * E, bc_t), 1e-4)
        an = np.sum(np.conj(lam) * E).real
        assert abs(fd - an) <= 1e-6 * abs(an)
