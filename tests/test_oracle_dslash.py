"""Pins of the FP64 oracle's staggered operator against facts outside the oracle.

* a hand-derived worked example (free links, point source; golden file) fixes the phase convention,
  the 1/2 and the antiperiodic time boundary;
* anti-Hermiticity D^dag = -D (fails on a wrong sign, a missing hop or U in place of U^dag);
* the parity block structure (D_ee = D_oo = 0);
* the free-field plane-wave eigenvalue sum_mu sin^2 p_mu of -D^2 (fails on a wrong eta or factor);
* gauge covariance D[U'] G chi = G D[U] chi (fails on a wrong link site or orientation);
* the even-odd operator A equals the even block of (m + D)^dag (m + D).
"""
import os

import numpy as np
import pytest

import lattice_inputs as li
from helpers import (coords, dense_operator, gauge_transform_links, gauge_transform_vec, half_rows,
                     lex_of, parity, to_full, to_half)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _unit_links(dims):
    V = li.volume(dims)
    return np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()


@pytest.mark.parametrize("bc_t", [0, 1])
def test_worked_example_point_source(oracle_lib, bc_t):
    dims = (4, 4, 4, 4)
    V = li.volume(dims)
    rows = np.loadtxt(os.path.join(GOLDEN, "free_delta_4x4x4x4.txt"))
    rows = rows[rows[:, 0] == bc_t]
    chi = np.zeros((V, 3), np.complex128)
    chi[lex_of(dims, (1, 1, 1, 0))] = 1.0
    out = oracle_lib.dslash(dims, _unit_links(dims), chi, bc_t=bc_t)
    expect = np.zeros((V, 3), np.complex128)
    for r in rows:
        expect[lex_of(dims, r[1:5].astype(int))] = r[5]
    np.testing.assert_allclose(out, expect, atol=1e-15)


def test_worked_example_link_orientation(oracle_lib):
    """One link U_x(n0) = e^{i theta} 1: the forward hop sees U, the backward hop sees U^dag."""
    dims = (4, 4, 4, 4)
    U = _unit_links(dims)
    n0 = (1, 2, 3, 1)
    theta = 0.3
    U[0, lex_of(dims, n0)] *= np.exp(1j * theta)
    V = li.volume(dims)
    n1 = (2, 2, 3, 1)
    # source at n0 + x: output at n0 = +1/2 eta_0 U_x(n0) = 0.5 e^{i theta}
    chi = np.zeros((V, 3), np.complex128)
    chi[lex_of(dims, n1)] = 1.0
    out = oracle_lib.dslash(dims, U, chi)
    np.testing.assert_allclose(out[lex_of(dims, n0)], 0.5 * np.exp(1j * theta) * np.ones(3), atol=1e-15)
    # source at n0: output at n0 + x = -1/2 eta_0 U_x(n0)^dag = -0.5 e^{-i theta}
    chi = np.zeros((V, 3), np.complex128)
    chi[lex_of(dims, n0)] = 1.0
    out = oracle_lib.dslash(dims, U, chi)
    np.testing.assert_allclose(out[lex_of(dims, n1)], -0.5 * np.exp(-1j * theta) * np.ones(3), atol=1e-15)


@pytest.mark.parametrize("dims,bc_t", [((4, 4, 4, 4), 0), ((4, 6, 2, 8), 1), ((2, 2, 2, 2), 0)])
def test_anti_hermitian(oracle_lib, dims, bc_t):
    V = li.volume(dims)
    U = li.haar_links(dims, 5)
    x = li.gaussian_vector(V, 6)
    y = li.gaussian_vector(V, 7)
    Dx = oracle_lib.dslash(dims, U, x, bc_t=bc_t)
    Dy = oracle_lib.dslash(dims, U, y, bc_t=bc_t)
    lhs = np.vdot(y, Dx)
    rhs = -np.vdot(Dy, x)
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_anti_hermitian_dense_2x2x2x2(oracle_lib):
    dims = (2, 2, 2, 2)
    V = li.volume(dims)
    U = li.haar_links(dims, 8)
    D = dense_operator(lambda e: oracle_lib.dslash(dims, U, e.reshape(V, 3)).ravel(), 3 * V)
    assert np.abs(D).max() > 0.1
    np.testing.assert_allclose(D + D.conj().T, 0, atol=1e-15)


def test_parity_blocks_vanish(oracle_lib):
    dims = (4, 4, 6, 4)
    V = li.volume(dims)
    U = li.haar_links(dims, 9)
    par = parity(dims)
    for p in (0, 1):
        x = li.gaussian_vector(V, 10 + p)
        x[par != p] = 0
        Dx = oracle_lib.dslash(dims, U, x)
        assert np.abs(Dx[par == p]).max() == 0.0
        assert np.abs(Dx[par != p]).max() > 0.1


@pytest.mark.parametrize("p", [0, 1])
def test_half_operator_matches_full(oracle_lib, p):
    """D_{p,1-p} acting on half vectors equals the full operator restricted to the parities."""
    dims = (4, 6, 4, 8)
    U = li.haar_links(dims, 13)
    V = li.volume(dims)
    xh = li.gaussian_vector(V // 2, 14)
    full = oracle_lib.dslash(dims, U, to_full(dims, xh, 1 - p), bc_t=1)
    half = oracle_lib.dslash_eo(dims, U, xh, p, bc_t=1)
    np.testing.assert_allclose(half, to_half(dims, full, p), atol=1e-14)
    cbs = np.array([0, 5, V // 2 - 1, 17, 17])
    np.testing.assert_allclose(oracle_lib.dslash_eo_sites(dims, U, xh, p, cbs, bc_t=1), half[cbs], atol=0)


@pytest.mark.parametrize("dims,bc_t", [((4, 6, 8, 10), 0), ((6, 4, 4, 8), 1)])
def test_free_field_plane_waves(oracle_lib, dims, bc_t):
    """-D^2 e^{ipn} v = sum_mu sin^2(p_mu) e^{ipn} v on free links (antiperiodic: p_t = (2k+1) pi / T)."""
    rng = np.random.default_rng(3)
    U = _unit_links(dims)
    n = coords(dims)
    for _ in range(4):
        k = np.array([rng.integers(0, L) for L in dims])
        p = 2 * np.pi * k / np.array(dims)
        if bc_t:
            p[3] = (2 * k[3] + 1) * np.pi / dims[3]
        v = rng.standard_normal(3) + 1j * rng.standard_normal(3)
        wave = np.exp(1j * (n @ p))[:, None] * v[None, :]
        D2 = oracle_lib.dslash(dims, U, oracle_lib.dslash(dims, U, wave, bc_t=bc_t), bc_t=bc_t)
        lam = np.sum(np.sin(p) ** 2)
        np.testing.assert_allclose(-D2, lam * wave, atol=1e-13)


def test_free_field_spectrum_of_A(oracle_lib):
    dims = (4, 4, 4, 4)
    V = li.volume(dims)
    m = 0.3
    U = _unit_links(dims)
    A = dense_operator(lambda e: oracle_lib.apply_A(dims, U, m, e.reshape(V // 2, 3)).ravel(), 3 * V // 2)
    np.testing.assert_allclose(A, A.conj().T, atol=1e-15)
    ev = np.linalg.eigvalsh(A)
    golden = np.loadtxt(os.path.join(GOLDEN, "free_spectrum_A_4x4x4x4.txt"))
    expect = np.concatenate([np.full(int(mult), m * m + j) for j, mult in golden])
    np.testing.assert_allclose(np.sort(ev), np.sort(expect), atol=1e-12)


@pytest.mark.parametrize("bc_t", [0, 1])
def test_gauge_covariance(oracle_lib, bc_t):
    dims = (4, 4, 6, 4)
    V = li.volume(dims)
    U = li.haar_links(dims, 15)
    G = li.random_gauge_transform(dims, 16)
    chi = li.gaussian_vector(V, 17)
    lhs = oracle_lib.dslash(dims, gauge_transform_links(dims, U, G), gauge_transform_vec(G, chi), bc_t=bc_t)
    rhs = gauge_transform_vec(G, oracle_lib.dslash(dims, U, chi, bc_t=bc_t))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)
    # the same on the half operator
    xh = li.gaussian_vector(V // 2, 18)
    lhs = oracle_lib.dslash_eo(dims, gauge_transform_links(dims, U, G),
                               gauge_transform_vec(half_rows(dims, G, 0), xh), 1, bc_t=bc_t)
    rhs = gauge_transform_vec(half_rows(dims, G, 1), oracle_lib.dslash_eo(dims, U, xh, 1, bc_t=bc_t))
    np.testing.assert_allclose(lhs, rhs, atol=1e-13)


def test_A_is_even_block_of_normal_operator(oracle_lib):
    """(m + D)^dag (m + D) = m^2 - D^2; its even block is A = m^2 - D_eo D_oe."""
    dims = (4, 4, 4, 6)
    V = li.volume(dims)
    U = li.haar_links(dims, 19)
    m = 0.07
    xh = li.gaussian_vector(V // 2, 20)
    xf = to_full(dims, xh, 0)
    M = lambda v: m * v + oracle_lib.dslash(dims, U, v, bc_t=1)
    Mdag = lambda v: m * v - oracle_lib.dslash(dims, U, v, bc_t=1)
    ref = to_half(dims, Mdag(M(xf)), 0)
    np.testing.assert_allclose(oracle_lib.apply_A(dims, U, m, xh, bc_t=1), ref, atol=1e-13)


def test_A_bounds_unitary_links(oracle_lib):
    """m^2 <= <x, A x>/<x, x> <= m^2 + 16 for unitary links; power iteration reaches below the top."""
    dims = (4, 4, 4, 4)
    V = li.volume(dims)
    U = li.haar_links(dims, 21)
    m = 0.2
    x = li.gaussian_vector(V // 2, 22)
    for _ in range(30):
        y = oracle_lib.apply_A(dims, U, m, x)
        lam = np.vdot(x, y).real / np.vdot(x, x).real
        assert m * m - 1e-12 <= lam <= m * m + 16 + 1e-12
        x = y / np.linalg.norm(y)
