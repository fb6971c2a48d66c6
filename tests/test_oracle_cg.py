"""Pins of the FP64 oracle's CG (and its full-system solve) against facts outside the oracle.

* numpy.linalg.solve on the dense matrix of A (2^4 and 4^4, Haar links);
* the free-field solution in momentum space by FFT: x = F^-1[F(b) / (m^2 + sum sin^2 p)];
* CG on free 4^4 converges in <= 5 iterations (A has exactly 5 distinct eigenvalues there);
* gauge covariance of the solution x[U', G b] = G x[U, b];
* a warm start from a looser solve reaches the same solution;
* the full system (m + D) psi = src by dense solve on 2^4 and 4^4.
"""
import numpy as np
import pytest

import lattice_inputs as li
from conftest import rel_err_2
from helpers import dense_operator, gauge_transform_links, gauge_transform_vec, half_rows, parity, to_full, to_half


@pytest.mark.parametrize("dims,seed,m", [((2, 2, 2, 2), 1, 0.1), ((4, 4, 4, 4), 11, 0.1), ((4, 2, 4, 2), 3, 0.02)])
def test_cg_matches_dense_solve(oracle_lib, dims, seed, m):
    V = li.volume(dims)
    U = li.haar_links(dims, seed)
    b = li.gaussian_even_source(dims, seed + 1)
    A = dense_operator(lambda e: oracle_lib.apply_A(dims, U, m, e.reshape(V // 2, 3)).ravel(), 3 * V // 2)
    x_ref = np.linalg.solve(A, b.ravel()).reshape(V // 2, 3)
    x, st, it, res = oracle_lib.cg_solve(dims, U, m, b, tol=1e-12)
    assert st == 0 and res <= 1e-12
    assert rel_err_2(x, x_ref) < 1e-10


def test_cfg0_converges(oracle_lib):
    c = li.cfg0()
    x, st, it, res = oracle_lib.cg_solve(c["dims"], c["links"], c["mass"], c["source"], tol=c["tol"])
    assert st == 0 and res <= 1e-10 and 0 < it < 1000


@pytest.mark.parametrize("dims,m", [((8, 8, 8, 8), 0.05), ((4, 6, 8, 10), 0.2)])
def test_free_field_fft_solution(oracle_lib, dims, m):
    V = li.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()
    b = li.gaussian_even_source(dims, 4)
    bf = to_full(dims, b, 0).reshape(dims[3], dims[2], dims[1], dims[0], 3)  # [t][z][y][x][c]
    ks = np.meshgrid(*[2 * np.pi * np.fft.fftfreq(L) for L in (dims[3], dims[2], dims[1], dims[0])],
                     indexing="ij")
    denom = m * m + sum(np.sin(k) ** 2 for k in ks)
    xf = np.fft.ifftn(np.fft.fftn(bf, axes=(0, 1, 2, 3)) / denom[..., None], axes=(0, 1, 2, 3))
    xf = xf.reshape(V, 3)
    assert np.abs(xf[parity(dims) == 1]).max() < 1e-12  # -D^2 keeps parity
    x_ref = to_half(dims, xf, 0)
    x, st, it, res = oracle_lib.cg_solve(dims, U, m, b, tol=1e-12)
    assert st == 0
    assert rel_err_2(x, x_ref) < 1e-10


def test_free_4x4x4x4_five_iterations(oracle_lib):
    dims = (4, 4, 4, 4)
    V = li.volume(dims)
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (4, V, 3, 3)).copy()
    b = li.gaussian_even_source(dims, 5)
    x, st, it, res = oracle_lib.cg_solve(dims, U, 0.1, b, tol=1e-10)
    assert st == 0 and it <= 5 and res <= 1e-10


def test_solution_gauge_covariance(oracle_lib):
    dims = (4, 4, 4, 6)
    U = li.haar_links(dims, 7)
    G = li.random_gauge_transform(dims, 8)
    b = li.gaussian_even_source(dims, 9)
    Ge = half_rows(dims, G, 0)
    x, st, _, _ = oracle_lib.cg_solve(dims, U, 0.1, b, tol=1e-12, bc_t=1)
    xg, st2, _, _ = oracle_lib.cg_solve(dims, gauge_transform_links(dims, U, G), 0.1,
                                        gauge_transform_vec(Ge, b), tol=1e-12, bc_t=1)
    assert st == 0 and st2 == 0
    assert rel_err_2(xg, gauge_transform_vec(Ge, x)) < 1e-10


def test_warm_start(oracle_lib):
    dims = (4, 4, 4, 4)
    U = li.near_identity_links(dims, 0.3, 10)
    b = li.gaussian_even_source(dims, 11)
    x1, st1, it1, r1 = oracle_lib.cg_solve(dims, U, 0.05, b, tol=1e-4)
    assert st1 == 0 and r1 <= 1e-4
    x2, st2, it2, r2 = oracle_lib.cg_solve(dims, U, 0.05, b, tol=1e-12, x0=x1)
    x3, st3, it3, r3 = oracle_lib.cg_solve(dims, U, 0.05, b, tol=1e-12)
    assert st2 == 0 and st3 == 0 and r2 <= 1e-12
    assert rel_err_2(x2, x3) < 1e-10


def test_cg_not_converged_and_breakdown(oracle_lib):
    dims = (4, 4, 4, 4)
    U = li.haar_links(dims, 12)
    b = li.gaussian_even_source(dims, 13)
    x, st, it, res = oracle_lib.cg_solve(dims, U, 0.01, b, tol=1e-12, max_iter=3)
    assert st == 1 and it == 3 and res > 1e-12
    bn = b.copy()
    bn[0, 0] = np.nan
    x, st, it, res = oracle_lib.cg_solve(dims, U, 0.01, bn, tol=1e-12)
    assert st == -6


@pytest.mark.parametrize("dims,m", [((2, 2, 2, 2), 0.3), ((4, 4, 4, 4), 0.1)])
def test_full_system_dense(oracle_lib, dims, m):
    V = li.volume(dims)
    U = li.haar_links(dims, 14)
    src = li.gaussian_vector(V, 15)
    M = dense_operator(lambda e: (m * e.reshape(V, 3) + oracle_lib.dslash(dims, U, e.reshape(V, 3))).ravel(), 3 * V)
    psi_ref = np.linalg.solve(M, src.ravel()).reshape(V, 3)
    psi, st, it = oracle_lib.full_solve(dims, U, m, src, tol=1e-13)
    assert st == 0
    assert rel_err_2(psi, psi_ref) < 1e-10
