"""Pins of the NPR contraction oracle (oracle/npr.py) against facts that do not come from the oracle itself.

* spin-taste matrices: identity for S = F = 0; entries in {0, +-1}, nonzero exactly when A xor B = S xor F;
  orthonormal under the trace inner product (the 256 matrices gamma_S x xi_F form a basis); unchanged under a
  change of Dirac representation; equal to a sign rule derived by hand from the anticommutation relations;
* path links: 1 on the unit field; G(z_A) G(z_D)^dag on a pure-gauge field (every path gives the same product,
  which fixes orientation and normalisation); the link or its dagger for one step; U_DA = U_AD^dag; gauge
  covariance;
* the contraction: gauge invariance, the symmetry that exchanges the two bilinears, linearity, locality to
  the hypercube, and a colour-crossing case with a closed form (the one-colour-trace pairing chib1 with chi4
  and chib3 with chi2, which vanishes for the two-trace pairing).
"""
import numpy as np
import pytest

import lattice_inputs as li
from oracle import npr

DIMS = (4, 4, 4, 4)


def _bits(x):
    return [(x >> k) & 1 for k in range(4)]


def _sigma(x, y):
    # number of pairs mu > nu with x_mu = y_nu = 1: gamma_X gamma_Y = (-1)^sigma gamma_{X xor Y}
    bx, by = _bits(x), _bits(y)
    return sum(bx[m] * by[n] for m in range(4) for n in range(m))


def _rev_sign(x):
    n = bin(x).count("1")
    return -1 if (n * (n - 1) // 2) % 2 else 1


def _sign_rule(S, F, A, B):
    if A ^ S ^ B ^ F:
        return 0
    e = _sigma(A, S) + _sigma(A ^ S, B) + _sigma(A ^ S ^ B, F)
    return _rev_sign(A) * _rev_sign(F) * (-1) ** e


def test_spin_taste_identity_support_and_sign_rule():
    assert np.allclose(npr.spin_taste(0, 0), np.eye(16), atol=1e-14)
    for S in range(16):
        for F in range(16):
            M = npr.spin_taste(S, F)
            ref = np.array([[_sign_rule(S, F, A, B) for B in range(16)] for A in range(16)], float)
            assert np.max(np.abs(M - ref)) < 1e-13, (S, F)


def test_spin_taste_orthonormal_basis():
    Ms = np.array([npr.spin_taste(S, F) for S in range(16) for F in range(16)]).reshape(256, 256)
    G = Ms.conj() @ Ms.T
    assert np.max(np.abs(G - 16 * np.eye(256))) < 1e-11


def test_spin_taste_representation_independent(monkeypatch):
    g = npr.euclidean_gammas()
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    g2 = np.array([Q @ x @ Q.conj().T for x in g])
    ref = {(S, F): npr.spin_taste(S, F) for S, F in ((3, 5), (15, 1), (6, 6))}
    monkeypatch.setattr(npr, "euclidean_gammas", lambda: g2)
    for (S, F), M in ref.items():
        assert np.max(np.abs(npr.spin_taste(S, F) - M)) < 1e-13


def _pure_gauge(dims, seed):
    G = li.random_gauge_transform(dims, seed)
    from helpers import shift_lex
    U = np.empty((4,) + G.shape, complex)
    for mu in range(4):
        U[mu] = G @ np.conj(np.swapaxes(G[shift_lex(dims, mu, +1)], -1, -2))
    return U, G


def test_path_links_unit_pure_gauge_single_step_and_reversal():
    V = li.volume(DIMS)
    U1 = np.broadcast_to(np.eye(3, dtype=complex), (4, V, 3, 3)).copy()
    assert np.max(np.abs(npr.path_links(DIMS, U1) - np.eye(3))) < 1e-14
    Ug, G = _pure_gauge(DIMS, 6)
    P = npr.path_links(DIMS, Ug)
    cs = npr.corner_sites(DIMS)
    ref = G[cs][:, :, None] @ np.conj(np.swapaxes(G[cs][:, None, :], -1, -2))
    assert np.max(np.abs(P - ref)) < 1e-13
    U = li.near_identity_links(DIMS, 0.7, 7)
    P = npr.path_links(DIMS, U)
    for mu in range(4):
        A, D = 0, 1 << mu
        assert np.max(np.abs(P[:, A, D] - U[mu][cs[:, A]])) < 1e-15
        assert np.max(np.abs(P[:, D, A] - np.conj(np.swapaxes(U[mu][cs[:, A]], -1, -2)))) < 1e-15
    assert np.max(np.abs(P - np.conj(np.swapaxes(np.swapaxes(P, 1, 2), -1, -2)))) < 1e-14


def _fields(n, V, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((n, V, 3)) + 1j * rng.standard_normal((n, V, 3)) for _ in range(4)]


def test_contraction_gauge_invariant():
    from helpers import gauge_transform_links

    V = li.volume(DIMS)
    U = li.near_identity_links(DIMS, 0.7, 8)
    G = li.random_gauge_transform(DIMS, 9)
    f = _fields(2, V, 10)
    O = npr.contract(DIMS, npr.path_links(DIMS, U), *f, 3, 5, 12, 9)
    Ug = gauge_transform_links(DIMS, U, G)
    # chi -> G chi, chib -> conj(G) chib
    fg = [np.einsum("vij,nvj->nvi", np.conj(G) if k in (0, 2) else G, f[k]) for k in range(4)]
    Og = npr.contract(DIMS, npr.path_links(DIMS, Ug), *fg, 3, 5, 12, 9)
    assert np.max(np.abs(O - Og)) < 1e-12 * np.max(np.abs(O))


def test_contraction_bilinear_exchange_symmetry_and_linearity():
    V = li.volume(DIMS)
    U = li.near_identity_links(DIMS, 0.7, 11)
    P = npr.path_links(DIMS, U)
    f = _fields(1, V, 12)
    O = npr.contract(DIMS, P, f[0], f[1], f[2], f[3], 6, 10, 1, 14)
    Ox = npr.contract(DIMS, P, f[2], f[3], f[0], f[1], 1, 14, 6, 10)
    assert np.max(np.abs(O - Ox)) < 1e-12 * np.max(np.abs(O))
    O2 = npr.contract(DIMS, P, f[0], (2 - 1j) * f[1], f[2], f[3], 6, 10, 1, 14)
    assert np.max(np.abs(O2 - (2 - 1j) * O)) < 1e-12 * np.max(np.abs(O))


def test_contraction_local_to_its_hypercube():
    V = li.volume(DIMS)
    U = li.near_identity_links(DIMS, 0.7, 13)
    f = _fields(1, V, 14)
    cs = npr.corner_sites(DIMS)
    O = npr.contract(DIMS, npr.path_links(DIMS, U), *f, 15, 15, 15, 15)
    z = 5
    inside = set(cs[z].tolist())
    g = [x.copy() for x in f]
    U2 = U.copy()
    for s in range(V):
        if s not in inside:
            for x in g:
                x[:, s] += 1.0
            U2[:, s] = li.haar_su3(4, np.random.default_rng(s))
    O2 = npr.contract(DIMS, npr.path_links(DIMS, U2), *g, 15, 15, 15, 15)
    assert O2[0, z] == O[0, z]
    assert np.all(np.abs(np.delete(O2[0] - O[0], z)) > 0)


def test_contraction_colour_crossing_closed_form():
    # unit links, chib1 = chi4 = colour 0 everywhere, chib3 = chi2 = colour 1: each crossed bilinear is 1,
    # so O = (sum of the entries of M1)(sum of the entries of M2); pairing chib1 with chi2 would give 0
    V = li.volume(DIMS)
    U1 = np.broadcast_to(np.eye(3, dtype=complex), (4, V, 3, 3)).copy()
    e0 = np.zeros((1, V, 3), complex)
    e0[..., 0] = 1
    e1 = np.zeros((1, V, 3), complex)
    e1[..., 1] = 1
    # the first three label sets have entry sums of 16 x 16, the last two sum to zero
    for S1, F1, S2, F2 in ((0, 0, 0, 0), (1, 8, 6, 3), (10, 5, 13, 14), (5, 5, 3, 12), (15, 0, 0, 15)):
        O = npr.contract(DIMS, npr.path_links(DIMS, U1), e0, e1, e1, e0, S1, F1, S2, F2)
        ref = npr.spin_taste(S1, F1).sum() * npr.spin_taste(S2, F2).sum()
        assert np.max(np.abs(O - ref)) < 1e-12
