"""Pins of the HYP-smearing oracle (oracle/hyp.py) against facts that do not come from the oracle itself.

* the projection's start is the unitary polar factor (scipy.linalg.polar) with its determinant's cube
  root divided out, and its result is a stationary maximum of Re tr(X^dag W) over SU(3);
* special cases: zero smearing weights give back SU(3) links; pure-gauge (flat) fields are fixed points;
* gauge covariance V[G U G^dag] = G V[U] G^dag;
* hypercubic locality: the smeared link depends on exactly the links of the 8 hypercubes that contain it;
* first order in the field: U = exp(i eps A) gives V = exp(i eps A' + O(eps^2)) with A' a linear
  smoothing of A whose momentum-space form factor follows from the definition by hand (below), and
  which, for the weights (7/8, 4/7, 1/4), vanishes at every momentum with transverse components 0 or pi
  (the tree-level equivalence of HYP with those weights to Fat7 smearing, Lee and Sharpe,
  Phys. Rev. D 66 (2002) 114501) -- a property of the whole three-level structure.
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import lattice_inputs as li
from oracle import hyp
from helpers import coords, gauge_transform_links

DIMS = (4, 4, 4, 4)


def _su3_random(n, rng):
    return li.haar_su3(n, rng)


def _objective(X, W):
    return np.real(np.trace(hyp.dag(X) @ W, axis1=-2, axis2=-1))


def _ta(M):
    A = 0.5 * (M - hyp.dag(M))
    tr = np.trace(A, axis1=-2, axis2=-1) / 3.0
    return A - tr[..., None, None] * np.eye(3)


def _generic_W(n, seed):
    rng = np.random.default_rng(seed)
    U = _su3_random(n, rng)
    staple = (_su3_random(n, rng) + _su3_random(n, rng)) / 2
    return 0.4 * U + 0.6 * staple


# ---------------------------------------------------------------------------------------------------------
# projection
# ---------------------------------------------------------------------------------------------------------
def test_projection_start_is_polar_factor_with_det_root_removed():
    W = _generic_W(200, 1)
    X0 = hyp.polar_start(W)
    for k in range(W.shape[0]):
        Up, _ = scipy.linalg.polar(W[k], side="right")  # W = Up P
        d = np.linalg.det(Up)
        ref = Up * np.exp(-1j * np.angle(d) / 3.0)
        assert np.max(np.abs(X0[k] - ref)) < 1e-12


def test_projection_is_stationary_maximum_in_su3():
    W = _generic_W(300, 2)
    X = hyp.proj_su3(W)
    assert np.max(np.abs(X @ hyp.dag(X) - np.eye(3))) < 1e-12
    assert np.max(np.abs(np.linalg.det(X) - 1.0)) < 1e-12
    # first-order optimality: the traceless anti-Hermitian part of W X^dag vanishes
    assert np.max(np.abs(_ta(W @ hyp.dag(X)))) < 1e-12
    # no SU(3) step in any direction improves the objective, and the sweeps improved on the start
    rng = np.random.default_rng(3)
    f = _objective(X, W)
    assert np.all(f >= _objective(hyp.polar_start(W), W) - 1e-13)
    lam = li.gell_mann()
    for _ in range(20):
        H = np.einsum("a,aij->ij", rng.standard_normal(8), lam)
        for t in (1e-3, -1e-3):
            step = scipy.linalg.expm(1j * t * H)
            assert np.all(_objective(step @ X, W) <= f + 1e-13)


def test_projection_special_cases():
    rng = np.random.default_rng(4)
    U = _su3_random(50, rng)
    c = rng.uniform(0.2, 3.0, 50)
    assert np.max(np.abs(hyp.proj_su3(c[:, None, None] * U) - U)) < 1e-13
    # a U(3) matrix e^{i theta} U with |theta| < pi/3 projects onto U
    th = rng.uniform(-1.0, 1.0, 50)
    assert np.max(np.abs(hyp.proj_su3(np.exp(1j * th)[:, None, None] * U) - U)) < 1e-13


# ---------------------------------------------------------------------------------------------------------
# smearing: special cases, covariance, locality
# ---------------------------------------------------------------------------------------------------------
def test_zero_weights_return_the_links():
    U = li.haar_links(DIMS, 11)
    V = hyp.hyp_smear(DIMS, U, alpha=(0.0, 0.0, 0.0))
    assert np.max(np.abs(V - U)) < 1e-13


def _pure_gauge(dims, seed):
    G = li.random_gauge_transform(dims, seed)  # [V][3][3]
    U = np.empty((4,) + G.shape, np.complex128)
    for mu in range(4):
        U[mu] = G @ hyp.dag(hyp.shift(G, mu, +1, dims))
    return U


def test_pure_gauge_field_is_a_fixed_point():
    U = _pure_gauge(DIMS, 7)
    V = hyp.hyp_smear(DIMS, U)
    assert np.max(np.abs(V - U)) < 1e-12


def test_gauge_covariance():
    U = li.near_identity_links(DIMS, 0.6, 43)
    G = li.random_gauge_transform(DIMS, 8)
    V = hyp.hyp_smear(DIMS, U)
    Vg = hyp.hyp_smear(DIMS, gauge_transform_links(DIMS, U, G))
    assert np.max(np.abs(Vg - gauge_transform_links(DIMS, V, G))) < 1e-12


def _hypercube_links(dims, x, mu):
    """Links (nu, lex) with both ends in one of the 8 hypercubes containing the link (x, mu)."""
    X, Y, Z, T = dims
    L = np.array(dims)
    trans = [d for d in range(4) if d != mu]
    out = set()
    for signs in itertools.product((1, -1), repeat=3):
        corners = []
        for a in (0, 1):
            for b in itertools.product((0, 1), repeat=3):
                c = np.array(x)
                c[mu] += a
                for d, s, bb in zip(trans, signs, b):
                    c[d] += s * bb
                corners.append(tuple(c % L))
        cs = set(corners)
        for c in cs:
            for nu in range(4):
                e = list(c)
                e[nu] = (e[nu] + 1) % L[nu]
                if tuple(e) in cs:
                    out.add((nu, c[0] + X * (c[1] + Y * (c[2] + Z * c[3]))))
    return out


def test_hypercube_locality():
    dims = DIMS
    U = li.near_identity_links(dims, 0.5, 45)
    x, mu = (1, 2, 1, 2), 2
    lex = x[0] + 4 * (x[1] + 4 * (x[2] + 4 * x[3]))
    inside = _hypercube_links(dims, x, mu)
    assert len(inside) == 135  # 54 sites: 27 links along mu, 2 x 3 x 18 transverse ones
    V0 = hyp.hyp_smear(dims, U)[mu, lex]
    rng = np.random.default_rng(9)
    lam = li.gell_mann()
    kick = lambda: scipy.linalg.expm(1j * 0.05 * np.einsum("a,aij->ij", rng.standard_normal(8), lam))  # noqa
    # every link outside the hypercubes at once: the smeared link does not move by a single bit
    Uo = U.copy()
    for nu in range(4):
        for s in range(U.shape[1]):
            if (nu, s) not in inside:
                Uo[nu, s] = kick() @ Uo[nu, s]
    assert np.array_equal(hyp.hyp_smear(dims, Uo)[mu, lex], V0)
    # each of a sample of links inside, one at a time, moves it
    sample = sorted(inside)
    idx = rng.choice(len(sample), 24, replace=False)
    for i in idx:
        nu, s = sample[i]
        Ui = U.copy()
        Ui[nu, s] = kick() @ Ui[nu, s]
        assert np.max(np.abs(hyp.hyp_smear(dims, Ui)[mu, lex] - V0)) > 1e-6, (nu, s)


# ---------------------------------------------------------------------------------------------------------
# first order in the field: momentum-space form factor
# ---------------------------------------------------------------------------------------------------------
def _staple_lin(s, t, kmu, keta):
    # staple of side links exp(i eps s) around top links exp(i eps t), to first order, for fields
    # f(x) = f_k e^{i k.x}: s(x) + t(x+eta) - s(x+mu) - s(x-eta) + t(x-eta) + s(x-eta+mu)
    return 2.0 * np.cos(keta) * t + (1.0 - np.exp(1j * kmu)) * (1.0 - np.exp(-1j * keta)) * s


def _form_factor(a, k, alpha):
    a1, a2, a3 = alpha
    l1 = {(m, e): (1 - a3) * a[m] + (a3 / 2) * _staple_lin(a[e], a[m], k[m], k[e])
          for m in range(4) for e in range(4) if e != m}
    l2 = {}
    for m in range(4):
        for n in range(4):
            if n == m:
                continue
            s = 0
            for r in range(4):
                if r not in (m, n):
                    sg = 6 - m - n - r
                    s = s + _staple_lin(l1[r, sg], l1[m, sg], k[m], k[r])
            l2[m, n] = (1 - a2) * a[m] + (a2 / 4) * s
    out = []
    for m in range(4):
        s = sum(_staple_lin(l2[n, m], l2[m, n], k[m], k[n]) for n in range(4) if n != m)
        out.append((1 - a1) * a[m] + (a1 / 6) * s)
    return out


def _su3_field_from(A, eps):
    w, v = np.linalg.eigh(A)
    return (v * np.exp(1j * eps * w)[..., None, :]) @ hyp.dag(v)


def _first_order(dims, A, alpha, eps):
    V = hyp.hyp_smear(dims, _su3_field_from(A, eps), alpha=alpha)
    B = (V - hyp.dag(V)) / (2j * eps)
    tr = np.trace(B, axis1=-2, axis2=-1) / 3.0
    return B - tr[..., None, None] * np.eye(3)


def _random_hermitian_field(dims, seed):
    rng = np.random.default_rng(seed)
    V = int(np.prod(dims))
    h = rng.standard_normal((4, V, 8))
    return np.einsum("mva,aij->mvij", h, li.gell_mann() / 2)


@pytest.mark.parametrize("alpha", [hyp.HYP_ALPHA, (0.5, 0.3, 0.9)])
def test_first_order_matches_momentum_space_form_factor(alpha):
    dims = DIMS
    X, Y, Z, T = dims
    A = _random_hermitian_field(dims, 12)
    B = _first_order(dims, A, alpha, 1e-6)
    Ah = np.fft.fftn(A.reshape(4, T, Z, Y, X, 3, 3), axes=(1, 2, 3, 4))
    kt, kz, ky, kx = np.meshgrid(*(2 * np.pi * np.arange(n) / n for n in (T, Z, Y, X)), indexing="ij")
    k = [q[..., None, None] for q in (kx, ky, kz, kt)]
    Bh = _form_factor([Ah[m] for m in range(4)], k, alpha)
    Bref = np.fft.ifftn(np.array(Bh), axes=(1, 2, 3, 4)).reshape(B.shape)
    assert np.max(np.abs(B - Bref)) / np.max(np.abs(Bref)) < 1e-4


def test_fat7_equivalent_weights_cancel_taste_changing_momenta():
    # a perturbation along direction mu with momentum pi in some transverse directions (0 along mu)
    # leaves the smeared mu link unchanged at first order for weights (7/8, 4/7, 1/4), not otherwise
    dims = DIMS
    c = coords(dims)  # [V][4]
    lam3 = li.gell_mann()[2] / 2
    for mu in (0, 3):
        trans = [d for d in range(4) if d != mu]
        for bits in ((1, 0, 0), (0, 1, 1), (1, 1, 1)):
            phase = np.cos(np.pi * sum(b * c[:, d] for b, d in zip(bits, trans)))
            A = np.zeros((4, c.shape[0], 3, 3), np.complex128)
            A[mu] = phase[:, None, None] * lam3
            Bf = _first_order(dims, A, (7 / 8, 4 / 7, 1 / 4), 1e-6)
            Bs = _first_order(dims, A, hyp.HYP_ALPHA, 1e-6)
            assert np.max(np.abs(Bf[mu])) < 1e-5
            assert np.max(np.abs(Bs[mu])) > 1e-2
