"""HYP smearing of SU(3) links, FP64 numpy oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this module; the GPU
library does not load it and nothing falls back to it.

The paper solves for "HYP-smeared" staggered quarks (Sec. 3) without defining the smearing. The definition
written out here is the hypercubic blocking of Hasenfratz and Knechtli (Phys. Rev. D 64 (2001) 034504):
three levels of staple smearing, each level's staples built only from links of the hypercubes that contain
the link being smeared, each sum projected back to SU(3):

  level 1, for the link (x, mu) and a staple direction eta != mu (the two remaining directions are the
  ones the decorated link excludes):
      W = (1 - a3) U_mu(x) + a3/2 * sum over +-eta of the staple of U_eta around U_mu
  level 2, for (x, mu) excluding nu != mu:  staples in the two directions rho not in {mu, nu}, built from
      level-1 links that exclude {rho, nu} (the mu link) and {nu, mu} (the rho links):
      W = (1 - a2) U_mu(x) + a2/4 * sum over +-rho
  level 3, for (x, mu): staples in the three directions nu != mu, built from level-2 links that exclude
      nu (the mu link) and mu (the nu links):
      W = (1 - a1) U_mu(x) + a1/6 * sum over +-nu

The staple of side links S and top links T around the link (x, mu), for direction eta, is
      S_eta(x) T_mu(x+eta) S_eta(x+mu)^dag  +  S_eta(x-eta)^dag T_mu(x-eta) S_eta(x-eta+mu).

Proj_SU(3)(W) is the SU(3) matrix X that maximises Re tr(X^dag W) (the projection of the original
definition). It is computed from the start X0 = unitary polar factor W (W^dag W)^(-1/2) divided by the
cube root (principal branch) of its determinant, by repeated maximisation over the three SU(2) subgroups
(Cabibbo-Marinari) until a sweep no longer changes X. The smearing is gauge-field-only, so every
direction is periodic (a fermion boundary sign is not a property of the links).

Layout: links [4][V][3][3] complex128 over lexicographic sites lex = x + X(y + Y(z + Z t)).
"""
from __future__ import annotations

import numpy as np

HYP_ALPHA = (0.75, 0.6, 0.3)  # (a1, a2, a3): the standard values of Hasenfratz and Knechtli

_AXIS = (3, 2, 1, 0)  # direction mu -> axis of a field reshaped to [T][Z][Y][X]


def shift(f: np.ndarray, mu: int, s: int, dims) -> np.ndarray:
    """g(x) = f(x + s mu-hat), periodic, for a field f[V][...] over lexicographic sites."""
    X, Y, Z, T = dims
    g = f.reshape((T, Z, Y, X) + f.shape[1:])
    return np.roll(g, -s, axis=_AXIS[mu]).reshape(f.shape)


def dag(a: np.ndarray) -> np.ndarray:
    return np.conj(np.swapaxes(a, -1, -2))


def staples(side: np.ndarray, top: np.ndarray, mu: int, eta: int, dims) -> np.ndarray:
    """Forward plus backward staple in direction eta around (x, mu); side, top are [V][3][3] fields of
    links in directions eta and mu."""
    fwd = side @ shift(top, eta, +1, dims) @ dag(shift(side, mu, +1, dims))
    sb = shift(side, eta, -1, dims)  # S_eta(x - eta)
    bwd = dag(sb) @ shift(top, eta, -1, dims) @ shift(sb, mu, +1, dims)
    return fwd + bwd


def polar_start(W: np.ndarray) -> np.ndarray:
    """The unitary polar factor W (W^dag W)^(-1/2) = P Q^dag from the singular value decomposition
    W = P S Q^dag, times the inverse cube root (principal branch) of its determinant."""
    P, _, Qh = np.linalg.svd(W)
    X = P @ Qh
    theta = np.angle(np.linalg.det(X))
    return X * np.exp(-1j * theta / 3.0)[..., None, None]


_SUBGROUPS = ((0, 1), (0, 2), (1, 2))


def su2_step(X: np.ndarray, W: np.ndarray, i: int, j: int) -> np.ndarray:
    """X -> g X with g in the SU(2) subgroup on rows (i, j) maximising Re tr((g X)^dag W)."""
    M = W @ dag(X)
    # Re tr(h^dag A) over h = b0 + i b.sigma in SU(2) is 2 (b0 Re A0 + b . Re A) with A = A0 + i A.sigma
    a0 = 0.5 * np.real(M[..., i, i] + M[..., j, j])
    a1 = 0.5 * np.imag(M[..., i, j] + M[..., j, i])
    a2 = 0.5 * np.real(M[..., i, j] - M[..., j, i])
    a3 = 0.5 * np.imag(M[..., i, i] - M[..., j, j])
    n = np.sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3)
    b0, b1, b2, b3 = a0 / n, a1 / n, a2 / n, a3 / n
    # h = b0 + i (b1 sigma1 + b2 sigma2 + b3 sigma3)
    h00, h01 = b0 + 1j * b3, b2 + 1j * b1
    h10, h11 = -b2 + 1j * b1, b0 - 1j * b3
    Xi, Xj = X[..., i, :].copy(), X[..., j, :].copy()
    out = X.copy()
    out[..., i, :] = h00[..., None] * Xi + h01[..., None] * Xj
    out[..., j, :] = h10[..., None] * Xi + h11[..., None] * Xj
    return out


def proj_su3(W: np.ndarray, max_sweeps: int = 500, tol: float = 1e-15) -> np.ndarray:
    """argmax over X in SU(3) of Re tr(X^dag W), from the polar start, by SU(2)-subgroup sweeps; each
    matrix stops at the first sweep that moves none of its elements by more than tol (so its result
    depends on its own W only)."""
    X = polar_start(W)
    live = np.ones(W.shape[:-2], dtype=bool)
    for _ in range(max_sweeps):
        Y = X[live]
        Wl = W[live]
        for i, j in _SUBGROUPS:
            Y = su2_step(Y, Wl, i, j)
        moved = np.max(np.abs(Y - X[live]), axis=(-2, -1)) > tol
        X[live] = Y
        idx = np.flatnonzero(live.ravel())
        flat = live.ravel()
        flat[idx[~moved]] = False
        live = flat.reshape(live.shape)
        if not live.any():
            break
    return X


def hyp_smear(dims, U: np.ndarray, alpha=HYP_ALPHA, max_sweeps: int = 500) -> np.ndarray:
    """HYP-smeared links V[4][V][3][3] of U[4][V][3][3] with alpha = (a1, a2, a3)."""
    a1, a2, a3 = alpha
    U = np.asarray(U, dtype=np.complex128)
    proj = lambda W: proj_su3(W, max_sweeps)  # noqa: E731
    # level 1: lv1[mu][eta], the mu link dressed with staples in direction eta
    lv1 = {}
    for mu in range(4):
        for eta in range(4):
            if eta != mu:
                lv1[mu, eta] = proj((1.0 - a3) * U[mu] + (a3 / 2.0) * staples(U[eta], U[mu], mu, eta, dims))
    # level 2: lv2[mu][nu], the mu link excluding nu
    lv2 = {}
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            s = np.zeros_like(U[mu])
            for rho in range(4):
                if rho in (mu, nu):
                    continue
                sigma = 6 - mu - nu - rho  # the direction outside {mu, nu, rho}
                s += staples(lv1[rho, sigma], lv1[mu, sigma], mu, rho, dims)
            lv2[mu, nu] = proj((1.0 - a2) * U[mu] + (a2 / 4.0) * s)
    # level 3
    V = np.empty_like(U)
    for mu in range(4):
        s = np.zeros_like(U[mu])
        for nu in range(4):
            if nu != mu:
                s += staples(lv2[nu, mu], lv2[mu, nu], mu, nu, dims)
        V[mu] = proj((1.0 - a1) * U[mu] + (a1 / 6.0) * s)
    return V
