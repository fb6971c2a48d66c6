"""Lattice bookkeeping used by the tests (index maps, parity masks, gauge transforms).

These helpers move data between layouts and build transformed inputs; none of them evaluates the
staggered operator.
"""
import numpy as np


def coords(dims):
    """[V][4] coordinates (x, y, z, t) in lex order, lex = x + X*(y + Y*(z + Z*t))."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel(), t.ravel()], axis=1)


def parity(dims):
    return coords(dims).sum(axis=1) % 2


def lex_of(dims, n):
    X, Y, Z, T = dims
    n = np.asarray(n)
    return n[..., 0] + X * (n[..., 1] + Y * (n[..., 2] + Z * n[..., 3]))


def shift_lex(dims, mu, d):
    """lex index of n + d*mu_hat for every lex n."""
    c = coords(dims)
    c[:, mu] = (c[:, mu] + d) % dims[mu]
    return lex_of(dims, c)


def to_full(dims, half, p):
    """Embed a parity-p half vector [V/2][3] into a full vector [V][3] (zeros elsewhere)."""
    V = int(np.prod(dims))
    full = np.zeros((V, 3), np.complex128)
    lex = np.arange(V)
    sel = parity(dims) == p
    full[lex[sel]] = half[lex[sel] >> 1]
    return full


def to_half(dims, full, p):
    V = int(np.prod(dims))
    lex = np.arange(V)
    sel = parity(dims) == p
    half = np.zeros((V // 2, 3), np.complex128)
    half[lex[sel] >> 1] = full[lex[sel]]
    return half


def gauge_transform_links(dims, U, G):
    """U'_mu(n) = G(n) U_mu(n) G(n+mu)^dag."""
    Up = np.empty_like(U)
    for mu in range(4):
        fw = shift_lex(dims, mu, +1)
        Up[mu] = G @ U[mu] @ np.conj(np.swapaxes(G[fw], -1, -2))
    return Up


def gauge_transform_vec(G, v):
    """v'(n) = G(n) v(n) for a full vector; for a half vector pass the matching rows of G."""
    return np.einsum("nij,nj->ni", G, v)


def half_rows(dims, G, p):
    """Rows of a per-site field [V]... restricted to parity p, in cb order."""
    V = int(np.prod(dims))
    lex = np.arange(V)
    sel = parity(dims) == p
    out = np.empty((V // 2,) + G.shape[1:], G.dtype)
    out[lex[sel] >> 1] = G[lex[sel]]
    return out


def dense_operator(apply, n):
    """Dense matrix of a linear map on C^n given as apply(vec) -> vec (vectors flattened)."""
    M = np.empty((n, n), np.complex128)
    for k in range(n):
        e = np.zeros(n, np.complex128)
        e[k] = 1.0
        M[:, k] = apply(e)
    return M
