"""One-colour-trace four-fermion contraction of the NPR code, FP64 numpy oracle -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this module; the GPU
library does not load it and nothing falls back to it.

The contraction is the general one-colour-trace operator of the paper's Eq. (1), Sec. 4: per hypercube z
(sites z_A = 2z + A, A in {0,1}^4) and per field set i,

  O_i(z) = sum_{A,B,C,D} M1_{AB} M2_{CD}  [chib1(z_A)^T U_{AD}(z) chi4(z_D)]  [chib3(z_C)^T U_{CB}(z) chi2(z_B)]

with chib^T U chi = sum_{c,c'} chib_c U_{cc'} chi_{c'}: colour c1 of the first bilinear's antiquark is tied to
colour c4 of the second bilinear's quark by U_{AD}, and c3 to c2 by U_{CB} (a single colour trace around the
four fields and two links). The paper prints the formula only; the conventions below are the readings taken:

* spin-taste matrices in the hypercube basis, M_{AB} = (1/4) tr(gamma_A^dag gamma_S gamma_B gamma_F^dag) with
  gamma_A = g1^A1 g2^A2 g3^A3 g4^A4 for Hermitian Euclidean Dirac matrices (the trace does not depend on the
  representation); S and F are 4-bit spin and taste labels;
* U_{AD}(z): the average over all shortest lattice paths from z_A to z_D inside the hypercube of the ordered
  product of links along the path (a step +mu from site x uses U_mu(x), a step -mu uses U_mu(x - mu)^dag);
  U_{AA} = 1;
* the fields chib and chi are given complex colour fields [n][V][3] (in the NPR code they are the quark
  propagators with their external labels folded into i); no conjugation is implied by the bar.

Layout: links [4][V][3][3] complex128 over lexicographic sites lex = x + X(y + Y(z + Z t)); hypercubes
ordered lexicographically on the coarse lattice (X/2, Y/2, Z/2, T/2); corner index A = A0 + 2 A1 + 4 A2 + 8 A3.
"""
from __future__ import annotations

import itertools

import numpy as np


def euclidean_gammas() -> np.ndarray:
    """Hermitian Euclidean Dirac matrices g1..g4 (chiral representation), [4][4][4]."""
    s = [np.array([[0, 1], [1, 0]], complex), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]], complex)]
    z = np.zeros((2, 2), complex)
    g = []
    for k in range(3):
        g.append(np.block([[z, -1j * s[k]], [1j * s[k], z]]))
    g.append(np.block([[z, np.eye(2)], [np.eye(2), z]]))
    return np.array(g)


def gamma_of(bits, g=None) -> np.ndarray:
    """g1^b0 g2^b1 g3^b2 g4^b3 for a corner / label index bits (int 0..15 or 4 bits)."""
    if g is None:
        g = euclidean_gammas()
    if isinstance(bits, (int, np.integer)):
        bits = [(int(bits) >> k) & 1 for k in range(4)]
    out = np.eye(4, dtype=complex)
    for mu in range(4):
        if bits[mu]:
            out = out @ g[mu]
    return out


def spin_taste(S: int, F: int) -> np.ndarray:
    """M_{AB} = (1/4) tr(gamma_A^dag gamma_S gamma_B gamma_F^dag), [16][16]."""
    g = euclidean_gammas()
    gS, gF = gamma_of(S, g), gamma_of(F, g)
    M = np.empty((16, 16), complex)
    for A in range(16):
        gA = gamma_of(A, g)
        for B in range(16):
            M[A, B] = 0.25 * np.trace(gA.conj().T @ gS @ gamma_of(B, g) @ gF.conj().T)
    return M


def _corner_coords(dims):
    X, Y, Z, T = dims
    Lc = (X // 2, Y // 2, Z // 2, T // 2)
    nz = Lc[0] * Lc[1] * Lc[2] * Lc[3]
    zc = np.stack(np.unravel_index(np.arange(nz), Lc[::-1])[::-1], axis=1)  # [nz][4] coarse (x,y,z,t)
    return Lc, nz, zc


def _lex(dims, c):
    X, Y, Z, T = dims
    c = np.asarray(c) % np.array(dims)
    return c[..., 0] + X * (c[..., 1] + Y * (c[..., 2] + Z * c[..., 3]))


def corner_sites(dims) -> np.ndarray:
    """lex index of z_A for every hypercube z and corner A, [nz][16]."""
    _, nz, zc = _corner_coords(dims)
    out = np.empty((nz, 16), np.int64)
    for A in range(16):
        a = np.array([(A >> k) & 1 for k in range(4)])
        out[:, A] = _lex(dims, 2 * zc + a)
    return out


def path_links(dims, U: np.ndarray) -> np.ndarray:
    """U_{AD}(z) for every hypercube, [nz][16][16][3][3]: the average over shortest paths of link products."""
    _, nz, zc = _corner_coords(dims)
    out = np.empty((nz, 16, 16, 3, 3), complex)
    for A in range(16):
        a = np.array([(A >> k) & 1 for k in range(4)])
        for D in range(16):
            d = np.array([(D >> k) & 1 for k in range(4)])
            dirs = [mu for mu in range(4) if a[mu] != d[mu]]
            acc = np.zeros((nz, 3, 3), complex)
            paths = list(itertools.permutations(dirs))
            for path in paths:
                prod = np.broadcast_to(np.eye(3, dtype=complex), (nz, 3, 3)).copy()
                pos = 2 * zc + a
                for mu in path:
                    if a[mu] == 0:  # step +mu
                        prod = prod @ U[mu][_lex(dims, pos)]
                        pos = pos.copy()
                        pos[:, mu] += 1
                    else:  # step -mu
                        pos = pos.copy()
                        pos[:, mu] -= 1
                        prod = prod @ np.conj(np.swapaxes(U[mu][_lex(dims, pos)], -1, -2))
                acc += prod
            out[:, A, D] = acc / len(paths)
    return out


def contract(dims, UAD: np.ndarray, chib1, chi2, chib3, chi4, S1: int, F1: int, S2: int, F2: int) -> np.ndarray:
    """O_i(z), [n][nz], for fields [n][V][3] and path links from path_links()."""
    cs = corner_sites(dims)
    M1, M2 = spin_taste(S1, F1), spin_taste(S2, F2)
    f = [np.asarray(v, complex)[:, cs] for v in (chib1, chi2, chib3, chi4)]  # [n][nz][16][3]
    # P14[n,z,A,D] = chib1(z_A)^T U_AD chi4(z_D);  P32[n,z,C,B] = chib3(z_C)^T U_CB chi2(z_B)
    P14 = np.einsum("nzac,zadce,nzde->nzad", f[0], UAD, f[3])
    P32 = np.einsum("nzcp,zcbpe,nzbe->nzcb", f[2], UAD, f[1])
    return np.einsum("ab,cd,nzad,nzcb->nz", M1, M2, P14, P32)
