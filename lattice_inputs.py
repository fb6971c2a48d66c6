"""Seeded synthetic inputs for the staggered even-odd CG: gauge links, sources, gauge transforms.

This module is the one thing the FP64 oracle and the GPU path share. It draws random numbers and shapes
them into lattice fields; it contains none of the solver's arithmetic (no Dirac operator, no CG, no
reductions, no gradient).

The paper benchmarks its CG on MILC asqtad 20^3x64 coarse lattices with HYP-smeared links (Sec. 3,
Fig. 1 and Table 2). Those ensembles are not available, so unitary SU(3) fields with the same shape
stand in for them:

* ``haar_links``: every link an independent Haar-random SU(3) matrix (QR of a complex Gaussian matrix,
  column phases fixed by R's diagonal, then the determinant divided out with its principal cube root).
* ``near_identity_links``: U = exp(i * eps * H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0, 1) and the
  Gell-Mann matrices lambda_a, followed by re-unitarisation (Gram-Schmidt of rows 0 and 1,
  row 2 = conj(row0 x row1)) so that det U = 1 to rounding. With eps = 0.3 this mimics smeared links
  (mean (1/3) Re tr U ~ 0.94).

Layouts (natural, complex128, the C-ABI layout):
* links ``[4][V][3][3]``: direction mu = 0..3 = x, y, z, t; site lex = x + X*(y + Y*(z + Z*t));
* even-site vectors ``[V/2][3]`` indexed by cb = lex >> 1 over sites with (x+y+z+t) even;
* full vectors ``[V][3]`` indexed by lex.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "gell_mann", "volume", "haar_su3", "near_identity_su3", "haar_links", "near_identity_links",
    "gaussian_even_source", "gaussian_vector", "random_gauge_transform", "BatchSystem", "uneven_batch",
    "cfg1", "cfg0", "cfg4",
]


def volume(dims) -> int:
    X, Y, Z, T = (int(d) for d in dims)
    return X * Y * Z * T


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices lambda_a, shape [8][3][3] complex128."""
    l = np.zeros((8, 3, 3), dtype=np.complex128)
    l[0][0, 1] = l[0][1, 0] = 1
    l[1][0, 1], l[1][1, 0] = -1j, 1j
    l[2][0, 0], l[2][1, 1] = 1, -1
    l[3][0, 2] = l[3][2, 0] = 1
    l[4][0, 2], l[4][2, 0] = -1j, 1j
    l[5][1, 2] = l[5][2, 1] = 1
    l[6][1, 2], l[6][2, 1] = -1j, 1j
    l[7][0, 0] = l[7][1, 1] = 1 / np.sqrt(3)
    l[7][2, 2] = -2 / np.sqrt(3)
    return l


def _complex_gaussian(rng: np.random.Generator, shape) -> np.ndarray:
    """(N(0,1) + i N(0,1)) / sqrt(2) per component."""
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    return (re + 1j * im) / np.sqrt(2.0)


def _reunitarize(m: np.ndarray) -> np.ndarray:
    """Project [..., 3, 3] onto SU(3): Gram-Schmidt rows 0 and 1, row 2 = conj(row0 x row1)."""
    r0 = m[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = m[..., 1, :]
    r1 = r1 - np.sum(np.conj(r0) * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.conj(np.cross(r0, r1))
    return np.stack([r0, r1, r2], axis=-2)


def haar_su3(n: int, rng: np.random.Generator) -> np.ndarray:
    """n Haar-distributed SU(3) matrices, [n][3][3] complex128."""
    z = _complex_gaussian(rng, (n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[..., None, :]
    det = np.linalg.det(q)
    q = q * (det ** (-1.0 / 3.0))[..., None, None]
    return q


def near_identity_su3(n: int, eps: float, rng: np.random.Generator) -> np.ndarray:
    """n matrices exp(i eps H), H = sum_a h_a lambda_a / 2, re-unitarised; [n][3][3] complex128."""
    h = rng.standard_normal((n, 8))
    H = (h @ (gell_mann() / 2.0).reshape(8, 9)).reshape(n, 3, 3)
    w, v = np.linalg.eigh(H)
    u = (v * np.exp(1j * eps * w)[:, None, :]) @ np.conj(np.swapaxes(v, -1, -2))
    return _reunitarize(u)


def haar_links(dims, seed: int) -> np.ndarray:
    """Haar SU(3) links, [4][V][3][3] complex128."""
    rng = np.random.default_rng(seed)
    V = volume(dims)
    return np.ascontiguousarray(haar_su3(4 * V, rng).reshape(4, V, 3, 3))


def near_identity_links(dims, eps: float, seed: int) -> np.ndarray:
    """Near-identity SU(3) links exp(i eps H), [4][V][3][3] complex128."""
    rng = np.random.default_rng(seed)
    V = volume(dims)
    return np.ascontiguousarray(near_identity_su3(4 * V, eps, rng).reshape(4, V, 3, 3))


def gaussian_even_source(dims, seed: int) -> np.ndarray:
    """Complex Gaussian even-site colour vector, [V/2][3] complex128."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_complex_gaussian(rng, (volume(dims) // 2, 3)))


def gaussian_vector(n_sites: int, seed: int) -> np.ndarray:
    """Complex Gaussian colour vector on n_sites sites, [n_sites][3] complex128."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(_complex_gaussian(rng, (n_sites, 3)))


def random_gauge_transform(dims, seed: int) -> np.ndarray:
    """Haar SU(3) matrix per site, [V][3][3] complex128 (for covariance checks)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(haar_su3(volume(dims), rng))


# ---------------------------------------------------------------------------------------------------------
# Named workloads. Dimensions, link recipes, masses and seeds of the benchmark configurations.
# ---------------------------------------------------------------------------------------------------------

def cfg0():
    """4^4, Haar links (seed 11), m = 0.1, one Gaussian even source (seed 12); FP64 CG to 1e-10."""
    dims = (4, 4, 4, 4)
    return dict(dims=dims, links=haar_links(dims, 11), mass=0.1, source=gaussian_even_source(dims, 12),
                tol=1e-10)


def cfg1(dims=(20, 20, 20, 64)):
    """20^3x64 near-identity links (eps 0.3, seed 21), m = 0.01, Gaussian source (seed 22); to 1e-8."""
    return dict(dims=tuple(dims), links=near_identity_links(dims, 0.3, 21), mass=0.01,
                source=gaussian_even_source(dims, 22), tol=1e-8)


def cfg4(dims=(16, 16, 16, 32), link_seed=41, src_seed=42):
    """16^3x32 near-identity links (eps 0.3), m = 0.05, Gaussian phi; loss Re phi^dag A^-1 phi."""
    return dict(dims=tuple(dims), links=near_identity_links(dims, 0.3, link_seed), mass=0.05,
                source=gaussian_even_source(dims, src_seed))


class BatchSystem:
    """One system of a batch: geometry, index of its gauge field, mass and source."""

    def __init__(self, dims, gauge_index: int, mass: float, source: np.ndarray):
        self.dims = tuple(int(d) for d in dims)
        self.gauge_index = int(gauge_index)
        self.mass = float(mass)
        self.source = source


def uneven_batch(big_dims=(20, 20, 20, 64), n_big=8, n_each=8,
                 small_dims=((8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32))):
    """The batched workload: n_big Gaussian sources on big_dims (links seed 21, sources seed 31+k,
    m = 0.01) plus n_each systems on each of small_dims (one near-identity gauge field per size,
    seeds 32, 33, 34; masses uniform in [0.01, 0.1] from seed 35; sources seeded 3500 + index).

    Returns (gauges, systems): gauges is a list of (dims, links) and systems a list of BatchSystem.
    """
    gauges = []
    systems = []
    if n_big > 0:
        gauges.append((tuple(big_dims), near_identity_links(big_dims, 0.3, 21)))
        for k in range(n_big):
            systems.append(BatchSystem(big_dims, 0, 0.01, gaussian_even_source(big_dims, 31 + k)))
    mass_rng = np.random.default_rng(35)
    masses = mass_rng.uniform(0.01, 0.1, size=n_each * len(small_dims))
    idx = 0
    for s, dims in enumerate(small_dims):
        gauges.append((tuple(dims), near_identity_links(dims, 0.3, 32 + s)))
        g = len(gauges) - 1
        for _ in range(n_each):
            systems.append(BatchSystem(dims, g, masses[idx], gaussian_even_source(dims, 3500 + idx)))
            idx += 1
    return gauges, systems
