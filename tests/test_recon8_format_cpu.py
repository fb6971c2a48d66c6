"""The recon-8 link format on the host: an FP32 numpy rendering of what the packing stores and of the unitarity
formulas the kernels rebuild the link from, over every link of the 20^3x64 near-identity workload field.

Stored: U01, U02, S = the smaller in modulus of U10 and U20, arg U00, and the phase f of the other one (L), plus 8
when S is U20. Rebuilt: n = |U01|^2 + |U02|^2, |U00| = sqrt(1 - n), |L| = sqrt(n - |S|^2), and from row 1 and row
2 orthogonal to row 0 with det U = 1:
  U11 = -(conj U20 conj U02 + U01 U10 conj U00) / n,   U12 = (conj U01 conj U20 - U02 U10 conj U00) / n,
  U21 = (conj U10 conj U02 - U01 U20 conj U00) / n,    U22 = -(U02 U20 conj U00 + conj U01 conj U10) / n.
Pins: every rebuilt entry within 1e-6 of the FP64 link (the FP32 operator's gate), and the alternative that
always stores U10 (rebuilding |U20| from the difference of squares) worse than 1e-5 on the same field, which is
why the smaller entry is stored."""
import numpy as np

import lattice_inputs as li

f32 = np.float32


def _rebuild(U, choose_smaller):
    a2 = U[:, 0, 1].astype(np.complex64)
    a3 = U[:, 0, 2].astype(np.complex64)
    s20 = (np.abs(U[:, 2, 0]) < np.abs(U[:, 1, 0])) if choose_smaller else np.zeros(len(U), bool)
    S = np.where(s20, U[:, 2, 0], U[:, 1, 0]).astype(np.complex64)
    f = np.where(s20, np.angle(U[:, 1, 0]) + 8.0, np.angle(U[:, 2, 0])).astype(f32)
    ph0 = np.angle(U[:, 0, 0]).astype(f32)
    flag = f > f32(4)
    f = np.where(flag, f - f32(8), f).astype(f32)
    n = (a2.real * a2.real + a2.imag * a2.imag + a3.real * a3.real + a3.imag * a3.imag).astype(f32)
    r0 = np.sqrt(np.maximum(f32(1) - n, f32(0)))
    rl = np.sqrt(np.maximum(n - (S.real * S.real + S.imag * S.imag), f32(0)))
    a1 = (r0 * np.cos(ph0) + 1j * r0 * np.sin(ph0)).astype(np.complex64)
    L = (rl * np.cos(f) + 1j * rl * np.sin(f)).astype(np.complex64)
    b1 = np.where(flag, L, S)
    c1 = np.where(flag, S, L)
    inv = (f32(1) / n).astype(f32)
    cj = np.conj
    R = np.empty(U.shape, np.complex64)
    R[:, 0] = np.stack([a1, a2, a3], -1)
    R[:, 1, 0], R[:, 2, 0] = b1, c1
    R[:, 1, 1] = -(cj(c1) * cj(a3) + a2 * b1 * cj(a1)) * inv
    R[:, 1, 2] = (cj(a2) * cj(c1) - a3 * b1 * cj(a1)) * inv
    R[:, 2, 1] = (cj(b1) * cj(a3) - a2 * c1 * cj(a1)) * inv
    R[:, 2, 2] = -(a3 * c1 * cj(a1) + cj(a2) * cj(b1)) * inv
    return np.abs(R.astype(np.complex128) - U).max()


def test_recon8_rebuild_error_on_the_workload_field():
    U = li.near_identity_links((20, 20, 20, 64), 0.3, 21).reshape(-1, 3, 3)
    assert _rebuild(U, True) <= 1e-6
    assert _rebuild(U, False) > 1e-5


def test_recon8_rebuild_on_haar_links():
    """On Haar links (|U00| spread over [0, 1]) the rebuilt entries stay within 1e-5 of the links."""
    U = li.haar_links((4, 4, 4, 4), 101).reshape(-1, 3, 3)
    assert _rebuild(U, True) <= 1e-5
