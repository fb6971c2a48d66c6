"""Packed link layouts, byte for byte: `sp_gauge_pack` of a gauge field against a numpy rendering of the layout
that `include/sp_api.h` and the kernels use, with the conversions written out.

Layout: 8 blocks, block (parity q, direction mu) at position 4 q + mu, each holding the V/2 links U_mu(n) of the
sites of parity q in checkerboard order (cb = lex / 2), split into planes of words, the reals of a link numbered
r[2k] = Re U[k / 3][k % 3], r[2k + 1] = Im U[k / 3][k % 3] (recon 12 keeps k < 6):
  FP64 r18: 9 planes of (r[2k], r[2k + 1]) as double2;
  FP32: planes of float4 (r[4k .. 4k + 3]), and for recon 18 a last plane of float2 (r[16], r[17]); recon 8:
  two planes of float4, (r[2], r[3], r[4], r[5]) and (S, atan2(r[1], r[0]), f), S = (r[6], r[7]) = U10 and
  f = atan2(r[13], r[12]) where |U10| <= |U20|, else S = (r[12], r[13]) = U20 and f = atan2(r[7], r[6]) + 8;
  16-bit (FP16, BF16, fixed point): word k = code(r[2k]) | code(r[2k + 1]) << 16; words 0-3 in a plane of uint4,
  then words 4-5 in a plane of uint2 (recon 12), or words 4-7 in a uint4 plane and word 8 in a uint32 plane.
Codes: the FP64 real rounded to FP32 (nearest even), then FP16 nearest even, BF16 nearest even, or fixed point
rint(32767 f) in FP32 clamped to [-32767, 32767]. Integer and byte work, so the comparison is exact."""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import paper_1511_00088_amd as sp
from gpu_common import DEV, announce, to_dev

pytestmark = pytest.mark.gpu


def _codes16(r32: np.ndarray, prec: str) -> np.ndarray:
    """16-bit codes of FP32 values."""
    if prec == "f16":
        return r32.astype(np.float16).view(np.uint16).astype(np.uint32)
    if prec == "bf16":
        u = r32.view(np.uint32).astype(np.uint64)
        return (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) & 0xFFFF).astype(np.uint32)
    q = np.clip(np.rint(r32 * np.float32(32767.0)), -32767, 32767).astype(np.int16)
    return q.view(np.uint16).astype(np.uint32)


def _reference(U: np.ndarray, dims, prec: str, recon: int) -> bytes:
    X, Y, Z, T = dims
    V = X * Y * Z * T
    Vh = V // 2
    lex = np.arange(V)
    x, y, z, t = lex % X, (lex // X) % Y, (lex // (X * Y)) % Z, lex // (X * Y * Z)
    q = (x + y + z + t) & 1
    cb = lex >> 1
    reals = np.stack([U.real, U.imag], axis=-1).reshape(4, V, 18)  # entry k = (row, col) row-major, then re, im
    nreal = 18 if prec == "f64" else recon
    blocks = []
    for par in (0, 1):
        sel = np.nonzero(q == par)[0]
        order = sel[np.argsort(cb[sel])]
        assert np.array_equal(cb[order], np.arange(Vh))
        for mu in range(4):
            r = reals[mu, order, :nreal]  # [Vh, nreal] in cb order
            if prec == "f64":
                planes = [np.ascontiguousarray(r[:, 2 * k:2 * k + 2]) for k in range(9)]
            elif prec == "f32" and recon == 8:
                full = reals[mu, order, :18]
                s20 = full[:, 12] ** 2 + full[:, 13] ** 2 < full[:, 6] ** 2 + full[:, 7] ** 2
                p1 = np.stack([np.where(s20, full[:, 12], full[:, 6]), np.where(s20, full[:, 13], full[:, 7]),
                               np.arctan2(full[:, 1], full[:, 0]),
                               np.where(s20, np.arctan2(full[:, 7], full[:, 6]) + 8.0,
                                        np.arctan2(full[:, 13], full[:, 12]))], axis=1)
                planes = [np.ascontiguousarray(full[:, 2:6].astype(np.float32)),
                          np.ascontiguousarray(p1.astype(np.float32))]
            elif prec == "f32":
                r32 = r.astype(np.float32)
                planes = [np.ascontiguousarray(r32[:, 4 * k:4 * k + 4]) for k in range(nreal // 4)]
                if recon == 18:
                    planes.append(np.ascontiguousarray(r32[:, 16:18]))
            else:
                c = _codes16(r.astype(np.float32), prec)
                w = (c[:, 0::2] | (c[:, 1::2] << 16)).astype(np.uint32)  # word k from reals 2k, 2k + 1
                planes = [np.ascontiguousarray(w[:, 0:4])]
                if recon == 18:
                    planes += [np.ascontiguousarray(w[:, 4:8]), np.ascontiguousarray(w[:, 8:9])]
                else:
                    planes.append(np.ascontiguousarray(w[:, 4:6]))
            blocks.append(b"".join(p.tobytes() for p in planes))
    return b"".join(blocks)


def _special_links(dims, seed):
    """A non-unitary field with the values the conversions treat specially: 0, +-1, +-1.5 and +-3 (the fixed
    point clamps), 1e-6 and 1e-9 (FP16 subnormal and underflow), beside Gaussian entries."""
    rng = np.random.default_rng(seed)
    V = li.volume(dims)
    U = rng.normal(size=(4, V, 3, 3)) + 1j * rng.normal(size=(4, V, 3, 3))
    special = np.array([0.0, 1.0, -1.0, 1.5, -1.5, 3.0, -3.0, 1e-6, -1e-9, 0.5, 1.0 / 32767.0])
    mask = rng.random(U.shape) < 0.3
    U.real[mask] = rng.choice(special, size=int(mask.sum()))
    mask = rng.random(U.shape) < 0.3
    U.imag[mask] = rng.choice(special, size=int(mask.sum()))
    return U


@pytest.mark.parametrize("prec,recon", [("f64", 18), ("f32", 18), ("f32", 12), ("f16", 18), ("f16", 12),
                                        ("bf16", 18), ("bf16", 12), ("i16", 18), ("i16", 12)])
@pytest.mark.parametrize("dims", [(4, 6, 2, 8), (2, 2, 2, 2)])
def test_gauge_packing_byte_for_byte(prec, recon, dims):
    announce(f"pack layout {prec} r{recon} dims={dims}")
    lat = sp.Lattice(dims)
    for U in (li.haar_links(dims, 731), _special_links(dims, 732)):
        packed = sp.pack_gauge(lat, to_dev(U), prec, recon)
        assert packed.numel() == lat.gauge_bytes(prec, recon)
        ref = np.frombuffer(_reference(U, dims, prec, recon), dtype=np.uint8)
        got = packed.cpu().numpy()
        assert got.size == ref.size
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, f"{bad.size} bytes differ, first at {bad[:8]}"


@pytest.mark.parametrize("dims", [(4, 6, 2, 8), (2, 2, 2, 2)])
def test_gauge_packing_recon8(dims):
    """FP32 recon 8: plane 0 (U01, U02) and plane 1 (S, arg U00, f) as float4, S the smaller of U10 and U20 in
    modulus and f the other one's phase, plus 8 when S is U20 (both choices occur in both fields). The entries are
    FP32 roundings of the FP64 reals, byte for byte; the phases come from the device's FP64 atan2, which may differ
    from numpy's by an ulp before the rounding to FP32, so they are compared to one FP32 ulp."""
    announce(f"pack layout f32 r8 dims={dims}")
    lat = sp.Lattice(dims)
    for U in (li.haar_links(dims, 736), li.near_identity_links(dims, 0.3, 737)):
        packed = sp.pack_gauge(lat, to_dev(U), "f32", 8)
        assert packed.numel() == lat.gauge_bytes("f32", 8) == 8 * lat.Vh * 32
        got = packed.cpu().numpy().view(np.float32).reshape(8, 2, lat.Vh, 4)
        ref = np.frombuffer(_reference(U, dims, "f32", 8), dtype=np.float32).reshape(8, 2, lat.Vh, 4)
        assert np.array_equal(got[:, 0], ref[:, 0]) and np.array_equal(got[:, 1, :, :2], ref[:, 1, :, :2])
        ulp = np.spacing(np.abs(ref[:, 1, :, 2:]).astype(np.float32))
        assert (np.abs(got[:, 1, :, 2:] - ref[:, 1, :, 2:]) <= ulp).all()
        flagged = got[:, 1, :, 3] > 4.0
        assert flagged.any() and not flagged.all()


def test_gauge_f64_field_of_a_gauge_is_the_recon18_packing():
    """The FP64 field every Gauge carries (used by the reliable updates) is the FP64 recon-18 layout."""
    dims = (4, 6, 2, 8)
    U = li.haar_links(dims, 733)
    G = sp.Gauge(sp.Lattice(dims), to_dev(U), lo_prec="i16", recon=12)
    ref = np.frombuffer(_reference(U, dims, "f64", 18), dtype=np.uint8)
    assert np.array_equal(G.f64.cpu().numpy(), ref)
    assert torch.equal(G.lo, sp.pack_gauge(G.lat, to_dev(U), "i16", 12))
    assert G.lo.device == torch.device(DEV)


# Half vectors (V/2 sites in checkerboard order, colour c = 0, 1, 2):
#   FP64: 3 planes of double2 (Re v_c, Im v_c);
#   FP32: a plane of float4 (v_0, v_1) and a plane of float2 (v_2);
#   FP16: one uint4 per site, words (v_0, v_1, v_2) of 16-bit codes of v_c / n and the FP32 site norm n = the
#         largest |component| (a site with n < 1e-30 is first scaled by 2^64, exactly: the codes are then of
#         (2^64 v) / (2^64 n)); n = 0 stores zeros;
#   BF16: a plane of uint2 (words of v_0, v_1) and a plane of uint32 (v_2), unscaled.
# Every step in FP32 with rounding to nearest even, as the kernel does: the FP64 input to FP32, then the products.
def _vec_reference(v: np.ndarray, prec: str) -> bytes:
    Vh = v.shape[0]
    r = np.stack([v.real, v.imag], axis=-1).reshape(Vh, 6)  # Re v0, Im v0, Re v1, ...
    if prec == "f64":
        return b"".join(np.ascontiguousarray(r[:, 2 * c:2 * c + 2]).tobytes() for c in range(3))
    r32 = r.astype(np.float32)
    if prec == "f32":
        return np.ascontiguousarray(r32[:, 0:4]).tobytes() + np.ascontiguousarray(r32[:, 4:6]).tobytes()
    if prec == "bf16":
        c = _codes16(r32, "bf16")
        w = (c[:, 0::2] | (c[:, 1::2] << 16)).astype(np.uint32)
        return np.ascontiguousarray(w[:, 0:2]).tobytes() + np.ascontiguousarray(w[:, 2:3]).tobytes()
    m = np.abs(r32).max(axis=1).astype(np.float32)
    k = np.where(m < np.float32(1e-30), np.float32(2.0 ** 64), np.float32(1.0)).astype(np.float32)
    with np.errstate(divide="ignore"):
        inv = np.where(m > 0, np.float32(1.0) / (m * k), np.float32(0.0)).astype(np.float32)
    scaled = (inv[:, None] * (k[:, None] * r32)).astype(np.float32)
    c = _codes16(scaled, "f16")
    w = (c[:, 0::2] | (c[:, 1::2] << 16)).astype(np.uint32)
    words = np.concatenate([w, m.view(np.uint32)[:, None]], axis=1)
    return np.ascontiguousarray(words).tobytes()


def _special_vector(n, seed):
    """Gaussian sites beside sites of zeros, of a norm below 1e-30, of mixed scales and of exact powers of two."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(n, 3)) + 1j * rng.normal(size=(n, 3))
    v[1] = 0.0
    v[2] = 3e-35 * (rng.normal(size=3) + 1j * rng.normal(size=3))
    v[3] = np.array([1e20, 1e-20, -0.5]) + 1j * np.array([2.0 ** -30, -1.0, 0.0])
    v[4] = np.array([1.0, 0.5, 0.25]) - 1j * np.array([0.125, 2.0, -4.0])
    v[5:9] *= 1e-12
    return v


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_vector_packing_byte_for_byte(prec):
    dims = (4, 6, 2, 8)
    lat = sp.Lattice(dims)
    for v in (li.gaussian_vector(lat.Vh, 734), _special_vector(lat.Vh, 735)):
        packed = sp.pack_vec(lat, to_dev(v), prec)
        assert packed.numel() == lat.vec_bytes(prec)
        ref = np.frombuffer(_vec_reference(v, prec), dtype=np.uint8)
        got = packed.cpu().numpy()
        bad = np.nonzero(got != ref)[0]
        assert bad.size == 0, f"{prec}: {bad.size} bytes differ, first at {bad[:8]}"
