"""GPU parity of the t-cut shard path (one GPU's share of the paper's multi-GPU CG, Sec. 3 / Fig. 2): face pack,
exchange, face unpack and the halo-fed half operator, through the C-ABI, against the FP64 oracle.

The loopback runs every shard's part on this GPU: the neighbouring slabs of a global field are packed as their
own shards, their faces are packed and copied (standing in for the transfer), unpacked into the ghost slices of
the shard under test, and the operator runs on its interior and then its boundary slices. Its output must match
the oracle's global half operator at the shard's sites, element by element, at the operator tolerances.
"""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1511_00088_amd as sp
from conftest import rel_err_max
from gpu_common import DEV, DSLASH_TOL, announce, to_dev, to_host

pytestmark = pytest.mark.gpu

# (vector precision, link precision, recon)
PACKINGS = [("f64", "f64", 18), ("f32", "f32", 12), ("f32", "f32", 18), ("f32", "f32", 8), ("f16", "f16", 12),
            ("bf16", "bf16", 18), ("f32", "f16", 12), ("f32", "i16", 12)]


def _tol(vp, lp):
    # 16-bit fixed-point links: every entry within 2^-16 (the gate of tests/test_gpu_links16.py)
    return max(DSLASH_TOL[vp], 1e-3 if lp == "i16" else DSLASH_TOL[lp])


def _shard_parts(dims, U, chi, t0, Tl, vp, lp, rc, bc_t):
    """Shard at t0 with Tl slices, its packed local links and ghost t-links, and its extended input vector with
    both ghost slices filled through the loopback exchange."""
    X, Y, Z, T = dims
    XYZ = X * Y * Z
    F = XYZ // 2

    def shard(t):
        return sp.Shard((X, Y, Z, Tl), t, T, bc_t)

    def slab(t):
        return to_dev(np.ascontiguousarray(chi[t * F:(t + Tl) * F]))

    me = shard(t0)
    links = to_dev(np.ascontiguousarray(U[:, t0 * XYZ:(t0 + Tl) * XYZ]))
    G = sp.Gauge(me.lat, links, lo_prec=lp, recon=rc)
    tb = (t0 - 1) % T
    ghost = me.ghost_pack(to_dev(np.ascontiguousarray(U[3, tb * XYZ:(tb + 1) * XYZ])), lp if vp != "f64" else "f64",
                          rc if vp != "f64" else 18)
    ext = me.pack_vec(slab(t0), vp)
    below, above = (t0 - Tl) % T, (t0 + Tl) % T
    sb, sa = shard(below), shard(above)
    face_b = sb.face_pack(vp, sb.pack_vec(slab(below), vp), 1)  # its highest slice -> our ghost below
    face_a = sa.face_pack(vp, sa.pack_vec(slab(above), vp), 0)  # its lowest slice -> our ghost above
    me.face_unpack(vp, face_b.clone(), 0, ext)
    me.face_unpack(vp, face_a.clone(), 1, ext)
    return me, G, ghost, ext


_C = {}


def _cfg1_links():
    if "U" not in _C:
        _C["U"] = li.near_identity_links((20, 20, 20, 64), 0.3, 21)
    return _C["U"]


@pytest.mark.parametrize("vp,lp,rc", PACKINGS)
@pytest.mark.parametrize("t0,bc_t", [(0, 1), (24, 0), (56, 1)])
def test_loopback_workload_shards(vp, lp, rc, t0, bc_t):
    """20^3x64 cut into 8 shards of 20^3x8: the shards at the global start (t0 = 0, its ghost below is the global
    last slice), in the middle and at the end, antiperiodic and periodic."""
    dims, Tl = (20, 20, 20, 64), 8
    U = _cfg1_links()
    F = 20 * 20 * 20 // 2
    for p in (1, 0):
        chi = li.gaussian_vector(li.volume(dims) // 2, 601 + p)
        announce(f"halo loopback {vp} links {lp} r{rc} t0={t0} bc_t={bc_t} parity {p}")
        me, G, ghost, ext = _shard_parts(dims, U, chi, t0, Tl, vp, lp, rc, bc_t)
        out = me.dslash(G, ghost, vp, ext, p, part=1)
        me.dslash(G, ghost, vp, ext, p, part=2, out=out)
        y = to_host(sp.unpack_vec(me.lat, out, vp))
        cbs = np.arange(t0 * F, (t0 + Tl) * F)
        ref = oracle.dslash_eo_sites(dims, U, chi, p, cbs, bc_t=bc_t)
        err = rel_err_max(y, ref)
        announce(f"  max rel err {err:.3e}")
        assert err <= _tol(vp, lp)
        # interior then boundary is the whole operator, bit for bit
        whole = me.dslash(G, ghost, vp, ext, p, part=0)
        assert torch.equal(whole, out)


@pytest.mark.parametrize("vp,lp,rc", PACKINGS)
@pytest.mark.parametrize("dims,bc_t", [((4, 4, 4, 4), 1), ((8, 6, 4, 10), 0), ((2, 6, 4, 2), 1)])
def test_single_shard_is_the_periodic_operator(vp, lp, rc, dims, bc_t):
    """T = Tl: the shard's ghosts hold its own opposite faces, which makes the shard the whole (anti)periodic
    lattice; every site against the oracle, and against the plain half operator of the library."""
    U = li.haar_links(dims, 611) if dims != (8, 6, 4, 10) else li.near_identity_links(dims, 0.3, 612)
    chi = li.gaussian_vector(li.volume(dims) // 2, 613)
    announce(f"halo single shard {vp} links {lp} r{rc} dims={dims} bc_t={bc_t}")
    me, G, ghost, ext = _shard_parts(dims, U, chi, 0, dims[3], vp, lp, rc, bc_t)
    for p in (0, 1):
        y = to_host(sp.unpack_vec(me.lat, me.dslash(G, ghost, vp, ext, p), vp))
        ref = oracle.dslash_eo(dims, U, chi, p, bc_t=bc_t)
        assert rel_err_max(y, ref) <= _tol(vp, lp)
        plain = to_host(sp.unpack_vec(me.lat, sp.dslash_packed(G, vp, sp.pack_vec(me.lat, to_dev(chi), vp), p), vp))
        assert rel_err_max(y, plain) <= _tol(vp, lp)


@pytest.mark.parametrize("vp,lp,rc", [("f32", "f32", 12), ("f64", "f64", 18), ("f16", "f16", 18)])
def test_two_slice_shards_are_all_boundary(vp, lp, rc):
    """4^4 cut into two shards of 4x4x4x2: no interior slice (the interior launch is empty); antiperiodic."""
    dims = (4, 4, 4, 4)
    U = li.haar_links(dims, 621)
    chi = li.gaussian_vector(li.volume(dims) // 2, 622)
    F = 32
    for t0 in (0, 2):
        me, G, ghost, ext = _shard_parts(dims, U, chi, t0, 2, vp, lp, rc, 1)
        out = me.dslash(G, ghost, vp, ext, 1, part=1)  # writes nothing
        me.dslash(G, ghost, vp, ext, 1, part=2, out=out)
        y = to_host(sp.unpack_vec(me.lat, out, vp))
        ref = oracle.dslash_eo_sites(dims, U, chi, 1, np.arange(t0 * F, (t0 + 2) * F), bc_t=1)
        assert rel_err_max(y, ref) <= _tol(vp, lp)


PLANES = {"f64": [16, 16, 16], "f32": [16, 8], "f16": [16], "bf16": [8, 4]}


@pytest.mark.parametrize("vp", ["f64", "f32", "f16", "bf16"])
def test_face_pack_unpack_move_words_unchanged(vp):
    """A face packed from one shard and unpacked into another's ghost slice carries the source slice's bytes
    unchanged, plane by plane (FP16 norms included): nothing is rounded on the way."""
    sh = sp.Shard((6, 4, 2, 6), 2, 12)
    Vh, F = sh.lat.Vh, sh.F
    Vx = Vh + 2 * F
    a = sh.pack_vec(to_dev(li.gaussian_vector(Vh, 631)), vp)
    b = torch.zeros_like(a)
    for side_src, side_dst in ((1, 0), (0, 1)):
        face = sh.face_pack(vp, a, side_src)
        sh.face_unpack(vp, face, side_dst, b)
        src0 = F if side_src == 0 else Vh
        dst0 = 0 if side_dst == 0 else F + Vh
        off = 0
        for w in PLANES[vp]:
            sa = a[off + src0 * w: off + (src0 + F) * w]
            sb = b[off + dst0 * w: off + (dst0 + F) * w]
            assert torch.equal(sa, sb)
            off += w * Vx
    assert sh.face_bytes(vp) == F * sum(PLANES[vp])
    assert sh.vec_bytes(vp) == Vx * sum(PLANES[vp])


def test_shard_argument_errors():
    lib = sp.load()
    import ctypes

    from paper_1511_00088_amd import _lib

    bad = [_lib.sp_shard(sp.Lattice((4, 4, 4, 4)).geom, 1, 8),  # odd t0
           _lib.sp_shard(sp.Lattice((4, 4, 4, 4)).geom, 6, 8),  # past the global extent
           _lib.sp_shard(sp.Lattice((4, 4, 4, 4)).geom, 0, 7)]  # odd global extent
    for s in bad:
        assert lib.sp_shard_face_bytes(ctypes.byref(s), 1) == 0
    sh = sp.Shard((4, 4, 4, 4), 0, 8)
    ext = sh.pack_vec(to_dev(li.gaussian_vector(sh.lat.Vh, 641)), "f32")
    face = torch.empty(sh.face_bytes("f32"), dtype=torch.uint8, device=DEV)
    assert lib.sp_face_pack(ctypes.byref(sh.struct), 1, ctypes.c_void_p(ext.data_ptr()), 2,
                            ctypes.c_void_p(face.data_ptr()), None) == _lib.SP_ERR_INVALID_ARG
    dims = (4, 4, 4, 4)
    U = li.haar_links(dims, 642)
    me, G, ghost, ext = _shard_parts(dims, U, li.gaussian_vector(128, 643), 0, 4, "f32", "f32", 12, 0)
    out = torch.empty(me.lat.vec_bytes("f32"), dtype=torch.uint8, device=DEV)
    rc = lib.sp_dslash_halo(ctypes.byref(me.struct), ctypes.byref(G.struct), ctypes.c_void_p(ghost.data_ptr()), 1,
                            ctypes.c_void_p(ext.data_ptr()), ctypes.c_void_p(out.data_ptr()), 1, 3, None)
    assert rc == _lib.SP_ERR_INVALID_ARG
