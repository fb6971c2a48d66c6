"""Torch-facing wrappers of libstagcg.so.

PyTorch provides device memory and streams only: every step of the operator, the solver and the
gradient runs in the library's HIP kernels. Tensors are complex128 in the natural layout of the C-ABI
(links [4][V][3][3], even-site vectors [V/2][3]) and must live on the current HIP device.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def _prec(p) -> int:
    if isinstance(p, str):
        return L.PREC[p]
    return int(p)


def _check_c128(t: torch.Tensor, shape, name):
    if not isinstance(t, torch.Tensor) or t.dtype != torch.complex128 or not t.is_cuda:
        raise TypeError(f"{name} must be a complex128 GPU tensor")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _check_packed(t: torch.Tensor, nbytes: int, name, device=None):
    """A packed buffer goes to the library as a bare pointer: check here what the kernels will read or write."""
    if not isinstance(t, torch.Tensor) or t.dtype != torch.uint8 or not t.is_cuda:
        raise TypeError(f"{name} must be a uint8 GPU tensor (a packed buffer)")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < nbytes:
        raise ValueError(f"{name} holds {t.numel()} bytes, the packed layout needs {nbytes}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the gauge field on {device}")


class Lattice:
    """Lattice extents (X, Y, Z, T), each even, and the time boundary (0 periodic, 1 antiperiodic)."""

    def __init__(self, dims, bc_t: int = 0):
        self.dims = tuple(int(d) for d in dims)
        if len(self.dims) != 4:
            raise ValueError("dims must have 4 entries")
        self.bc_t = int(bc_t)
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        self.Vh = self.V // 2
        self.geom = L.sp_geom((ctypes.c_int32 * 4)(*self.dims), self.bc_t)

    def vec_bytes(self, prec) -> int:
        return int(L.load().sp_vec_bytes(ctypes.byref(self.geom), _prec(prec)))

    def gauge_bytes(self, prec, recon=18) -> int:
        return int(L.load().sp_gauge_bytes(ctypes.byref(self.geom), _prec(prec), int(recon)))


def _refuse_recon8_singular(links: torch.Tensor) -> None:
    """Recon 8 rebuilds the lower 2x2 block by dividing by n = |U01|^2 + |U02|^2: a link whose first row is a
    phase times (1, 0, 0) has n = 0 and cannot be stored this way."""
    n = links[..., 0, 1].abs().square() + links[..., 0, 2].abs().square()
    if bool((n == 0).any()):
        raise ValueError("recon 8 cannot store links whose first row is a phase times (1, 0, 0)")


def pack_gauge(lat: Lattice, links: torch.Tensor, prec, recon: int = 18) -> torch.Tensor:
    _check_c128(links, (4, lat.V, 3, 3), "links")
    nbytes = lat.gauge_bytes(prec, recon)
    if nbytes == 0:
        raise ValueError(f"unsupported packing prec={prec} recon={recon}")
    if int(recon) == 8:
        _refuse_recon8_singular(links)
    out = torch.empty(nbytes, dtype=torch.uint8, device=links.device)
    L.check(L.load().sp_gauge_pack(ctypes.byref(lat.geom), _ptr(links), _prec(prec), int(recon), _ptr(out),
                                   _stream()), "sp_gauge_pack")
    return out


class Gauge:
    """A gauge field packed for the GPU: FP64 (recon 18) plus an optional low-precision packing (recon 18, 12, or
    8 for FP32 links)."""

    def __init__(self, lat: Lattice, links: torch.Tensor, lo_prec="f32", recon: int = 18):
        self.lat = lat
        self.f64 = pack_gauge(lat, links, "f64", 18)
        self.lo_prec = _prec(lo_prec)
        self.recon = int(recon) if self.lo_prec != L.SP_F64 else 18
        self.lo = self.f64 if self.lo_prec == L.SP_F64 else pack_gauge(lat, links, self.lo_prec, self.recon)
        self.struct = L.sp_gauge(self.f64.data_ptr(), self.lo.data_ptr(), self.lo_prec, self.recon)


def pack_vec(lat: Lattice, v: torch.Tensor, prec) -> torch.Tensor:
    _check_c128(v, (lat.Vh, 3), "vector")
    out = torch.empty(lat.vec_bytes(prec), dtype=torch.uint8, device=v.device)
    L.check(L.load().sp_vec_pack(ctypes.byref(lat.geom), _ptr(v), _prec(prec), _ptr(out), _stream()),
            "sp_vec_pack")
    return out


def unpack_vec(lat: Lattice, packed: torch.Tensor, prec) -> torch.Tensor:
    _check_packed(packed, lat.vec_bytes(prec), "packed vector")
    out = torch.empty((lat.Vh, 3), dtype=torch.complex128, device=packed.device)
    L.check(L.load().sp_vec_unpack(ctypes.byref(lat.geom), _ptr(packed), _prec(prec), _ptr(out), _stream()),
            "sp_vec_unpack")
    return out


def dslash_packed(gauge: Gauge, prec, inp: torch.Tensor, out_parity: int, out: torch.Tensor | None = None):
    """out (parity out_parity) = D_{p,1-p} inp on packed vectors of precision prec."""
    lat = gauge.lat
    nbytes = lat.vec_bytes(prec)
    _check_packed(inp, nbytes, "inp", gauge.f64.device)
    if out is None:
        out = torch.empty(nbytes, dtype=torch.uint8, device=inp.device)
    _check_packed(out, nbytes, "out", gauge.f64.device)
    L.check(L.load().sp_dslash(ctypes.byref(lat.geom), ctypes.byref(gauge.struct), _prec(prec), _ptr(inp),
                               _ptr(out), int(out_parity), _stream()), "sp_dslash")
    return out


def dslash(gauge: Gauge, v: torch.Tensor, out_parity: int, prec="f64") -> torch.Tensor:
    """Half operator on a natural complex128 vector: pack to prec, apply, unpack."""
    lat = gauge.lat
    return unpack_vec(lat, dslash_packed(gauge, prec, pack_vec(lat, v, prec), out_parity), prec)


def _links_serve(gauge: "Gauge", inner_p: int) -> bool:
    """Whether the gauge field's low-precision packing can serve iterations of precision inner_p: its own
    precision, or (for FP32 iterations) links stored in FP16, BF16 or 16-bit fixed point with FP32 vectors."""
    return (inner_p == L.SP_F64 or inner_p == gauge.lo_prec
            or (inner_p == L.SP_F32 and gauge.lo_prec in (L.SP_F16, L.SP_BF16, L.SP_I16)))


@dataclass
class SolveStats:
    iters: int
    reliable_updates: int
    converged: bool
    status: int
    true_rel_resid: float
    seconds: float


def _params(tol, max_iter, inner, delta, ru_every, poll_chunk, use_x0, use_graph):
    return L.sp_cg_params(float(tol), int(max_iter), _prec(inner), float(delta), int(ru_every), int(poll_chunk),
                          int(use_x0), int(use_graph))


def _stats(s: L.sp_cg_stats) -> SolveStats:
    return SolveStats(int(s.iters), int(s.reliable_updates), bool(s.converged), int(s.status),
                      float(s.true_rel_resid), float(s.seconds))


class Workspace:
    """A reusable device workspace (grown on demand)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device) -> torch.Tensor:
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != torch.device(device):
            self.buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        return self.buf


_default_ws = Workspace()


def cg_solve(gauge: Gauge, mass: float, b: torch.Tensor, tol: float = 1e-8, inner="f32", max_iter: int = 100000,
             delta: float = 0.1, ru_every: int = 0, poll_chunk: int = 0, x0: torch.Tensor | None = None,
             use_graph: bool = True, workspace: Workspace | None = None, out: torch.Tensor | None = None,
             raise_on_not_converged: bool = False):
    """Solve (m^2 - D_eo D_oe) x = b on even sites. Returns (x, SolveStats)."""
    lat = gauge.lat
    _check_c128(b, (lat.Vh, 3), "b")
    inner_p = _prec(inner)
    if not _links_serve(gauge, inner_p):
        raise ValueError("the gauge field's low-precision packing cannot serve the inner precision")
    if out is not None:
        _check_c128(out, (lat.Vh, 3), "out")
    x = out if out is not None else torch.empty_like(b)
    if x0 is not None:
        _check_c128(x0, (lat.Vh, 3), "x0")
        x.copy_(x0)
    prm = _params(tol, max_iter, inner_p, delta, ru_every, poll_chunk, x0 is not None, use_graph)
    sysd = L.sp_system(ctypes.pointer(lat.geom), ctypes.pointer(gauge.struct), float(mass), b.data_ptr(),
                       x.data_ptr())
    lib = L.load()
    nbytes = lib.sp_cg_workspace_bytes(1, ctypes.byref(sysd), ctypes.byref(prm))
    if nbytes == 0:
        raise L.StagError(L.SP_ERR_INVALID_ARG, "sp_cg_workspace_bytes")
    ws = (workspace or _default_ws).get(nbytes, b.device)
    st = L.sp_cg_stats()
    rc = lib.sp_cg_solve(ctypes.byref(lat.geom), ctypes.byref(gauge.struct), float(mass), _ptr(b), _ptr(x),
                         ctypes.byref(prm), ctypes.byref(st), _ptr(ws), ctypes.c_size_t(ws.numel()), _stream())
    L.check(rc, "sp_cg_solve", allow_not_converged=not raise_on_not_converged)
    return x, _stats(st)


def cg_solve_batched(systems, tol: float = 1e-8, inner="f32", max_iter: int = 100000, delta: float = 0.1,
                     ru_every: int = 0, poll_chunk: int = 0, use_graph: bool = True,
                     workspace: Workspace | None = None, raise_on_breakdown: bool = True):
    """Solve many systems together. systems: list of (Gauge, mass, b). Returns (list of x, list of stats).
    With raise_on_breakdown=False a breakdown of some systems does not raise: their stats carry the status
    SP_ERR_BREAKDOWN and the other systems' solutions and stats are valid."""
    n = len(systems)
    if n == 0:
        return [], []
    inner_p = _prec(inner)
    arr = (L.sp_system * n)()
    xs = []
    for i, (gauge, mass, b) in enumerate(systems):
        _check_c128(b, (gauge.lat.Vh, 3), f"b[{i}]")
        if not _links_serve(gauge, inner_p):
            raise ValueError("a gauge field's low-precision packing cannot serve the inner precision")
        x = torch.empty_like(b)
        xs.append(x)
        arr[i] = L.sp_system(ctypes.pointer(gauge.lat.geom), ctypes.pointer(gauge.struct), float(mass),
                             b.data_ptr(), x.data_ptr())
    prm = _params(tol, max_iter, inner_p, delta, ru_every, poll_chunk, 0, use_graph)
    lib = L.load()
    nbytes = lib.sp_cg_workspace_bytes(n, arr, ctypes.byref(prm))
    if nbytes == 0:
        raise L.StagError(L.SP_ERR_INVALID_ARG, "sp_cg_workspace_bytes")
    dev = systems[0][2].device
    ws = (workspace or _default_ws).get(nbytes, dev)
    st = (L.sp_cg_stats * n)()
    rc = lib.sp_cg_solve_batched(n, arr, ctypes.byref(prm), st, _ptr(ws), ctypes.c_size_t(ws.numel()), _stream())
    if not (rc == L.SP_ERR_BREAKDOWN and not raise_on_breakdown):
        L.check(rc, "sp_cg_solve_batched", allow_not_converged=True)
    return xs, [_stats(s) for s in st]


def full_solve(gauge: Gauge, mass: float, src: torch.Tensor, tol: float = 1e-8, inner="f32",
               max_iter: int = 100000, delta: float = 0.1, ru_every: int = 0, poll_chunk: int = 0,
               use_graph: bool = True):
    """Solve (m + D) psi = src on the whole lattice (src, psi: complex128 [V][3] in lex order) through the
    even-odd system. Returns (psi, SolveStats of the even solve)."""
    lat = gauge.lat
    _check_c128(src, (lat.V, 3), "src")
    inner_p = _prec(inner)
    if not _links_serve(gauge, inner_p):
        raise ValueError("the gauge field's low-precision packing cannot serve the inner precision")
    prm = _params(tol, max_iter, inner_p, delta, ru_every, poll_chunk, 0, use_graph)
    lib = L.load()
    nbytes = lib.sp_full_workspace_bytes(ctypes.byref(lat.geom), ctypes.byref(gauge.struct), ctypes.byref(prm))
    if nbytes == 0:
        raise L.StagError(L.SP_ERR_INVALID_ARG, "sp_full_workspace_bytes")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=src.device)
    psi = torch.empty_like(src)
    st = L.sp_cg_stats()
    rc = lib.sp_full_solve(ctypes.byref(lat.geom), ctypes.byref(gauge.struct), float(mass), _ptr(src), _ptr(psi),
                           ctypes.byref(prm), ctypes.byref(st), _ptr(ws), ctypes.c_size_t(nbytes), _stream())
    L.check(rc, "sp_full_solve", allow_not_converged=True)
    return psi, _stats(st)


def cg_force(gauge: Gauge, mass: float, x: torch.Tensor, lam: torch.Tensor, want_force: bool = True):
    """Link gradient gamma = dl/dU, su(3) force TA(U gamma^dag) and dl/dm = -2 m Re<lam, x>."""
    lat = gauge.lat
    _check_c128(x, (lat.Vh, 3), "x")
    _check_c128(lam, (lat.Vh, 3), "lambda")
    dev = x.device
    gamma = torch.empty((4, lat.V, 3, 3), dtype=torch.complex128, device=dev)
    force = torch.empty_like(gamma) if want_force else None
    dmass = torch.empty((), dtype=torch.float64, device=dev)
    lib = L.load()
    nbytes = lib.sp_force_workspace_bytes(ctypes.byref(lat.geom))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    rc = lib.sp_cg_force(ctypes.byref(lat.geom), ctypes.byref(gauge.struct), float(mass), _ptr(x), _ptr(lam),
                         _ptr(gamma), _ptr(force) if force is not None else None, _ptr(dmass), _ptr(ws),
                         ctypes.c_size_t(nbytes), _stream())
    L.check(rc, "sp_cg_force")
    return gamma, force, dmass



def cg_force_noalloc(gauge: Gauge, mass: float, x: torch.Tensor, lam: torch.Tensor, gamma: torch.Tensor,
                     force: torch.Tensor | None, dmass: torch.Tensor | None):
    """sp_cg_force_noalloc: the gradient of cg_force into caller-provided outputs (gamma and force complex128
    [4][V][3][3], dmass a float64 scalar), with the library allocating nothing; asynchronous on the current
    stream. Lattices whose scratch exceeds the library's fixed array (64 MiB) raise SP_ERR_WORKSPACE."""
    lat = gauge.lat
    _check_c128(x, (lat.Vh, 3), "x")
    _check_c128(lam, (lat.Vh, 3), "lambda")
    _check_c128(gamma, (4, lat.V, 3, 3), "gamma")
    if force is not None:
        _check_c128(force, (4, lat.V, 3, 3), "force")
    if dmass is not None and (dmass.dtype != torch.float64 or not dmass.is_cuda or dmass.numel() != 1):
        raise TypeError("dmass must be a float64 GPU scalar")
    rc = L.load().sp_cg_force_noalloc(ctypes.byref(lat.geom), ctypes.byref(gauge.struct), float(mass), _ptr(x),
                                      _ptr(lam), _ptr(gamma), _ptr(force) if force is not None else None,
                                      _ptr(dmass) if dmass is not None else None, _stream())
    L.check(rc, "sp_cg_force_noalloc")
    return gamma, force, dmass

HYP_ALPHA = (0.75, 0.6, 0.3)


def hyp_smear(lat: Lattice, links: torch.Tensor, alpha=HYP_ALPHA, out: torch.Tensor | None = None,
              workspace: Workspace | None = None) -> torch.Tensor:
    """HYP-smeared links (sp_hyp_smear): links complex128 [4][V][3][3] on the GPU -> a new tensor of the same
    shape (or `out`). alpha = (a1, a2, a3), the weights of levels 3, 2 and 1."""
    _check_c128(links, (4, lat.V, 3, 3), "links")
    if out is None:
        out = torch.empty_like(links)
    else:
        _check_c128(out, (4, lat.V, 3, 3), "out")
    lib = L.load()
    nbytes = int(lib.sp_hyp_workspace_bytes(ctypes.byref(lat.geom)))
    ws = (workspace or _default_ws).get(nbytes, links.device)
    a = (ctypes.c_double * 3)(*[float(x) for x in alpha])
    L.check(lib.sp_hyp_smear(ctypes.byref(lat.geom), _ptr(links), a, _ptr(out), _ptr(ws), ctypes.c_size_t(nbytes),
                             _stream()), "sp_hyp_smear")
    return out


def npr_path_links(lat: Lattice, links: torch.Tensor) -> torch.Tensor:
    """U_AD(z) of the NPR contraction (sp_npr_path_links): complex128 [V/16][16][16][3][3]."""
    _check_c128(links, (4, lat.V, 3, 3), "links")
    out = torch.empty(lat.V // 16, 16, 16, 3, 3, dtype=torch.complex128, device=links.device)
    L.check(L.load().sp_npr_path_links(ctypes.byref(lat.geom), _ptr(links), _ptr(out), _stream()), "sp_npr_path_links")
    return out


def npr_contract_links(lat: Lattice, links: torch.Tensor, chib1, chi2, chib3, chi4, labels) -> torch.Tensor:
    """O_i(z) as npr_contract, with the path links built inside the contraction from the links [4][V][3][3]
    (sp_npr_contract_links): nothing but the result is written."""
    _check_c128(links, (4, lat.V, 3, 3), "links")
    n = chib1.shape[0]
    for name, f in (("chib1", chib1), ("chi2", chi2), ("chib3", chib3), ("chi4", chi4)):
        _check_c128(f, (n, lat.V, 3), name)
    out = torch.empty(n, lat.V // 16, dtype=torch.complex128, device=links.device)
    lab = (ctypes.c_int32 * 4)(*[int(x) for x in labels])
    L.check(L.load().sp_npr_contract_links(ctypes.byref(lat.geom), _ptr(links), int(n), _ptr(chib1), _ptr(chi2),
                                           _ptr(chib3), _ptr(chi4), lab, _ptr(out), _stream()), "sp_npr_contract_links")
    return out


def npr_contract(lat: Lattice, uad: torch.Tensor, chib1, chi2, chib3, chi4, labels) -> torch.Tensor:
    """O_i(z) of the one-colour-trace four-fermion contraction (sp_npr_contract): fields complex128 [n][V][3],
    labels (S1, F1, S2, F2) -> complex128 [n][V/16]."""
    _check_c128(uad, (lat.V // 16, 16, 16, 3, 3), "uad")
    n = chib1.shape[0]
    for name, f in (("chib1", chib1), ("chi2", chi2), ("chib3", chib3), ("chi4", chi4)):
        _check_c128(f, (n, lat.V, 3), name)
    out = torch.empty(n, lat.V // 16, dtype=torch.complex128, device=uad.device)
    lab = (ctypes.c_int32 * 4)(*[int(x) for x in labels])
    L.check(L.load().sp_npr_contract(ctypes.byref(lat.geom), _ptr(uad), int(n), _ptr(chib1), _ptr(chi2), _ptr(chib3),
                                     _ptr(chi4), lab, _ptr(out), _stream()), "sp_npr_contract")
    return out


class Shard:
    """One GPU's share of a lattice cut in time (sp_shard): local extents (X, Y, Z, Tl), the global time of its
    first slice t0 and the global time extent T; bc_t is the global time boundary. Vectors of a shard are
    extended (ghost slices t0 - 1 and t0 + Tl around the local ones); faces are one slice of one parity."""

    def __init__(self, local_dims, t0: int, T: int, bc_t: int = 0):
        self.lat = Lattice(local_dims, bc_t)
        self.t0, self.T = int(t0), int(T)
        self.struct = L.sp_shard(self.lat.geom, self.t0, self.T)
        self.F = self.lat.dims[0] * self.lat.dims[1] * self.lat.dims[2] // 2

    def face_bytes(self, prec) -> int:
        return int(L.load().sp_shard_face_bytes(ctypes.byref(self.struct), _prec(prec)))

    def vec_bytes(self, prec) -> int:
        return int(L.load().sp_shard_vec_bytes(ctypes.byref(self.struct), _prec(prec)))

    def ghost_bytes(self, prec, recon) -> int:
        return int(L.load().sp_shard_ghost_bytes(ctypes.byref(self.struct), _prec(prec), int(recon)))

    def pack_vec(self, v: torch.Tensor, prec, ext: torch.Tensor | None = None) -> torch.Tensor:
        """Local natural half vector [Vh][3] -> an extended vector (a new one, ghosts unset, or ext)."""
        _check_c128(v, (self.lat.Vh, 3), "vector")
        nbytes = self.vec_bytes(prec)
        if ext is None:
            ext = torch.zeros(nbytes, dtype=torch.uint8, device=v.device)
        _check_packed(ext, nbytes, "ext")
        L.check(L.load().sp_shard_vec_pack(ctypes.byref(self.struct), _ptr(v), _prec(prec), _ptr(ext), _stream()),
                "sp_shard_vec_pack")
        return ext

    def face_pack(self, prec, ext: torch.Tensor, side: int, face: torch.Tensor | None = None) -> torch.Tensor:
        _check_packed(ext, self.vec_bytes(prec), "ext")
        nbytes = self.face_bytes(prec)
        if face is None:
            face = torch.empty(nbytes, dtype=torch.uint8, device=ext.device)
        _check_packed(face, nbytes, "face")
        L.check(L.load().sp_face_pack(ctypes.byref(self.struct), _prec(prec), _ptr(ext), int(side), _ptr(face),
                                      _stream()), "sp_face_pack")
        return face

    def face_unpack(self, prec, face: torch.Tensor, side: int, ext: torch.Tensor) -> torch.Tensor:
        _check_packed(face, self.face_bytes(prec), "face")
        _check_packed(ext, self.vec_bytes(prec), "ext")
        L.check(L.load().sp_face_unpack(ctypes.byref(self.struct), _prec(prec), _ptr(face), int(side), _ptr(ext),
                                        _stream()), "sp_face_unpack")
        return ext

    def ghost_pack(self, tlinks: torch.Tensor, prec, recon: int) -> torch.Tensor:
        """U_t on global slice t0 - 1, complex128 [X Y Z][3][3] -> packed ghost links."""
        _check_c128(tlinks, (2 * self.F, 3, 3), "tlinks")
        nbytes = self.ghost_bytes(prec, recon)
        if nbytes == 0:
            raise ValueError(f"unsupported packing prec={prec} recon={recon}")
        if int(recon) == 8:
            _refuse_recon8_singular(tlinks)
        out = torch.empty(nbytes, dtype=torch.uint8, device=tlinks.device)
        L.check(L.load().sp_shard_ghost_pack(ctypes.byref(self.struct), _ptr(tlinks), _prec(prec), int(recon),
                                             _ptr(out), _stream()), "sp_shard_ghost_pack")
        return out

    def dslash(self, gauge: Gauge, ghost: torch.Tensor, prec, ext: torch.Tensor, out_parity: int, part: int = 0,
               out: torch.Tensor | None = None) -> torch.Tensor:
        """Halo-fed half operator (sp_dslash_halo) into a local packed vector; part 0 all, 1 interior, 2 boundary."""
        lat = self.lat
        if gauge.lat.dims != lat.dims:
            raise ValueError("the gauge field must be packed on the shard's local geometry")
        _check_packed(ext, self.vec_bytes(prec), "ext", gauge.f64.device)
        nbytes = lat.vec_bytes(prec)
        if out is None:
            out = torch.empty(nbytes, dtype=torch.uint8, device=ext.device)
        _check_packed(out, nbytes, "out", gauge.f64.device)
        lp = L.SP_F64 if _prec(prec) == L.SP_F64 else gauge.lo_prec
        rc = 18 if _prec(prec) == L.SP_F64 else gauge.recon
        _check_packed(ghost, self.ghost_bytes(lp, rc), "ghost", gauge.f64.device)
        L.check(L.load().sp_dslash_halo(ctypes.byref(self.struct), ctypes.byref(gauge.struct), _ptr(ghost), _prec(prec),
                                        _ptr(ext), _ptr(out), int(out_parity), int(part), _stream()), "sp_dslash_halo")
        return out

STREAM_KINDS = {"read": 0, "copy": 1, "triad": 2}


def stream_probe(kind: str, k: int, a: torch.Tensor, b: torch.Tensor, c: torch.Tensor | None = None) -> None:
    """One launch of the library's streaming-bandwidth probe (sp_stream_probe) over a's 16-byte words: "read"
    (b receives one float per block, sp_stream_out_bytes), "copy" (b = a) or "triad" (b = a + 0.5 c), k words
    per lane. Asynchronous on the current stream."""
    for name, t in (("a", a), ("b", b), ("c", c)):
        if t is None:
            continue
        if not isinstance(t, torch.Tensor) or not t.is_cuda or not t.is_contiguous():
            raise TypeError(f"{name} must be a contiguous GPU tensor")
    n16 = a.numel() * a.element_size() // 16
    lib = L.load()
    kd = STREAM_KINDS[kind]
    need = lib.sp_stream_out_bytes(n16, int(k)) if kd == 0 else n16 * 16
    if b.numel() * b.element_size() < need or (c is not None and c.numel() * c.element_size() < n16 * 16):
        raise ValueError("output or second input too small for the probe")
    if kd == 2 and c is None:
        raise ValueError("triad needs c")
    L.check(lib.sp_stream_probe(kd, int(k), _ptr(a), _ptr(b), _ptr(c) if c is not None else None,
                                ctypes.c_size_t(n16), _stream()), "sp_stream_probe")

def tune_dslash(gauge: Gauge, prec) -> float:
    """Pick the fastest launch shape of the half operator for this lattice and precision (ms per call)."""
    lat = gauge.lat
    dev = gauge.f64.device
    a = torch.zeros(lat.vec_bytes(prec), dtype=torch.uint8, device=dev)
    b = torch.zeros_like(a)
    best = ctypes.c_double(0)
    L.check(L.load().sp_tune_dslash(ctypes.byref(lat.geom), ctypes.byref(gauge.struct), _prec(prec), _ptr(a), _ptr(b),
                                    _stream(), ctypes.byref(best)), "sp_tune_dslash")
    return float(best.value)


def tune_save(path: str):
    L.check(L.load().sp_tune_save(path.encode()), "sp_tune_save")


def tune_load(path: str):
    L.check(L.load().sp_tune_load(path.encode()), "sp_tune_load")


def release_cache():
    L.load().sp_release_cache()
