"""FP64 CPU oracle for the even-odd staggered CG -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this package. The
GPU library does not load it and there is no fallback from the GPU path to it.

``build()`` compiles ``oracle.c`` with gcc into ``liboracle.so`` beside it; the wrappers below take and
return numpy complex128 arrays in the natural layout described in ``oracle.h``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, plain C11, no threads)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra",
                               os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.c_void_p
        I = ctypes.c_int32
        D = ctypes.c_double
        lib.or_dslash.argtypes = [P, I, P, P, P]
        lib.or_dslash_eo.argtypes = [P, I, P, P, P, I]
        lib.or_dslash_eo_sites.argtypes = [P, I, P, P, I, P, ctypes.c_int64, P]
        lib.or_apply_A.argtypes = [P, I, P, D, P, P]
        lib.or_cg_solve.argtypes = [P, I, P, D, P, P, D, I, I, P, P]
        lib.or_cg_solve.restype = I
        lib.or_grad.argtypes = [P, I, P, D, P, P, P, P, P]
        lib.or_full_solve.argtypes = [P, I, P, D, P, P, D, I, P]
        lib.or_full_solve.restype = I
        _lib = lib
    return _lib


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,) and np.all(d % 2 == 0) and np.all(d >= 2), "dims must be 4 even extents >= 2"
    return d


def _c128(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    if shape is not None:
        assert a.shape == tuple(shape), (a.shape, shape)
    return a


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _V(d):
    return int(np.prod(d.astype(np.int64)))


def dslash(dims, U, chi, bc_t=0):
    """Full-lattice D chi; chi [V][3] -> [V][3]."""
    d = _dims(dims)
    V = _V(d)
    U = _c128(U, (4, V, 3, 3))
    chi = _c128(chi, (V, 3))
    out = np.empty((V, 3), np.complex128)
    _load().or_dslash(_ptr(d), bc_t, _ptr(U), _ptr(chi), _ptr(out))
    return out


def dslash_eo(dims, U, chi, out_parity, bc_t=0):
    """Half operator D_{p,1-p}: chi on parity 1-p [V/2][3] -> parity p [V/2][3]."""
    d = _dims(dims)
    V = _V(d)
    U = _c128(U, (4, V, 3, 3))
    chi = _c128(chi, (V // 2, 3))
    out = np.empty((V // 2, 3), np.complex128)
    _load().or_dslash_eo(_ptr(d), bc_t, _ptr(U), _ptr(chi), _ptr(out), int(out_parity))
    return out


def dslash_eo_sites(dims, U, chi, out_parity, cbs, bc_t=0):
    """D_{p,1-p} chi at the checkerboard indices cbs only; -> [len(cbs)][3]."""
    d = _dims(dims)
    V = _V(d)
    U = _c128(U, (4, V, 3, 3))
    chi = _c128(chi, (V // 2, 3))
    cbs = np.ascontiguousarray(np.asarray(cbs, dtype=np.int64))
    assert cbs.ndim == 1 and (cbs.size == 0 or (cbs.min() >= 0 and cbs.max() < V // 2))
    out = np.empty((cbs.size, 3), np.complex128)
    _load().or_dslash_eo_sites(_ptr(d), bc_t, _ptr(U), _ptr(chi), int(out_parity), _ptr(cbs), cbs.size,
                               _ptr(out))
    return out


def apply_A(dims, U, mass, x, bc_t=0):
    """(m^2 - D_eo D_oe) x on even sites."""
    d = _dims(dims)
    V = _V(d)
    U = _c128(U, (4, V, 3, 3))
    x = _c128(x, (V // 2, 3))
    y = np.empty_like(x)
    _load().or_apply_A(_ptr(d), bc_t, _ptr(U), float(mass), _ptr(x), _ptr(y))
    return y


def cg_solve(dims, U, mass, b, tol=1e-12, max_iter=100000, x0=None, bc_t=0):
    """FP64 CG on A x = b. Returns (x, status, iters, true_rel_resid)."""
    d = _dims(dims)
    V = _V(d)
    U = _c128(U, (4, V, 3, 3))
    b = _c128(b, (V // 2, 3))
    x = np.zeros_like(b) if x0 is None else _c128(x0, (V // 2, 3)).copy()
    iters = ctypes.c_int32(0)
    res = ctypes.c_double(0)
    st = _load().or_cg_solve(_ptr(d), bc_t, _ptr(U), float(mass), _ptr(b), _ptr(x), float(tol),
                             int(max_iter), 0 if x0 is None else 1, ctypes.byref(iters), ctypes.byref(res))
    return x, int(st), int(iters.value), float(res.value)


def grad(dims, U, mass, x, lam, bc_t=0, want_force=True):
    """Adjoint gradient: (gamma [4][V][3][3], force or None, dl/dm)."""
    d = _dims(dims)
    V = _V(d)
    U = _c128(U, (4, V, 3, 3))
    x = _c128(x, (V // 2, 3))
    lam = _c128(lam, (V // 2, 3))
    gamma = np.empty((4, V, 3, 3), np.complex128)
    force = np.empty((4, V, 3, 3), np.complex128) if want_force else None
    dm = ctypes.c_double(0)
    _load().or_grad(_ptr(d), bc_t, _ptr(U), float(mass), _ptr(x), _ptr(lam), _ptr(gamma),
                    _ptr(force) if want_force else None, ctypes.byref(dm))
    return gamma, force, float(dm.value)


def full_solve(dims, U, mass, src, tol=1e-12, max_iter=100000, bc_t=0):
    """(m + D) psi = src on the full lattice via the even-odd system. Returns (psi, status, iters)."""
    d = _dims(dims)
    V = _V(d)
    U = _c128(U, (4, V, 3, 3))
    src = _c128(src, (V, 3))
    psi = np.empty_like(src)
    iters = ctypes.c_int32(0)
    st = _load().or_full_solve(_ptr(d), bc_t, _ptr(U), float(mass), _ptr(src), _ptr(psi), float(tol),
                               int(max_iter), ctypes.byref(iters))
    return psi, int(st), int(iters.value)
