"""ctypes declarations of libstagcg.so (the C-ABI in include/sp_api.h).

Loading fails loudly when the library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstagcg.so")

SP_F64, SP_F32, SP_F16, SP_BF16, SP_I16 = 0, 1, 2, 3, 4
# "i16": 16-bit fixed-point link storage (FP32 iterations only)
PREC = {"f64": SP_F64, "f32": SP_F32, "f16": SP_F16, "bf16": SP_BF16, "i16": SP_I16}

SP_OK = 0
SP_NOT_CONVERGED = 1
SP_ERR_INVALID_ARG = -1
SP_ERR_ODD_EXTENT = -2
SP_ERR_UNSUPPORTED = -3
SP_ERR_WORKSPACE = -4
SP_ERR_HIP = -5
SP_ERR_BREAKDOWN = -6

# bytes of the fixed device array of sp_cg_force_noalloc (SP_NOALLOC_SCRATCH_BYTES)
NOALLOC_SCRATCH_BYTES = 64 << 20


class sp_geom(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("bc_t", ctypes.c_int32)]


class sp_shard(ctypes.Structure):
    _fields_ = [("local", sp_geom), ("t0", ctypes.c_int32), ("T", ctypes.c_int32)]


class sp_gauge(ctypes.Structure):
    _fields_ = [("f64", ctypes.c_void_p), ("lo", ctypes.c_void_p), ("lo_prec", ctypes.c_int32),
                ("recon", ctypes.c_int32)]


class sp_cg_params(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("max_iter", ctypes.c_int32), ("inner", ctypes.c_int32),
                ("delta", ctypes.c_double), ("ru_every", ctypes.c_int32), ("poll_chunk", ctypes.c_int32),
                ("use_x0", ctypes.c_int32), ("use_graph", ctypes.c_int32)]


class sp_cg_stats(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("reliable_updates", ctypes.c_int32), ("converged", ctypes.c_int32),
                ("status", ctypes.c_int32), ("true_rel_resid", ctypes.c_double), ("seconds", ctypes.c_double)]


class sp_system(ctypes.Structure):
    _fields_ = [("g", ctypes.POINTER(sp_geom)), ("U", ctypes.POINTER(sp_gauge)), ("mass", ctypes.c_double),
                ("b_e", ctypes.c_void_p), ("x_e", ctypes.c_void_p)]


# name -> (restype, argtypes); every function declared in include/sp_api.h
P = ctypes.c_void_p
I = ctypes.c_int
SZ = ctypes.c_size_t
D = ctypes.c_double
PG = ctypes.POINTER(sp_geom)
PU = ctypes.POINTER(sp_gauge)
PP = ctypes.POINTER(sp_cg_params)
PS = ctypes.POINTER(sp_cg_stats)
PY = ctypes.POINTER(sp_system)
SIGNATURES = {
    "sp_version": (I, []),
    "sp_strerror": (ctypes.c_char_p, [I]),
    "sp_last_error": (ctypes.c_char_p, []),
    "sp_gauge_bytes": (SZ, [PG, I, I]),
    "sp_gauge_pack": (I, [PG, P, I, I, P, P]),
    "sp_vec_bytes": (SZ, [PG, I]),
    "sp_vec_pack": (I, [PG, P, I, P, P]),
    "sp_vec_unpack": (I, [PG, P, I, P, P]),
    "sp_dslash": (I, [PG, PU, I, P, P, I, P]),
    "sp_cg_workspace_bytes": (SZ, [I, PY, PP]),
    "sp_cg_solve": (I, [PG, PU, D, P, P, PP, PS, P, SZ, P]),
    "sp_cg_solve_batched": (I, [I, PY, PP, PS, P, SZ, P]),
    "sp_force_workspace_bytes": (SZ, [PG]),
    "sp_cg_force": (I, [PG, PU, D, P, P, P, P, P, P, SZ, P]),
    "sp_cg_force_noalloc": (I, [PG, PU, D, P, P, P, P, P, P]),
    "sp_full_workspace_bytes": (SZ, [PG, PU, PP]),
    "sp_full_solve": (I, [PG, PU, D, P, P, PP, PS, P, SZ, P]),
    "sp_hyp_workspace_bytes": (SZ, [PG]),
    "sp_hyp_smear": (I, [PG, P, ctypes.POINTER(D), P, P, SZ, P]),
    "sp_npr_path_bytes": (SZ, [PG]),
    "sp_npr_path_links": (I, [PG, P, P, P]),
    "sp_npr_contract": (I, [PG, P, I, P, P, P, P, ctypes.POINTER(ctypes.c_int32), P, P]),
    "sp_npr_contract_links": (I, [PG, P, I, P, P, P, P, ctypes.POINTER(ctypes.c_int32), P, P]),
    "sp_tune_dslash": (I, [PG, PU, I, P, P, P, ctypes.POINTER(D)]),
    "sp_tune_save": (I, [ctypes.c_char_p]),
    "sp_tune_load": (I, [ctypes.c_char_p]),
    "sp_release_cache": (None, []),
    "sp_shard_face_bytes": (SZ, [ctypes.POINTER(sp_shard), I]),
    "sp_shard_vec_bytes": (SZ, [ctypes.POINTER(sp_shard), I]),
    "sp_shard_vec_pack": (I, [ctypes.POINTER(sp_shard), P, I, P, P]),
    "sp_face_pack": (I, [ctypes.POINTER(sp_shard), I, P, I, P, P]),
    "sp_face_unpack": (I, [ctypes.POINTER(sp_shard), I, P, I, P, P]),
    "sp_shard_ghost_bytes": (SZ, [ctypes.POINTER(sp_shard), I, I]),
    "sp_shard_ghost_pack": (I, [ctypes.POINTER(sp_shard), P, I, I, P, P]),
    "sp_dslash_halo": (I, [ctypes.POINTER(sp_shard), PU, P, I, P, P, I, I, P]),
    "sp_stream_out_bytes": (SZ, [SZ, I]),
    "sp_stream_probe": (I, [I, I, P, P, P, SZ, P]),
}

_lib = None


class StagError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        lib = load()
        super().__init__(f"{where}: {lib.sp_strerror(code).decode()} ({code}): {lib.sp_last_error().decode()}")


def load():
    """Load libstagcg.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1511_00088_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def check(code: int, where: str, allow_not_converged: bool = False) -> int:
    if code == SP_OK or (allow_not_converged and code == SP_NOT_CONVERGED):
        return code
    raise StagError(code, where)
