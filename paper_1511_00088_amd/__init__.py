"""MI355X-native even-odd mixed-precision CG for staggered quarks (HIP kernels behind a C-ABI).

The compute path lives in libstagcg.so (built from csrc/ by ``paper_1511_00088_amd.build``); this package
only marshals torch tensors into its C-ABI.
"""
from ._lib import PREC, SP_BF16, SP_F16, SP_F32, SP_F64, SP_I16, StagError, load  # noqa: F401
from .api import (Gauge, Lattice, Shard, SolveStats, Workspace, cg_force, cg_force_noalloc, cg_solve, cg_solve_batched,  # noqa: F401
                  HYP_ALPHA, dslash, dslash_packed, full_solve, hyp_smear, npr_contract, npr_contract_links, npr_path_links, pack_gauge, pack_vec, release_cache, stream_probe, tune_dslash, tune_load, tune_save,
                  unpack_vec)
from .autograd import StaggeredSolve, staggered_solve  # noqa: F401
