// Host-side launch wrappers: map runtime precision / reconstruction choices onto kernel instantiations.
#pragma once

#include <hip/hip_runtime.h>

#include "sp_kernels.h"

namespace sp {

struct LaunchCfg {
    int nt = 256;    // threads per block (64, 128 or 256)
    int remap = 1;   // XCD-aware block order
    int stream = 0;  // link loads of the single-system half operator: 0 cached, 1 streaming (non-temporal)
};

// Maximum systems per group in batched launches.
static constexpr int NB = 4;

inline int blocks_for(int n, int nt) { return (n + nt - 1) / nt; }

// The fused single-system iteration has every block sum all block partials of the previous launch (in the same
// order in every block): at most this many per thread. 32 admits 8,192 blocks of 256 threads (V/2 up to 2^21:
// the 32^3x64 control and the 28^3x96 production lattice). The partials are loaded before the gather, so their
// latency overlaps the link loads; each block reads them all (8 bytes per block of the launch) from L2.
static constexpr int FUSED_PARTIALS = 32;

// Half operator (see k_dslash; mode DS_PLAIN, DS_NORM or DS_UPDATE). D = DescSingle (one system) or
// DescBatch (up to NB per group).
template <class D>
hipError_t launch_dslash(const D& d, int nblocks, LaunchCfg c, int lp, int recon, int vp, int p, int in_slot,
                         int out_slot, int mode, int gate, int use64, hipStream_t s);
template <class D>
hipError_t launch_resid(const D& d, int nblocks, LaunchCfg c, int op, int init, hipStream_t s);
template <class D>
hipError_t launch_xpay(const D& d, int nblocks, LaunchCfg c, int vp, int gate, hipStream_t s);
template <class D>
hipError_t launch_accum(const D& d, int nblocks, LaunchCfg c, hipStream_t s);
template <class D>
hipError_t launch_norm_b(const D& d, int nblocks, LaunchCfg c, hipStream_t s);
// Fused p update of one system (k_xpay_fused): reads d's state, writes the advanced state to st_out.
hipError_t launch_xpay_fused(const DescSingle& d, SolverState* st_out, int chunk_end, int nblocks, LaunchCfg c, int vp,
                             hipStream_t s);
hipError_t launch_state_copy(const SolverState* src, SolverState* dst, hipStream_t s);
hipError_t launch_state_publish(const SolverState* src, SolverState* dst, int n, hipStream_t s);
// First launch of the two-launch iteration of one system in FP32 or FP64 (k_norm_rec).
hipError_t launch_norm_rec(const DescSingle& d, SolverState* st_out, int nblocks, LaunchCfg c, int lp, int recon, int vp,
                           hipStream_t s);
// Second reduction stage (k_finalize), one block per group.
template <class D>
hipError_t launch_finalize(const D& d, int ngroups, int kind, int gate, hipStream_t s);

hipError_t launch_pack_gauge(const Geom& g, const double* nat, int prec, int recon, void* out, hipStream_t s);
hipError_t launch_pack_vec(int Vh, const double* nat, int prec, void* out, hipStream_t s);
hipError_t launch_unpack_vec(int Vh, const void* in, int prec, double* nat, hipStream_t s);
hipError_t launch_zero(void* p, size_t bytes, hipStream_t s);  // bytes multiple of 16

// Force: gamma / force in natural layout from packed FP64 x, lambda (even) and y_x, y_l (odd).
hipError_t launch_force(const Geom& g, const void* links64, const void* x, const void* lam, const void* yx,
                        const void* yl, double* gamma, double* force, hipStream_t s);
// out = -2 m Re<lam, x> (device scalar), two-stage reduction through partials[mass_grad_blocks(g)].
hipError_t launch_mass_grad(const Geom& g, double mass, const void* x, const void* lam, double* partials,
                            double* out, hipStream_t s);
int mass_grad_blocks(const Geom& g);

// Full-lattice solve helpers (sp_full.hip): split a natural full vector into packed FP64 halves, form
// b_e = m src_e - t_e in the natural half layout, merge psi_e with psi_o = (src_o - t_o) / m.
hipError_t launch_full_split(const Geom& g, const double* src, void* se, void* so, hipStream_t s);
hipError_t launch_full_source(const Geom& g, double m, const void* se, const void* te, double* be, hipStream_t s);
hipError_t launch_full_merge(const Geom& g, double m, const double* psie, const void* so, const void* to,
                             double* psi, hipStream_t s);

// HYP smearing (sp_hyp.hip): three launches, intermediate levels in ws (hyp_workspace_bytes).
size_t hyp_workspace_bytes(const Geom& g);
hipError_t launch_hyp(const Geom& g, const double* links, const double alpha[3], double* out, void* ws,
                      hipStream_t s);

// NPR contraction (sp_npr.hip): path links per hypercube, then the contraction of n field sets.
size_t npr_path_bytes(const Geom& g);
hipError_t launch_npr_paths(const Geom& g, const double* links, void* uad, hipStream_t s);
hipError_t launch_npr_contract(const Geom& g, const void* uad, int n, const double* const f[4], const int labels[4],
                               double* out, hipStream_t s);
// The same contraction from stored path links (uad, links null) or fused with their construction from the natural
// links (links non-null, uad ignored).
hipError_t launch_npr_contract_from(const Geom& g, const void* uad, const double* links, int n, const double* const f[4],
                                    const int labels[4], double* out, hipStream_t s);

}  // namespace sp
