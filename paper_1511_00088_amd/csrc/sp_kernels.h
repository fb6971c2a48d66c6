// Kernel templates of the even-odd staggered CG.
//
// Every solver kernel runs over a list of "groups": a group is a set of up to N systems (right-hand
// sides) that share one gauge field and geometry. A launch covers the blocks of every group; a block
// handles blockDim.x consecutive sites of one group for all of its systems, so the half operator loads
// each link once per group rather than once per system. A single solve is one group with one system,
// its descriptor passed by value (DescSingle); batches keep their descriptors in device memory
// (DescBatch).
//
// Global dot products use a two-stage reduction: each block reduces its sites in FP64 (wave64 shuffles,
// then LDS across waves) and stores one partial per system; the next launch, k_finalize (one block per
// group), sums the partials in a fixed order and updates each system's device-resident state (alpha,
// beta, flags). The kernel boundary makes the partials visible without any in-kernel fence, sums have a
// fixed order and results are bitwise reproducible.
#pragma once

#include "sp_device.h"

namespace sp {

// Vector slots of a system.
enum Slot : int { S_B64 = 0, S_X64, S_T64, S_XLO, S_P, S_R, S_T, NSLOT };

// Which systems a kernel works on.
enum Gate : int {
    G_NONE = 0,   // no state (stand-alone operator application)
    G_ITER = 1,   // CG iteration: not done, not paused for a reliable update
    G_RU = 2,     // reliable update requested by the last iteration (ST_PENDING)
    G_XPAY = 3,   // the paused iteration's p update is due after the reliable update
    G_ALIVE = 4,  // not done (set-up kernels)
};

struct SysDev {
    void* v[NSLOT];
    SolverState* st;
};

struct GroupDev {
    Geom g;
    const void* links_lo;
    const void* links64;
    double* partials;   // [nblk][2 N] block partials of the last reducing launch
    double* partials_p; // [nblk][N]   block partials of |p|^2 from the last p update
    double* partials_r; // [nblk]      block partials of |r|^2 from DS_UPDATE_FUSED
    double* rec;        // [2]         Re<p,Ap> and alpha of the last DS_UPDATE_FUSED (block 0 writes them)
    int nrhs, sys0, blk0, nblk;
};

struct DescSingle {
    GroupDev grp;
    SysDev sys;
};

struct DescBatch {
    const GroupDev* grp;
    const SysDev* sys;
    int ngroups;
};

// --- descriptor access ---------------------------------------------------------------------------------
__device__ __forceinline__ int find_group(const DescSingle&, int) { return 0; }
// The group of a logical block: the number of groups that start at or before it, minus one (group starts
// increase strictly). Lane l tests group l (then l + 64, ...), so the starts load in parallel instead of
// one after the other. Called by whole waves at kernel entry.
__device__ __forceinline__ int find_group(const DescBatch& d, int lblk) {
    int count = 0;
    for (int g0 = 0; g0 < d.ngroups; g0 += 64) {
        const int g = g0 + (int)(threadIdx.x & 63);
        const bool started = g < d.ngroups && d.grp[g].blk0 <= lblk;
        count += __popcll(__ballot(started));
    }
    return __builtin_amdgcn_readfirstlane(count - 1);
}
__device__ __forceinline__ const GroupDev& grp_of(const DescSingle& d, int) { return d.grp; }
__device__ __forceinline__ const GroupDev& grp_of(const DescBatch& d, int g) { return d.grp[g]; }
__device__ __forceinline__ const SysDev& sys_of(const DescSingle& d, int) { return d.sys; }
__device__ __forceinline__ const SysDev& sys_of(const DescBatch& d, int i) { return d.sys[i]; }

// Block order: with remap, consecutive logical blocks (neighbouring lattice slabs) go to the same XCD.
// The hardware hands block b to XCD b % 8; logical block = start of that XCD's contiguous range + b / 8.
// A bijection of [0, nb) for every nb (XCD x owns nb / 8 blocks, plus one for the first nb % 8 XCDs).
__host__ __device__ __forceinline__ int remap_block(int b, int nb) {
    const int q = nb >> 3, rem = nb & 7, x = b & 7, i = b >> 3;
    return x * q + (x < rem ? x : rem) + i;
}
__device__ __forceinline__ int logical_block(int remap) {
    return remap ? remap_block(blockIdx.x, gridDim.x) : (int)blockIdx.x;
}

// Whether a launch gated by `gate` works on a system whose state flags are f.
__device__ __forceinline__ bool gate_flags_open(int f, int gate) {
    if (gate == G_NONE) return true;
    if (f & ST_DONE) return false;
    if (gate == G_ITER) return !(f & ST_PENDING);
    if (gate == G_RU) return (f & ST_PENDING) != 0;
    if (gate == G_XPAY) return (f & ST_XPAY_DUE) != 0;
    return true;
}

// Per-launch view of the systems of this block's group.
template <int N>
struct Rhs {
    bool act[N];
    SolverState* st[N];
    bool any;
};

// The state pointers and flags of the group's systems load unconditionally (slots beyond the group's count
// repeat its first system and are marked inactive), so the loads of all systems are in flight together.
template <int N, class D>
__device__ __forceinline__ Rhs<N> rhs_of(const D& d, const GroupDev& G, int gate) {
    Rhs<N> h;
    if constexpr (N == 1) {
        h.st[0] = sys_of(d, G.sys0).st;
        h.act[0] = G.nrhs > 0 && (gate == G_NONE || h.st[0] == nullptr || gate_flags_open(h.st[0]->flags, gate));
        h.any = h.act[0];
        return h;
    }
    h.any = false;
#pragma unroll
    for (int r = 0; r < N; ++r) h.st[r] = sys_of(d, G.sys0 + (r < G.nrhs ? r : 0)).st;
    int f[N];
#pragma unroll
    for (int r = 0; r < N; ++r) f[r] = (gate == G_NONE || h.st[r] == nullptr) ? 0 : h.st[r]->flags;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        h.act[r] = r < G.nrhs && (h.st[r] == nullptr || gate_flags_open(f[r], gate));
        h.any |= h.act[r];
    }
    return h;
}

// This thread's share of the second reduction stage over n block partials of NV arrays: acc[q] += a[q][b] for
// b = b_first, + blockDim.x, ... < n, added in increasing b (the order that makes every block of a launch
// reach the same total, bit for bit). The loads go out eight at a time: a plain loop of dependent adds waits
// for each load in turn, one memory round trip per partial.
template <int NV>
__device__ __forceinline__ void strided_sums_from(double (&acc)[NV], const double* const (&a)[NV], int n,
                                                  int b_first) {
    constexpr int K = 8;
    const int nt = blockDim.x;
    for (int b0 = b_first; b0 < n; b0 += K * nt) {
        double v[K][NV];
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int q = 0; q < NV; ++q) v[j][q] = b0 + j * nt < n ? a[q][b0 + j * nt] : 0.0;
#pragma unroll
        for (int j = 0; j < K; ++j)
#pragma unroll
            for (int q = 0; q < NV; ++q)
                if (b0 + j * nt < n) acc[q] += v[j][q];
    }
}

// The same sums split around the caller's own loads, when every thread has at most HEAD partials (up to
// HEAD x blockDim.x blocks): strided_head loads them with no branch (indices clamped to n - 1) and leaves them
// unused, so that the loads the caller issues next do not wait for them, and strided_tail adds those below n
// in the same increasing order. With more partials strided_head sums them all at once, eight loads in flight
// (moving them after the operator's gathers put two or more dependent rounds of loads after it: 2% slower
// iterations on 32^3x64), and strided_tail adds nothing.
constexpr int HEAD = 4;
template <int NV>
__device__ __forceinline__ void strided_head(double (&acc)[NV], double (&v)[HEAD][NV], const double* const (&a)[NV],
                                             int n) {
    const int nt = blockDim.x;
    if (n <= HEAD * nt) {
#pragma unroll
        for (int j = 0; j < HEAD; ++j) {
            const int b = threadIdx.x + j * nt;
            const int c = b < n ? b : n - 1;
#pragma unroll
            for (int q = 0; q < NV; ++q) v[j][q] = a[q][c];
        }
    } else {
        strided_sums_from<NV>(acc, a, n, threadIdx.x);
#pragma unroll
        for (int j = 0; j < HEAD; ++j)
#pragma unroll
            for (int q = 0; q < NV; ++q) v[j][q] = 0.0;
    }
}
template <int NV>
__device__ __forceinline__ void strided_tail(double (&acc)[NV], const double (&v)[HEAD][NV], int n) {
    if (n <= HEAD * (int)blockDim.x) {
#pragma unroll
        for (int j = 0; j < HEAD; ++j)
            if (threadIdx.x + j * blockDim.x < n) {
#pragma unroll
                for (int q = 0; q < NV; ++q) acc[q] += v[j][q];
            }
    }
}

// First reduction stage: block totals of NV values per thread, stored by thread 0 as dst[gblk][NV].
template <int NV>
__device__ __forceinline__ void block_partials(double* dst, int gblk, double (&v)[NV]) {
    block_sum<NV>(v);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) dst[(size_t)gblk * NV + k] = v[k];
    }
}

// ------------------------------------------------------------------------------------------------------
// Half operator, N right-hand sides sharing each link load. MODE:
//   DS_PLAIN : out = D_{p,1-p} in
//   DS_NORM  : t = D_oe p (out), block partials of Re<t, t_stored>; with |p|^2 from the last p update this
//              gives Re<p, A p> = m^2 |p|^2 + |D_oe p|^2 and alpha, since D_eo = -D_oe^dag for any links
//   DS_UPDATE: q = m^2 p - D_eo t (not stored); x += alpha p; r -= alpha q; block partials of |r|^2
//   DS_UPDATE_FUSED (one system): as DS_UPDATE, but every block forms alpha itself from the partials of
//              |D_oe p|^2 and |p|^2 (summed in the same order in every block, so all blocks agree bit for
//              bit); the first partials are loaded before the gathers and summed after them. Saves the
//              alpha finalize launch when the partials are few; |r|^2 partials go to partials_r, Re<p,Ap>
//              and alpha to rec for k_xpay_fused, which takes the place of the update finalize.
// ------------------------------------------------------------------------------------------------------
enum DsMode : int { DS_PLAIN = 0, DS_NORM = 1, DS_UPDATE = 2, DS_UPDATE_FUSED = 3 };

// Multi-system launches keep every load unconditional so that the compiler can keep all of them in flight:
// right-hand sides beyond the group's count read the last system's vectors and store nothing, and systems
// that are stopped or paused are computed with zero coefficients (x += 0 p, r -= 0 q, p = 0 r + 1 p leave
// their stored values unchanged). Only temporaries (t) are overwritten for them.
template <int LP, int RECON, int VP, int N, class D, int MODE, bool NT = false>
__global__ __launch_bounds__(256) void k_dslash(D d, int p, int in_slot, int out_slot, int gate, int use64,
                                                int remap) {
    using R = typename Real<VP>::T;
    using LF = LinkFmt<LP, RECON>;
    using VF = VecFmt<VP>;
    constexpr int XP = VP == F64 ? F64 : F32;  // x: FP64 in place for plain FP64 CG, else the FP32 x_lo
    using RX = typename Real<XP>::T;
    using XF = VecFmt<XP>;
    const int lblk = logical_block(remap);
    const int gi = find_group(d, lblk);
    const GroupDev& G = grp_of(d, gi);
    const int gblk = lblk - G.blk0;
    const Rhs<N> h = rhs_of<N>(d, G, gate);
    if (!h.any) return;
    const Geom g = G.g;
    const int nr = G.nrhs;
    const void* links = use64 ? G.links64 : G.links_lo;
    const void* in[N];
#pragma unroll
    for (int r = 0; r < N; ++r) in[r] = sys_of(d, G.sys0 + (r < nr ? r : nr - 1)).v[in_slot];
    const int cb = gblk * blockDim.x + threadIdx.x;
    double dots[N];
#pragma unroll
    for (int r = 0; r < N; ++r) dots[r] = 0.0;
    constexpr bool FUSED = MODE == DS_UPDATE_FUSED;
    static_assert(!FUSED || N == 1, "alpha is formed in-block for one system only");
    double pre[2] = {0.0, 0.0};  // FUSED: this thread's share of the |D_oe p|^2 and |p|^2 partials
    double head[HEAD][2];
    const double* const psrc[2] = {G.partials, G.partials_p};
    if constexpr (FUSED) strided_head<2>(pre, head, psrc, G.nblk);
    const bool live = cb < g.Vh;
    Vec3<R> acc[N];
#pragma unroll
    for (int r = 0; r < N; ++r) acc[r] = vzero<R>();

    if (live) {
        const Site s = site_of(g, p, cb);
// several systems: two directions at a time (FP32 and 16-bit vectors; 105-158 VGPRs for four systems, 1% faster
// batches than one at a time), one in FP64 (its four-system update holds 216 VGPRs already); one system: two at a time
// in FP64, where all four put 384 values in flight and leave one wave per SIMD, and for FP32 recon-12 with
// cached link loads, whose row rebuild makes four at a time cost 125-136 VGPRs (measured 3-4% slower)
        constexpr int UNROLL = N == 1 ? unroll_dirs(LP, RECON, VP, NT) : (VP == F64 ? 1 : 2);
#pragma unroll UNROLL
        for (int mu = 0; mu < 4; ++mu) {
            R e = (R)eta_sign(s, mu);
            R sf = e, sb = -e;
            if (mu == 3 && g.bc_t) {
                if (s.t == g.T - 1) sf = -sf;
                if (s.t == 0) sb = -sb;
            }
            const int nf = nbr(g, s, mu, +1);
            const int nb = nbr(g, s, mu, -1);
            const Su3<R> Uf = LF::template load<NT>(link_block<LF>(links, g.Vh, p, mu), g.Vh, cb);
            Vec3<R> v[N];
#pragma unroll
            for (int r = 0; r < N; ++r) v[r] = VF::load(in[r], g.Vh, nf);
#pragma unroll
            for (int r = 0; r < N; ++r) mv_acc(acc[r], Uf, v[r], sf);
            const Su3<R> Ub = LF::template load<NT>(link_block<LF>(links, g.Vh, 1 - p, mu), g.Vh, nb);
#pragma unroll
            for (int r = 0; r < N; ++r) v[r] = VF::load(in[r], g.Vh, nb);
#pragma unroll
            for (int r = 0; r < N; ++r) mdv_acc(acc[r], Ub, v[r], sb);
        }
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                acc[r].c[i].re *= R(0.5);
                acc[r].c[i].im *= R(0.5);
            }
    }
    R alpha_blk = R(0);
    if constexpr (FUSED) {
        __shared__ double a_sh;
        strided_tail<2>(pre, head, G.nblk);
        block_sum<2>(pre);
        if (threadIdx.x == 0) {
            const SolverState* st = h.st[0];
            const double pq = st->m2 * pre[1] + pre[0];
            a_sh = (pq > 0.0 && isfinite(pq)) ? st->rho / pq : 0.0;  // breakdown: no update, flagged later
            if (gblk == 0) {
                G.rec[0] = pq;
                G.rec[1] = a_sh;
            }
        }
        __syncthreads();
        alpha_blk = (R)a_sh;
    }
    if (live) {
        if constexpr (MODE == DS_PLAIN) {
#pragma unroll
            for (int r = 0; r < N; ++r)
                if (r < nr) VF::store(sys_of(d, G.sys0 + r).v[out_slot], g.Vh, cb, acc[r]);
        } else if constexpr (MODE == DS_NORM) {
#pragma unroll
            for (int r = 0; r < N; ++r) {
                if (r >= nr) continue;
                const Vec3<R> ts = VF::store_rt(sys_of(d, G.sys0 + r).v[out_slot], g.Vh, cb, acc[r]);
                double dd = 0.0;
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    dd += (double)acc[r].c[i].re * (double)ts.c[i].re + (double)acc[r].c[i].im * (double)ts.c[i].im;
                dots[r] = dd;
            }
        } else {
            // per group of up to four systems: loads first, then arithmetic, then stores
            constexpr int NG = N < 4 ? N : 4;
#pragma unroll
            for (int r0 = 0; r0 < N; r0 += NG) {
                Vec3<R> pc[NG], rv[NG];
                Vec3<RX> xv[NG];
#pragma unroll
                for (int j = 0; j < NG; ++j) {
                    const int r = r0 + j;
                    const SysDev& S = sys_of(d, G.sys0 + (r < nr ? r : nr - 1));
                    pc[j] = VF::load(S.v[S_P], g.Vh, cb);
                    rv[j] = VF::load(S.v[S_R], g.Vh, cb);
                    xv[j] = XF::load(S.v[XP == F64 ? S_X64 : S_XLO], g.Vh, cb);
                }
#pragma unroll
                for (int j = 0; j < NG; ++j) {
                    const int r = r0 + j;
                    const R m2 = h.act[r] ? (R)h.st[r]->m2 : R(0);
                    const R a = h.act[r] ? (FUSED ? alpha_blk : (R)h.st[r]->alpha) : R(0);
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const R qre = m2 * pc[j].c[i].re - acc[r].c[i].re;
                        const R qim = m2 * pc[j].c[i].im - acc[r].c[i].im;
                        xv[j].c[i].re += (RX)a * (RX)pc[j].c[i].re;
                        xv[j].c[i].im += (RX)a * (RX)pc[j].c[i].im;
                        rv[j].c[i].re -= a * qre;
                        rv[j].c[i].im -= a * qim;
                    }
                }
#pragma unroll
                for (int j = 0; j < NG; ++j) {
                    const int r = r0 + j;
                    if (r >= nr) continue;
                    const SysDev& S = sys_of(d, G.sys0 + r);
                    XF::store(S.v[XP == F64 ? S_X64 : S_XLO], g.Vh, cb, xv[j]);
                    const Vec3<R> rs = VF::store_rt(S.v[S_R], g.Vh, cb, rv[j]);
                    double dd = 0.0;
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        dd += (double)rs.c[i].re * (double)rs.c[i].re + (double)rs.c[i].im * (double)rs.c[i].im;
                    dots[r] = dd;
                }
            }
        }
    }
    if constexpr (MODE == DS_UPDATE_FUSED) block_partials<N>(G.partials_r, gblk, dots);
    else if constexpr (MODE != DS_PLAIN) block_partials<N>(G.partials, gblk, dots);
}

// ------------------------------------------------------------------------------------------------------
// FP64 true residual on even sites: r = b - m^2 x + D_eo t64, t64 = D_oe x (previous launch).
// Writes R (inner precision OP); block partials of |r|^2 and Re<r, p> (p unused when init). init: 0 a reliable
// update, 1 the start of a solve from a given x0, 2 the start from x0 = 0, where r = b needs no operator (t64 is
// then neither read nor needed).
// ------------------------------------------------------------------------------------------------------
template <int OP, int N, class D>
__global__ __launch_bounds__(256) void k_resid(D d, int init, int remap) {
    using LF = LinkFmt<F64, 18>;
    using VO = VecFmt<OP>;
    using RO = typename Real<OP>::T;
    const int lblk = logical_block(remap);
    const int gi = find_group(d, lblk);
    const GroupDev& G = grp_of(d, gi);
    const int gblk = lblk - G.blk0;
    const Rhs<N> h = rhs_of<N>(d, G, init ? G_ALIVE : G_RU);
    if (!h.any) return;
    const Geom g = G.g;
    const int cb = gblk * blockDim.x + threadIdx.x;
    double dots[2 * N];
#pragma unroll
    for (int r = 0; r < 2 * N; ++r) dots[r] = 0.0;
    const bool zero_x = init == 2;
    if (cb < g.Vh) {
        const Site s = site_of(g, 0, cb);
        Vec3<double> acc[N];
        const void* tin[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            acc[r] = vzero<double>();
            tin[r] = h.act[r] ? sys_of(d, G.sys0 + r).v[S_T64] : nullptr;
        }
        // two directions at a time for one system, as in the FP64 half operator (all four put the kernel past 256
        // registers, one wave per SIMD)
        constexpr int UNROLL = N == 1 ? 2 : 4;
#pragma unroll UNROLL
        for (int mu = 0; mu < (zero_x ? 0 : 4); ++mu) {
            double e = (double)eta_sign(s, mu);
            double sf = e, sb = -e;
            if (mu == 3 && g.bc_t) {
                if (s.t == g.T - 1) sf = -sf;
                if (s.t == 0) sb = -sb;
            }
            const int nf = nbr(g, s, mu, +1);
            const int nb = nbr(g, s, mu, -1);
            const Su3<double> Uf = LF::load(link_block<LF>(G.links64, g.Vh, 0, mu), g.Vh, cb);
#pragma unroll
            for (int r = 0; r < N; ++r)
                if (h.act[r]) mv_acc(acc[r], Uf, VecFmt<F64>::load(tin[r], g.Vh, nf), sf);
            const Su3<double> Ub = LF::load(link_block<LF>(G.links64, g.Vh, 1, mu), g.Vh, nb);
#pragma unroll
            for (int r = 0; r < N; ++r)
                if (h.act[r]) mdv_acc(acc[r], Ub, VecFmt<F64>::load(tin[r], g.Vh, nb), sb);
        }
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if (!h.act[r]) continue;
            const SysDev& S = sys_of(d, G.sys0 + r);
            const Vec3<double> b = VecFmt<F64>::load(S.v[S_B64], g.Vh, cb);
            const Vec3<double> x = zero_x ? vzero<double>() : VecFmt<F64>::load(S.v[S_X64], g.Vh, cb);
            const double m2 = h.st[r]->m2;
            Vec3<RO> ro, pv;
            if (!init) pv = VO::load(S.v[S_P], g.Vh, cb);
            double dd = 0.0, rp = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const double re = b.c[i].re - m2 * x.c[i].re + 0.5 * acc[r].c[i].re;
                const double im = b.c[i].im - m2 * x.c[i].im + 0.5 * acc[r].c[i].im;
                dd += re * re + im * im;
                if (!init) rp += re * (double)pv.c[i].re + im * (double)pv.c[i].im;
                ro.c[i].re = (RO)re;
                ro.c[i].im = (RO)im;
            }
            dots[2 * r] = dd;
            dots[2 * r + 1] = rp;
            VO::store(S.v[S_R], g.Vh, cb, ro);
        }
    }
    block_partials<2 * N>(G.partials, gblk, dots);
}

// p = r + beta p inside an iteration (gate G_ITER); p = a r + beta p after a reliable update or at the
// start (G_XPAY). Block partials of |p|^2 (as stored) feed the next alpha.
template <int VP, int N, class D>
__global__ __launch_bounds__(256) void k_xpay(D d, int gate, int remap) {
    using R = typename Real<VP>::T;
    using VF = VecFmt<VP>;
    const int lblk = logical_block(remap);
    const int gi = find_group(d, lblk);
    const GroupDev& G = grp_of(d, gi);
    const int gblk = lblk - G.blk0;
    const Rhs<N> h = rhs_of<N>(d, G, gate);
    if (!h.any) return;
    const int Vh = G.g.Vh;
    const int nr = G.nrhs;
    const int cb = gblk * blockDim.x + threadIdx.x;
    double dots[N];
#pragma unroll
    for (int r = 0; r < N; ++r) dots[r] = 0.0;
    if (cb < Vh) {
        // every load first (systems that do not update take p = 0 r + 1 p), then arithmetic, then stores
        Vec3<R> rv[N], pv[N];
        R a[N], beta[N];
#pragma unroll
        for (int r = 0; r < N; ++r) {
            const SysDev& S = sys_of(d, G.sys0 + (r < nr ? r : nr - 1));
            beta[r] = h.act[r] ? (R)h.st[r]->beta : R(1);
            a[r] = h.act[r] ? (gate == G_XPAY ? (R)h.st[r]->xpay_a : R(1)) : R(0);
            rv[r] = VF::load(S.v[S_R], Vh, cb);
            // beta = 0 (start of a solve, restart): p is not read, it may hold anything
            pv[r] = beta[r] != R(0) ? VF::load(S.v[S_P], Vh, cb) : vzero<R>();
        }
#pragma unroll
        for (int r = 0; r < N; ++r) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                pv[r].c[i].re = a[r] * rv[r].c[i].re + beta[r] * pv[r].c[i].re;
                pv[r].c[i].im = a[r] * rv[r].c[i].im + beta[r] * pv[r].c[i].im;
            }
        }
#pragma unroll
        for (int r = 0; r < N; ++r) {
            if (r >= nr) continue;
            const Vec3<R> ps = VF::store_rt(sys_of(d, G.sys0 + r).v[S_P], Vh, cb, pv[r]);
            double dd = 0.0;
#pragma unroll
            for (int i = 0; i < 3; ++i)
                dd += (double)ps.c[i].re * (double)ps.c[i].re + (double)ps.c[i].im * (double)ps.c[i].im;
            dots[r] = dd;
        }
    }
    block_sum<N>(dots);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int r = 0; r < N; ++r) G.partials_p[(size_t)gblk * N + r] = dots[r];
    }
}

// One system, after DS_UPDATE_FUSED: every block sums the |r|^2 partials (same order in every block) and
// takes the decisions of the update finalize itself (breakdown, convergence and reliable-update triggers,
// beta), then p = r + beta p with |p|^2 partials. The state is double-buffered: all blocks read st_in
// (the descriptor's state) and block 0 writes the advanced state to st_out, which the next iteration's
// launches read, so no block can see a half-written state. At a chunk end (chunk_end != 0) with a reliable
// update due, the launch instead performs the update's first step, x64 += x_lo and x_lo = 0.
template <int VP>
__global__ __launch_bounds__(256) void k_xpay_fused(DescSingle d, SolverState* __restrict__ st_out, int chunk_end,
                                                     int remap) {
    using R = typename Real<VP>::T;
    using VF = VecFmt<VP>;
    const int gblk = logical_block(remap);
    const GroupDev& G = d.grp;
    const SolverState* st = d.sys.st;
    const int Vh = G.g.Vh;
    const int cb = gblk * blockDim.x + threadIdx.x;
    const bool live = cb < Vh;
    // loads that do not depend on the state go first
    double part[1] = {0.0};
    double head[HEAD][1];
    const double* const src[1] = {G.partials_r};
    strided_head<1>(part, head, src, G.nblk);
    Vec3<R> rv = vzero<R>(), pv = vzero<R>();
    if (live) {
        rv = VF::load(d.sys.v[S_R], Vh, cb);
        pv = VF::load(d.sys.v[S_P], Vh, cb);
    }
    strided_tail<1>(part, head, G.nblk);
    block_sum<1>(part);
    __shared__ double beta_sh;
    __shared__ int go_sh, ru_sh;
    if (threadIdx.x == 0) {
        SolverState s = *st;
        bool go = false;
        if (!(s.flags & (ST_DONE | ST_PENDING))) {
            fin_alpha(&s, G.rec[0]);
            if (!(s.flags & ST_DONE)) fin_update(&s, part[0], chunk_end != 0);
            go = !(s.flags & (ST_DONE | ST_PENDING));
            if (go) s.flags |= ST_T_STALE;  // p formed here: a following k_norm_rec applies D_oe to it
        }
        if (gblk == 0) *st_out = s;
        beta_sh = s.beta;
        go_sh = go;
        ru_sh = chunk_end != 0 && (s.flags & ST_PENDING) && !(s.flags & ST_DONE);
    }
    __syncthreads();
    if constexpr (VP != F64) {
        if (ru_sh) {
            // the reliable update that follows the chunk starts here: x64 += x_lo; x_lo = 0 (k_accum's step)
            if (live) {
                Vec3<double> x = VecFmt<F64>::load(d.sys.v[S_X64], Vh, cb);
                const Vec3<float> xl = VecFmt<F32>::load(d.sys.v[S_XLO], Vh, cb);
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    x.c[i].re += (double)xl.c[i].re;
                    x.c[i].im += (double)xl.c[i].im;
                }
                VecFmt<F64>::store(d.sys.v[S_X64], Vh, cb, x);
                VecFmt<F32>::store(d.sys.v[S_XLO], Vh, cb, vzero<float>());
            }
            return;
        }
    }
    if (!go_sh) return;  // paused or stopped: p and its partials stay as they are
    const R beta = (R)beta_sh;
    double dots[1] = {0.0};
    if (live) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            pv.c[i].re = rv.c[i].re + beta * pv.c[i].re;
            pv.c[i].im = rv.c[i].im + beta * pv.c[i].im;
        }
        const Vec3<R> ps = VF::store_rt(d.sys.v[S_P], Vh, cb, pv);
#pragma unroll
        for (int i = 0; i < 3; ++i)
            dots[0] += (double)ps.c[i].re * (double)ps.c[i].re + (double)ps.c[i].im * (double)ps.c[i].im;
    }
    block_partials<1>(G.partials_p, gblk, dots);
}

// The first launch of an iteration of one system in FP32 or FP64 (with DS_UPDATE_FUSED the second). It
// replaces the p update and t = D_oe p of the three-launch iteration by the recurrence
//   p_i = r_i + beta p_{i-1},   t_i = D_oe p_i = D_oe r_i + beta t_{i-1},
// so that the operator is applied to r_i, which is complete when the launch starts, while p_i is formed in
// the same launch (each thread also updates the even site with its own index). Every block first takes the
// decisions of the last update from its |r|^2 partials (as k_xpay_fused does); block 0 writes the advanced
// state to st_out. When p was formed elsewhere (start, reliable update, end of the last chunk: ST_T_STALE)
// the launch applies D_oe to p directly and takes no decision. Partials: Re<D_oe in, t> as DS_NORM, and
// |p_i|^2 from the recurrence (the other paths leave the |p|^2 partials of the launch that formed p).
template <int LP, int RECON, int VP, bool NT = false>
__global__ __launch_bounds__(256) void k_norm_rec(DescSingle d, SolverState* __restrict__ st_out, int remap) {
    using R = typename Real<VP>::T;
    using VF = VecFmt<VP>;
    const int gblk = logical_block(remap);
    const GroupDev& G = d.grp;
    const SysDev& S = d.sys;
    const SolverState* st = S.st;
    const Geom g = G.g;
    const int cb = gblk * blockDim.x + threadIdx.x;
    const bool live = cb < g.Vh;
    const int flags = st->flags;
    if (flags & (ST_DONE | ST_PENDING)) {
        if (gblk == 0 && threadIdx.x == 0) *st_out = *st;
        return;
    }
    const bool direct = (flags & ST_T_STALE) != 0;
    double part[1] = {0.0};
    double head[HEAD][1];
    const double* const psrc[1] = {G.partials_r};
    if (!direct) strided_head<1>(part, head, psrc, G.nblk);
    Vec3<R> acc = vzero<R>(), told = vzero<R>(), rv = vzero<R>(), pv = vzero<R>();
    if (live) {
        acc = dslash_site<LP, RECON, VP, NT>(g, G.links_lo, direct ? S.v[S_P] : S.v[S_R], 1, site_of(g, 1, cb));
        if (!direct) {
            told = VF::load(S.v[S_T], g.Vh, cb);
            rv = VF::load(S.v[S_R], g.Vh, cb);
            pv = VF::load(S.v[S_P], g.Vh, cb);
        }
    }
    __shared__ double beta_sh;
    __shared__ int go_sh;
    if (!direct) {
        strided_tail<1>(part, head, G.nblk);
        block_sum<1>(part);
    }
    if (threadIdx.x == 0) {
        SolverState s = *st;
        bool go = true;
        if (direct) {
            s.flags &= ~ST_T_STALE;
        } else {
            fin_alpha(&s, G.rec[0]);
            if (!(s.flags & ST_DONE)) fin_update(&s, part[0], false);
            go = !(s.flags & (ST_DONE | ST_PENDING));
        }
        if (gblk == 0) *st_out = s;
        beta_sh = direct ? 0.0 : s.beta;
        go_sh = go;
    }
    __syncthreads();
    if (!go_sh) return;  // paused or stopped: t, p and their partials stay as they are
    const R beta = (R)beta_sh;
    double dots[2] = {0.0, 0.0};
    if (live) {
        Vec3<R> t = acc;
        if (!direct) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                t.c[i].re += beta * told.c[i].re;
                t.c[i].im += beta * told.c[i].im;
                pv.c[i].re = rv.c[i].re + beta * pv.c[i].re;
                pv.c[i].im = rv.c[i].im + beta * pv.c[i].im;
            }
            const Vec3<R> ps = VF::store_rt(S.v[S_P], g.Vh, cb, pv);
#pragma unroll
            for (int i = 0; i < 3; ++i)
                dots[1] += (double)ps.c[i].re * (double)ps.c[i].re + (double)ps.c[i].im * (double)ps.c[i].im;
        }
        const Vec3<R> ts = VF::store_rt(S.v[S_T], g.Vh, cb, t);
#pragma unroll
        for (int i = 0; i < 3; ++i)
            dots[0] += (double)t.c[i].re * (double)ts.c[i].re + (double)t.c[i].im * (double)ts.c[i].im;
    }
    block_sum<2>(dots);
    if (threadIdx.x == 0) {
        G.partials[gblk] = dots[0];
        if (!direct) G.partials_p[gblk] = dots[1];
    }
}

// x64 += xlo; xlo = 0 (reliable update).
template <int N, class D>
__global__ __launch_bounds__(256) void k_accum(D d, int remap) {
    const int lblk = logical_block(remap);
    const int gi = find_group(d, lblk);
    const GroupDev& G = grp_of(d, gi);
    const int gblk = lblk - G.blk0;
    const Rhs<N> h = rhs_of<N>(d, G, G_RU);
    if (!h.any) return;
    const int Vh = G.g.Vh;
    const int cb = gblk * blockDim.x + threadIdx.x;
    if (cb >= Vh) return;
#pragma unroll
    for (int r = 0; r < N; ++r) {
        if (!h.act[r]) continue;
        const SysDev& S = sys_of(d, G.sys0 + r);
        Vec3<double> x = VecFmt<F64>::load(S.v[S_X64], Vh, cb);
        const Vec3<float> xl = VecFmt<F32>::load(S.v[S_XLO], Vh, cb);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            x.c[i].re += (double)xl.c[i].re;
            x.c[i].im += (double)xl.c[i].im;
        }
        VecFmt<F64>::store(S.v[S_X64], Vh, cb, x);
        VecFmt<F32>::store(S.v[S_XLO], Vh, cb, vzero<float>());
    }
}

// Block partials of |b|^2 (-> bnorm2 and the stopping threshold tol^2 |b|^2).
template <int N, class D>
__global__ __launch_bounds__(256) void k_norm_b(D d, int remap) {
    const int lblk = logical_block(remap);
    const int gi = find_group(d, lblk);
    const GroupDev& G = grp_of(d, gi);
    const int gblk = lblk - G.blk0;
    const Rhs<N> h = rhs_of<N>(d, G, G_ALIVE);
    if (!h.any) return;
    const int Vh = G.g.Vh;
    const int cb = gblk * blockDim.x + threadIdx.x;
    double dots[N];
#pragma unroll
    for (int r = 0; r < N; ++r) {
        dots[r] = 0.0;
        if (!h.act[r] || cb >= Vh) continue;
        const Vec3<double> b = VecFmt<F64>::load(sys_of(d, G.sys0 + r).v[S_B64], Vh, cb);
#pragma unroll
        for (int i = 0; i < 3; ++i) dots[r] += b.c[i].re * b.c[i].re + b.c[i].im * b.c[i].im;
    }
    block_partials<N>(G.partials, gblk, dots);
}

// ------------------------------------------------------------------------------------------------------
// Second reduction stage, one block per group: sum the partials of the previous launch in block order and
// update the state of every system that launch worked on (same gate, and no state changed in between).
// ------------------------------------------------------------------------------------------------------
enum FinKind : int {
    FIN_ALPHA = 0,
    FIN_UPDATE = 1,      // inside a chunk
    FIN_RESID = 2,
    FIN_RESID_INIT = 3,
    FIN_NORM_B = 4,
    FIN_UPDATE_END = 5,  // last iteration of a chunk: also the delta and ru_every triggers
};

// partials of FIN_ALPHA: |D_oe p|^2 (from DS_NORM) and |p|^2 (from k_xpay)
//
// The launch is latency bound: 1024 threads put every partial load in flight at once (a few per thread);
// then thread r updates the state of system r.
template <int N, class D>
__global__ __launch_bounds__(1024) void k_finalize(D d, int kind, int gate) {
    const GroupDev& G = grp_of(d, blockIdx.x);
    const Rhs<N> h = rhs_of<N>(d, G, gate);
    if (!h.any) return;
    const bool two = kind == FIN_RESID || kind == FIN_RESID_INIT;
    const int nv = two ? 2 * N : N;
    // s[0..nv) from partials; for FIN_ALPHA s[N..2N) holds the |p|^2 partials
    double s[2 * N];
#pragma unroll
    for (int k = 0; k < 2 * N; ++k) s[k] = 0.0;
    for (int b = threadIdx.x; b < G.nblk; b += blockDim.x) {
#pragma unroll
        for (int k = 0; k < 2 * N; ++k) {
            if (k < nv) s[k] += G.partials[(size_t)b * nv + k];
            else if (kind == FIN_ALPHA) s[k] += G.partials_p[(size_t)b * N + (k - N)];
        }
    }
    block_sum<2 * N>(s);
    // thread r updates system r (the states are independent, their loads overlap)
    __shared__ double tot[2 * N];
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < 2 * N; ++k) tot[k] = s[k];
    }
    __syncthreads();
    const int r = threadIdx.x;
    if (r >= N || r >= G.nrhs) return;
    bool act = false;
    SolverState* st = nullptr;
#pragma unroll
    for (int q = 0; q < N; ++q)
        if (q == r) {
            act = h.act[q];
            st = h.st[q];
        }
    if (!act) return;
    if (kind == FIN_ALPHA) fin_alpha(st, st->m2 * tot[N + r] + tot[r]);
    else if (kind == FIN_UPDATE || kind == FIN_UPDATE_END) fin_update(st, tot[r], kind == FIN_UPDATE_END);
    else if (kind == FIN_NORM_B) {
        st->bnorm2 = tot[r];
        st->stop2 = st->tol2 * tot[r];
    } else fin_resid(st, tot[2 * r], tot[2 * r + 1], kind == FIN_RESID_INIT);
}

// ------------------------------------------------------------------------------------------------------
// Packing: natural complex128 <-> planes.
// ------------------------------------------------------------------------------------------------------
template <int P, int RECON>
__global__ __launch_bounds__(256) void k_pack_gauge(Geom g, const double* __restrict__ nat, void* out) {
    using LF = LinkFmt<P, RECON>;
    const long V = 2L * g.Vh;
    const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;  // mu * V + lex
    if (l >= 4 * V) return;
    const int mu = (int)(l / V);
    const int lex = (int)(l - (long)mu * V);
    const int x = lex % g.X, r1 = lex / g.X, y = r1 % g.Y, r2 = r1 / g.Y, z = r2 % g.Z, t = r2 / g.Z;
    const int q = (x + y + z + t) & 1;
    double r[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) r[k] = nat[l * 18 + k];
    LF::store((void*)link_block<LF>(out, g.Vh, q, mu), g.Vh, lex >> 1, r);
}

template <int P>
__global__ __launch_bounds__(256) void k_pack_vec(int Vh, const double* __restrict__ nat, void* out) {
    using R = typename Real<P>::T;
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    if (cb >= Vh) return;
    Vec3<R> v;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v.c[c].re = (R)nat[(size_t)cb * 6 + 2 * c];
        v.c[c].im = (R)nat[(size_t)cb * 6 + 2 * c + 1];
    }
    VecFmt<P>::store(out, Vh, cb, v);
}

template <int P>
__global__ __launch_bounds__(256) void k_unpack_vec(int Vh, const void* in, double* __restrict__ nat) {
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    if (cb >= Vh) return;
    const auto v = VecFmt<P>::load(in, Vh, cb);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        nat[(size_t)cb * 6 + 2 * c] = (double)v.c[c].re;
        nat[(size_t)cb * 6 + 2 * c + 1] = (double)v.c[c].im;
    }
}

}  // namespace sp
