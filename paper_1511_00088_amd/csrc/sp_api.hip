// C-ABI of libstagcg.so: argument checks, workspace layout, the CG drivers (single and batched), hipGraph
// chunk replay, the launch autotuner, and the force, full-lattice solve, HYP smearing and NPR contraction
// entry points.
//
// Solver schedule (mixed precision, after the FP64 set-up r = b - A x0):
//   chunk = poll_chunk iterations of
//             t = D_oe p                  (inner precision)
//             q = m^2 p - D_eo t, Re<p,q>  -> alpha (device)
//             x_lo += alpha p, r -= alpha q, |r|^2 -> beta, triggers (device)
//             p = r + beta p
//           then a reliable update when due (every ru_every iterations, when |r| drops below
//           delta * |r at the last update|, at apparent convergence and at the iteration cap):
//             x64 += x_lo, x_lo = 0; r = b - A x64 in FP64; r_lo = round(r); converged if |r| <= tol |b|
//   The host replays chunks (one hipGraph launch each) and reads the device state once per chunk. A single
//   system in FP32 or FP64 takes two launches per iteration: beta (with the stopping decisions), the p
//   update and t = D_oe r + beta t (the recurrence of t = D_oe p) in one, alpha and the x and r updates in
//   the other, each block forming the scalars from the block partials of the launch before; the chunk
//   ends with a p update alone, after which t is formed from p directly. With 16-bit storage a single
//   system takes three (t = D_oe p, the update, the p update), and batched groups take five: two one-block
//   finalize launches between them.
// Plain FP64 CG is the same schedule with FP64 vectors, x updated in place and the FP64 true residual
// computed only at apparent convergence.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include <dlfcn.h>

#include "sp_entry.h"

using namespace sp;

namespace {

thread_local std::string g_last_error;

// ---------------------------------------------------------------------------------------------------
// Diagnostics: a host log on stderr (SP_LOG=1: one line per solve; SP_LOG=2: also one per chunk poll) and roctx
// ranges per solve and per chunk for rocprofv3 --marker-trace, from the roctx library when it can be loaded (no
// link-time dependency; SP_ROCTX=0 turns the ranges off).
// ---------------------------------------------------------------------------------------------------
int log_level() {
    static const int level = [] {
        const char* e = getenv("SP_LOG");
        return e ? atoi(e) : 0;
    }();
    return level;
}

void log_line(int level, const char* fmt, ...) {
    if (log_level() < level) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    fprintf(stderr, "[libstagcg] %s\n", buf);
}

struct Roctx {
    int (*push)(const char*) = nullptr;
    int (*pop)() = nullptr;
    Roctx() {
        const char* e = getenv("SP_ROCTX");
        if (e && atoi(e) == 0) return;
        void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL | RTLD_NOLOAD);
        if (!h) h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_LOCAL);
        if (!h) return;
        push = (int (*)(const char*))dlsym(h, "roctxRangePushA");
        pop = (int (*)())dlsym(h, "roctxRangePop");
        if (!push || !pop) push = nullptr, pop = nullptr;
    }
};
const Roctx& roctx() {
    static const Roctx r;
    return r;
}

// A roctx range for the lifetime of the object.
struct TraceRange {
    bool on;
    explicit TraceRange(const char* msg) : on(roctx().push != nullptr) {
        if (on) roctx().push(msg);
    }
    ~TraceRange() {
        if (on) roctx().pop();
    }
};

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                                  \
    do {                                                                                               \
        hipError_t e_ = (expr);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(SP_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__,   \
                        __LINE__);                                                                     \
    } while (0)

inline size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

bool valid_prec(int p) { return p >= SP_F64 && p <= SP_BF16; }
// link storage also admits 16-bit fixed point
bool valid_link_prec(int p) { return valid_prec(p) || p == SP_I16; }
bool is_16bit_link(int p) { return p == SP_F16 || p == SP_BF16 || p == SP_I16; }

int check_geom(const sp_geom* g, Geom* out) {
    if (!g) return fail(SP_ERR_INVALID_ARG, "geometry is null");
    long V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        int L = g->dims[mu];
        if (L < 2 || (L & 1)) return fail(SP_ERR_ODD_EXTENT, "extent %d of direction %d is odd or < 2", L, mu);
        V *= L;
    }
    if (g->bc_t != 0 && g->bc_t != 1) return fail(SP_ERR_INVALID_ARG, "bc_t must be 0 or 1");
    if (V / 2 >= (1L << 24)) return fail(SP_ERR_UNSUPPORTED, "lattice too large: V/2 = %ld >= 2^24", V / 2);
    if (out) {
        out->X = g->dims[0];
        out->Y = g->dims[1];
        out->Z = g->dims[2];
        out->T = g->dims[3];
        out->Xh = g->dims[0] / 2;
        out->Vh = (int)(V / 2);
        out->bc_t = g->bc_t;
        out->rXh = 1.0f / (float)out->Xh;
        out->rY = 1.0f / (float)out->Y;
        out->rZ = 1.0f / (float)out->Z;
    }
    return SP_OK;
}

size_t link_bytes(int prec, int recon) {
    if (prec == SP_F64) return recon == 18 ? 144 : 0;
    if (prec == SP_F32) return recon == 18 ? 72 : recon == 12 ? 48 : recon == 8 ? 32 : 0;
    if (prec == SP_F16 || prec == SP_BF16 || prec == SP_I16) return recon == 18 ? 36 : recon == 12 ? 24 : 0;
    return 0;
}

size_t vec_site_bytes(int prec) {
    switch (prec) {
        case SP_F64: return 48;
        case SP_F32: return 24;
        case SP_F16: return 16;
        case SP_BF16: return 12;
    }
    return 0;
}

// ---------------------------------------------------------------------------------------------------
// Tuned launch configurations
// ---------------------------------------------------------------------------------------------------
std::mutex g_mu;  // guards every cache below and the pinned staging buffers
std::map<std::string, LaunchCfg> g_tune;

std::string tune_key(const Geom& g, int lp, int recon, int vp) {
    char b[128];
    snprintf(b, sizeof b, "%dx%dx%dx%d/l%d/r%d/v%d", g.X, g.Y, g.Z, g.T, lp, recon, vp);
    return b;
}

LaunchCfg tuned_cfg(const Geom& g, int lp, int recon, int vp) {
    auto it = g_tune.find(tune_key(g, lp, recon, vp));
    return it == g_tune.end() ? LaunchCfg{} : it->second;
}

// Launch shape of the NB-right-hand-side operator ("/n4" entry), else the single-system one.
LaunchCfg tuned_cfg_batched(const Geom& g, int lp, int recon, int vp) {
    auto it = g_tune.find(tune_key(g, lp, recon, vp) + "/n4");
    return it == g_tune.end() ? tuned_cfg(g, lp, recon, vp) : it->second;
}

// Launch shape of a single solve's iteration ("/solve" entry: block order and link-load policy timed on the
// solver's own launches, by the tuning driver), else the plain operator's.
LaunchCfg tuned_cfg_solve(const Geom& g, int lp, int recon, int vp) {
    auto it = g_tune.find(tune_key(g, lp, recon, vp) + "/solve");
    return it == g_tune.end() ? tuned_cfg(g, lp, recon, vp) : it->second;
}

// ---------------------------------------------------------------------------------------------------
// Pinned host staging (control block upload, state polls)
// ---------------------------------------------------------------------------------------------------
struct Pinned {
    void* p = nullptr;
    size_t n = 0;
    hipError_t ensure(size_t bytes) {
        if (bytes <= n) return hipSuccess;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
        // coherent: the poll slots are written by a kernel (the last node of a chunk's graph) and read by the host
        hipError_t e = hipHostMalloc(&p, bytes, hipHostMallocCoherent);
        if (e == hipSuccess) n = bytes;
        return e;
    }
};
Pinned g_upload, g_poll;

struct Events {
    hipEvent_t e[2] = {nullptr, nullptr};
    hipError_t create() {
        for (auto& x : e) {
            hipError_t r = hipEventCreateWithFlags(&x, hipEventDisableTiming);
            if (r) return r;
        }
        return hipSuccess;
    }
    ~Events() {
        for (auto& x : e)
            if (x) (void)hipEventDestroy(x);
    }
};

// ---------------------------------------------------------------------------------------------------
// Workspace layout of a solve over a list of systems grouped by (gauge, geometry)
// ---------------------------------------------------------------------------------------------------
struct GroupPlan {
    Geom g;
    const sp_gauge* U;
    std::vector<int> sys;  // indices into the caller's system list
    int nblk = 0, blk0 = 0;
    size_t partials_off = 0, partials_p_off = 0, partials_r_off = 0, rec_off = 0;
};

struct Layout {
    std::vector<GroupPlan> groups;
    std::vector<size_t> sys_off;  // byte offset of each system's vector block
    std::vector<int> sys_group;
    size_t states_off = 0, gdesc_off = 0, sdesc_off = 0, ctrl_bytes = 0;
    size_t total = 0;
    int inner = SP_F32, nbatch_rhs = 1;
    int total_blocks = 0;
    LaunchCfg cfg;
};

// Per-system vector block: B64 X64 T64 (48 B/site), XLO (24 B/site, mixed only), P R T (inner).
size_t sys_block_bytes(int Vh, int inner, size_t slot_off[NSLOT]) {
    size_t off = 0;
    const size_t v64 = align256((size_t)Vh * 48);
    const size_t vin = align256((size_t)Vh * vec_site_bytes(inner));
    slot_off[S_B64] = off; off += v64;
    slot_off[S_X64] = off; off += v64;
    slot_off[S_T64] = off; off += v64;
    slot_off[S_XLO] = off; if (inner != SP_F64) off += align256((size_t)Vh * 24);
    slot_off[S_P] = off; off += vin;
    slot_off[S_R] = off; off += vin;
    slot_off[S_T] = off; off += vin;
    return off;
}

// Groups systems and computes the workspace layout. n_rhs_max: 1 for a single solve, NB for batches.
int make_layout(int nsys, const sp_system* systems, const sp_cg_params* prm, int n_rhs_max, Layout* L) {
    if (nsys <= 0 || !systems) return fail(SP_ERR_INVALID_ARG, "no systems");
    if (!prm) return fail(SP_ERR_INVALID_ARG, "params is null");
    if (!valid_prec(prm->inner)) return fail(SP_ERR_INVALID_ARG, "bad inner precision %d", prm->inner);
    L->inner = prm->inner;
    L->nbatch_rhs = n_rhs_max;
    L->groups.clear();
    for (int i = 0; i < nsys; ++i) {
        const sp_system& s = systems[i];
        Geom g;
        int rc = check_geom(s.g, &g);
        if (rc) return rc;
        if (!s.U) return fail(SP_ERR_INVALID_ARG, "system %d: gauge is null", i);
        int gi = -1;
        for (size_t k = 0; k < L->groups.size(); ++k) {
            GroupPlan& G = L->groups[k];
            if ((int)G.sys.size() < n_rhs_max && G.U->f64 == s.U->f64 && G.U->lo == s.U->lo &&
                G.U->recon == s.U->recon && G.U->lo_prec == s.U->lo_prec && !memcmp(&G.g, &g, sizeof g)) {
                gi = (int)k;
                break;
            }
        }
        if (gi < 0) {
            GroupPlan G;
            G.g = g;
            G.U = s.U;
            L->groups.push_back(G);
            gi = (int)L->groups.size() - 1;
        }
        L->groups[gi].sys.push_back(i);
    }
    // launch shape: the tuned block size of the largest group's operator
    int big = 0;
    for (size_t k = 1; k < L->groups.size(); ++k)
        if (L->groups[k].g.Vh > L->groups[big].g.Vh) big = (int)k;
    {
        const GroupPlan& G = L->groups[big];
        const int lp = prm->inner == SP_F64 ? SP_F64 : G.U->lo_prec;
        const int rc = prm->inner == SP_F64 ? 18 : G.U->recon;
        L->cfg = n_rhs_max > 1 ? tuned_cfg_batched(G.g, lp, rc, prm->inner) : tuned_cfg_solve(G.g, lp, rc, prm->inner);
        // one system: 256-thread blocks whenever they admit the fused iteration, whose launches have every block
        // sum the partials of all blocks (smaller blocks mean more partials per block); the block order and the
        // link-load policy stay the tuned ones. Measured: FP16 links with 128-thread blocks (the plain operator's
        // tuned shape) took the 20^3x64 solve from 21.9 to 25.8 ms.
        if (n_rhs_max == 1 && blocks_for(G.g.Vh, 256) <= FUSED_PARTIALS * 256) L->cfg.nt = 256;
    }
    int blk = 0;
    for (auto& G : L->groups) {
        G.nblk = blocks_for(G.g.Vh, L->cfg.nt);
        G.blk0 = blk;
        blk += G.nblk;
    }
    L->total_blocks = blk;
    // control block: states, descriptors
    size_t off = 0;
    // states: nsys current ones, then nsys spares (the second buffer of the fused single-system iteration)
    L->states_off = off;
    off += align256(sizeof(SolverState) * 2 * nsys);
    L->gdesc_off = off;
    off += align256(sizeof(GroupDev) * L->groups.size());
    L->sdesc_off = off;
    off += align256(sizeof(SysDev) * nsys);
    L->ctrl_bytes = off;
    // partials: sized for the smallest block size so that retuning never overflows them
    for (auto& G : L->groups) {
        G.partials_off = off;
        off += align256(sizeof(double) * (size_t)(2 * NB) * blocks_for(G.g.Vh, 64));
        G.partials_p_off = off;
        off += align256(sizeof(double) * (size_t)NB * blocks_for(G.g.Vh, 64));
        G.partials_r_off = off;
        off += align256(sizeof(double) * (size_t)blocks_for(G.g.Vh, 64));
        G.rec_off = off;
        off += align256(sizeof(double) * 2);
    }
    L->sys_off.assign(nsys, 0);
    L->sys_group.assign(nsys, 0);
    for (size_t k = 0; k < L->groups.size(); ++k)
        for (int i : L->groups[k].sys) {
            size_t so[NSLOT];
            L->sys_off[i] = off;
            L->sys_group[i] = (int)k;
            off += sys_block_bytes(L->groups[k].g.Vh, L->inner, so);
        }
    L->total = off;
    return SP_OK;
}

int check_gauge(const sp_gauge* U, int inner) {
    if (!U->f64) return fail(SP_ERR_INVALID_ARG, "gauge f64 packing is null");
    if (inner == SP_F64) return SP_OK;
    if (!U->lo) return fail(SP_ERR_INVALID_ARG, "gauge lo packing is null");
    // FP32 iterations also take links stored at 16 bits (FP32 vectors and arithmetic); 16-bit vector storage
    // needs links of its own precision
    const bool links_ok = U->lo_prec == inner || (inner == SP_F32 && is_16bit_link(U->lo_prec));
    if (!links_ok)
        return fail(SP_ERR_UNSUPPORTED, "gauge lo precision %d cannot serve inner precision %d", U->lo_prec, inner);
    if (U->recon != 18 && U->recon != 12 && U->recon != 8)
        return fail(SP_ERR_INVALID_ARG, "recon must be 18, 12 or 8");
    if (U->recon == 8 && U->lo_prec != SP_F32) return fail(SP_ERR_UNSUPPORTED, "recon 8 is built for FP32 links only");
    return SP_OK;
}

// ---------------------------------------------------------------------------------------------------
// Enqueue helpers
// ---------------------------------------------------------------------------------------------------
struct Plan {
    int inner, lp, recon, nblocks, ngroups;
    LaunchCfg cfg;
};

// One system with at most FUSED_PARTIALS partials per thread: every block of the update forms alpha itself and
// every block of the launch that updates p forms beta and the stopping decisions itself, so no finalize
// launch is needed (FP32/FP64: k_norm_rec, k_dslash DS_UPDATE_FUSED; 16-bit: k_dslash DS_NORM,
// DS_UPDATE_FUSED, k_xpay_fused).
template <class D>
bool fused_single(const Plan& pl) {
    return std::is_same<D, DescSingle>::value && pl.nblocks <= FUSED_PARTIALS * pl.cfg.nt;
}

// One CG iteration: t = D_oe p (|t|^2) -> alpha -> x += alpha p, r -= alpha (m^2 p - D_eo t) (|r|^2) -> beta
// and triggers -> p = r + beta p (|p|^2).
template <class D>
hipError_t enqueue_iterations(const D& d, const Plan& pl, int count, hipStream_t s) {
    const int use64 = pl.inner == SP_F64;
    for (int i = 0; i < count; ++i) {
        hipError_t e;
        if ((e = launch_dslash(d, pl.nblocks, pl.cfg, pl.lp, pl.recon, pl.inner, 1, S_P, S_T, DS_NORM, G_ITER, use64,
                               s)))
            return e;
        if ((e = launch_finalize(d, pl.ngroups, FIN_ALPHA, G_ITER, s))) return e;
        if ((e = launch_dslash(d, pl.nblocks, pl.cfg, pl.lp, pl.recon, pl.inner, 0, S_T, S_R, DS_UPDATE, G_ITER,
                               use64, s)))
            return e;
        if ((e = launch_finalize(d, pl.ngroups, i + 1 == count ? FIN_UPDATE_END : FIN_UPDATE, G_ITER, s))) return e;
        if ((e = launch_xpay(d, pl.nblocks, pl.cfg, pl.inner, G_ITER, s))) return e;
    }
    return hipSuccess;
}

// The fused single-system iteration. Iteration i reads state buffer i % 2 (the descriptor's state and the
// spare right after it) and writes the other; an odd count ends with a copy back, so that between chunks
// the state is always in the descriptor's buffer.
hipError_t enqueue_iterations_fused(const DescSingle& d0, const Plan& pl, int count, hipStream_t s) {
    const int use64 = pl.inner == SP_F64;
    DescSingle d[2] = {d0, d0};
    d[1].sys.st = d0.sys.st + 1;
    if (pl.inner == SP_F32 || pl.inner == SP_F64) {
        // two launches per iteration (t and p by recurrence in k_norm_rec); the chunk's last p update is
        // k_xpay_fused, so the next chunk starts from a p and t that the chunk boundary leaves consistent
        for (int i = 0; i < count; ++i) {
            hipError_t e;
            if ((e = launch_norm_rec(d[i & 1], d[(i + 1) & 1].sys.st, pl.nblocks, pl.cfg, pl.lp, pl.recon, pl.inner,
                                     s)))
                return e;
            if ((e = launch_dslash(d[(i + 1) & 1], pl.nblocks, pl.cfg, pl.lp, pl.recon, pl.inner, 0, S_T, S_R,
                                   DS_UPDATE_FUSED, G_ITER, use64, s)))
                return e;
        }
        hipError_t e = launch_xpay_fused(d[count & 1], d[(count + 1) & 1].sys.st, 1, pl.nblocks, pl.cfg, pl.inner, s);
        if (e) return e;
        if ((count + 1) & 1) return launch_state_copy(d[1].sys.st, d[0].sys.st, s);
        return hipSuccess;
    }
    for (int i = 0; i < count; ++i) {
        const DescSingle& di = d[i & 1];
        hipError_t e;
        if ((e = launch_dslash(di, pl.nblocks, pl.cfg, pl.lp, pl.recon, pl.inner, 1, S_P, S_T, DS_NORM, G_ITER,
                               use64, s)))
            return e;
        if ((e = launch_dslash(di, pl.nblocks, pl.cfg, pl.lp, pl.recon, pl.inner, 0, S_T, S_R, DS_UPDATE_FUSED,
                               G_ITER, use64, s)))
            return e;
        if ((e = launch_xpay_fused(di, d[(i + 1) & 1].sys.st, i + 1 == count, pl.nblocks, pl.cfg, pl.inner, s)))
            return e;
    }
    if (count & 1) return launch_state_copy(d[1].sys.st, d[0].sys.st, s);
    return hipSuccess;
}

// Reliable update (runs only for systems whose last iteration requested it): x64 += x_lo; t64 = D_oe x64;
// r = b - A x64 in FP64 (|r|^2, Re<r,p>) -> state; p = a r + beta p.
template <class D>
hipError_t enqueue_reliable(const D& d, const Plan& pl, bool accum_done, hipStream_t s) {
    hipError_t e;
    if (pl.inner != SP_F64 && !accum_done && (e = launch_accum(d, pl.nblocks, pl.cfg, s))) return e;
    if ((e = launch_dslash(d, pl.nblocks, pl.cfg, SP_F64, 18, SP_F64, 1, S_X64, S_T64, DS_PLAIN, G_RU, 1, s)))
        return e;
    if ((e = launch_resid(d, pl.nblocks, pl.cfg, pl.inner, 0, s))) return e;
    if ((e = launch_finalize(d, pl.ngroups, FIN_RESID, G_RU, s))) return e;
    return launch_xpay(d, pl.nblocks, pl.cfg, pl.inner, G_XPAY, s);
}

// Start of a solve: |b|^2; r = b - A x0 in FP64 (r = b when there is no x0: no operator); p = r.
template <class D>
hipError_t enqueue_setup(const D& d, const Plan& pl, bool zero_x0, hipStream_t s) {
    hipError_t e;
    if ((e = launch_norm_b(d, pl.nblocks, pl.cfg, s))) return e;
    if ((e = launch_finalize(d, pl.ngroups, FIN_NORM_B, G_ALIVE, s))) return e;
    if (!zero_x0 &&
        (e = launch_dslash(d, pl.nblocks, pl.cfg, SP_F64, 18, SP_F64, 1, S_X64, S_T64, DS_PLAIN, G_ALIVE, 1, s)))
        return e;
    if ((e = launch_resid(d, pl.nblocks, pl.cfg, pl.inner, zero_x0 ? 2 : 1, s))) return e;
    if ((e = launch_finalize(d, pl.ngroups, FIN_RESID_INIT, G_ALIVE, s))) return e;
    return launch_xpay(d, pl.nblocks, pl.cfg, pl.inner, G_XPAY, s);
}

template <class D>
hipError_t enqueue_chunk(const D& d, const Plan& pl, int iters, hipStream_t s) {
    hipError_t e;
    // the fused iteration's chunk-end k_xpay_fused already folds x_lo into x64 when an update is due
    const bool fused = fused_single<D>(pl);
    if constexpr (std::is_same<D, DescSingle>::value)
        e = fused ? enqueue_iterations_fused(d, pl, iters, s) : enqueue_iterations(d, pl, iters, s);
    else
        e = enqueue_iterations(d, pl, iters, s);
    if (e) return e;
    return enqueue_reliable(d, pl, fused, s);
}

// ---------------------------------------------------------------------------------------------------
// hipGraph cache: one executable graph per (descriptor bytes, plan, chunk length)
// ---------------------------------------------------------------------------------------------------
std::map<std::string, hipGraphExec_t> g_graphs;
constexpr size_t kMaxGraphs = 64;
hipStream_t g_capture_stream = nullptr;
int g_capture_device = -1;

template <class D>
std::string graph_key(const D& d, const Plan& pl, int iters, const SolverState* states, SolverState* publish,
                      int nsys) {
    std::string k((const char*)&d, sizeof d);
    k.append((const char*)&pl, sizeof pl);
    k.append((const char*)&iters, sizeof iters);
    k.append((const char*)&states, sizeof states);
    k.append((const char*)&publish, sizeof publish);
    k.append((const char*)&nsys, sizeof nsys);
    int dev = 0;
    (void)hipGetDevice(&dev);
    k.append((const char*)&dev, sizeof dev);
    return k;
}

void release_graphs();

// The graph of one chunk: its iterations, then the systems' states copied to `publish` (pinned host memory the
// host polls), so that no separate copy, with its own submission gap, follows each chunk.
template <class D>
hipError_t chunk_graph(const D& d, const Plan& pl, int iters, const SolverState* states, SolverState* publish,
                       int nsys, hipGraphExec_t* out) {
    const std::string key = graph_key(d, pl, iters, states, publish, nsys);
    auto it = g_graphs.find(key);
    if (it != g_graphs.end()) {
        *out = it->second;
        return hipSuccess;
    }
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e) return e;
    if (!g_capture_stream || g_capture_device != dev) {
        if (g_capture_stream) (void)hipStreamDestroy(g_capture_stream);
        g_capture_stream = nullptr;
        if ((e = hipStreamCreateWithFlags(&g_capture_stream, hipStreamNonBlocking))) return e;
        g_capture_device = dev;
    }
    if ((e = hipStreamBeginCapture(g_capture_stream, hipStreamCaptureModeThreadLocal))) return e;
    hipError_t ee = enqueue_chunk(d, pl, iters, g_capture_stream);
    if (!ee) ee = launch_state_publish(states, publish, nsys, g_capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g_capture_stream, &graph);
    if (ee) {
        if (graph) (void)hipGraphDestroy(graph);
        return ee;
    }
    if (e) return e;
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e) return e;
    g_graphs[key] = exec;
    *out = exec;
    return hipSuccess;
}

void release_graphs() {
    for (auto& kv : g_graphs) (void)hipGraphExecDestroy(kv.second);
    g_graphs.clear();
}

// ---------------------------------------------------------------------------------------------------
// Solve driver shared by sp_cg_solve (DescSingle) and sp_cg_solve_batched (DescBatch)
// ---------------------------------------------------------------------------------------------------
SolverState initial_state(const sp_system& s, const sp_cg_params* prm, int chunk) {
    SolverState st;
    memset(&st, 0, sizeof st);
    st.tol2 = prm->tol * prm->tol;
    // plain FP64 CG recomputes the true residual only when the iterated one says it has converged
    st.delta2 = (prm->delta > 0 && prm->inner != SP_F64) ? prm->delta * prm->delta : 0.0;
    st.floor2 = prm->inner != SP_F64 ? 1e-6 : 0.0;  // |r| three decades below the last true residual
    st.m2 = s.mass * s.mass;
    st.max_iter = prm->max_iter;
    // FP32 iterations on FP32 or 16-bit fixed-point links keep the direction across a reliable update unless
    // the true |r|^2 exceeds the recursive one by more than 1.5x; the fixed-point links (within 2^-16 of the
    // true ones) update every 50 iterations, or at every end of the 75-iteration chunks of large single solves.
    // FP16 and BF16 storage, of the vectors or of the links, moves the inner operator by about 2^-11 |A| and
    // 2^-8 |A|, far more than the smallest eigenvalue m^2 of a light-quark system: FP16 keeps the direction
    // unless the residual has drifted by 1.25x (a kept direction without that check stalls the solve), BF16
    // restarts it at every update (fewer iterations at the default schedule than any drift factor measured)
    const bool fixed16_links = prm->inner == SP_F32 && s.U && s.U->lo_prec == SP_I16;
    const bool f16 = prm->inner == SP_F16 || (prm->inner == SP_F32 && s.U && s.U->lo_prec == SP_F16);
    const bool bf16 = prm->inner == SP_BF16 || (prm->inner == SP_F32 && s.U && s.U->lo_prec == SP_BF16);
    int every = prm->ru_every;
    if (prm->inner == SP_F64) every = INT_MAX;
    else if (every <= 0) every = fixed16_links ? (chunk == 75 ? 75 : 50) : 100;
    st.ru_every = every;
    st.drift = bf16 ? 0.0 : f16 ? 1.25 : 1.5;
    return st;
}

int status_of(const SolverState& st) {
    if (st.flags & ST_BREAKDOWN) return SP_ERR_BREAKDOWN;
    if (st.flags & ST_CONVERGED) return SP_OK;
    return SP_NOT_CONVERGED;
}

int solve_impl(int nsys, const sp_system* systems, const sp_cg_params* prm, sp_cg_stats* stats, void* ws,
               size_t ws_bytes, hipStream_t stream, bool batched) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!prm) return fail(SP_ERR_INVALID_ARG, "params is null");
    if (!(prm->tol > 0.0) || !(prm->tol < 1.0)) return fail(SP_ERR_INVALID_ARG, "tol must be in (0, 1)");
    if (prm->max_iter <= 0) return fail(SP_ERR_INVALID_ARG, "max_iter must be > 0");
    if (prm->delta < 0.0 || prm->delta >= 1.0) return fail(SP_ERR_INVALID_ARG, "delta must be in [0, 1)");
    for (int i = 0; i < nsys; ++i) {
        if (!systems[i].b_e || !systems[i].x_e) return fail(SP_ERR_INVALID_ARG, "system %d: b or x is null", i);
        if (!std::isfinite(systems[i].mass)) return fail(SP_ERR_INVALID_ARG, "system %d: mass not finite", i);
        if (!systems[i].U) return fail(SP_ERR_INVALID_ARG, "system %d: gauge is null", i);
        int rc = check_gauge(systems[i].U, prm->inner);
        if (rc) return rc;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    Layout L;
    int rc = make_layout(nsys, systems, prm, batched ? NB : 1, &L);
    if (rc) return rc;
    char range[160];
    snprintf(range, sizeof range, "%s %dx%dx%dx%d inner=%d links=%d/r%d systems=%d", batched ? "sp_cg_solve_batched" : "sp_cg_solve",
             L.groups[0].g.X, L.groups[0].g.Y, L.groups[0].g.Z, L.groups[0].g.T, prm->inner,
             prm->inner == SP_F64 ? SP_F64 : L.groups[0].U->lo_prec, prm->inner == SP_F64 ? 18 : L.groups[0].U->recon, nsys);
    const TraceRange solve_range(range);
    if (!ws) return fail(SP_ERR_WORKSPACE, "workspace is null");
    if (ws_bytes < L.total) return fail(SP_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, L.total);
    if (((uintptr_t)ws) & 255) return fail(SP_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    char* base = (char*)ws;
    for (auto& G : L.groups)
        if ((L.inner != SP_F64) && (G.U->recon != L.groups[0].U->recon || G.U->lo_prec != L.groups[0].U->lo_prec))
            return fail(SP_ERR_UNSUPPORTED, "all systems of a batch must share the link packing");

    // Iterations per chunk, when the caller leaves it, for single solves of at least 2^16 even sites, where each
    // chunk boundary costs a graph launch and a state poll (about 17 us): 100 with FP32 iterations on FP32 links
    // (or plain FP64 CG), where the t recurrence and the kept direction need no earlier reset (20^3x64: 499
    // iterations at any length from 20 to 100, 23.7 -> 23.4 ms); 75 on fixed-point links, with a reliable update
    // at every chunk end (20^3x64: 511-514 iterations and 8 updates, 18.0 ms, against 502 and 11, 18.1 ms, with
    // chunks of 25 and an update every 50). 25 otherwise: with FP16 or BF16 links or vectors the reliable-update
    // triggers, checked at chunk ends, set the iteration count, and small or batched solves keep the finer polling.
    const int lo0 = L.inner == SP_F64 ? SP_F64 : L.groups[0].U->lo_prec;
    int chunk = prm->poll_chunk;
    if (chunk <= 0) {
        const bool full_links = L.inner == SP_F64 || (L.inner == SP_F32 && lo0 == SP_F32);
        const bool fixed_links = L.inner == SP_F32 && lo0 == SP_I16;
        const bool large = !batched && L.groups[0].g.Vh >= (1 << 16);
        chunk = large && full_links ? 100 : large && fixed_links ? 75 : 25;
    }

    // ---- control block on the host ----
    HIP_TRY(g_upload.ensure(L.ctrl_bytes));
    char* h = (char*)g_upload.p;
    memset(h, 0, L.ctrl_bytes);
    SolverState* hst = (SolverState*)(h + L.states_off);
    for (int i = 0; i < nsys; ++i) hst[i] = initial_state(systems[i], prm, chunk);
    GroupDev* hg = (GroupDev*)(h + L.gdesc_off);
    SysDev* hs = (SysDev*)(h + L.sdesc_off);
    int sys_counter = 0;
    std::vector<int> order(nsys);  // descriptor index -> caller index
    for (size_t k = 0; k < L.groups.size(); ++k) {
        const GroupPlan& G = L.groups[k];
        GroupDev gd;
        memset(&gd, 0, sizeof gd);
        gd.g = G.g;
        gd.links64 = G.U->f64;
        gd.links_lo = prm->inner == SP_F64 ? G.U->f64 : G.U->lo;
        gd.partials = (double*)(base + G.partials_off);
        gd.partials_p = (double*)(base + G.partials_p_off);
        gd.partials_r = (double*)(base + G.partials_r_off);
        gd.rec = (double*)(base + G.rec_off);
        gd.nrhs = (int)G.sys.size();
        gd.sys0 = sys_counter;
        gd.blk0 = G.blk0;
        gd.nblk = G.nblk;
        hg[k] = gd;
        for (int i : G.sys) {
            size_t so[NSLOT];
            sys_block_bytes(G.g.Vh, L.inner, so);
            SysDev sd;
            for (int sl = 0; sl < NSLOT; ++sl) sd.v[sl] = base + L.sys_off[i] + so[sl];
            sd.st = (SolverState*)(base + L.states_off) + i;
            hs[sys_counter] = sd;
            order[sys_counter] = i;
            ++sys_counter;
        }
    }
    HIP_TRY(hipMemcpyAsync(base, h, L.ctrl_bytes, hipMemcpyHostToDevice, stream));

    // ---- pack b and x0 ----
    for (int i = 0; i < nsys; ++i) {
        const GroupPlan& G = L.groups[L.sys_group[i]];
        size_t so[NSLOT];
        sys_block_bytes(G.g.Vh, L.inner, so);
        char* sb = base + L.sys_off[i];
        HIP_TRY(launch_pack_vec(G.g.Vh, systems[i].b_e, SP_F64, sb + so[S_B64], stream));
        if (prm->use_x0) HIP_TRY(launch_pack_vec(G.g.Vh, systems[i].x_e, SP_F64, sb + so[S_X64], stream));
        else HIP_TRY(launch_zero(sb + so[S_X64], align256((size_t)G.g.Vh * 48), stream));
        if (L.inner != SP_F64) HIP_TRY(launch_zero(sb + so[S_XLO], align256((size_t)G.g.Vh * 24), stream));
    }

    Plan pl;
    pl.inner = L.inner;
    pl.lp = L.inner == SP_F64 ? SP_F64 : L.groups[0].U->lo_prec;
    pl.recon = L.inner == SP_F64 ? 18 : L.groups[0].U->recon;
    pl.nblocks = L.total_blocks;
    pl.ngroups = (int)L.groups.size();
    pl.cfg = L.cfg;

    HIP_TRY(g_poll.ensure(2 * sizeof(SolverState) * nsys));
    SolverState* slots[2] = {(SolverState*)g_poll.p, (SolverState*)g_poll.p + nsys};

    DescSingle ds;
    DescBatch db;
    memset(&ds, 0, sizeof ds);
    memset(&db, 0, sizeof db);
    if (!batched) {
        ds.grp = hg[0];
        ds.sys = hs[0];
    } else {
        db.grp = (const GroupDev*)(base + L.gdesc_off);
        db.sys = (const SysDev*)(base + L.sdesc_off);
        db.ngroups = (int)L.groups.size();
    }
    const bool zero_x0 = !prm->use_x0;
    auto setup = [&]() {
        return batched ? enqueue_setup(db, pl, zero_x0, stream) : enqueue_setup(ds, pl, zero_x0, stream);
    };
    HIP_TRY(setup());

    // with graphs, one per poll slot: each ends by copying the states into its slot. Near convergence the
    // chunks are shorter (tail iterations), so that the last one does not run many iterations past the point
    // where every system stopped: those return at once, but each still costs a launch.
    const int tail = std::min(chunk, 25);
    const SolverState* dev_states = (const SolverState*)(base + L.states_off);
    hipGraphExec_t exec[2] = {nullptr, nullptr}, exec_tail[2] = {nullptr, nullptr};
    auto graphs = [&](int len, hipGraphExec_t* out) -> hipError_t {
        for (int k = 0; k < 2; ++k) {
            hipError_t e = batched ? chunk_graph(db, pl, len, dev_states, slots[k], nsys, &out[k])
                                   : chunk_graph(ds, pl, len, dev_states, slots[k], nsys, &out[k]);
            if (e) return e;
        }
        return hipSuccess;
    };
    // the cache is trimmed before this solve takes any graph from it (its two chunk lengths add at most four),
    // never while one it holds may be queued
    if (prm->use_graph && g_graphs.size() + 4 > kMaxGraphs) release_graphs();
    if (prm->use_graph) HIP_TRY(graphs(chunk, exec));
    Events ev;
    HIP_TRY(ev.create());
    // Chunks are pipelined: chunk c is queued before the state written by chunk c-1 is inspected, so the
    // GPU does not wait for the host. Near convergence (estimated from the residual decay between polls)
    // the host waits for each chunk before queueing the next one, so that no chunk is launched only to
    // find every system stopped, and the chunks take `tail` iterations.
    const long max_chunks = (long)prm->max_iter / tail + 64;
    SolverState* poll = nullptr;
    std::vector<double> last_rho(nsys, -1.0);
    std::vector<int> last_iter(nsys, 0);
    bool careful = false;
    auto all_done = [&](const SolverState* st) {
        for (int i = 0; i < nsys; ++i)
            if (!(st[i].flags & ST_DONE)) return false;
        return true;
    };
    for (long c = 0;; ++c) {
        if (careful && c > 0) {
            HIP_TRY(hipEventSynchronize(ev.e[(c - 1) & 1]));
            if (all_done(slots[(c - 1) & 1])) {
                poll = slots[(c - 1) & 1];
                break;
            }
        }
        {
            char cr[48];
            snprintf(cr, sizeof cr, "chunk %ld", c);
            const TraceRange chunk_range(cr);
            const int len = careful ? tail : chunk;
            if (prm->use_graph && len != chunk && !exec_tail[0]) HIP_TRY(graphs(len, exec_tail));
            hipGraphExec_t g = len != chunk ? exec_tail[c & 1] : exec[c & 1];
            if (g) {
                HIP_TRY(hipGraphLaunch(g, stream));
            } else {
                HIP_TRY(batched ? enqueue_chunk(db, pl, len, stream) : enqueue_chunk(ds, pl, len, stream));
                HIP_TRY(hipMemcpyAsync(slots[c & 1], dev_states, sizeof(SolverState) * nsys, hipMemcpyDeviceToHost,
                                       stream));
            }
        }
        HIP_TRY(hipEventRecord(ev.e[c & 1], stream));
        if (c > max_chunks) {
            // cannot happen unless the device state is corrupted: every system stops at max_iter
            HIP_TRY(hipStreamSynchronize(stream));
            return fail(SP_ERR_HIP, "solver did not stop after %ld chunks", c);
        }
        if (careful || c == 0) continue;
        HIP_TRY(hipEventSynchronize(ev.e[(c - 1) & 1]));
        SolverState* prev = slots[(c - 1) & 1];
        log_line(2, "poll after chunk %ld: system 0 iter %d |r|^2 %.3e flags %d", c - 1, prev[0].iter, prev[0].rho_new,
                 prev[0].flags);
        if (all_done(prev)) {
            poll = prev;
            break;
        }
        // iterations still needed, from the decay of the iterated |r|^2 since the previous poll
        double need = 0.0;
        for (int i = 0; i < nsys; ++i) {
            const SolverState& st = prev[i];
            if (st.flags & ST_DONE) continue;
            const double rho = st.rho_new > 0 ? st.rho_new : st.rho;
            double est = 1e30;
            if (last_rho[i] > 0 && rho > 0 && rho < last_rho[i] && st.iter > last_iter[i] && st.stop2 > 0) {
                const double rate = std::log(last_rho[i] / rho) / (st.iter - last_iter[i]);
                est = rho <= st.stop2 ? 0.0 : std::log(rho / st.stop2) / rate;
            }
            need = std::max(need, est);
            last_rho[i] = rho;
            last_iter[i] = st.iter;
        }
        // chunk c is in flight: switch when what is left fits in it and the next one
        careful = need <= 1.5 * chunk;
    }

    // ---- unpack x ----
    for (int i = 0; i < nsys; ++i) {
        const GroupPlan& G = L.groups[L.sys_group[i]];
        size_t so[NSLOT];
        sys_block_bytes(G.g.Vh, L.inner, so);
        HIP_TRY(launch_unpack_vec(G.g.Vh, base + L.sys_off[i] + so[S_X64], SP_F64, systems[i].x_e, stream));
    }
    HIP_TRY(hipStreamSynchronize(stream));
    const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();

    int worst = SP_OK;
    for (int i = 0; i < nsys; ++i) {
        const SolverState& st = poll[i];
        const int s = status_of(st);
        if (s < 0 && worst >= 0) worst = s;
        else if (s > 0 && worst == SP_OK) worst = s;
        if (stats) {
            sp_cg_stats& o = stats[i];
            o.iters = st.iter;
            o.reliable_updates = st.ru_count;
            o.converged = (st.flags & ST_CONVERGED) ? 1 : 0;
            o.status = s;
            o.true_rel_resid = st.bnorm2 > 0 ? std::sqrt(st.true_rho / st.bnorm2) : 0.0;
            o.seconds = secs;
        }
    }
    for (int i = 0; i < nsys && log_level() >= 1; ++i) {
        const SolverState& st = poll[i];
        log_line(1, "%s: system %d of %d: status %d, %d iterations, %d reliable updates, true residual %.3e, %.3f ms",
                 range, i, nsys, status_of(st), st.iter, st.ru_count,
                 st.bnorm2 > 0 ? std::sqrt(st.true_rho / st.bnorm2) : 0.0, secs * 1e3);
    }
    if (worst < 0) return fail(worst, "CG breakdown (Re<p,Ap> <= 0 or non-finite scalar)");
    return worst;
}

}  // namespace

namespace sp {

int set_error(int code, const char* msg) { return fail(code, "%s", msg); }

int geom_check(const sp_geom* g, Geom* G) { return check_geom(g, G); }

LaunchCfg tuned_launch(const Geom& G, int lp, int recon, int vp) {
    std::lock_guard<std::mutex> lock(g_mu);
    return tuned_cfg(G, lp, recon, vp);
}

// Argument checks shared by sp_cg_force and its allocation-free variant.
int force_check(const sp_geom* g, const sp_gauge* U, double mass, const double* x_e, const double* lambda_e,
                const double* gamma, Geom* G) {
    int rc = check_geom(g, G);
    if (rc) return rc;
    if (!U || !U->f64 || !x_e || !lambda_e || !gamma) return fail(SP_ERR_INVALID_ARG, "null pointer");
    if (!std::isfinite(mass)) return fail(SP_ERR_INVALID_ARG, "mass not finite");
    return SP_OK;
}

// The gradient's launches, with the scratch at base (force_scratch_bytes(G) bytes, 256-byte aligned): pack x
// and lambda to FP64 planes, y_x = D_oe x and y_l = D_oe lambda, gamma and the force link by link, and the
// two-stage reduction of dl/dm. Every scratch word is written before it is read. Asynchronous on s.
int force_enqueue(const sp_geom* g, const Geom& G, const sp_gauge* U, double mass, const double* x_e,
                  const double* lambda_e, double* gamma, double* force, double* grad_mass, char* base, hipStream_t s) {
    const size_t v = align256((size_t)G.Vh * 48);
    void* xp = base;
    void* lp = base + v;
    void* yx = base + 2 * v;
    void* yl = base + 3 * v;
    double* partials = (double*)(base + 4 * v);
    HIP_TRY(launch_pack_vec(G.Vh, x_e, SP_F64, xp, s));
    HIP_TRY(launch_pack_vec(G.Vh, lambda_e, SP_F64, lp, s));
    sp_gauge Ug = *U;
    Ug.lo = U->f64;
    Ug.lo_prec = SP_F64;
    int rc = sp_dslash(g, &Ug, SP_F64, xp, yx, 1, s);
    if (rc) return rc;
    rc = sp_dslash(g, &Ug, SP_F64, lp, yl, 1, s);
    if (rc) return rc;
    HIP_TRY(launch_force(G, U->f64, xp, lp, yx, yl, gamma, force, s));
    if (grad_mass) HIP_TRY(launch_mass_grad(G, mass, xp, lp, partials, grad_mass, s));
    return SP_OK;
}

size_t force_scratch_bytes(const Geom& G) {
    return 4 * align256((size_t)G.Vh * 48) + align256(sizeof(double) * (size_t)mass_grad_blocks(G));
}

}  // namespace sp

// =====================================================================================================
// C-ABI
// =====================================================================================================
extern "C" {

int sp_version(void) { return 10000; }

const char* sp_strerror(int code) {
    switch (code) {
        case SP_OK: return "ok";
        case SP_NOT_CONVERGED: return "not converged";
        case SP_ERR_INVALID_ARG: return "invalid argument";
        case SP_ERR_ODD_EXTENT: return "lattice extent odd or < 2";
        case SP_ERR_UNSUPPORTED: return "unsupported combination";
        case SP_ERR_WORKSPACE: return "workspace missing or too small";
        case SP_ERR_HIP: return "HIP runtime error";
        case SP_ERR_BREAKDOWN: return "CG breakdown";
    }
    return "unknown status";
}

const char* sp_last_error(void) { return g_last_error.c_str(); }

size_t sp_gauge_bytes(const sp_geom* g, int prec, int recon) {
    Geom G;
    if (check_geom(g, &G) || !valid_link_prec(prec)) return 0;
    return 8 * (size_t)G.Vh * link_bytes(prec, recon);
}

int sp_gauge_pack(const sp_geom* g, const double* links_nat, int prec, int recon, void* out, void* stream) {
    Geom G;
    int rc = check_geom(g, &G);
    if (rc) return rc;
    if (!valid_link_prec(prec)) return fail(SP_ERR_INVALID_ARG, "bad precision %d", prec);
    if (link_bytes(prec, recon) == 0) return fail(SP_ERR_UNSUPPORTED, "precision %d with recon %d", prec, recon);
    if (!links_nat || !out) return fail(SP_ERR_INVALID_ARG, "null pointer");
    HIP_TRY(launch_pack_gauge(G, links_nat, prec, recon, out, (hipStream_t)stream));
    return SP_OK;
}

size_t sp_vec_bytes(const sp_geom* g, int prec) {
    Geom G;
    if (check_geom(g, &G) || !valid_prec(prec)) return 0;
    return (size_t)G.Vh * vec_site_bytes(prec);
}

int sp_vec_pack(const sp_geom* g, const double* v_nat, int prec, void* out, void* stream) {
    Geom G;
    int rc = check_geom(g, &G);
    if (rc) return rc;
    if (!valid_prec(prec)) return fail(SP_ERR_INVALID_ARG, "bad precision %d", prec);
    if (!v_nat || !out) return fail(SP_ERR_INVALID_ARG, "null pointer");
    HIP_TRY(launch_pack_vec(G.Vh, v_nat, prec, out, (hipStream_t)stream));
    return SP_OK;
}

int sp_vec_unpack(const sp_geom* g, const void* v, int prec, double* v_nat, void* stream) {
    Geom G;
    int rc = check_geom(g, &G);
    if (rc) return rc;
    if (!valid_prec(prec)) return fail(SP_ERR_INVALID_ARG, "bad precision %d", prec);
    if (!v || !v_nat) return fail(SP_ERR_INVALID_ARG, "null pointer");
    HIP_TRY(launch_unpack_vec(G.Vh, v, prec, v_nat, (hipStream_t)stream));
    return SP_OK;
}

static int dslash_desc(const sp_geom* g, const sp_gauge* U, int prec, const void* in, void* out, int out_parity,
                       Geom* G, DescSingle* d, int* lp, int* recon) {
    int rc = check_geom(g, G);
    if (rc) return rc;
    if (!valid_prec(prec)) return fail(SP_ERR_INVALID_ARG, "bad precision %d", prec);
    if (!U || !in || !out) return fail(SP_ERR_INVALID_ARG, "null pointer");
    if (out_parity != 0 && out_parity != 1) return fail(SP_ERR_INVALID_ARG, "out_parity must be 0 or 1");
    if (in == out) return fail(SP_ERR_INVALID_ARG, "in and out must differ");
    const void* links;
    if (prec == SP_F64) {
        links = U->f64;
        *lp = SP_F64;
        *recon = 18;
    } else {
        const bool links_ok = U->lo_prec == prec || (prec == SP_F32 && is_16bit_link(U->lo_prec));
        if (!links_ok) return fail(SP_ERR_UNSUPPORTED, "gauge lo precision %d with vectors of precision %d", U->lo_prec, prec);
        if (U->recon != 18 && U->recon != 12 && U->recon != 8)
            return fail(SP_ERR_INVALID_ARG, "recon must be 18, 12 or 8");
        if (U->recon == 8 && U->lo_prec != SP_F32)
            return fail(SP_ERR_UNSUPPORTED, "recon 8 is built for FP32 links only");
        links = U->lo;
        *lp = U->lo_prec;
        *recon = U->recon;
    }
    if (!links) return fail(SP_ERR_INVALID_ARG, "gauge field of precision %d is null", prec);
    memset(d, 0, sizeof *d);
    d->grp.g = *G;
    d->grp.links_lo = links;
    d->grp.links64 = links;
    d->grp.nrhs = 1;
    d->sys.v[S_P] = const_cast<void*>(in);
    d->sys.v[S_T] = out;
    return SP_OK;
}

int sp_dslash(const sp_geom* g, const sp_gauge* U, int prec, const void* in, void* out, int out_parity, void* stream) {
    Geom G;
    DescSingle d;
    int lp, recon;
    int rc = dslash_desc(g, U, prec, in, out, out_parity, &G, &d, &lp, &recon);
    if (rc) return rc;
    LaunchCfg c;
    {
        std::lock_guard<std::mutex> lock(g_mu);
        c = tuned_cfg(G, lp, recon, prec);
    }
    const int nb = blocks_for(G.Vh, c.nt);
    d.grp.nblk = nb;
    HIP_TRY(launch_dslash(d, nb, c, lp, recon, prec, out_parity, S_P, S_T, DS_PLAIN, G_NONE, prec == SP_F64,
                          (hipStream_t)stream));
    return SP_OK;
}

int sp_tune_dslash(const sp_geom* g, const sp_gauge* U, int prec, void* in, void* out, void* stream, double* best_ms) {
    Geom G;
    DescSingle d;
    int lp, recon;
    int rc = dslash_desc(g, U, prec, in, out, 1, &G, &d, &lp, &recon);
    if (rc) return rc;
    hipStream_t s = (hipStream_t)stream;
    // timing events, destroyed on every return path
    struct TimingEvents {
        hipEvent_t a = nullptr, b = nullptr;
        ~TimingEvents() {
            if (a) (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
        }
    } ev;
    HIP_TRY(hipEventCreate(&ev.a));
    HIP_TRY(hipEventCreate(&ev.b));
    hipEvent_t e0 = ev.a, e1 = ev.b;
    const int nts[3] = {64, 128, 256};
    const int reps = 10, trials = 5;
    const int use64 = prec == SP_F64;
    // For every block size, block order and (for the one-right-hand-side operator) link-load policy: 3 warm-up
    // launches, then `trials` timings of `reps` back-to-back launches; the median trial's time per launch
    // counts and the fastest configuration wins. Back-to-back launches are the solver's situation (a link field
    // that fits in the Infinity Cache stays there between the iteration's launches).
    auto sweep = [&](auto launch, bool policies, LaunchCfg* best, float* best_t) -> hipError_t {
        *best_t = 1e30f;
        for (int stream_links = 0; stream_links <= (policies ? 1 : 0); ++stream_links)
            for (int remap = 0; remap <= 1; ++remap)
                for (int nt : nts) {
                    LaunchCfg c;
                    c.nt = nt;
                    c.remap = remap;
                    c.stream = stream_links;
                    hipError_t e;
                    for (int w = 0; w < 3; ++w)
                        if ((e = launch(c))) return e;
                    float t[trials];
                    for (int k = 0; k < trials; ++k) {
                        if ((e = hipEventRecord(e0, s))) return e;
                        for (int r = 0; r < reps; ++r)
                            if ((e = launch(c))) return e;
                        if ((e = hipEventRecord(e1, s))) return e;
                        if ((e = hipEventSynchronize(e1))) return e;
                        if ((e = hipEventElapsedTime(&t[k], e0, e1))) return e;
                    }
                    std::sort(t, t + trials);
                    const float ms = t[trials / 2] / reps;
                    if (ms < *best_t) {
                        *best_t = ms;
                        *best = c;
                    }
                }
        return hipSuccess;
    };
    LaunchCfg best, best4;
    float best_t = 0, best4_t = 0;
    HIP_TRY(sweep(
        [&](LaunchCfg c) {
            const int nb = blocks_for(G.Vh, c.nt);
            d.grp.nblk = nb;
            return launch_dslash(d, nb, c, lp, recon, prec, 1, S_P, S_T, DS_PLAIN, G_NONE, use64, s);
        },
        true, &best, &best_t));
    // The NB-right-hand-side operator of batched solves has its own register use and therefore its own
    // best shape (key suffix "/n4"). It is timed on NB copies of the input into NB outputs, in a temporary
    // device buffer that also holds the group and system descriptors; the buffer is freed before return.
    {
        const size_t vb = align256((size_t)G.Vh * vec_site_bytes(prec));
        const size_t gb = align256(sizeof(GroupDev)), sb = align256(NB * sizeof(SysDev));
        char* buf = nullptr;
        HIP_TRY(hipMalloc((void**)&buf, 2 * NB * vb + gb + sb));
        GroupDev hg = {};
        hg.g = G;
        hg.links_lo = d.grp.links_lo;
        hg.links64 = d.grp.links64;
        hg.nrhs = NB;
        SysDev hs[NB] = {};
        hipError_t e = hipSuccess;
        for (int r = 0; r < NB && !e; ++r) {
            hs[r].v[S_P] = buf + (size_t)r * vb;
            hs[r].v[S_T] = buf + (size_t)(NB + r) * vb;
            e = hipMemcpyAsync(hs[r].v[S_P], in, (size_t)G.Vh * vec_site_bytes(prec), hipMemcpyDeviceToDevice, s);
        }
        GroupDev* dg = (GroupDev*)(buf + 2 * NB * vb);
        SysDev* ds = (SysDev*)(buf + 2 * NB * vb + gb);
        if (!e) e = hipMemcpyAsync(ds, hs, sizeof hs, hipMemcpyHostToDevice, s);
        DescBatch db;
        db.grp = dg;
        db.sys = ds;
        db.ngroups = 1;
        if (!e)
            e = sweep(
                [&](LaunchCfg c) {
                    const int nb = blocks_for(G.Vh, c.nt);
                    if (hg.nblk != nb) {  // the descriptor lives in device memory: rewrite it per shape
                        hg.nblk = nb;
                        hipError_t ee = hipMemcpyAsync(dg, &hg, sizeof hg, hipMemcpyHostToDevice, s);
                        if (!ee) ee = hipStreamSynchronize(s);
                        if (ee) return ee;
                    }
                    return launch_dslash(db, nb, c, lp, recon, prec, 1, S_P, S_T, DS_PLAIN, G_NONE, use64, s);
                },
                false, &best4, &best4_t);
        const hipError_t es = hipStreamSynchronize(s);
        (void)hipFree(buf);
        HIP_TRY(e);
        HIP_TRY(es);
    }
    {
        std::lock_guard<std::mutex> lock(g_mu);
        g_tune[tune_key(G, lp, recon, prec)] = best;
        g_tune[tune_key(G, lp, recon, prec) + "/n4"] = best4;
    }
    if (best_ms) *best_ms = best_t;
    return SP_OK;
}

int sp_tune_save(const char* path) {
    if (!path) return fail(SP_ERR_INVALID_ARG, "path is null");
    std::lock_guard<std::mutex> lock(g_mu);
    std::ofstream f(path);
    if (!f) return fail(SP_ERR_INVALID_ARG, "cannot write %s", path);
    f << "{\n";
    size_t i = 0;
    for (auto& kv : g_tune) {
        f << "  \"" << kv.first << "\": {\"nt\": " << kv.second.nt << ", \"remap\": " << kv.second.remap
          << ", \"stream\": " << kv.second.stream << "}" << (++i < g_tune.size() ? ",\n" : "\n");
    }
    f << "}\n";
    return SP_OK;
}

int sp_tune_load(const char* path) {
    if (!path) return fail(SP_ERR_INVALID_ARG, "path is null");
    std::ifstream f(path);
    if (!f) return fail(SP_ERR_INVALID_ARG, "cannot read %s", path);
    std::stringstream ss;
    ss << f.rdbuf();
    const std::string txt = ss.str();
    // entries are parsed into a temporary table and take effect only if the whole file parses
    std::map<std::string, LaunchCfg> parsed;
    size_t pos = 0;
    while ((pos = txt.find('"', pos)) != std::string::npos) {
        const size_t end = txt.find('"', pos + 1);
        if (end == std::string::npos) return fail(SP_ERR_INVALID_ARG, "unterminated key in %s", path);
        const std::string key = txt.substr(pos + 1, end - pos - 1);
        LaunchCfg c;
        int nt = 0, remap = 0, stream_links = 0;
        const size_t brace = txt.find('{', end);
        if (brace == std::string::npos) return fail(SP_ERR_INVALID_ARG, "tuning key %s has no entry", key.c_str());
        const size_t close = txt.find('}', brace);
        if (close == std::string::npos) return fail(SP_ERR_INVALID_ARG, "malformed tuning entry for %s", key.c_str());
        const std::string entry = txt.substr(brace, close - brace + 1);
        // {"nt": N, "remap": R, "stream": S}; tables written before the link-load policy existed omit "stream"
        // the whole entry must match one of the two forms (%n: characters consumed up to the closing brace)
        int used3 = -1, used2 = -1;
        sscanf(entry.c_str(), "{\"nt\": %d, \"remap\": %d, \"stream\": %d}%n", &nt, &remap, &stream_links, &used3);
        if (used3 != (int)entry.size()) {
            stream_links = 0;
            sscanf(entry.c_str(), "{\"nt\": %d, \"remap\": %d}%n", &nt, &remap, &used2);
            if (used2 != (int)entry.size())
                return fail(SP_ERR_INVALID_ARG, "malformed tuning entry for %s", key.c_str());
        }
        if (nt != 64 && nt != 128 && nt != 256) return fail(SP_ERR_INVALID_ARG, "bad block size %d", nt);
        c.nt = nt;
        c.remap = remap ? 1 : 0;
        c.stream = stream_links ? 1 : 0;
        parsed[key] = c;
        pos = close + 1;
    }
    std::lock_guard<std::mutex> lock(g_mu);
    for (const auto& kv : parsed) g_tune[kv.first] = kv.second;
    return SP_OK;
}

void sp_release_cache(void) {
    std::lock_guard<std::mutex> lock(g_mu);
    release_graphs();
    g_tune.clear();
}

size_t sp_cg_workspace_bytes(int nsys, const sp_system* systems, const sp_cg_params* params) {
    std::lock_guard<std::mutex> lock(g_mu);
    Layout L;
    if (make_layout(nsys, systems, params, nsys > 1 ? NB : 1, &L)) return 0;
    return L.total;
}

int sp_cg_solve(const sp_geom* g, const sp_gauge* U, double mass, const double* b_e, double* x_e,
                const sp_cg_params* params, sp_cg_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    sp_system s;
    s.g = g;
    s.U = U;
    s.mass = mass;
    s.b_e = b_e;
    s.x_e = x_e;
    return solve_impl(1, &s, params, stats, ws, ws_bytes, (hipStream_t)stream, false);
}

int sp_cg_solve_batched(int nsys, const sp_system* systems, const sp_cg_params* params, sp_cg_stats* stats,
                        void* ws, size_t ws_bytes, void* stream) {
    if (nsys <= 0 || !systems) return fail(SP_ERR_INVALID_ARG, "no systems");
    return solve_impl(nsys, systems, params, stats, ws, ws_bytes, (hipStream_t)stream, true);
}

size_t sp_force_workspace_bytes(const sp_geom* g) {
    Geom G;
    if (check_geom(g, &G)) return 0;
    return sp::force_scratch_bytes(G);
}

int sp_cg_force(const sp_geom* g, const sp_gauge* U, double mass, const double* x_e, const double* lambda_e,
                double* gamma, double* force, double* grad_mass, void* ws, size_t ws_bytes, void* stream) {
    Geom G;
    int rc = sp::force_check(g, U, mass, x_e, lambda_e, gamma, &G);
    if (rc) return rc;
    if (!ws) return fail(SP_ERR_WORKSPACE, "workspace is null");
    if (ws_bytes < sp_force_workspace_bytes(g)) return fail(SP_ERR_WORKSPACE, "workspace too small");
    if (((uintptr_t)ws) & 255) return fail(SP_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    rc = sp::force_enqueue(g, G, U, mass, x_e, lambda_e, gamma, force, grad_mass, (char*)ws, s);
    if (rc) return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return SP_OK;
}

}  // extern "C"

extern "C" {

size_t sp_full_workspace_bytes(const sp_geom* g, const sp_gauge* U, const sp_cg_params* params) {
    Geom G;
    if (check_geom(g, &G) || !U || !params) return 0;
    sp_system s;
    s.g = g;
    s.U = U;
    s.mass = 1.0;
    s.b_e = nullptr;
    s.x_e = nullptr;
    const size_t cg = sp_cg_workspace_bytes(1, &s, params);
    if (cg == 0) return 0;
    return 6 * align256((size_t)G.Vh * 48) + cg;
}

int sp_full_solve(const sp_geom* g, const sp_gauge* U, double mass, const double* src, double* psi,
                  const sp_cg_params* params, sp_cg_stats* stats, void* ws, size_t ws_bytes, void* stream) {
    Geom G;
    int rc = check_geom(g, &G);
    if (rc) return rc;
    if (!U || !U->f64 || !src || !psi || !params) return fail(SP_ERR_INVALID_ARG, "null pointer");
    if (!std::isfinite(mass) || mass == 0.0) return fail(SP_ERR_INVALID_ARG, "mass must be finite and non-zero");
    const size_t need = sp_full_workspace_bytes(g, U, params);
    if (need == 0) return fail(SP_ERR_INVALID_ARG, "bad parameters");
    if (!ws || ws_bytes < need) return fail(SP_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
    if (((uintptr_t)ws) & 255) return fail(SP_ERR_INVALID_ARG, "workspace not 256-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const size_t v = align256((size_t)G.Vh * 48);
    char* base = (char*)ws;
    void* se = base;
    void* so = base + v;
    void* t = base + 2 * v;
    void* pe = base + 3 * v;
    double* be = (double*)(base + 4 * v);
    double* xe = (double*)(base + 5 * v);
    void* wcg = base + 6 * v;
    sp_gauge U64 = *U;
    U64.lo = U->f64;
    U64.lo_prec = SP_F64;
    U64.recon = 18;
    HIP_TRY(launch_full_split(G, src, se, so, s));
    if ((rc = sp_dslash(g, &U64, SP_F64, so, t, 0, stream))) return rc;  // t = D_eo src_o
    HIP_TRY(launch_full_source(G, mass, se, t, be, s));
    sp_cg_params prm = *params;
    prm.use_x0 = 0;  // psi_e starts from zero (the buffer is workspace, not a guess)
    const int st = sp_cg_solve(g, U, mass, be, xe, &prm, stats, wcg, ws_bytes - 6 * v, stream);
    if (st < 0) return st;
    HIP_TRY(launch_pack_vec(G.Vh, xe, SP_F64, pe, s));
    if ((rc = sp_dslash(g, &U64, SP_F64, pe, t, 1, stream))) return rc;  // t = D_oe psi_e
    HIP_TRY(launch_full_merge(G, mass, xe, so, t, psi, s));
    HIP_TRY(hipStreamSynchronize(s));
    return st;
}

size_t sp_hyp_workspace_bytes(const sp_geom* g) {
    Geom G;
    if (check_geom(g, &G)) return 0;
    return hyp_workspace_bytes(G);
}

int sp_hyp_smear(const sp_geom* g, const double* links_nat, const double* alpha, double* out_nat, void* ws,
                 size_t ws_bytes, void* stream) {
    Geom G;
    int rc = check_geom(g, &G);
    if (rc) return rc;
    if (!links_nat || !alpha || !out_nat) return fail(SP_ERR_INVALID_ARG, "null pointer");
    for (int k = 0; k < 3; ++k)
        if (!(alpha[k] >= 0.0 && alpha[k] <= 1.0)) return fail(SP_ERR_INVALID_ARG, "alpha[%d] not in [0, 1]", k);
    const size_t field = 4ull * 2 * G.Vh * 18 * sizeof(double);
    const char *a0 = (const char*)links_nat, *b0 = (const char*)out_nat;
    if (a0 < b0 + field && b0 < a0 + field) return fail(SP_ERR_INVALID_ARG, "links and output overlap");
    const size_t need = hyp_workspace_bytes(G);
    if (!ws || ws_bytes < need) return fail(SP_ERR_WORKSPACE, "workspace %zu bytes < required %zu", ws_bytes, need);
    if (((uintptr_t)ws) & 15) return fail(SP_ERR_INVALID_ARG, "workspace not 16-byte aligned");
    if (((uintptr_t)links_nat) & 15 || ((uintptr_t)out_nat) & 15)
        return fail(SP_ERR_INVALID_ARG, "links or output not 16-byte aligned");
    HIP_TRY(launch_hyp(G, links_nat, alpha, out_nat, ws, (hipStream_t)stream));
    return SP_OK;
}

size_t sp_npr_path_bytes(const sp_geom* g) {
    Geom G;
    if (check_geom(g, &G)) return 0;
    return npr_path_bytes(G);
}

int sp_npr_path_links(const sp_geom* g, const double* links_nat, void* uad, void* stream) {
    Geom G;
    int rc = check_geom(g, &G);
    if (rc) return rc;
    if (!links_nat || !uad) return fail(SP_ERR_INVALID_ARG, "null pointer");
    if (((uintptr_t)links_nat) & 15 || ((uintptr_t)uad) & 15) return fail(SP_ERR_INVALID_ARG, "pointers not 16-byte aligned");
    HIP_TRY(launch_npr_paths(G, links_nat, uad, (hipStream_t)stream));
    return SP_OK;
}

static int npr_contract_any(const sp_geom* g, const void* uad, const double* links_nat, int n, const double* chib1,
                            const double* chi2, const double* chib3, const double* chi4, const int32_t* labels,
                            double* out, void* stream) {
    Geom G;
    int rc = check_geom(g, &G);
    if (rc) return rc;
    if (!(uad || links_nat) || !chib1 || !chi2 || !chib3 || !chi4 || !labels || !out)
        return fail(SP_ERR_INVALID_ARG, "null pointer");
    if (n < 1) return fail(SP_ERR_INVALID_ARG, "n must be >= 1");
    int lab[4];
    for (int k = 0; k < 4; ++k) {
        if (labels[k] < 0 || labels[k] > 15) return fail(SP_ERR_INVALID_ARG, "label %d not in [0, 16)", k);
        lab[k] = labels[k];
    }
    const double* f[4] = {chib1, chi2, chib3, chi4};
    for (int k = 0; k < 4; ++k)
        if (((uintptr_t)f[k]) & 15) return fail(SP_ERR_INVALID_ARG, "field %d not 16-byte aligned", k);
    if (((uintptr_t)uad) & 15 || ((uintptr_t)links_nat) & 15) return fail(SP_ERR_INVALID_ARG, "pointers not 16-byte aligned");
    HIP_TRY(launch_npr_contract_from(G, uad, links_nat, n, f, lab, out, (hipStream_t)stream));
    return SP_OK;
}

int sp_npr_contract(const sp_geom* g, const void* uad, int n, const double* chib1, const double* chi2,
                    const double* chib3, const double* chi4, const int32_t* labels, double* out, void* stream) {
    if (!uad) return fail(SP_ERR_INVALID_ARG, "null pointer");
    return npr_contract_any(g, uad, nullptr, n, chib1, chi2, chib3, chi4, labels, out, stream);
}

int sp_npr_contract_links(const sp_geom* g, const double* links_nat, int n, const double* chib1, const double* chi2,
                          const double* chib3, const double* chi4, const int32_t* labels, double* out, void* stream) {
    if (!links_nat) return fail(SP_ERR_INVALID_ARG, "null pointer");
    return npr_contract_any(g, nullptr, links_nat, n, chib1, chi2, chib3, chi4, labels, out, stream);
}

}  // extern "C"
