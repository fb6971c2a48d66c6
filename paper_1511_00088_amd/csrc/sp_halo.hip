// One GPU's share of a lattice cut in time across GPUs, the decomposition of the paper's multi-GPU CG (Sec. 3,
// Fig. 2, Table 2: each GPU exchanges the vector with its nearest neighbours every iteration).
//
// A shard holds the time slices [t0, t0 + Tl) of an X x Y x Z x T lattice (t0 and Tl even, so local and global
// parities agree and the shard's checkerboard indices are the global ones minus t0 X Y Z / 2). Each time slice of
// one parity is F = X Y Z / 2 consecutive checkerboard indices, so a face is a contiguous range of every plane.
//   * Extended vector: the packed planes of Vh + 2F sites, [ghost below: slice t0 - 1][the Tl local slices]
//     [ghost above: slice t0 + Tl]; local site cb sits at F + cb, and its t-neighbours at F + cb -+ F with no wrap.
//   * Face: one slice of one parity, packed with plane stride F (the wire format of the exchange, identical
//     to the packed format, so pack and unpack move raw 16-bit, 32-bit or 64-bit words and never round).
//   * Ghost links: U_t(x, y, z, t0 - 1) of both parities (the backward t-link of slice t0 lives below the
//     shard), two blocks of F links in the packed link format; exchanged once per gauge field.
// The halo-fed half operator runs over the interior slices 1 .. Tl-2 (no ghost read: can overlap the exchange),
// the boundary slices 0 and Tl-1, or all; the antiperiodic sign applies at the global time boundary.
#include <hip/hip_runtime.h>

#include "sp_entry.h"

namespace sp {

struct Shard {
    Geom g;     // local geometry: X, Y, Z, Tl
    int t0, T;  // global time of local slice 0, global time extent
    int F;      // sites of one parity in one time slice
};

// Raw plane structure of the packed vector formats (VecFmt): plane k holds w[k] bytes per site.
template <int P>
struct Planes;
template <>
struct Planes<F64> {
    static constexpr int n = 3;
    __device__ static constexpr int w(int) { return 16; }
};
template <>
struct Planes<F32> {
    static constexpr int n = 2;
    __device__ static constexpr int w(int k) { return k == 0 ? 16 : 8; }
};
template <>
struct Planes<F16> {
    static constexpr int n = 1;
    __device__ static constexpr int w(int) { return 16; }
};
template <>
struct Planes<BF16> {
    static constexpr int n = 2;
    __device__ static constexpr int w(int k) { return k == 0 ? 8 : 4; }
};

// Copies sites [src0, src0 + n) of a packed vector with plane stride ssrc to sites [dst0, dst0 + n) of one with
// plane stride sdst, word for word. One thread per site.
template <int P>
__global__ __launch_bounds__(256) void k_copy_sites(const char* __restrict__ src, long ssrc, long src0,
                                                    char* __restrict__ dst, long sdst, long dst0, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    long offs = 0, offd = 0;
#pragma unroll
    for (int k = 0; k < Planes<P>::n; ++k) {
        const int w = Planes<P>::w(k);
        const char* a = src + offs + (src0 + i) * w;
        char* b = dst + offd + (dst0 + i) * w;
        if (w == 16) *(uint4*)b = *(const uint4*)a;
        else if (w == 8) *(uint2*)b = *(const uint2*)a;
        else *(uint32_t*)b = *(const uint32_t*)a;
        offs += w * ssrc;
        offd += w * sdst;
    }
}

// Natural local half vector -> the local part of an extended vector.
template <int P>
__global__ __launch_bounds__(256) void k_pack_ext(int Vh, int F, const double* __restrict__ nat, void* ext) {
    using R = typename Real<P>::T;
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    if (cb >= Vh) return;
    Vec3<R> v;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v.c[c].re = (R)nat[(size_t)cb * 6 + 2 * c];
        v.c[c].im = (R)nat[(size_t)cb * 6 + 2 * c + 1];
    }
    VecFmt<P>::store(ext, Vh + 2 * F, F + cb, v);
}

// Ghost t-links: natural U_t of the slice below, [X Y Z][3][3] in lex order of (x, y, z), into two parity blocks.
template <int P, int RECON>
__global__ __launch_bounds__(256) void k_pack_ghost(Geom g, int tb, const double* __restrict__ nat, void* out) {
    using LF = LinkFmt<P, RECON>;
    const int F = g.Xh * g.Y * g.Z;
    const int l = blockIdx.x * blockDim.x + threadIdx.x;  // x + X (y + Y z)
    if (l >= 2 * F) return;
    const int x = l % g.X, r1 = l / g.X, y = r1 % g.Y, z = r1 / g.Y;
    const int q = (x + y + z + tb) & 1;
    double r[18];
#pragma unroll
    for (int k = 0; k < 18; ++k) r[k] = nat[(size_t)l * 18 + k];
    LF::store((char*)out + (size_t)q * F * LF::bytes, F, l >> 1, r);
}

// out(n) = 1/2 sum_mu eta_mu(n) [ s_f U_mu(n) in(n+mu) - s_b U_mu(n-mu)^dag in(n-mu) ] on local sites of parity
// p, with in(n +- t) read from the extended vector (ghost slices at the shard's edges) and the backward t-link
// of slice 0 from the ghost links. Sites: cb0 + i for i < n1, then cb1 + i - n1 (interior: one range;
// boundary: slice 0 and slice Tl-1).
template <int LP, int RECON, int VP, bool NT>
__global__ __launch_bounds__(256) void k_dslash_halo(Shard sh, const void* links, const void* ghost, const void* ext,
                                                     void* out, int p, int cb0, int n1, int cb1, int n, int remap) {
    using R = typename Real<VP>::T;
    using LF = LinkFmt<LP, RECON>;
    using VF = VecFmt<VP>;
    const Geom g = sh.g;
    const int i = logical_block(remap) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cb = i < n1 ? cb0 + i : cb1 + (i - n1);
    const int F = sh.F, Vx = g.Vh + 2 * F;
    const Site s = site_of(g, p, cb);
    const int tg = sh.t0 + s.t;
    Vec3<R> acc = vzero<R>();
    constexpr int UNROLL = unroll_dirs(LP, RECON, VP, NT);
#pragma unroll UNROLL
    for (int mu = 0; mu < 4; ++mu) {
        const R e = (R)eta_sign(s, mu);
        R sf = e, sb = -e;
        int nf, nb;
        const char* bblk;
        int bidx, bstride;
        if (mu < 3) {
            nf = F + nbr(g, s, mu, +1);
            nb = nbr(g, s, mu, -1);
            bblk = link_block<LF>(links, g.Vh, 1 - p, mu);
            bidx = nb;
            bstride = g.Vh;
            nb += F;
        } else {
            if (g.bc_t) {
                if (tg == sh.T - 1) sf = -sf;
                if (tg == 0) sb = -sb;
            }
            nf = F + cb + F;
            nb = cb;  // F + cb - F
            if (s.t > 0) {
                bblk = link_block<LF>(links, g.Vh, 1 - p, 3);
                bidx = cb - F;
                bstride = g.Vh;
            } else {
                bblk = (const char*)ghost + (size_t)(1 - p) * F * LF::bytes;
                bidx = cb;
                bstride = F;
            }
        }
        const Su3<R> Uf = LF::template load<NT>(link_block<LF>(links, g.Vh, p, mu), g.Vh, cb);
        const Vec3<R> vf = VF::load(ext, Vx, nf);
        const Su3<R> Ub = LF::template load<NT>(bblk, bstride, bidx);
        const Vec3<R> vb = VF::load(ext, Vx, nb);
        mv_acc(acc, Uf, vf, sf);
        mdv_acc(acc, Ub, vb, sb);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        acc.c[c].re *= R(0.5);
        acc.c[c].im *= R(0.5);
    }
    VF::store(out, g.Vh, cb, acc);
}

// ---------------------------------------------------------------------------------------------------------
// launches
// ---------------------------------------------------------------------------------------------------------
template <int P>
hipError_t copy_sites_p(const void* src, long ssrc, long src0, void* dst, long sdst, long dst0, int n, hipStream_t s) {
    hipLaunchKernelGGL((k_copy_sites<P>), dim3(blocks_for(n, 256)), dim3(256), 0, s, (const char*)src, ssrc, src0,
                       (char*)dst, sdst, dst0, n);
    return hipGetLastError();
}

hipError_t launch_copy_sites(int prec, const void* src, long ssrc, long src0, void* dst, long sdst, long dst0, int n,
                             hipStream_t s) {
    switch (prec) {
        case F64: return copy_sites_p<F64>(src, ssrc, src0, dst, sdst, dst0, n, s);
        case F32: return copy_sites_p<F32>(src, ssrc, src0, dst, sdst, dst0, n, s);
        case F16: return copy_sites_p<F16>(src, ssrc, src0, dst, sdst, dst0, n, s);
        case BF16: return copy_sites_p<BF16>(src, ssrc, src0, dst, sdst, dst0, n, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_pack_ext(int prec, int Vh, int F, const double* nat, void* ext, hipStream_t s) {
    const int nb = blocks_for(Vh, 256);
#define SP_LAUNCH(P)                                                                                        \
    do {                                                                                                    \
        hipLaunchKernelGGL((k_pack_ext<P>), dim3(nb), dim3(256), 0, s, Vh, F, nat, ext);                   \
        return hipGetLastError();                                                                           \
    } while (0)
    if (prec == F64) SP_LAUNCH(F64);
    if (prec == F32) SP_LAUNCH(F32);
    if (prec == F16) SP_LAUNCH(F16);
    if (prec == BF16) SP_LAUNCH(BF16);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_pack_ghost(const Geom& g, int tb, const double* nat, int prec, int recon, void* out, hipStream_t s) {
    const int nb = blocks_for(2 * g.Xh * g.Y * g.Z, 256);
#define SP_LAUNCH(P, RC)                                                                                    \
    do {                                                                                                    \
        hipLaunchKernelGGL((k_pack_ghost<P, RC>), dim3(nb), dim3(256), 0, s, g, tb, nat, out);             \
        return hipGetLastError();                                                                           \
    } while (0)
    if (prec == F64 && recon == 18) SP_LAUNCH(F64, 18);
    if (prec == F32 && recon == 18) SP_LAUNCH(F32, 18);
    if (prec == F32 && recon == 12) SP_LAUNCH(F32, 12);
    if (prec == F32 && recon == 8) SP_LAUNCH(F32, 8);
    if (prec == F16 && recon == 18) SP_LAUNCH(F16, 18);
    if (prec == F16 && recon == 12) SP_LAUNCH(F16, 12);
    if (prec == BF16 && recon == 18) SP_LAUNCH(BF16, 18);
    if (prec == BF16 && recon == 12) SP_LAUNCH(BF16, 12);
    if (prec == I16 && recon == 18) SP_LAUNCH(I16, 18);
    if (prec == I16 && recon == 12) SP_LAUNCH(I16, 12);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_dslash_halo(const Shard& sh, int lp, int recon, int vp, const void* links, const void* ghost,
                              const void* ext, void* out, int p, int cb0, int n1, int cb1, int n, LaunchCfg c,
                              hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const int nb = blocks_for(n, c.nt);
#define SP_LAUNCH(LP, RC, VP)                                                                               \
    do {                                                                                                    \
        if (c.stream)                                                                                       \
            hipLaunchKernelGGL((k_dslash_halo<LP, RC, VP, true>), dim3(nb), dim3(c.nt), 0, s, sh, links, ghost, ext, \
                               out, p, cb0, n1, cb1, n, c.remap);                                           \
        else                                                                                                \
            hipLaunchKernelGGL((k_dslash_halo<LP, RC, VP, false>), dim3(nb), dim3(c.nt), 0, s, sh, links, ghost, \
                               ext, out, p, cb0, n1, cb1, n, c.remap);                                      \
        return hipGetLastError();                                                                           \
    } while (0)
    if (lp == F64 && recon == 18 && vp == F64) SP_LAUNCH(F64, 18, F64);
    if (lp == F32 && recon == 18 && vp == F32) SP_LAUNCH(F32, 18, F32);
    if (lp == F32 && recon == 12 && vp == F32) SP_LAUNCH(F32, 12, F32);
    if (lp == F32 && recon == 8 && vp == F32) SP_LAUNCH(F32, 8, F32);
    if (lp == F16 && recon == 18 && vp == F16) SP_LAUNCH(F16, 18, F16);
    if (lp == F16 && recon == 12 && vp == F16) SP_LAUNCH(F16, 12, F16);
    if (lp == BF16 && recon == 18 && vp == BF16) SP_LAUNCH(BF16, 18, BF16);
    if (lp == BF16 && recon == 12 && vp == BF16) SP_LAUNCH(BF16, 12, BF16);
    if (lp == F16 && recon == 12 && vp == F32) SP_LAUNCH(F16, 12, F32);
    if (lp == F16 && recon == 18 && vp == F32) SP_LAUNCH(F16, 18, F32);
    if (lp == BF16 && recon == 12 && vp == F32) SP_LAUNCH(BF16, 12, F32);
    if (lp == BF16 && recon == 18 && vp == F32) SP_LAUNCH(BF16, 18, F32);
    if (lp == I16 && recon == 12 && vp == F32) SP_LAUNCH(I16, 12, F32);
    if (lp == I16 && recon == 18 && vp == F32) SP_LAUNCH(I16, 18, F32);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace sp

// ---------------------------------------------------------------------------------------------------------
// C-ABI
// ---------------------------------------------------------------------------------------------------------
namespace {

size_t vec_site_bytes_of(int prec) {
    switch (prec) {
        case SP_F64: return 48;
        case SP_F32: return 24;
        case SP_F16: return 16;
        case SP_BF16: return 12;
    }
    return 0;
}

size_t link_bytes_of(int prec, int recon) {
    if (prec == SP_F64) return recon == 18 ? 144 : 0;
    if (prec == SP_F32) return recon == 18 ? 72 : recon == 12 ? 48 : recon == 8 ? 32 : 0;
    if (prec == SP_F16 || prec == SP_BF16 || prec == SP_I16) return recon == 18 ? 36 : recon == 12 ? 24 : 0;
    return 0;
}

int shard_check(const sp_shard* s, sp::Shard* sh) {
    if (!s) return sp::set_error(SP_ERR_INVALID_ARG, "shard is null");
    int rc = sp::geom_check(&s->local, &sh->g);
    if (rc) return rc;
    const int Tl = s->local.dims[3];
    if (s->T < 2 || (s->T & 1)) return sp::set_error(SP_ERR_ODD_EXTENT, "global time extent odd or < 2");
    if (s->t0 < 0 || (s->t0 & 1) || s->t0 + Tl > s->T)
        return sp::set_error(SP_ERR_INVALID_ARG, "t0 must be even and the shard must lie inside the global extent");
    sh->t0 = s->t0;
    sh->T = s->T;
    sh->F = sh->g.Xh * sh->g.Y * sh->g.Z;
    return SP_OK;
}

int hip_status(hipError_t e) {
    return e == hipSuccess ? SP_OK : sp::set_error(SP_ERR_HIP, hipGetErrorString(e));
}

}  // namespace

extern "C" {

size_t sp_shard_face_bytes(const sp_shard* s, int prec) {
    sp::Shard sh;
    if (shard_check(s, &sh)) return 0;
    return (size_t)sh.F * vec_site_bytes_of(prec);
}

size_t sp_shard_vec_bytes(const sp_shard* s, int prec) {
    sp::Shard sh;
    if (shard_check(s, &sh)) return 0;
    return ((size_t)sh.g.Vh + 2 * (size_t)sh.F) * vec_site_bytes_of(prec);
}

int sp_shard_vec_pack(const sp_shard* s, const double* v_nat, int prec, void* ext, void* stream) {
    sp::Shard sh;
    int rc = shard_check(s, &sh);
    if (rc) return rc;
    if (!vec_site_bytes_of(prec)) return sp::set_error(SP_ERR_INVALID_ARG, "bad precision");
    if (!v_nat || !ext) return sp::set_error(SP_ERR_INVALID_ARG, "null pointer");
    return hip_status(sp::launch_pack_ext(prec, sh.g.Vh, sh.F, v_nat, ext, (hipStream_t)stream));
}

int sp_face_pack(const sp_shard* s, int prec, const void* ext, int side, void* face, void* stream) {
    sp::Shard sh;
    int rc = shard_check(s, &sh);
    if (rc) return rc;
    if (!vec_site_bytes_of(prec)) return sp::set_error(SP_ERR_INVALID_ARG, "bad precision");
    if (side != 0 && side != 1) return sp::set_error(SP_ERR_INVALID_ARG, "side must be 0 (lowest slice) or 1 (highest)");
    if (!ext || !face) return sp::set_error(SP_ERR_INVALID_ARG, "null pointer");
    const long Vx = (long)sh.g.Vh + 2L * sh.F;
    const long src0 = side == 0 ? sh.F : sh.g.Vh;  // local slice 0 or Tl - 1 inside the extended planes
    return hip_status(sp::launch_copy_sites(prec, ext, Vx, src0, face, sh.F, 0, sh.F, (hipStream_t)stream));
}

int sp_face_unpack(const sp_shard* s, int prec, const void* face, int side, void* ext, void* stream) {
    sp::Shard sh;
    int rc = shard_check(s, &sh);
    if (rc) return rc;
    if (!vec_site_bytes_of(prec)) return sp::set_error(SP_ERR_INVALID_ARG, "bad precision");
    if (side != 0 && side != 1) return sp::set_error(SP_ERR_INVALID_ARG, "side must be 0 (ghost below) or 1 (above)");
    if (!ext || !face) return sp::set_error(SP_ERR_INVALID_ARG, "null pointer");
    const long Vx = (long)sh.g.Vh + 2L * sh.F;
    const long dst0 = side == 0 ? 0 : (long)sh.F + sh.g.Vh;
    return hip_status(sp::launch_copy_sites(prec, face, sh.F, 0, ext, Vx, dst0, sh.F, (hipStream_t)stream));
}

size_t sp_shard_ghost_bytes(const sp_shard* s, int prec, int recon) {
    sp::Shard sh;
    if (shard_check(s, &sh)) return 0;
    return 2 * (size_t)sh.F * link_bytes_of(prec, recon);
}

int sp_shard_ghost_pack(const sp_shard* s, const double* tlinks_nat, int prec, int recon, void* ghost, void* stream) {
    sp::Shard sh;
    int rc = shard_check(s, &sh);
    if (rc) return rc;
    if (!link_bytes_of(prec, recon)) return sp::set_error(SP_ERR_UNSUPPORTED, "precision and recon not built");
    if (!tlinks_nat || !ghost) return sp::set_error(SP_ERR_INVALID_ARG, "null pointer");
    const int tb = (sh.t0 - 1 + sh.T) % sh.T;
    return hip_status(sp::launch_pack_ghost(sh.g, tb, tlinks_nat, prec, recon, ghost, (hipStream_t)stream));
}

int sp_dslash_halo(const sp_shard* s, const sp_gauge* U, const void* ghost, int prec, const void* ext_in, void* out,
                   int out_parity, int part, void* stream) {
    sp::Shard sh;
    int rc = shard_check(s, &sh);
    if (rc) return rc;
    if (!vec_site_bytes_of(prec)) return sp::set_error(SP_ERR_INVALID_ARG, "bad precision");
    if (!U || !ghost || !ext_in || !out) return sp::set_error(SP_ERR_INVALID_ARG, "null pointer");
    if (out_parity != 0 && out_parity != 1) return sp::set_error(SP_ERR_INVALID_ARG, "out_parity must be 0 or 1");
    if (part < 0 || part > 2) return sp::set_error(SP_ERR_INVALID_ARG, "part must be 0 (all), 1 (interior) or 2 (boundary)");
    int lp, recon;
    const void* links;
    if (prec == SP_F64) {
        links = U->f64;
        lp = SP_F64;
        recon = 18;
    } else {
        const bool ok = U->lo_prec == prec ||
                        (prec == SP_F32 && (U->lo_prec == SP_F16 || U->lo_prec == SP_BF16 || U->lo_prec == SP_I16));
        if (!ok) return sp::set_error(SP_ERR_UNSUPPORTED, "gauge precision cannot serve these vectors");
        if (U->recon != 18 && U->recon != 12 && U->recon != 8)
            return sp::set_error(SP_ERR_INVALID_ARG, "recon must be 18, 12 or 8");
        if (U->recon == 8 && U->lo_prec != SP_F32)
            return sp::set_error(SP_ERR_UNSUPPORTED, "recon 8 is built for FP32 links only");
        links = U->lo;
        lp = U->lo_prec;
        recon = U->recon;
    }
    if (!links) return sp::set_error(SP_ERR_INVALID_ARG, "gauge field is null");
    const int Vh = sh.g.Vh, F = sh.F;
    int cb0 = 0, n1 = Vh, cb1 = 0, n = Vh;
    if (part == 1) {
        cb0 = F;
        n1 = n = Vh - 2 * F;
    } else if (part == 2) {
        n1 = F;
        cb1 = Vh - F;
        n = 2 * F;
    }
    const sp::LaunchCfg c = sp::tuned_launch(sh.g, lp, recon, prec);
    return hip_status(sp::launch_dslash_halo(sh, lp, recon, prec, links, ghost, ext_in, out, out_parity, cb0, n1, cb1,
                                             n, c, (hipStream_t)stream));
}

}  // extern "C"
