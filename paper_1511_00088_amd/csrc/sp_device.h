// Device building blocks for the staggered even-odd CG on CDNA4 (gfx950): complex / SU(3) arithmetic,
// structure-of-arrays storage formats, checkerboard geometry, wave64 reductions and the device-resident
// solver state.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sp {

// I16: 16-bit fixed point q / 32767 (link storage only: SU(3) entries lie in [-1, 1])
enum Prec : int { F64 = 0, F32 = 1, F16 = 2, BF16 = 3, I16 = 4 };

// ------------------------------------------------------------------------------------------------------
// Complex colour vectors and 3x3 links
// ------------------------------------------------------------------------------------------------------
template <class R>
struct Cx {
    R re, im;
};

template <class R>
struct Vec3 {
    Cx<R> c[3];
};

template <class R>
struct Su3 {
    Cx<R> e[3][3];
};

template <class R>
__device__ __forceinline__ Vec3<R> vzero() {
    Vec3<R> v;
#pragma unroll
    for (int i = 0; i < 3; ++i) v.c[i].re = v.c[i].im = R(0);
    return v;
}

// acc += s * (U v)
template <class R>
__device__ __forceinline__ void mv_acc(Vec3<R>& acc, const Su3<R>& U, const Vec3<R>& v, R s) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        R re = R(0), im = R(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            re += U.e[i][j].re * v.c[j].re - U.e[i][j].im * v.c[j].im;
            im += U.e[i][j].re * v.c[j].im + U.e[i][j].im * v.c[j].re;
        }
        acc.c[i].re += s * re;
        acc.c[i].im += s * im;
    }
}

// acc += s * (U^dag v)
template <class R>
__device__ __forceinline__ void mdv_acc(Vec3<R>& acc, const Su3<R>& U, const Vec3<R>& v, R s) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        R re = R(0), im = R(0);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            re += U.e[j][i].re * v.c[j].re + U.e[j][i].im * v.c[j].im;
            im += U.e[j][i].re * v.c[j].im - U.e[j][i].im * v.c[j].re;
        }
        acc.c[i].re += s * re;
        acc.c[i].im += s * im;
    }
}

// Third row of an SU(3) matrix from the first two: row2 = conj(row0 x row1).
template <class R>
__device__ __forceinline__ void rebuild_row2(Su3<R>& U) {
    auto cross = [](Cx<R> a, Cx<R> b, Cx<R> c, Cx<R> d) {  // conj(a*b - c*d)
        Cx<R> r;
        r.re = (a.re * b.re - a.im * b.im) - (c.re * d.re - c.im * d.im);
        r.im = -((a.re * b.im + a.im * b.re) - (c.re * d.im + c.im * d.re));
        return r;
    };
    U.e[2][0] = cross(U.e[0][1], U.e[1][2], U.e[0][2], U.e[1][1]);
    U.e[2][1] = cross(U.e[0][2], U.e[1][0], U.e[0][0], U.e[1][2]);
    U.e[2][2] = cross(U.e[0][0], U.e[1][1], U.e[0][1], U.e[1][0]);
}

// ------------------------------------------------------------------------------------------------------
// Scalar conversions for 16-bit storage (round to nearest even)
// ------------------------------------------------------------------------------------------------------
__device__ __forceinline__ uint32_t f32_to_bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (u >> 16) | 0x40u;  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_bits_to_f32(uint32_t b) { return __uint_as_float(b << 16); }

__device__ __forceinline__ uint32_t f32_to_f16_bits(float f) {
    _Float16 h = (_Float16)f;
    return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ __forceinline__ float f16_bits_to_f32(uint32_t b) {
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(b & 0xffffu));
}

// 16-bit fixed point: q = round(32767 v) clamped to [-32767, 32767]; the absolute error is at most 2^-16 for
// every |v| <= 1, where FP16 keeps a relative 2^-11 (an error of 2^-12 near 1, the size of smeared links'
// diagonal entries)
__device__ __forceinline__ uint32_t f32_to_i16_bits(float f) {
    const float q = fminf(fmaxf(rintf(f * 32767.0f), -32767.0f), 32767.0f);
    return (uint32_t)(uint16_t)(int16_t)q;
}
__device__ __forceinline__ float i16_bits_to_f32(uint32_t b) {
    return (float)(int16_t)(uint16_t)(b & 0xffffu) * (1.0f / 32767.0f);
}

template <int P>
__device__ __forceinline__ uint32_t pack2(float a, float b) {
    if constexpr (P == F16)
        return f32_to_f16_bits(a) | (f32_to_f16_bits(b) << 16);
    else if constexpr (P == I16)
        return f32_to_i16_bits(a) | (f32_to_i16_bits(b) << 16);
    else
        return f32_to_bf16_bits(a) | (f32_to_bf16_bits(b) << 16);
}
template <int P>
__device__ __forceinline__ float unpack_lo(uint32_t w) {
    if constexpr (P == F16) return f16_bits_to_f32(w);
    else if constexpr (P == I16) return i16_bits_to_f32(w);
    else return bf16_bits_to_f32(w & 0xffffu);
}
template <int P>
__device__ __forceinline__ float unpack_hi(uint32_t w) {
    if constexpr (P == F16) return f16_bits_to_f32(w >> 16);
    else if constexpr (P == I16) return i16_bits_to_f32(w >> 16);
    else return bf16_bits_to_f32(w >> 16);
}

template <int P>
struct Real {
    using T = float;
};
template <>
struct Real<F64> {
    using T = double;
};

// ------------------------------------------------------------------------------------------------------
// Vector storage: one parity-half vector of Vh sites, 3 complex colours per site, as planes so that a
// wavefront reads 64 consecutive sites with one wide load per plane.
//   F64 : 3 planes of double2 (one per colour)                                        48 B/site
//   F32 : plane float4 (colours 0,1) + plane float2 (colour 2)                         24 B/site
//   F16 : one plane uint4 per site: 6 halves (colours 0..2) and the float norm, so one
//         16-byte load; stored value = half * norm, norm = max |component| of the site   16 B/site
//   BF16: plane uint2 + plane uint, unscaled                                          12 B/site
// ------------------------------------------------------------------------------------------------------
template <int P>
struct VecFmt;

template <>
struct VecFmt<F64> {
    static constexpr int bytes = 48;
    __device__ static Vec3<double> load(const void* base, int Vh, int cb) {
        const double2* p = (const double2*)base;
        Vec3<double> v;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double2 a = p[(size_t)c * Vh + cb];
            v.c[c].re = a.x;
            v.c[c].im = a.y;
        }
        return v;
    }
    __device__ static void store(void* base, int Vh, int cb, const Vec3<double>& v) {
        double2* p = (double2*)base;
#pragma unroll
        for (int c = 0; c < 3; ++c) p[(size_t)c * Vh + cb] = make_double2(v.c[c].re, v.c[c].im);
    }
    // store and return the value as stored
    __device__ static Vec3<double> store_rt(void* base, int Vh, int cb, const Vec3<double>& v) {
        store(base, Vh, cb, v);
        return v;
    }
};

template <>
struct VecFmt<F32> {
    static constexpr int bytes = 24;
    __device__ static Vec3<float> load(const void* base, int Vh, int cb) {
        const float4* p4 = (const float4*)base;
        const float2* p2 = (const float2*)(p4 + Vh);
        float4 a = p4[cb];
        float2 b = p2[cb];
        Vec3<float> v;
        v.c[0].re = a.x; v.c[0].im = a.y; v.c[1].re = a.z; v.c[1].im = a.w;
        v.c[2].re = b.x; v.c[2].im = b.y;
        return v;
    }
    __device__ static void store(void* base, int Vh, int cb, const Vec3<float>& v) {
        float4* p4 = (float4*)base;
        float2* p2 = (float2*)(p4 + Vh);
        p4[cb] = make_float4(v.c[0].re, v.c[0].im, v.c[1].re, v.c[1].im);
        p2[cb] = make_float2(v.c[2].re, v.c[2].im);
    }
    __device__ static Vec3<float> store_rt(void* base, int Vh, int cb, const Vec3<float>& v) {
        store(base, Vh, cb, v);
        return v;
    }
};

template <int P>
struct VecFmt16 {
    static constexpr bool scaled = (P == F16);
    static constexpr int bytes = scaled ? 16 : 12;
    __device__ static Vec3<float> load(const void* base, int Vh, int cb) {
        uint32_t w0, w1, w2;
        float s = 1.0f;
        if constexpr (scaled) {
            const uint4 q = ((const uint4*)base)[cb];  // three packed pairs and the site norm: one load
            w0 = q.x; w1 = q.y; w2 = q.z;
            s = __uint_as_float(q.w);
        } else {
            const uint2* pa = (const uint2*)base;
            const uint2 a = pa[cb];
            w0 = a.x; w1 = a.y;
            w2 = ((const uint32_t*)(pa + Vh))[cb];
        }
        Vec3<float> v;
        v.c[0].re = s * unpack_lo<P>(w0); v.c[0].im = s * unpack_hi<P>(w0);
        v.c[1].re = s * unpack_lo<P>(w1); v.c[1].im = s * unpack_hi<P>(w1);
        v.c[2].re = s * unpack_lo<P>(w2); v.c[2].im = s * unpack_hi<P>(w2);
        return v;
    }
    __device__ static void store(void* base, int Vh, int cb, const Vec3<float>& v) { (void)store_rt(base, Vh, cb, v); }
    // store and return the value as stored (rounded to 16 bits, scaled by the site norm)
    __device__ static Vec3<float> store_rt(void* base, int Vh, int cb, const Vec3<float>& v) {
        float inv = 1.0f, m = 1.0f, k = 1.0f;
        if constexpr (scaled) {
            m = 0.0f;
#pragma unroll
            for (int c = 0; c < 3; ++c) m = fmaxf(m, fmaxf(fabsf(v.c[c].re), fabsf(v.c[c].im)));
            // a site norm near the bottom of the FP32 range (the last residuals of a source of norm ~1e-30)
            // would overflow 1/m: scale the site by 2^64 (exact) before dividing
            k = m < 1.0e-30f ? 18446744073709551616.0f : 1.0f;
            inv = m > 0.0f ? 1.0f / (m * k) : 0.0f;
        }
        const uint32_t w0 = pack2<P>(inv * (k * v.c[0].re), inv * (k * v.c[0].im));
        const uint32_t w1 = pack2<P>(inv * (k * v.c[1].re), inv * (k * v.c[1].im));
        const uint32_t w2 = pack2<P>(inv * (k * v.c[2].re), inv * (k * v.c[2].im));
        if constexpr (scaled) {
            ((uint4*)base)[cb] = make_uint4(w0, w1, w2, __float_as_uint(m));
        } else {
            uint2* pa = (uint2*)base;
            pa[cb] = make_uint2(w0, w1);
            ((uint32_t*)(pa + Vh))[cb] = w2;
        }
        Vec3<float> o;
        o.c[0].re = m * unpack_lo<P>(w0); o.c[0].im = m * unpack_hi<P>(w0);
        o.c[1].re = m * unpack_lo<P>(w1); o.c[1].im = m * unpack_hi<P>(w1);
        o.c[2].re = m * unpack_lo<P>(w2); o.c[2].im = m * unpack_hi<P>(w2);
        return o;
    }
};
template <>
struct VecFmt<F16> : VecFmt16<F16> {};
template <>
struct VecFmt<BF16> : VecFmt16<BF16> {};

// ------------------------------------------------------------------------------------------------------
// Loads of packed link words. NT = false: ordinary cached loads. NT = true: non-temporal (streaming) loads,
// which mark the lines for early eviction: a link field read once per launch then does not push the
// neighbour vectors (each read by eight sites) out of the caches. Cached loads keep a link field that fits
// in the Infinity Cache there between launches; which one is faster depends on the lattice size, and the
// launch autotuner chooses.
// ------------------------------------------------------------------------------------------------------
template <bool NT>
__device__ __forceinline__ float4 ldw(const float4* p) {
    if constexpr (NT) {
        typedef float v4 __attribute__((ext_vector_type(4)));
        const v4 v = __builtin_nontemporal_load((const v4*)p);
        return make_float4(v.x, v.y, v.z, v.w);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ float2 ldw(const float2* p) {
    if constexpr (NT) {
        typedef float v2 __attribute__((ext_vector_type(2)));
        const v2 v = __builtin_nontemporal_load((const v2*)p);
        return make_float2(v.x, v.y);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ double2 ldw(const double2* p) {
    if constexpr (NT) {
        typedef double v2 __attribute__((ext_vector_type(2)));
        const v2 v = __builtin_nontemporal_load((const v2*)p);
        return make_double2(v.x, v.y);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ uint4 ldw(const uint4* p) {
    if constexpr (NT) {
        typedef unsigned int v4 __attribute__((ext_vector_type(4)));
        const v4 v = __builtin_nontemporal_load((const v4*)p);
        return make_uint4(v.x, v.y, v.z, v.w);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ uint2 ldw(const uint2* p) {
    if constexpr (NT) {
        typedef unsigned int v2 __attribute__((ext_vector_type(2)));
        const v2 v = __builtin_nontemporal_load((const v2*)p);
        return make_uint2(v.x, v.y);
    } else {
        return *p;
    }
}
template <bool NT>
__device__ __forceinline__ uint32_t ldw(const uint32_t* p) {
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}

// ------------------------------------------------------------------------------------------------------
// Link storage. The packed field is 8 blocks (parity q = 0,1) x (mu = 0..3), block (q, mu) holding
// U_mu(n) for the Vh sites n of parity q in cb order, as planes:
//   F64  r18: 9 planes double2                         144 B/link
//   F32  r18: 4 planes float4 + 1 plane float2          72 B/link
//   F32  r12: 3 planes float4 (rows 0,1)                48 B/link
//   F32  r8 : 2 planes float4 (U01, U02; U10, 2 phases) 32 B/link
//   16b  r18: 2 planes uint4 (16 values) + 1 plane uint  36 B/link
//   16b  r12: 1 plane uint4 + 1 plane uint2             24 B/link
// Real parts and imaginary parts alternate, row-major: e00.re e00.im e01.re ... e22.im.
// ------------------------------------------------------------------------------------------------------
template <int P, int RECON>
struct LinkFmt;

template <>
struct LinkFmt<F64, 18> {
    static constexpr int bytes = 144;
    template <bool NT = false>
    __device__ static Su3<double> load(const void* blk, int Vh, int cb) {
        const double2* p = (const double2*)blk;
        Su3<double> U;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            double2 a = ldw<NT>(p + (size_t)k * Vh + cb);
            U.e[k / 3][k % 3].re = a.x;
            U.e[k / 3][k % 3].im = a.y;
        }
        return U;
    }
    __device__ static void store(void* blk, int Vh, int cb, const double* r) {
        double2* p = (double2*)blk;
#pragma unroll
        for (int k = 0; k < 9; ++k) p[(size_t)k * Vh + cb] = make_double2(r[2 * k], r[2 * k + 1]);
    }
};

template <int RECON>
struct LinkFmtF32 {
    static constexpr int nq = RECON == 18 ? 4 : 3;  // float4 planes
    static constexpr int bytes = RECON == 18 ? 72 : 48;
    template <bool NT = false>
    __device__ static Su3<float> load(const void* blk, int Vh, int cb) {
        const float4* p = (const float4*)blk;
        float f[18];
#pragma unroll
        for (int k = 0; k < nq; ++k) {
            float4 a = ldw<NT>(p + (size_t)k * Vh + cb);
            f[4 * k] = a.x; f[4 * k + 1] = a.y; f[4 * k + 2] = a.z; f[4 * k + 3] = a.w;
        }
        if constexpr (RECON == 18) {
            float2 b = ldw<NT>((const float2*)(p + (size_t)4 * Vh) + cb);
            f[16] = b.x; f[17] = b.y;
        }
        Su3<float> U;
#pragma unroll
        for (int k = 0; k < RECON / 2; ++k) {
            U.e[k / 3][k % 3].re = f[2 * k];
            U.e[k / 3][k % 3].im = f[2 * k + 1];
        }
        if constexpr (RECON == 12) rebuild_row2(U);
        return U;
    }
    __device__ static void store(void* blk, int Vh, int cb, const double* r) {
        float4* p = (float4*)blk;
#pragma unroll
        for (int k = 0; k < nq; ++k)
            p[(size_t)k * Vh + cb] = make_float4((float)r[4 * k], (float)r[4 * k + 1], (float)r[4 * k + 2], (float)r[4 * k + 3]);
        if constexpr (RECON == 18) ((float2*)(p + (size_t)4 * Vh))[cb] = make_float2((float)r[16], (float)r[17]);
    }
};
template <>
struct LinkFmt<F32, 18> : LinkFmtF32<18> {};
template <>
struct LinkFmt<F32, 12> : LinkFmtF32<12> {};

// FP32 recon 8: plane 0 holds (U01, U02) and plane 1 (S, arg U00, f), 32 B per link, where S is the smaller in
// modulus of U10 and U20 and f the phase of the other one, L; f is stored plus 8 when S is U20 (phases lie in
// [-pi, pi], so the offset marks the case; subtracting it again is exact, and the phase keeps a quantum of
// 9.5e-7). With n = |U01|^2 + |U02|^2 the moduli follow from the unit norms of row 0 and column 0,
// |U00| = sqrt(1 - n) and |L| = sqrt(n - |S|^2) >= sqrt(n / 2) (so the difference of squares loses nothing;
// rebuilding the smaller entry from it instead leaves errors up to 1e-4 on near-identity fields), and the four
// remaining entries from row 1 and row 2 being orthogonal to row 0 with det U = 1 (each row the conjugate cross
// product of the other two), two 2x2 systems of determinant -n and n:
//   U11 = -(conj U20 conj U02 + U01 U10 conj U00) / n,   U12 = (conj U01 conj U20 - U02 U10 conj U00) / n,
//   U21 = (conj U10 conj U02 - U01 U20 conj U00) / n,    U22 = -(U02 U20 conj U00 + conj U01 conj U10) / n.
// Every product is of stored or rebuilt entries of size <= sqrt(n) against the divisor n, so small n costs no
// precision; n = 0 (row 0 a phase times (1, 0, 0)) leaves the lower block undetermined, and such fields are
// refused when packed from Python (the C packing's caller must not pass them: the operator would be NaN and the
// solve would stop with a breakdown). |U00| = sqrt(1 - n) loses precision as |U00| -> 0, which near-identity
// (smeared) fields never approach. On the 20^3x64 near-identity field the rebuilt entries are within 6e-7 of
// the FP64 links (FP32 rounding 4e-8, phase quantum and hardware sine and cosine the rest).
template <>
struct LinkFmt<F32, 8> {
    static constexpr int bytes = 32;
    template <bool NT = false>
    __device__ static Su3<float> load(const void* blk, int Vh, int cb) {
        using Cf = Cx<float>;
        const float4* p = (const float4*)blk;
        const float4 u = ldw<NT>(p + cb);
        const float4 v = ldw<NT>(p + (size_t)Vh + cb);
        const Cf a2 = {u.x, u.y}, a3 = {u.z, u.w}, sm = {v.x, v.y};
        const bool s_is_u20 = v.w > 4.0f;
        const float f = s_is_u20 ? v.w - 8.0f : v.w;
        const float n = a2.re * a2.re + a2.im * a2.im + a3.re * a3.re + a3.im * a3.im;
        const float ra1 = sqrtf(fmaxf(1.0f - n, 0.0f));
        const float rl = sqrtf(fmaxf(n - (sm.re * sm.re + sm.im * sm.im), 0.0f));
        float s1, k1, s2, k2;
        __sincosf(v.z, &s1, &k1);
        __sincosf(f, &s2, &k2);
        const Cf a1 = {ra1 * k1, ra1 * s1}, lg = {rl * k2, rl * s2};
        const Cf b1 = s_is_u20 ? lg : sm, c1 = s_is_u20 ? sm : lg;
        const float inv = 1.0f / n;
        auto mul = [](Cf x, Cf y) { return Cf{x.re * y.re - x.im * y.im, x.re * y.im + x.im * y.re}; };
        auto cj = [](Cf x) { return Cf{x.re, -x.im}; };
        const Cf b1a = mul(b1, cj(a1)), c1a = mul(c1, cj(a1));
        const Cf t1 = mul(cj(c1), cj(a3)), t2 = mul(a2, b1a), t3 = mul(cj(a2), cj(c1)), t4 = mul(a3, b1a);
        const Cf t5 = mul(cj(b1), cj(a3)), t6 = mul(a2, c1a), t7 = mul(a3, c1a), t8 = mul(cj(a2), cj(b1));
        Su3<float> U;
        U.e[0][0] = a1;
        U.e[0][1] = a2;
        U.e[0][2] = a3;
        U.e[1][0] = b1;
        U.e[1][1] = {-(t1.re + t2.re) * inv, -(t1.im + t2.im) * inv};
        U.e[1][2] = {(t3.re - t4.re) * inv, (t3.im - t4.im) * inv};
        U.e[2][0] = c1;
        U.e[2][1] = {(t5.re - t6.re) * inv, (t5.im - t6.im) * inv};
        U.e[2][2] = {-(t7.re + t8.re) * inv, -(t7.im + t8.im) * inv};
        return U;
    }
    // r: the 18 reals of the link, row-major, re and im alternating; the phases in FP64, then rounded
    __device__ static void store(void* blk, int Vh, int cb, const double* r) {
        float4* p = (float4*)blk;
        p[cb] = make_float4((float)r[2], (float)r[3], (float)r[4], (float)r[5]);
        const bool s_is_u20 = r[12] * r[12] + r[13] * r[13] < r[6] * r[6] + r[7] * r[7];
        const double sr = s_is_u20 ? r[12] : r[6], si = s_is_u20 ? r[13] : r[7];
        const double f = s_is_u20 ? atan2(r[7], r[6]) + 8.0 : atan2(r[13], r[12]);
        p[(size_t)Vh + cb] = make_float4((float)sr, (float)si, (float)atan2(r[1], r[0]), (float)f);
    }
};

template <int P, int RECON>
struct LinkFmt16 {
    static constexpr int bytes = RECON == 18 ? 36 : 24;
    template <bool NT = false>
    __device__ static Su3<float> load(const void* blk, int Vh, int cb) {
        const uint4* p = (const uint4*)blk;
        uint32_t w[9];
        uint4 a = ldw<NT>(p + cb);
        w[0] = a.x; w[1] = a.y; w[2] = a.z; w[3] = a.w;
        if constexpr (RECON == 18) {
            uint4 b = ldw<NT>(p + (size_t)Vh + cb);
            w[4] = b.x; w[5] = b.y; w[6] = b.z; w[7] = b.w;
            w[8] = ldw<NT>((const uint32_t*)(p + (size_t)2 * Vh) + cb);
        } else {
            uint2 b = ldw<NT>((const uint2*)(p + (size_t)Vh) + cb);
            w[4] = b.x; w[5] = b.y;
        }
        Su3<float> U;
#pragma unroll
        for (int k = 0; k < RECON / 2; ++k) {
            U.e[k / 3][k % 3].re = unpack_lo<P>(w[k]);
            U.e[k / 3][k % 3].im = unpack_hi<P>(w[k]);
        }
        if constexpr (RECON == 12) rebuild_row2(U);
        return U;
    }
    __device__ static void store(void* blk, int Vh, int cb, const double* r) {
        uint32_t w[9];
#pragma unroll
        for (int k = 0; k < RECON / 2; ++k) w[k] = pack2<P>((float)r[2 * k], (float)r[2 * k + 1]);
        uint4* p = (uint4*)blk;
        p[cb] = make_uint4(w[0], w[1], w[2], w[3]);
        if constexpr (RECON == 18) {
            p[(size_t)Vh + cb] = make_uint4(w[4], w[5], w[6], w[7]);
            ((uint32_t*)(p + (size_t)2 * Vh))[cb] = w[8];
        } else {
            ((uint2*)(p + (size_t)Vh))[cb] = make_uint2(w[4], w[5]);
        }
    }
};
template <>
struct LinkFmt<F16, 18> : LinkFmt16<F16, 18> {};
template <>
struct LinkFmt<F16, 12> : LinkFmt16<F16, 12> {};
template <>
struct LinkFmt<BF16, 18> : LinkFmt16<BF16, 18> {};
template <>
struct LinkFmt<BF16, 12> : LinkFmt16<BF16, 12> {};
template <>
struct LinkFmt<I16, 18> : LinkFmt16<I16, 18> {};
template <>
struct LinkFmt<I16, 12> : LinkFmt16<I16, 12> {};

// Address of block (q, mu) of a packed gauge field.
template <class LF>
__device__ __forceinline__ const char* link_block(const void* links, int Vh, int q, int mu) {
    return (const char*)links + (size_t)(q * 4 + mu) * (size_t)Vh * LF::bytes;
}

// ------------------------------------------------------------------------------------------------------
// Checkerboard geometry
// ------------------------------------------------------------------------------------------------------
struct Geom {
    int X, Y, Z, T;
    int Xh;   // X / 2
    int Vh;   // X*Y*Z*T / 2
    int bc_t; // 1: antiperiodic in t
    float rXh, rY, rZ;  // reciprocals for the index division
};

// floor(a / d) for 0 <= a < 2^24, 1 <= d: the float estimate is within one of the quotient.
__host__ __device__ __forceinline__ int divq(int a, int d, float rd) {
    int q = (int)((float)a * rd);
    int r = a - q * d;
    q += (r >= d) - (r < 0);
    return q;
}

struct Site {
    int cb;
    int x, y, z, t;
    int row;  // cb - x/2: first cb of this (y,z,t) row
};

__host__ __device__ __forceinline__ Site site_of(const Geom& g, int p, int cb) {
    Site s;
    s.cb = cb;
    int r = divq(cb, g.Xh, g.rXh);
    int xh = cb - r * g.Xh;
    int r2 = divq(r, g.Y, g.rY);
    s.y = r - r2 * g.Y;
    s.t = divq(r2, g.Z, g.rZ);
    s.z = r2 - s.t * g.Z;
    s.x = 2 * xh + ((p + s.y + s.z + s.t) & 1);
    s.row = cb - xh;
    return s;
}

// cb index of n + mu (dir = +1) or n - mu (dir = -1); the neighbour has the opposite parity.
__host__ __device__ __forceinline__ int nbr(const Geom& g, const Site& s, int mu, int dir) {
    if (mu == 0) {
        int x1 = dir > 0 ? (s.x + 1 == g.X ? 0 : s.x + 1) : (s.x == 0 ? g.X - 1 : s.x - 1);
        return s.row + (x1 >> 1);
    }
    int stride, c, L;
    if (mu == 1) { stride = g.Xh; c = s.y; L = g.Y; }
    else if (mu == 2) { stride = g.Xh * g.Y; c = s.z; L = g.Z; }
    else { stride = g.Xh * g.Y * g.Z; c = s.t; L = g.T; }
    if (dir > 0) return c == L - 1 ? s.cb - (L - 1) * stride : s.cb + stride;
    return c == 0 ? s.cb + (L - 1) * stride : s.cb - stride;
}

// eta_mu(n): +1 or -1
__host__ __device__ __forceinline__ float eta_sign(const Site& s, int mu) {
    int e = mu == 0 ? 0 : mu == 1 ? s.x : mu == 2 ? s.x + s.y : s.x + s.y + s.z;
    return (e & 1) ? -1.0f : 1.0f;
}

// Directions whose gathers a single-system half operator keeps in flight together (the unroll of its direction
// loop), by measurement: two where all four put too many values in registers (FP64: 384 values; FP32 recon-12
// and recon-8 and 16-bit links with FP32 vectors: the rebuild of rows and the unpacking lower the waves per SIMD)
// unless the links stream past the caches, four otherwise.
constexpr int unroll_dirs(int lp, int recon, int vp, bool nt) {
    return (vp == F64 || (!nt && ((lp == F32 && recon != 18) || (vp == F32 && lp != F32)))) ? 2 : 4;
}

// ------------------------------------------------------------------------------------------------------
// The half operator at one site:
//   out(n) = 1/2 sum_mu eta_mu(n) [ s_f U_mu(n) in(n+mu) - s_b U_mu(n-mu)^dag in(n-mu) ]
// with s_f, s_b the antiperiodic-time signs of the two links. Links of parity p are the forward links;
// the backward link U_mu(n-mu) sits at the neighbour's cb in the parity 1-p block.
// ------------------------------------------------------------------------------------------------------
template <int LP, int RECON, int VP, bool NT = false>
__device__ __forceinline__ Vec3<typename Real<VP>::T> dslash_site(const Geom g, const void* links, const void* in,
                                                                  int p, const Site s) {
    using R = typename Real<VP>::T;
    using LF = LinkFmt<LP, RECON>;
    using VF = VecFmt<VP>;
    Vec3<R> acc = vzero<R>();
    constexpr int UNROLL = unroll_dirs(LP, RECON, VP, NT);
#pragma unroll UNROLL
    for (int mu = 0; mu < 4; ++mu) {
        R e = (R)eta_sign(s, mu);
        R sf = e, sb = e;
        if (mu == 3 && g.bc_t) {
            if (s.t == g.T - 1) sf = -sf;
            if (s.t == 0) sb = -sb;
        }
        int nf = nbr(g, s, mu, +1);
        int nb = nbr(g, s, mu, -1);
        Su3<R> Uf = LF::template load<NT>(link_block<LF>(links, g.Vh, p, mu), g.Vh, s.cb);
        Vec3<R> vf = VF::load(in, g.Vh, nf);
        Su3<R> Ub = LF::template load<NT>(link_block<LF>(links, g.Vh, 1 - p, mu), g.Vh, nb);
        Vec3<R> vb = VF::load(in, g.Vh, nb);
        mv_acc(acc, Uf, vf, sf);
        mdv_acc(acc, Ub, vb, -sb);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        acc.c[i].re *= R(0.5);
        acc.c[i].im *= R(0.5);
    }
    return acc;
}

// ------------------------------------------------------------------------------------------------------
// Reductions (FP64, fixed order: deterministic for a fixed launch shape)
// ------------------------------------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sums NV values per thread across the block; results valid in thread 0. blockDim.x <= 1024.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV]) {
    __shared__ double sm[NV][16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) sm[k][wid] = v[k];
    }
    __syncthreads();
    if (wid == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double a = lane < nw ? sm[k][lane] : 0.0;
            v[k] = wave_sum(a);
        }
    }
    __syncthreads();
}

// ------------------------------------------------------------------------------------------------------
// Device-resident CG state of one system. Written by the one-block finalize launch, or, in the fused
// single-system iteration, by block 0 into a second buffer that only later launches read; either way every
// block of a launch sees the same values.
// ------------------------------------------------------------------------------------------------------
enum : int {
    ST_DONE = 1,        // stop: every kernel of this system returns at entry
    ST_BREAKDOWN = 2,   // Re<p,Ap> <= 0 or a non-finite scalar
    ST_PENDING = 4,     // iterations paused until the next reliable update
    ST_MAXIT = 8,       // iteration cap reached
    ST_STALL = 16,      // true residual stopped improving
    ST_CONVERGED = 32,  // true residual <= tol |b|
    ST_XPAY_DUE = 64,   // p = a r + beta p is due (after a reliable update, or p = r at the start)
    ST_T_STALE = 128,   // p was formed outside the t recurrence: the next t must be D_oe p itself
};

struct alignas(64) SolverState {
    double rho;       // |r|^2 entering the current iteration
    double alpha, beta, pq, rho_new;
    double xpay_a;    // p = xpay_a r + beta p after a reliable update
    double rr_ru;     // true |r|^2 at the last reliable update (delta trigger)
    double bnorm2;    // |b|^2
    double stop2;     // tol^2 |b|^2
    double tol2;      // tol^2
    double delta2;    // delta^2
    double floor2;    // any-iteration trigger: |r|^2 below floor2 * rr_ru (0: off)
    double true_rho;  // last true |r|^2
    double best_rho;  // best true |r|^2 so far (stagnation)
    double m2;        // mass^2
    double drift;     // a reliable update restarts the direction (p = r) when the true |r|^2 exceeds the
                      // recursive one by more than this factor (0: at every update)
    int iter, iter_last_ru, ru_count, flags;
    int stall, max_iter, ru_every;
};

static constexpr int STALL_LIMIT = 6;

__device__ __forceinline__ void fin_alpha(SolverState* st, double pq) {
    st->pq = pq;
    st->flags &= ~ST_XPAY_DUE;
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(st->rho)) {
        st->flags |= ST_BREAKDOWN | ST_DONE;
        return;
    }
    st->alpha = st->rho / pq;
}

// After r -= alpha q. A reliable update is requested (the iteration's p update is then left to it) on
// apparent convergence, at the iteration cap and when |r| fell three decades below |r_true at the last
// update| at any iteration; on the last iteration of a chunk also when |r| fell below delta |r_true at the
// last update| or ru_every iterations have passed. Keeping the
// last two triggers at chunk ends means a chunk never stops early for them.
__device__ __forceinline__ void fin_update(SolverState* st, double rho_new, bool chunk_end) {
    st->iter += 1;
    st->rho_new = rho_new;
    if (!isfinite(rho_new)) {
        st->flags |= ST_BREAKDOWN | ST_DONE;
        return;
    }
    bool pause = rho_new <= st->stop2 || st->iter >= st->max_iter;
    // the recursive residual has fallen three decades below the last true one: further than a low-precision
    // recursion stays accurate; left until the chunk end, it can run many decades below the true residual
    // in a fast-converging solve, and the update would then restart from a direction scaled by their ratio
    pause |= rho_new < st->floor2 * st->rr_ru;
    if (chunk_end) {
        pause |= st->delta2 > 0.0 && rho_new < st->delta2 * st->rr_ru;
        pause |= st->iter - st->iter_last_ru >= st->ru_every;
    }
    if (pause) {
        st->flags |= ST_PENDING;
        return;
    }
    st->beta = rho_new / st->rho;
    st->rho = rho_new;
}

// After a true residual r (|r|^2 = rho_true, rp = Re<r, p> with the current direction p). init = 1 for the
// initial residual of a solve, which is followed by p = r. Otherwise the paused iteration's direction
// update becomes
//   p = r + beta (p - c r), beta = rho_true / rho, c = Re<r,p> / rho_true
// which restores the orthogonality of the old direction to the new residual, or p = r (restart) when the
// true residual has drifted from the recursive one by more than the factor st->drift: a kept direction assumes
// that the recursion tracked the true residual, and once the inner operator's error dominates the residual it
// no longer does.
__device__ __forceinline__ void fin_resid(SolverState* st, double rho_true, double rp, int init) {
    st->true_rho = rho_true;
    if (!init) st->ru_count += 1;
    st->iter_last_ru = st->iter;
    st->flags &= ~ST_PENDING;
    if (!isfinite(rho_true) || !isfinite(rp)) {
        st->flags |= ST_BREAKDOWN | ST_DONE;
        return;
    }
    if (rho_true <= st->stop2) {
        st->flags |= ST_CONVERGED | ST_DONE;
        return;
    }
    if (st->iter >= st->max_iter) {
        st->flags |= ST_MAXIT | ST_DONE;
        return;
    }
    if (init || rho_true < st->best_rho) {
        st->best_rho = rho_true;
        st->stall = 0;
    } else if (++st->stall > STALL_LIMIT) {
        st->flags |= ST_STALL | ST_DONE;
        return;
    }
    st->rr_ru = rho_true;
    if (init) {
        st->beta = 0.0;  // p = r
        st->xpay_a = 1.0;
    } else {
        if (rho_true > st->drift * st->rho_new) {
            st->beta = 0.0;
            st->xpay_a = 1.0;
        } else {
            const double beta = rho_true / st->rho;
            st->beta = beta;
            st->xpay_a = 1.0 - beta * (rp / rho_true);
        }
    }
    st->flags |= ST_XPAY_DUE | ST_T_STALE;
    st->rho = rho_true;
}

}  // namespace sp
