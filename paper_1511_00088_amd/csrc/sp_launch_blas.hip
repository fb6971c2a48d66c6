// Instantiations and launches of the fused vector updates, reductions and packing kernels.
#include "sp_launch.h"

namespace sp {

// Fill n 16-byte words with zeros (used instead of memset so that it can sit inside a graph).
__global__ __launch_bounds__(256) void k_zero16(uint4* p, long n) {
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// *dst = *src for the double-buffered state of k_xpay_fused (one thread).
__global__ void k_state_copy(const SolverState* __restrict__ src, SolverState* __restrict__ dst) {
    if (threadIdx.x == 0) *dst = *src;
}

// dst[0..n) = src[0..n), one block: the systems' states copied to the pinned host buffer that the solver polls,
// as the last node of a chunk's graph (in 16-byte words; the state's size is a multiple of 64 bytes).
__global__ __launch_bounds__(256) void k_state_publish(const uint4* __restrict__ src, uint4* __restrict__ dst, int words) {
    for (int i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
}
static_assert(sizeof(SolverState) % sizeof(uint4) == 0, "states copy as 16-byte words");

template <class D>
struct NOf {
    static constexpr int value = NB;
};
template <>
struct NOf<DescSingle> {
    static constexpr int value = 1;
};

template <class D>
hipError_t launch_xpay(const D& d, int nblocks, LaunchCfg c, int vp, int gate, hipStream_t s) {
    constexpr int N = NOf<D>::value;
#define SP_LAUNCH(VP)                                                                                      \
    do {                                                                                                   \
        hipLaunchKernelGGL((k_xpay<VP, N, D>), dim3(nblocks), dim3(c.nt), 0, s, d, gate, c.remap);          \
        return hipGetLastError();                                                                          \
    } while (0)
    if (vp == F64) SP_LAUNCH(F64);
    if (vp == F32) SP_LAUNCH(F32);
    if (vp == F16) SP_LAUNCH(F16);
    if (vp == BF16) SP_LAUNCH(BF16);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_xpay_fused(const DescSingle& d, SolverState* st_out, int chunk_end, int nblocks, LaunchCfg c, int vp,
                             hipStream_t s) {
#define SP_LAUNCH(VP)                                                                                      \
    do {                                                                                                   \
        hipLaunchKernelGGL((k_xpay_fused<VP>), dim3(nblocks), dim3(c.nt), 0, s, d, st_out, chunk_end, c.remap); \
        return hipGetLastError();                                                                          \
    } while (0)
    if (vp == F64) SP_LAUNCH(F64);
    if (vp == F32) SP_LAUNCH(F32);
    if (vp == F16) SP_LAUNCH(F16);
    if (vp == BF16) SP_LAUNCH(BF16);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_state_publish(const SolverState* src, SolverState* dst, int n, hipStream_t s) {
    const int words = (int)(n * sizeof(SolverState) / sizeof(uint4));
    hipLaunchKernelGGL(k_state_publish, dim3(1), dim3(256), 0, s, (const uint4*)src, (uint4*)dst, words);
    return hipGetLastError();
}

hipError_t launch_state_copy(const SolverState* src, SolverState* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_state_copy, dim3(1), dim3(64), 0, s, src, dst);
    return hipGetLastError();
}

template <class D>
hipError_t launch_accum(const D& d, int nblocks, LaunchCfg c, hipStream_t s) {
    constexpr int N = NOf<D>::value;
    hipLaunchKernelGGL((k_accum<N, D>), dim3(nblocks), dim3(c.nt), 0, s, d, c.remap);
    return hipGetLastError();
}

template <class D>
hipError_t launch_norm_b(const D& d, int nblocks, LaunchCfg c, hipStream_t s) {
    constexpr int N = NOf<D>::value;
    hipLaunchKernelGGL((k_norm_b<N, D>), dim3(nblocks), dim3(c.nt), 0, s, d, c.remap);
    return hipGetLastError();
}

template <class D>
hipError_t launch_finalize(const D& d, int ngroups, int kind, int gate, hipStream_t s) {
    constexpr int N = NOf<D>::value;
    hipLaunchKernelGGL((k_finalize<N, D>), dim3(ngroups), dim3(1024), 0, s, d, kind, gate);
    return hipGetLastError();
}

#define SP_INST(D)                                                                                         \
    template hipError_t launch_finalize<D>(const D&, int, int, int, hipStream_t);                          \
    template hipError_t launch_xpay<D>(const D&, int, LaunchCfg, int, int, hipStream_t);                   \
    template hipError_t launch_accum<D>(const D&, int, LaunchCfg, hipStream_t);                            \
    template hipError_t launch_norm_b<D>(const D&, int, LaunchCfg, hipStream_t);
SP_INST(DescSingle)
SP_INST(DescBatch)
#undef SP_INST

hipError_t launch_pack_gauge(const Geom& g, const double* nat, int prec, int recon, void* out, hipStream_t s) {
    const long n = 8L * g.Vh;
    const int nb = (int)((n + 255) / 256);
#define SP_LAUNCH(P, RC)                                                                                   \
    do {                                                                                                   \
        hipLaunchKernelGGL((k_pack_gauge<P, RC>), dim3(nb), dim3(256), 0, s, g, nat, out);                 \
        return hipGetLastError();                                                                          \
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

hipError_t launch_pack_vec(int Vh, const double* nat, int prec, void* out, hipStream_t s) {
    const int nb = blocks_for(Vh, 256);
#define SP_LAUNCH(P)                                                                                       \
    do {                                                                                                   \
        hipLaunchKernelGGL((k_pack_vec<P>), dim3(nb), dim3(256), 0, s, Vh, nat, out);                      \
        return hipGetLastError();                                                                          \
    } while (0)
    if (prec == F64) SP_LAUNCH(F64);
    if (prec == F32) SP_LAUNCH(F32);
    if (prec == F16) SP_LAUNCH(F16);
    if (prec == BF16) SP_LAUNCH(BF16);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_unpack_vec(int Vh, const void* in, int prec, double* nat, hipStream_t s) {
    const int nb = blocks_for(Vh, 256);
#define SP_LAUNCH(P)                                                                                       \
    do {                                                                                                   \
        hipLaunchKernelGGL((k_unpack_vec<P>), dim3(nb), dim3(256), 0, s, Vh, in, nat);                     \
        return hipGetLastError();                                                                          \
    } while (0)
    if (prec == F64) SP_LAUNCH(F64);
    if (prec == F32) SP_LAUNCH(F32);
    if (prec == F16) SP_LAUNCH(F16);
    if (prec == BF16) SP_LAUNCH(BF16);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

hipError_t launch_zero(void* p, size_t bytes, hipStream_t s) {
    const long n = (long)(bytes / 16);
    if (n == 0) return hipSuccess;
    const int nb = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_zero16, dim3(nb), dim3(256), 0, s, (uint4*)p, n);
    return hipGetLastError();
}

}  // namespace sp
