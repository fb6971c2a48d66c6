// Streaming-bandwidth probe: the attainable HBM rate that the bandwidth-bound kernels of this library are
// measured against (the paper, Sec. 4 and Table 3, argues CG performance from memory bandwidth per flop).
// Three kernels over n 16-byte words, each lane moving whole 16-byte words, K words per lane in flight:
//   read  : s += a[i]        (one 16-byte word read per element; a per-block sum is written so that the loads
//                             are not removed)
//   copy  : b[i] = a[i]      (read + write)
//   triad : b[i] = a[i] + q c[i]  (two reads + one write, FP32 lanes)
// Lane l of block k handles words k K T + j T + l, j < K (T threads per block): each load instruction of a wave
// covers 1 KB of consecutive memory.
#include <hip/hip_runtime.h>

#include "sp_entry.h"

namespace sp {

template <int K>
__global__ __launch_bounds__(256) void k_stream_read(const float4* __restrict__ a, size_t n, float* __restrict__ out) {
    const size_t base = (size_t)blockIdx.x * K * blockDim.x + threadIdx.x;
    float4 v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const size_t i = base + (size_t)j * blockDim.x;
        v[j] = i < n ? a[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < K; ++j) s += (v[j].x + v[j].y) + (v[j].z + v[j].w);
    // one word per block: a wave sum by shuffles, lane 0 of wave 0 stores it (the rest is dead without it)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (threadIdx.x == 0) out[blockIdx.x] = s;
}

template <int K>
__global__ __launch_bounds__(256) void k_stream_copy(const float4* __restrict__ a, float4* __restrict__ b, size_t n) {
    const size_t base = (size_t)blockIdx.x * K * blockDim.x + threadIdx.x;
    float4 v[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const size_t i = base + (size_t)j * blockDim.x;
        if (i < n) v[j] = a[i];
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const size_t i = base + (size_t)j * blockDim.x;
        if (i < n) b[i] = v[j];
    }
}

template <int K>
__global__ __launch_bounds__(256) void k_stream_triad(const float4* __restrict__ a, float4* __restrict__ b,
                                                      const float4* __restrict__ c, float q, size_t n) {
    const size_t base = (size_t)blockIdx.x * K * blockDim.x + threadIdx.x;
    float4 v[K], w[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const size_t i = base + (size_t)j * blockDim.x;
        if (i < n) {
            v[j] = a[i];
            w[j] = c[i];
        }
    }
#pragma unroll
    for (int j = 0; j < K; ++j) {
        const size_t i = base + (size_t)j * blockDim.x;
        if (i < n)
            b[i] = make_float4(v[j].x + q * w[j].x, v[j].y + q * w[j].y, v[j].z + q * w[j].z, v[j].w + q * w[j].w);
    }
}

size_t stream_blocks(size_t n16, int k) { return (n16 + (size_t)k * 256 - 1) / ((size_t)k * 256); }

hipError_t launch_stream(int kind, int k, const void* a, void* b, const void* c, size_t n16, hipStream_t s) {
    const size_t nb = stream_blocks(n16, k);
    if (nb == 0 || nb > 0x7fffffffu) return hipErrorInvalidValue;
#define SP_LAUNCH(K)                                                                                          \
    do {                                                                                                      \
        if (kind == 0)                                                                                        \
            hipLaunchKernelGGL((k_stream_read<K>), dim3((unsigned)nb), dim3(256), 0, s, (const float4*)a, n16, \
                               (float*)b);                                                                    \
        else if (kind == 1)                                                                                   \
            hipLaunchKernelGGL((k_stream_copy<K>), dim3((unsigned)nb), dim3(256), 0, s, (const float4*)a,      \
                               (float4*)b, n16);                                                              \
        else                                                                                                  \
            hipLaunchKernelGGL((k_stream_triad<K>), dim3((unsigned)nb), dim3(256), 0, s, (const float4*)a,     \
                               (float4*)b, (const float4*)c, 0.5f, n16);                                      \
        return hipGetLastError();                                                                             \
    } while (0)
    if (k == 1) SP_LAUNCH(1);
    if (k == 2) SP_LAUNCH(2);
    if (k == 4) SP_LAUNCH(4);
    if (k == 8) SP_LAUNCH(8);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace sp

extern "C" size_t sp_stream_out_bytes(size_t n16, int k) {
    if (k != 1 && k != 2 && k != 4 && k != 8) return 0;
    return sp::stream_blocks(n16, k) * sizeof(float);
}

extern "C" int sp_stream_probe(int kind, int k, const void* a, void* b, const void* c, size_t n16, void* stream) {
    if (kind < 0 || kind > 2) return sp::set_error(SP_ERR_INVALID_ARG, "kind must be 0 (read), 1 (copy) or 2 (triad)");
    if (k != 1 && k != 2 && k != 4 && k != 8) return sp::set_error(SP_ERR_INVALID_ARG, "words per lane must be 1, 2, 4 or 8");
    if (n16 == 0 || !a || !b || (kind == 2 && !c)) return sp::set_error(SP_ERR_INVALID_ARG, "null buffer or n16 = 0");
    if ((((uintptr_t)a) | ((uintptr_t)b) | ((uintptr_t)c)) & 15)
        return sp::set_error(SP_ERR_INVALID_ARG, "buffers must be 16-byte aligned");
    const hipError_t e = sp::launch_stream(kind, k, a, b, c, n16, (hipStream_t)stream);
    if (e != hipSuccess) return sp::set_error(SP_ERR_HIP, hipGetErrorString(e));
    return SP_OK;
}
