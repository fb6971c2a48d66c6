// Instantiations and launches of the half operator and the FP64 residual kernel.
#include "sp_launch.h"

namespace sp {

template <class D>
struct NOf {
    static constexpr int value = NB;
};
template <>
struct NOf<DescSingle> {
    static constexpr int value = 1;
};

template <class D>
hipError_t launch_dslash(const D& d, int nblocks, LaunchCfg c, int lp, int recon, int vp, int p, int in_slot,
                         int out_slot, int mode, int gate, int use64, hipStream_t s) {
    constexpr int N = NOf<D>::value;
// The streaming link loads are built for the single-system operator (N == 1) only; batched groups share each
// link load among their right-hand sides and take the cached loads.
#define SP_LAUNCH_NT(LP, RC, VP, NT)                                                                       \
    do {                                                                                                   \
        if (mode == DS_PLAIN)                                                                              \
            hipLaunchKernelGGL((k_dslash<LP, RC, VP, N, D, DS_PLAIN, NT>), dim3(nblocks), dim3(c.nt), 0, s, d, \
                               p, in_slot, out_slot, gate, use64, c.remap);                               \
        else if (mode == DS_NORM)                                                                          \
            hipLaunchKernelGGL((k_dslash<LP, RC, VP, N, D, DS_NORM, NT>), dim3(nblocks), dim3(c.nt), 0, s, d, \
                               p, in_slot, out_slot, gate, use64, c.remap);                               \
        else if (mode == DS_UPDATE)                                                                        \
            hipLaunchKernelGGL((k_dslash<LP, RC, VP, N, D, DS_UPDATE, NT>), dim3(nblocks), dim3(c.nt), 0, s, \
                               d, p, in_slot, out_slot, gate, use64, c.remap);                            \
        else if constexpr (N == 1)                                                                         \
            hipLaunchKernelGGL((k_dslash<LP, RC, VP, N, D, DS_UPDATE_FUSED, NT>), dim3(nblocks), dim3(c.nt), 0, \
                               s, d, p, in_slot, out_slot, gate, use64, c.remap);                         \
        else                                                                                               \
            return hipErrorInvalidValue;                                                                   \
        return hipGetLastError();                                                                          \
    } while (0)
#define SP_LAUNCH(LP, RC, VP)                                                                              \
    do {                                                                                                   \
        if constexpr (N == 1) {                                                                            \
            if (c.stream) SP_LAUNCH_NT(LP, RC, VP, true);                                                  \
        }                                                                                                  \
        SP_LAUNCH_NT(LP, RC, VP, false);                                                                   \
    } while (0)
    if (lp == F64 && recon == 18 && vp == F64) SP_LAUNCH(F64, 18, F64);
    if (lp == F32 && recon == 18 && vp == F32) SP_LAUNCH(F32, 18, F32);
    if (lp == F32 && recon == 12 && vp == F32) SP_LAUNCH(F32, 12, F32);
    if (lp == F32 && recon == 8 && vp == F32) SP_LAUNCH(F32, 8, F32);
    if (lp == F16 && recon == 18 && vp == F16) SP_LAUNCH(F16, 18, F16);
    if (lp == F16 && recon == 12 && vp == F16) SP_LAUNCH(F16, 12, F16);
    if (lp == BF16 && recon == 18 && vp == BF16) SP_LAUNCH(BF16, 18, BF16);
    if (lp == BF16 && recon == 12 && vp == BF16) SP_LAUNCH(BF16, 12, BF16);
    // 16-bit links with FP32 vectors
    if (lp == F16 && recon == 12 && vp == F32) SP_LAUNCH(F16, 12, F32);
    if (lp == F16 && recon == 18 && vp == F32) SP_LAUNCH(F16, 18, F32);
    if (lp == BF16 && recon == 12 && vp == F32) SP_LAUNCH(BF16, 12, F32);
    if (lp == BF16 && recon == 18 && vp == F32) SP_LAUNCH(BF16, 18, F32);
    if (lp == I16 && recon == 12 && vp == F32) SP_LAUNCH(I16, 12, F32);
    if (lp == I16 && recon == 18 && vp == F32) SP_LAUNCH(I16, 18, F32);
#undef SP_LAUNCH
#undef SP_LAUNCH_NT
    return hipErrorInvalidValue;
}

hipError_t launch_norm_rec(const DescSingle& d, SolverState* st_out, int nblocks, LaunchCfg c, int lp, int recon, int vp,
                           hipStream_t s) {
#define SP_LAUNCH(LP, RC, VP)                                                                              \
    do {                                                                                                   \
        if (c.stream)                                                                                      \
            hipLaunchKernelGGL((k_norm_rec<LP, RC, VP, true>), dim3(nblocks), dim3(c.nt), 0, s, d, st_out,  \
                               c.remap);                                                                   \
        else                                                                                               \
            hipLaunchKernelGGL((k_norm_rec<LP, RC, VP, false>), dim3(nblocks), dim3(c.nt), 0, s, d, st_out, \
                               c.remap);                                                                   \
        return hipGetLastError();                                                                          \
    } while (0)
    if (lp == F64 && recon == 18 && vp == F64) SP_LAUNCH(F64, 18, F64);
    if (lp == F32 && recon == 18 && vp == F32) SP_LAUNCH(F32, 18, F32);
    if (lp == F32 && recon == 12 && vp == F32) SP_LAUNCH(F32, 12, F32);
    if (lp == F32 && recon == 8 && vp == F32) SP_LAUNCH(F32, 8, F32);
    if (lp == F16 && recon == 12 && vp == F32) SP_LAUNCH(F16, 12, F32);
    if (lp == F16 && recon == 18 && vp == F32) SP_LAUNCH(F16, 18, F32);
    if (lp == BF16 && recon == 12 && vp == F32) SP_LAUNCH(BF16, 12, F32);
    if (lp == BF16 && recon == 18 && vp == F32) SP_LAUNCH(BF16, 18, F32);
    if (lp == I16 && recon == 12 && vp == F32) SP_LAUNCH(I16, 12, F32);
    if (lp == I16 && recon == 18 && vp == F32) SP_LAUNCH(I16, 18, F32);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

template <class D>
hipError_t launch_resid(const D& d, int nblocks, LaunchCfg c, int op, int init, hipStream_t s) {
    constexpr int N = NOf<D>::value;
#define SP_LAUNCH(OP)                                                                                      \
    do {                                                                                                   \
        hipLaunchKernelGGL((k_resid<OP, N, D>), dim3(nblocks), dim3(c.nt), 0, s, d, init, c.remap);         \
        return hipGetLastError();                                                                          \
    } while (0)
    if (op == F64) SP_LAUNCH(F64);
    if (op == F32) SP_LAUNCH(F32);
    if (op == F16) SP_LAUNCH(F16);
    if (op == BF16) SP_LAUNCH(BF16);
#undef SP_LAUNCH
    return hipErrorInvalidValue;
}

template hipError_t launch_dslash<DescSingle>(const DescSingle&, int, LaunchCfg, int, int, int, int, int, int, int,
                                              int, int, hipStream_t);
template hipError_t launch_dslash<DescBatch>(const DescBatch&, int, LaunchCfg, int, int, int, int, int, int, int,
                                             int, int, hipStream_t);
template hipError_t launch_resid<DescSingle>(const DescSingle&, int, LaunchCfg, int, int, hipStream_t);
template hipError_t launch_resid<DescBatch>(const DescBatch&, int, LaunchCfg, int, int, hipStream_t);

}  // namespace sp
