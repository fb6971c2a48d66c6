// Full-lattice solve (m + D) psi = src around the even-odd solver.
//
// With M = m + D split by parity, the even rows give (m^2 - D_eo D_oe) psi_e = m src_e - D_eo src_o and the
// odd rows give psi_o = (src_o - D_oe psi_e) / m. These kernels split the natural source by parity, form
// the even right-hand side and merge the reconstructed odd half with the even solution.
#include "sp_launch.h"

namespace sp {

// Natural full vector [V][3] complex128 -> packed FP64 even and odd halves.
__global__ __launch_bounds__(256) void k_full_split(Geom g, const double* __restrict__ src, void* se, void* so) {
    const int lex = blockIdx.x * blockDim.x + threadIdx.x;
    if (lex >= 2 * g.Vh) return;
    const int x = lex % g.X, r1 = lex / g.X, y = r1 % g.Y, r2 = r1 / g.Y, z = r2 % g.Z, t = r2 / g.Z;
    Vec3<double> v;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v.c[c].re = src[(size_t)lex * 6 + 2 * c];
        v.c[c].im = src[(size_t)lex * 6 + 2 * c + 1];
    }
    VecFmt<F64>::store(((x + y + z + t) & 1) ? so : se, g.Vh, lex >> 1, v);
}

// b_e = m src_e - t_e (t_e = D_eo src_o), written in the natural half layout [V/2][3].
__global__ __launch_bounds__(256) void k_full_source(int Vh, double m, const void* se, const void* te,
                                                     double* __restrict__ be) {
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    if (cb >= Vh) return;
    const Vec3<double> s = VecFmt<F64>::load(se, Vh, cb);
    const Vec3<double> t = VecFmt<F64>::load(te, Vh, cb);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        be[(size_t)cb * 6 + 2 * c] = m * s.c[c].re - t.c[c].re;
        be[(size_t)cb * 6 + 2 * c + 1] = m * s.c[c].im - t.c[c].im;
    }
}

// psi (natural full) from psi_e (natural half) and psi_o = (src_o - t_o) / m, t_o = D_oe psi_e.
__global__ __launch_bounds__(256) void k_full_merge(Geom g, double m, const double* __restrict__ psie, const void* so,
                                                    const void* to, double* __restrict__ psi) {
    const int lex = blockIdx.x * blockDim.x + threadIdx.x;
    if (lex >= 2 * g.Vh) return;
    const int x = lex % g.X, r1 = lex / g.X, y = r1 % g.Y, r2 = r1 / g.Y, z = r2 % g.Z, t = r2 / g.Z;
    const int cb = lex >> 1;
    if (((x + y + z + t) & 1) == 0) {
#pragma unroll
        for (int k = 0; k < 6; ++k) psi[(size_t)lex * 6 + k] = psie[(size_t)cb * 6 + k];
        return;
    }
    const Vec3<double> s = VecFmt<F64>::load(so, g.Vh, cb);
    const Vec3<double> d = VecFmt<F64>::load(to, g.Vh, cb);
    const double inv = 1.0 / m;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        psi[(size_t)lex * 6 + 2 * c] = (s.c[c].re - d.c[c].re) * inv;
        psi[(size_t)lex * 6 + 2 * c + 1] = (s.c[c].im - d.c[c].im) * inv;
    }
}

hipError_t launch_full_split(const Geom& g, const double* src, void* se, void* so, hipStream_t s) {
    hipLaunchKernelGGL(k_full_split, dim3(blocks_for(2 * g.Vh, 256)), dim3(256), 0, s, g, src, se, so);
    return hipGetLastError();
}

hipError_t launch_full_source(const Geom& g, double m, const void* se, const void* te, double* be, hipStream_t s) {
    hipLaunchKernelGGL(k_full_source, dim3(blocks_for(g.Vh, 256)), dim3(256), 0, s, g.Vh, m, se, te, be);
    return hipGetLastError();
}

hipError_t launch_full_merge(const Geom& g, double m, const double* psie, const void* so, const void* to,
                             double* psi, hipStream_t s) {
    hipLaunchKernelGGL(k_full_merge, dim3(blocks_for(2 * g.Vh, 256)), dim3(256), 0, s, g, m, psie, so, to, psi);
    return hipGetLastError();
}

}  // namespace sp
