// Adjoint link gradient (fermion force) and mass gradient, FP64.
//
// For a real loss l(x), x = A^-1 b, A = m^2 - D_eo D_oe, with lambda = A^-1 dl/dx, y_x = D_oe x and
// y_l = D_oe lambda, varying one link U_mu(n) changes D_eo (output at n or n+mu) and D_oe; collecting the
// two terms gives
//   n even:  Gamma_mu(n) =  1/2 eta_mu(n) s [ lambda(n) y_x(n+mu)^dag + x(n) y_l(n+mu)^dag ]
//   n odd:   Gamma_mu(n) = -1/2 eta_mu(n) s [ y_x(n) lambda(n+mu)^dag + y_l(n) x(n+mu)^dag ]
// (s: antiperiodic-time sign of the link), and F = TA(U Gamma^dag) is its projection on su(3).
#include "sp_launch.h"

namespace sp {

__device__ __forceinline__ void outer_acc(Cx<double> (&G)[3][3], double c, const Vec3<double>& a,
                                          const Vec3<double>& b) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            // a_i conj(b_j)
            G[i][j].re += c * (a.c[i].re * b.c[j].re + a.c[i].im * b.c[j].im);
            G[i][j].im += c * (a.c[i].im * b.c[j].re - a.c[i].re * b.c[j].im);
        }
}

__global__ __launch_bounds__(256) void k_force(Geom g, const void* links64, const void* x, const void* lam,
                                               const void* yx, const void* yl, double* gamma, double* force) {
    using VF = VecFmt<F64>;
    using LF = LinkFmt<F64, 18>;
    const long V = 2L * g.Vh;
    const long l = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= 4 * V) return;
    const int mu = (int)(l / V);
    const int lex = (int)(l - (long)mu * V);
    const int x0 = lex % g.X, r1 = lex / g.X, y0 = r1 % g.Y, r2 = r1 / g.Y, z0 = r2 % g.Z, t0 = r2 / g.Z;
    const int p = (x0 + y0 + z0 + t0) & 1;
    const int cb = lex >> 1;
    const Site s = site_of(g, p, cb);
    const int nf = nbr(g, s, mu, +1);
    double c = 0.5 * (double)eta_sign(s, mu);
    if (mu == 3 && g.bc_t && s.t == g.T - 1) c = -c;
    Cx<double> G[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) G[i][j].re = G[i][j].im = 0.0;
    if (p == 0) {
        outer_acc(G, c, VF::load(lam, g.Vh, cb), VF::load(yx, g.Vh, nf));
        outer_acc(G, c, VF::load(x, g.Vh, cb), VF::load(yl, g.Vh, nf));
    } else {
        outer_acc(G, -c, VF::load(yx, g.Vh, cb), VF::load(lam, g.Vh, nf));
        outer_acc(G, -c, VF::load(yl, g.Vh, cb), VF::load(x, g.Vh, nf));
    }
    double* go = gamma + l * 18;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        go[2 * k] = G[k / 3][k % 3].re;
        go[2 * k + 1] = G[k / 3][k % 3].im;
    }
    if (force) {
        const Su3<double> U = LF::load(link_block<LF>(links64, g.Vh, p, mu), g.Vh, cb);
        // W = U Gamma^dag, W_ij = sum_k U_ik conj(G_jk)
        Cx<double> W[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double re = 0.0, im = 0.0;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    re += U.e[i][k].re * G[j][k].re + U.e[i][k].im * G[j][k].im;
                    im += U.e[i][k].im * G[j][k].re - U.e[i][k].re * G[j][k].im;
                }
                W[i][j].re = re;
                W[i][j].im = im;
            }
        // TA(W) = (W - W^dag)/2 - tr(W - W^dag)/6; tr(W - W^dag) = 2 i Im tr W
        const double imtr = W[0][0].im + W[1][1].im + W[2][2].im;
        double* fo = force + l * 18;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                double re = 0.5 * (W[i][j].re - W[j][i].re);
                double im = 0.5 * (W[i][j].im + W[j][i].im);
                if (i == j) im -= imtr / 3.0;
                fo[2 * (3 * i + j)] = re;
                fo[2 * (3 * i + j) + 1] = im;
            }
    }
}

__global__ __launch_bounds__(256) void k_mass_grad_partials(int Vh, const void* x, const void* lam,
                                                            double* partials) {
    using VF = VecFmt<F64>;
    const int cb = blockIdx.x * blockDim.x + threadIdx.x;
    double v[1] = {0.0};
    if (cb < Vh) {
        const Vec3<double> a = VF::load(lam, Vh, cb);
        const Vec3<double> b = VF::load(x, Vh, cb);
#pragma unroll
        for (int i = 0; i < 3; ++i) v[0] += a.c[i].re * b.c[i].re + a.c[i].im * b.c[i].im;
    }
    block_sum<1>(v);
    if (threadIdx.x == 0) partials[blockIdx.x] = v[0];
}

// out = -2 m sum(partials), summed in block order by one block.
__global__ __launch_bounds__(256) void k_mass_grad_final(int nblk, double mass, const double* partials,
                                                         double* out) {
    double s[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) s[0] += partials[b];
    block_sum<1>(s);
    if (threadIdx.x == 0) *out = -2.0 * mass * s[0];
}

int mass_grad_blocks(const Geom& g) { return blocks_for(g.Vh, 256); }

hipError_t launch_force(const Geom& g, const void* links64, const void* x, const void* lam, const void* yx,
                        const void* yl, double* gamma, double* force, hipStream_t s) {
    const long n = 8L * g.Vh;
    hipLaunchKernelGGL(k_force, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g, links64, x, lam, yx, yl,
                       gamma, force);
    return hipGetLastError();
}

hipError_t launch_mass_grad(const Geom& g, double mass, const void* x, const void* lam, double* partials,
                            double* out, hipStream_t s) {
    const int nb = mass_grad_blocks(g);
    hipLaunchKernelGGL(k_mass_grad_partials, dim3(nb), dim3(256), 0, s, g.Vh, x, lam, partials);
    hipError_t e = hipGetLastError();
    if (e) return e;
    hipLaunchKernelGGL(k_mass_grad_final, dim3(1), dim3(256), 0, s, nb, mass, partials, out);
    return hipGetLastError();
}

}  // namespace sp
