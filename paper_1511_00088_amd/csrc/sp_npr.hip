// One-colour-trace four-fermion contraction of the NPR code (Eq. (1) of the paper, Sec. 4), FP64.
//
// Per hypercube z (corners z_A = 2z + A, A in {0,1}^4) and field set i:
//   O_i(z) = sum_{A,B,C,D} M1_{AB} M2_{CD} [chib1(z_A)^T U_AD(z) chi4(z_D)] [chib3(z_C)^T U_CB(z) chi2(z_B)]
// with M_{AB} = (1/4) tr(gamma_A^dag gamma_S gamma_B gamma_F^dag) and U_AD(z) the average over the shortest
// paths from z_A to z_D of the ordered link products.
//
// Two launches, or one fused:
//  * k_npr_paths: one block per hypercube, one thread per corner pair; the path average is built by the
//    first-step recursion in LDS (U_mu(x) for a step +mu, U_mu(x - mu)^dag for a step -mu). Output
//    [nz][256][9] double2: a hypercube's 256 matrices are one contiguous 36 KB block, written and read
//    whole.
//  * k_npr_contract: one block per hypercube, one thread per (A, C). M_{AB} is nonzero only for
//    B = A xor S xor F, where it is a sign, so each thread owns one term: it keeps U_{A,D} and U_{C,B}
//    (D = C xor S2 xor F2) in registers for every field set; the hypercube's 192 field values of up to
//    NPR_CHUNK field sets are staged in LDS together, and one block reduction gives their O_i(z).
//  * k_npr_fused: both in one block per hypercube; the path links stay in LDS (for a few field sets per call this
//    saves the 36 KB per hypercube written by k_npr_paths and read back by k_npr_contract).
// The signs come from the anticommutation relations: gamma_X gamma_Y = (-1)^s(X,Y) gamma_{X xor Y} with
// s(X,Y) = #{mu > nu : X_mu = Y_nu = 1}, gamma_X^dag = (-1)^{n(n-1)/2} gamma_X for n = |X|, tr gamma_0 = 4.
#include "sp_launch.h"

namespace sp {
namespace {

using C = Cx<double>;

__device__ __forceinline__ C cmul(C a, C b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }

struct NprGeom {
    int L[4];   // fine extents X, Y, Z, T
    int Lc[4];  // coarse extents L / 2
    int nz;     // number of hypercubes
    int V;
};

__device__ __forceinline__ int lex4(const NprGeom& g, const int* c) {
    return c[0] + g.L[0] * (c[1] + g.L[1] * (c[2] + g.L[2] * c[3]));
}

__device__ __forceinline__ void coarse_coords(const NprGeom& g, int z, int* c) {
    c[0] = z % g.Lc[0];
    z /= g.Lc[0];
    c[1] = z % g.Lc[1];
    z /= g.Lc[1];
    c[2] = z % g.Lc[2];
    c[3] = z / g.Lc[2];
}

// corner X with bit mu cleared -> index 0..7 of the remaining three bits
__device__ __forceinline__ int squeeze(int X, int mu) { return (X & ((1 << mu) - 1)) | ((X >> (mu + 1)) << mu); }

__device__ __forceinline__ void mat_ld(const double2* p, C (&m)[3][3], bool dag) {
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const double2 v = p[j];
        if (dag) m[j % 3][j / 3] = {v.x, -v.y};
        else m[j / 3][j % 3] = {v.x, v.y};
    }
}

// The path links of hypercube z into P (LDS, pair A * 16 + D), by the 256 threads of a block, one per corner pair
// (A, D). The average over the k! shortest paths is built from the first step: U_AD = (1/k) sum over the k
// directions mu in which A and D differ of L(A -> A^mu) U_{A^mu, D}, where L is U_mu(z_A) when A_mu = 0 and
// U_mu(z_A - mu)^dag otherwise. Pairs are filled in order of k, so every U_{A^mu, D} a thread needs is complete one
// barrier earlier. lk (LDS) receives the hypercube's 32 links: [mu][corner with bit mu = 0, squeezed]. Ends with a
// barrier.
__device__ __forceinline__ void build_paths(const NprGeom& g, const double2* __restrict__ U, int z, double2 (*lk)[9],
                                            double2 (*P)[9]) {
    const int t = threadIdx.x, A = t >> 4, D = t & 15;
    int zc[4];
    coarse_coords(g, z, zc);
    for (int e = t; e < 32 * 9; e += 256) {
        const int l = e / 9, j = e % 9, mu = l >> 3, c8 = l & 7;
        const int X = (c8 & ((1 << mu) - 1)) | ((c8 >> mu) << (mu + 1));  // bit mu = 0
        int c[4];
        for (int nu = 0; nu < 4; ++nu) c[nu] = 2 * zc[nu] + ((X >> nu) & 1);
        lk[l][j] = U[((long)mu * g.V + lex4(g, c)) * 9 + j];
    }
    const int diff = A ^ D, k = __builtin_popcount(diff);
    __syncthreads();
    for (int level = 0; level <= 4; ++level) {
        if (k == level) {
            C acc[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) acc[i][j] = {level == 0 && i == j ? 1.0 : 0.0, 0.0};
            for (int mu = 0; mu < 4; ++mu) {
                if (!((diff >> mu) & 1)) continue;
                const int A1 = A ^ (1 << mu);
                const bool up = ((A >> mu) & 1) == 0;  // step +mu from z_A, else -mu
                C L[3][3], R[3][3];
                mat_ld(lk[mu * 8 + squeeze(up ? A : A1, mu)], L, !up);
                if (level == 1) {
#pragma unroll
                    for (int i = 0; i < 3; ++i)
#pragma unroll
                        for (int j = 0; j < 3; ++j) acc[i][j] = L[i][j];
                    break;
                }
                mat_ld(P[A1 * 16 + D], R, false);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        const C a = cmul(L[i][0], R[0][j]), b = cmul(L[i][1], R[1][j]), c = cmul(L[i][2], R[2][j]);
                        acc[i][j].re += a.re + b.re + c.re;
                        acc[i][j].im += a.im + b.im + c.im;
                    }
            }
            const double w = level > 1 ? 1.0 / level : 1.0;
#pragma unroll
            for (int j = 0; j < 9; ++j) P[t][j] = make_double2(w * acc[j / 3][j % 3].re, w * acc[j / 3][j % 3].im);
        }
        __syncthreads();
    }
}

// One block per hypercube: the path links, written as one contiguous 36 KB block per hypercube.
__global__ __launch_bounds__(256) void k_npr_paths(NprGeom g, const double2* __restrict__ U, double2* __restrict__ out) {
    __shared__ double2 lk[32][9];
    __shared__ double2 P[256][9];
    build_paths(g, U, blockIdx.x, lk, P);
    double2* o = out + (long)blockIdx.x * 256 * 9;
    const double2* src = &P[0][0];
    for (int e = threadIdx.x; e < 256 * 9; e += 256) o[e] = src[e];
}

struct NprArgs {
    NprGeom g;
    const double2* uad;                   // [nz][256][9]
    const double2* f[4];                  // chib1, chi2, chib3, chi4: [n][V][3]
    double2* out;                         // [n][nz]
    int n;
    int d1, d2;                           // S1 xor F1, S2 xor F2
    unsigned neg1, neg2;                  // bit A set: M_{A, A xor d} = -1
};

// Field sets per pass of k_npr_contract: their field values are staged together, so a pass pays one load
// latency, and one block reduction covers all of them.
constexpr int NPR_CHUNK = 4;

// The contraction of hypercube z for every field set, by thread (A, C) of a block holding U_{A,D} and U_{C,B} in
// registers; fs (LDS) stages the hypercube's field values of NPR_CHUNK field sets at a time.
__device__ __forceinline__ void contract_sets(const NprArgs& a, int z, const C (&uad)[3][3], const C (&ucb)[3][3],
                                              double2 (*fs)[4][16][3]) {
    const int A = threadIdx.x >> 4, Cc = threadIdx.x & 15;
    const int B = A ^ a.d1, D = Cc ^ a.d2;
    int zc[4];
    coarse_coords(a.g, z, zc);
    const int c0[4] = {2 * zc[0], 2 * zc[1], 2 * zc[2], 2 * zc[3]};
    const int base = lex4(a.g, c0);  // z_0
    const double sgn = (((a.neg1 >> A) ^ (a.neg2 >> Cc)) & 1) ? -1.0 : 1.0;
    for (int i0 = 0; i0 < a.n; i0 += NPR_CHUNK) {
        const int m = min(NPR_CHUNK, a.n - i0);
        for (int e = threadIdx.x; e < m * 192; e += 256) {
            const int s = e / 192, r0 = e % 192, fi = r0 / 48, r = r0 % 48, corner = r / 3, c = r % 3;
            // corner offset of z_corner from z_0 (no wrap: 2 z_mu + 1 < L_mu)
            const int off = (corner & 1) + a.g.L[0] * (((corner >> 1) & 1) + a.g.L[1] * (((corner >> 2) & 1) +
                                                                                    a.g.L[2] * (corner >> 3)));
            fs[s][fi][corner][c] = a.f[fi][((long)(i0 + s) * a.g.V + base + off) * 3 + c];
        }
        __syncthreads();
        double v[2 * NPR_CHUNK];
#pragma unroll
        for (int s = 0; s < NPR_CHUNK; ++s) {
            v[2 * s] = v[2 * s + 1] = 0.0;
            if (s >= m) continue;
            // chib1(A)^T U_AD chi4(D) and chib3(C)^T U_CB chi2(B)
            C b1 = {0.0, 0.0}, b2 = {0.0, 0.0};
#pragma unroll
            for (int r = 0; r < 3; ++r) {
                C s1 = {0.0, 0.0}, s2 = {0.0, 0.0};
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    const double2 x4 = fs[s][3][D][c], x2 = fs[s][1][B][c];
                    const C p = cmul(uad[r][c], {x4.x, x4.y}), q = cmul(ucb[r][c], {x2.x, x2.y});
                    s1 = {s1.re + p.re, s1.im + p.im};
                    s2 = {s2.re + q.re, s2.im + q.im};
                }
                const double2 y1 = fs[s][0][A][r], y3 = fs[s][2][Cc][r];
                const C p = cmul({y1.x, y1.y}, s1), q = cmul({y3.x, y3.y}, s2);
                b1 = {b1.re + p.re, b1.im + p.im};
                b2 = {b2.re + q.re, b2.im + q.im};
            }
            const C term = cmul(b1, b2);
            v[2 * s] = sgn * term.re;
            v[2 * s + 1] = sgn * term.im;
        }
        block_sum<2 * NPR_CHUNK>(v);  // ends with a barrier, so the staged values can be replaced next
        if (threadIdx.x == 0)
            for (int s = 0; s < m; ++s) a.out[(long)(i0 + s) * a.g.nz + z] = make_double2(v[2 * s], v[2 * s + 1]);
    }
}

// From stored path links: thread (A, C) loads U_{A,D} and U_{C,B} from the hypercube's block.
__global__ __launch_bounds__(256) void k_npr_contract(NprArgs a) {
    const int z = blockIdx.x;
    const int A = threadIdx.x >> 4, Cc = threadIdx.x & 15;
    const int B = A ^ a.d1, D = Cc ^ a.d2;
    __shared__ double2 fs[NPR_CHUNK][4][16][3];  // the hypercube's field values of a pass
    C uad[3][3], ucb[3][3];
    const double2* blk = a.uad + (long)z * 256 * 9;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const double2 v = blk[(A * 16 + D) * 9 + j];
        const double2 w = blk[(Cc * 16 + B) * 9 + j];
        uad[j / 3][j % 3] = {v.x, v.y};
        ucb[j / 3][j % 3] = {w.x, w.y};
    }
    contract_sets(a, z, uad, ucb, fs);
}

// Fused: the hypercube's path links are built in LDS (as k_npr_paths does) and contracted at once, so the 36 KB
// of path links per hypercube never travel to memory and back. Once every thread holds its two matrices the path
// area is reused for the field staging (a barrier separates the two uses).
__global__ __launch_bounds__(256) void k_npr_fused(NprArgs a, const double2* __restrict__ U) {
    const int z = blockIdx.x;
    const int A = threadIdx.x >> 4, Cc = threadIdx.x & 15;
    const int B = A ^ a.d1, D = Cc ^ a.d2;
    __shared__ double2 lk[32][9];
    __shared__ double2 P[256][9];
    static_assert(sizeof(double2) * NPR_CHUNK * 4 * 16 * 3 <= sizeof(double2) * 256 * 9, "staging fits the path area");
    build_paths(a.g, U, z, lk, P);
    C uad[3][3], ucb[3][3];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const double2 v = P[A * 16 + D][j];
        const double2 w = P[Cc * 16 + B][j];
        uad[j / 3][j % 3] = {v.x, v.y};
        ucb[j / 3][j % 3] = {w.x, w.y};
    }
    __syncthreads();  // every thread has read its matrices: the path area becomes the field staging
    contract_sets(a, z, uad, ucb, (double2(*)[4][16][3])&P[0][0]);
}

// Sign of M_{A, A xor S xor F} = (1/4) tr(gamma_A^dag gamma_S gamma_B gamma_F^dag), B = A xor S xor F.
int st_swaps(int x, int y) {
    int s = 0;
    for (int m = 0; m < 4; ++m)
        for (int n = 0; n < m; ++n) s += ((x >> m) & 1) & ((y >> n) & 1);
    return s;
}
int rev_parity(int x) {
    const int n = __builtin_popcount(x);
    return (n * (n - 1) / 2) & 1;
}
unsigned negative_corners(int S, int F) {
    unsigned neg = 0;
    for (int A = 0; A < 16; ++A) {
        const int B = A ^ S ^ F;
        const int e = rev_parity(A) + rev_parity(F) + st_swaps(A, S) + st_swaps(A ^ S, B) + st_swaps(A ^ S ^ B, F);
        if (e & 1) neg |= 1u << A;
    }
    return neg;
}

NprGeom npr_geom(const Geom& g) {
    NprGeom n;
    n.L[0] = g.X;
    n.L[1] = g.Y;
    n.L[2] = g.Z;
    n.L[3] = g.T;
    for (int mu = 0; mu < 4; ++mu) n.Lc[mu] = n.L[mu] / 2;
    n.nz = n.Lc[0] * n.Lc[1] * n.Lc[2] * n.Lc[3];
    n.V = 2 * g.Vh;
    return n;
}

}  // namespace

size_t npr_path_bytes(const Geom& g) { return (size_t)npr_geom(g).nz * 256 * 9 * sizeof(double2); }

hipError_t launch_npr_paths(const Geom& g, const double* links, void* uad, hipStream_t s) {
    const NprGeom n = npr_geom(g);
    hipLaunchKernelGGL(k_npr_paths, dim3(n.nz), dim3(256), 0, s, n, (const double2*)links, (double2*)uad);
    return hipGetLastError();
}

hipError_t launch_npr_contract(const Geom& g, const void* uad, int n, const double* const f[4], const int labels[4],
                               double* out, hipStream_t s) {
    return launch_npr_contract_from(g, uad, nullptr, n, f, labels, out, s);
}

hipError_t launch_npr_contract_from(const Geom& g, const void* uad, const double* links, int n, const double* const f[4],
                                    const int labels[4], double* out, hipStream_t s) {
    NprArgs a;
    a.g = npr_geom(g);
    a.uad = (const double2*)uad;
    for (int k = 0; k < 4; ++k) a.f[k] = (const double2*)f[k];
    a.out = (double2*)out;
    a.n = n;
    a.d1 = labels[0] ^ labels[1];
    a.d2 = labels[2] ^ labels[3];
    a.neg1 = negative_corners(labels[0], labels[1]);
    a.neg2 = negative_corners(labels[2], labels[3]);
    if (links) hipLaunchKernelGGL(k_npr_fused, dim3(a.g.nz), dim3(256), 0, s, a, (const double2*)links);
    else hipLaunchKernelGGL(k_npr_contract, dim3(a.g.nz), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sp
