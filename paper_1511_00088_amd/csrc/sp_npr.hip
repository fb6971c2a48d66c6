// One-colour-trace four-fermion contraction of the NPR code (Eq. (1) of the paper, Sec. 4), FP64.
//
// Per hypercube z (corners z_A = 2z + A, A in {0,1}^4) and field set i:
//   O_i(z) = sum_{A,B,C,D} M1_{AB} M2_{CD} [chib1(z_A)^T U_AD(z) chi4(z_D)] [chib3(z_C)^T U_CB(z) chi2(z_B)]
// with M_{AB} = (1/4) tr(gamma_A^dag gamma_S gamma_B gamma_F^dag) and U_AD(z) the average over the shortest
// paths from z_A to z_D of the ordered link products.
//
// Two launches, or one fused:
//  * k_npr_paths: one block per hypercube; the path average is built by the first-step recursion in LDS
//    (U_mu(x) for a step +mu, U_mu(x - mu)^dag for a step -mu), one thread per row of a corner pair's matrix,
//    the 256 matrices held there as nine planes, one per matrix element, with the pairs swizzled across LDS
//    banks. Output
//    [nz][256][9] double2: a hypercube's 256 matrices are one contiguous 36 KB block, written and read
//    whole.
//  * k_npr_contract: one block per hypercube, one thread per (A, C). M_{AB} is nonzero only for
//    B = A xor S xor F, where it is a sign, so each thread owns one term: it keeps U_{A,D} and U_{C,B}
//    (D = C xor S2 xor F2) in registers for every field set; the hypercube's 192 field values of up to
//    NPR_CHUNK field sets are staged in LDS together, and one block reduction gives their O_i(z).
//  * k_npr_fused: both in one block per hypercube; the path links stay in LDS (for a few field sets per call this
//    saves the 36 KB per hypercube written by k_npr_paths and read back by k_npr_contract).
// Every kernel takes its hypercubes in XCD-aware order (block b on XCD b % 8 gets one of a contiguous range), so
// that neighbouring hypercubes, which share cache lines of the fields and links, meet in one L2.
// The signs come from the anticommutation relations: gamma_X gamma_Y = (-1)^s(X,Y) gamma_{X xor Y} with
// s(X,Y) = #{mu > nu : X_mu = Y_nu = 1}, gamma_X^dag = (-1)^{n(n-1)/2} gamma_X for n = |X|, tr gamma_0 = 4.
#include "sp_launch.h"
#include "sp_npr_layout.h"

namespace sp {
namespace {

using C = Cx<double>;

// Every floating-point operation of this file is written out: the compiler fuses nothing by itself
// (contraction off below), and the products are fused multiply-adds in a fixed order (cmac). The two-launch
// and the fused contraction inline the same arithmetic, so their results agree bit for bit whatever the
// surrounding code; left to itself the compiler fuses differently in each kernel.
#pragma clang fp contract(off)

// acc + a b as four fused multiply-adds
__device__ __forceinline__ C cmac(C acc, C a, C b) {
    return {fma(a.re, b.re, fma(-a.im, b.im, acc.re)), fma(a.re, b.im, fma(a.im, b.re, acc.im))};
}

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

// The path area: element j (row j / 3, column j % 3) of the 256 path matrices as nine planes, pair (X, Y) at
// ppos(X, Y) in each (sp_npr_layout.h).
using Paths = double2[9][NPR_PLANE];

__device__ __forceinline__ void path_ld(const Paths& P, int X, int Y, C (&m)[3][3]) {
    const int q = ppos(X, Y);
#pragma unroll
    for (int j = 0; j < 9; ++j) m[j / 3][j % 3] = {P[j][q].x, P[j][q].y};
}

// The pairs at corner distance LEVEL (2, 3 or 4), each U_AD the average over the LEVEL directions mu in which A
// and D differ of L(A -> A^mu) U_{A^mu, D} (see build_paths). The work is cut into items of NC columns of one row
// of one pair (NC = 3: a row; NC = 1: one element), numbered with A fastest, so the 16 lanes of a quarter
// wavefront share the corner difference, the row and the columns and differ in A: their reads of U_{A, A^mu}
// and U_{A^mu, D} and their writes of U_{A, D} fall in distinct LDS banks (sp_npr_layout.h). Every lane takes
// the set bits of its difference in increasing order, so all lanes run the same LEVEL steps and the products
// are summed in the same order whatever the cut.
template <int LEVEL, int NC>
__device__ __forceinline__ void path_level(Paths& P) {
    // the corner differences with LEVEL bits set, in increasing order, four bits each
    constexpr int nd = LEVEL == 2 ? 6 : LEVEL == 3 ? 4 : 1;
    constexpr unsigned tab = LEVEL == 2 ? 0xCA9653u : LEVEL == 3 ? 0xEDB7u : 0xFu;
    constexpr int per = 9 / NC;  // items per pair
    const double w = 1.0 / LEVEL;
    for (int it = threadIdx.x; it < 16 * nd * per; it += 256) {
        const int A = it & 15, sub = (it >> 4) % per, diff = (tab >> (4 * ((it >> 4) / per))) & 15, D = A ^ diff;
        const int i = sub * NC / 3, j0 = (sub * NC) % 3;
        C acc[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) acc[c] = {0.0, 0.0};
        int left = diff;
#pragma unroll
        for (int k = 0; k < LEVEL; ++k) {
            const int mu = __builtin_ctz(left);
            left &= left - 1;
            const int A1 = A ^ (1 << mu), ql = ppos(A, A1), qr = ppos(A1, D);
            C L[3];
#pragma unroll
            for (int k2 = 0; k2 < 3; ++k2) L[k2] = {P[i * 3 + k2][ql].x, P[i * 3 + k2][ql].y};
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                const int j = j0 + c;
                const C R0 = {P[j][qr].x, P[j][qr].y}, R1 = {P[3 + j][qr].x, P[3 + j][qr].y},
                        R2 = {P[6 + j][qr].x, P[6 + j][qr].y};
                acc[c] = cmac(cmac(cmac(acc[c], L[0], R0), L[1], R1), L[2], R2);
            }
        }
        const int q = ppos(A, D);
#pragma unroll
        for (int c = 0; c < NC; ++c) P[i * 3 + j0 + c][q] = make_double2(w * acc[c].re, w * acc[c].im);
    }
    __syncthreads();
}

// The path links of hypercube z into P (LDS), by the 256 threads of a block. The average over the k! shortest
// paths is built from the first step: U_AD = (1/k) sum over the k directions mu in which A and D differ of
// L(A -> A^mu) U_{A^mu, D}, where L(A -> A^mu) = U_{A, A^mu} is U_mu(z_A) when A_mu = 0 and U_mu(z_A - mu)^dag
// otherwise. Distance 0 is the identity and distance 1 the hypercube's 32 links and their conjugate transposes,
// stored straight from memory; pairs at distance 2, 3, 4 follow in that order, so every U_{A^mu, D} and
// U_{A, A^mu} a thread needs is complete one barrier earlier. Distances 2 and 4 are cut into single elements
// (864 and 144 items over the 256 threads), distance 3 into rows (192 items), which keeps each level's longest
// chain of products short. Ends with a barrier.
__device__ __forceinline__ void build_paths(const NprGeom& g, const double2* __restrict__ U, int z, Paths& P) {
    const int t = threadIdx.x;
    int zc[4];
    coarse_coords(g, z, zc);
    for (int e = t; e < 32 * 9; e += 256) {
        const int l = e / 9, j = e % 9, mu = l >> 3, c8 = l & 7;
        const int X = (c8 & ((1 << mu) - 1)) | ((c8 >> mu) << (mu + 1));  // bit mu = 0
        int c[4];
        for (int nu = 0; nu < 4; ++nu) c[nu] = 2 * zc[nu] + ((X >> nu) & 1);
        const double2 v = U[((long)mu * g.V + lex4(g, c)) * 9 + j];
        const int Y = X | (1 << mu);
        P[j][ppos(X, Y)] = v;                                          // step +mu from z_X
        P[(j % 3) * 3 + j / 3][ppos(Y, X)] = make_double2(v.x, -v.y);  // step -mu from z_Y: the dagger
    }
    if (t < 16)
#pragma unroll
        for (int j = 0; j < 9; ++j) P[j][ppos(t, t)] = make_double2(j % 4 == 0 ? 1.0 : 0.0, 0.0);
    __syncthreads();
    path_level<2, 1>(P);
    path_level<3, 3>(P);
    path_level<4, 1>(P);
}

// One block per hypercube: the path links, written as one contiguous 36 KB block per hypercube (pair A * 16 + D,
// then the nine elements).
__global__ __launch_bounds__(256) void k_npr_paths(NprGeom g, const double2* __restrict__ U, double2* __restrict__ out) {
    __shared__ Paths P;
    const int z = remap_block(blockIdx.x, gridDim.x);
    build_paths(g, U, z, P);
    double2* o = out + (long)z * 256 * 9;
    for (int e = threadIdx.x; e < 256 * 9; e += 256) {
        const int pair = e / 9, j = e % 9;
        o[e] = P[j][ppos(pair >> 4, pair & 15)];
    }
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

// Field sets per pass of the contraction: their field values are staged together, so a pass pays one load
// latency, and one block reduction covers all of them.
constexpr int NPR_CHUNK = 4;
// The 192 field values per set and hypercube (4 fields x 16 corners x 3 colours) of a pass, over 256 threads.
static_assert(NPR_CHUNK * 192 == 3 * 256, "a pass's field values are three per thread");

// Offset of corner X of a hypercube from its corner 0 in the lattice (no wrap: 2 z_mu + 1 < L_mu).
__device__ __forceinline__ int corner_offset(const NprGeom& g, int X) {
    return (X & 1) + g.L[0] * (((X >> 1) & 1) + g.L[1] * (((X >> 2) & 1) + g.L[2] * (X >> 3)));
}

// Field value q of this thread's share (element threadIdx.x + 256 q) of the pass starting at set i0. The load is
// always issued: an element past the pass reads the pass's first element instead, and stage_put does not store
// it (loads under a branch would each wait for their data before the next one).
__device__ __forceinline__ double2 stage_get(const NprArgs& a, int base, int i0, int q) {
    const int m = min(NPR_CHUNK, a.n - i0);
    const int e0 = threadIdx.x + 256 * q, e = e0 < m * 192 ? e0 : 0;
    const int s = e / 192, r0 = e % 192, fi = r0 / 48, r = r0 % 48, corner = r / 3, c = r % 3;
    return a.f[fi][((long)(i0 + s) * a.g.V + base + corner_offset(a.g, corner)) * 3 + c];
}

__device__ __forceinline__ void stage_put(const NprArgs& a, int i0, int q, double2 v, double2 (*fs)[4][16][3]) {
    const int m = min(NPR_CHUNK, a.n - i0);
    const int e = threadIdx.x + 256 * q;
    if (e < m * 192) fs[e / 192][(e % 192) / 48][(e % 48) / 3][e % 3] = v;
}

// Lattice index of corner 0 of hypercube z.
__device__ __forceinline__ int npr_base(const NprGeom& g, int z) {
    int zc[4];
    coarse_coords(g, z, zc);
    const int c0[4] = {2 * zc[0], 2 * zc[1], 2 * zc[2], 2 * zc[3]};
    return lex4(g, c0);
}

// The contraction of hypercube z for every field set, by thread (A, C) of a block holding U_{A,D} and U_{C,B} in
// registers; fs (LDS) stages the hypercube's field values of NPR_CHUNK field sets at a time. When staged, the
// caller has put the first pass's values in fs already (loaded early, so that their latency overlaps other
// work); otherwise, and for later passes, the values are copied one at a time as a pass starts
// (register staging there, or prefetching across the arithmetic, raises the kernel's registers past three
// waves per SIMD; staging ahead of the path-link loads of k_npr_contract made it slower).
__device__ __forceinline__ void contract_sets(const NprArgs& a, int z, int base, const C (&uad)[3][3],
                                              const C (&ucb)[3][3], double2 (*fs)[4][16][3], bool staged) {
    const int A = threadIdx.x >> 4, Cc = threadIdx.x & 15;
    const int B = A ^ a.d1, D = Cc ^ a.d2;
    const double sgn = (((a.neg1 >> A) ^ (a.neg2 >> Cc)) & 1) ? -1.0 : 1.0;
    for (int i0 = 0; i0 < a.n; i0 += NPR_CHUNK) {
        const int m = min(NPR_CHUNK, a.n - i0);
        if (i0 > 0 || !staged)
            for (int e = threadIdx.x; e < m * 192; e += 256) {
                const int s = e / 192, r0 = e % 192, fi = r0 / 48, r = r0 % 48, corner = r / 3, c = r % 3;
                fs[s][fi][corner][c] = a.f[fi][((long)(i0 + s) * a.g.V + base + corner_offset(a.g, corner)) * 3 + c];
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
                    s1 = cmac(s1, uad[r][c], {x4.x, x4.y});
                    s2 = cmac(s2, ucb[r][c], {x2.x, x2.y});
                }
                const double2 y1 = fs[s][0][A][r], y3 = fs[s][2][Cc][r];
                b1 = cmac(b1, {y1.x, y1.y}, s1);
                b2 = cmac(b2, {y3.x, y3.y}, s2);
            }
            const C term = cmac({0.0, 0.0}, b1, b2);
            v[2 * s] = sgn * term.re;
            v[2 * s + 1] = sgn * term.im;
        }
        block_sum<2 * NPR_CHUNK>(v);  // ends with a barrier, so the staged values can be replaced next
        if (threadIdx.x == 0)
#pragma unroll
            for (int s = 0; s < NPR_CHUNK; ++s)
                if (s < m) a.out[(long)(i0 + s) * a.g.nz + z] = make_double2(v[2 * s], v[2 * s + 1]);
    }
}

// From stored path links: thread (A, C) loads U_{A,D} and U_{C,B} from the hypercube's block.
__global__ __launch_bounds__(256) void k_npr_contract(NprArgs a) {
    const int z = remap_block(blockIdx.x, gridDim.x);
    const int A = threadIdx.x >> 4, Cc = threadIdx.x & 15;
    const int B = A ^ a.d1, D = Cc ^ a.d2;
    __shared__ double2 fs[NPR_CHUNK][4][16][3];  // the hypercube's field values of a pass
    const int base = npr_base(a.g, z);
    C uad[3][3], ucb[3][3];
    const double2* blk = a.uad + (long)z * 256 * 9;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const double2 v = blk[(A * 16 + D) * 9 + j];
        const double2 w = blk[(Cc * 16 + B) * 9 + j];
        uad[j / 3][j % 3] = {v.x, v.y};
        ucb[j / 3][j % 3] = {w.x, w.y};
    }
    contract_sets(a, z, base, uad, ucb, fs, false);
}

// Fused: the hypercube's path links are built in LDS (as k_npr_paths does) and contracted at once, so the 36 KB
// of path links per hypercube never travel to memory and back. The first pass's field values are loaded before
// the paths are built; once every thread holds its two matrices the path area is reused for the field staging
// (a barrier separates the two uses).
__global__ __launch_bounds__(256) void k_npr_fused(NprArgs a, const double2* __restrict__ U) {
    const int z = remap_block(blockIdx.x, gridDim.x);
    const int A = threadIdx.x >> 4, Cc = threadIdx.x & 15;
    const int B = A ^ a.d1, D = Cc ^ a.d2;
    __shared__ Paths P;
    static_assert(sizeof(double2) * NPR_CHUNK * 4 * 16 * 3 <= sizeof(Paths), "staging fits the path area");
    const int base = npr_base(a.g, z);
    const double2 f0 = stage_get(a, base, 0, 0), f1 = stage_get(a, base, 0, 1), f2 = stage_get(a, base, 0, 2);
    build_paths(a.g, U, z, P);
    C uad[3][3], ucb[3][3];
    path_ld(P, A, D, uad);
    path_ld(P, Cc, B, ucb);
    __syncthreads();  // every thread has read its matrices: the path area becomes the field staging
    double2(*fs)[4][16][3] = (double2(*)[4][16][3])&P[0][0];
    stage_put(a, 0, 0, f0, fs);
    stage_put(a, 0, 1, f1, fs);
    stage_put(a, 0, 2, f2, fs);
    contract_sets(a, z, base, uad, ucb, fs, true);
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
