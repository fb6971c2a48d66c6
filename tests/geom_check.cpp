// CPU check of the library's checkerboard index arithmetic (host build of the __host__ __device__ helpers
// in sp_device.h and sp_kernels.h; compiled and run by tests/test_geometry_cpu.py).
//
//  1. divq(a, d, 1/d) == a / d. The float estimate of a / d is within (a / d) 2^-22 of the quotient, under
//     4 / d for a < 2^24, so it can only truncate to a wrong integer when a lies within 4 of a multiple of d.
//     Checked: every a < 2^24 for d <= 64, and a = k d + j, |j| <= 4, for every k and every d < 2^22 (the
//     largest divisor an admitted lattice produces: X/2, Y or Z with the other extents >= 2 and V/2 < 2^24).
//  2. site_of, nbr and eta_sign against plain lexicographic arithmetic, every site of both parities, on
//     lattices with extents of 2, unequal extents, and the workload shapes (sampled on the largest).
//  3. remap_block is a permutation of [0, nb) for every nb up to 20,000 and for the launch sizes of the
//     workload lattices.
// Prints one line per part and exits non-zero at the first mismatch.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../paper_1511_00088_amd/csrc/sp_kernels.h"

using namespace sp;

static Geom make_geom(int X, int Y, int Z, int T, int bc_t) {
    Geom g;
    g.X = X; g.Y = Y; g.Z = Z; g.T = T;
    g.Xh = X / 2;
    g.Vh = (int)((long)X * Y * Z * T / 2);
    g.bc_t = bc_t;
    g.rXh = 1.0f / (float)g.Xh;
    g.rY = 1.0f / (float)Y;
    g.rZ = 1.0f / (float)Z;
    return g;
}

static bool check_divq() {
    const int A = 1 << 24;
    long n = 0;
    for (int d = 1; d <= 64; ++d) {
        const float rd = 1.0f / (float)d;
        for (int a = 0; a < A; ++a) {
            if (divq(a, d, rd) != a / d) {
                printf("divq(%d, %d) = %d, expected %d\n", a, d, divq(a, d, rd), a / d);
                return false;
            }
        }
        n += A;
    }
    for (int d = 65; d < (1 << 22); ++d) {
        const float rd = 1.0f / (float)d;
        for (long k = 0; k * d - 4 < A; ++k) {
            for (int j = -4; j <= 4; ++j) {
                const long a = k * d + j;
                if (a < 0 || a >= A) continue;
                ++n;
                if (divq((int)a, d, rd) != (int)(a / d)) {
                    printf("divq(%ld, %d) = %d, expected %ld\n", a, d, divq((int)a, d, rd), a / d);
                    return false;
                }
            }
        }
    }
    printf("divq: %ld quotients exact\n", n);
    return true;
}

// Plain lexicographic reference: coordinates of lex, neighbour lex with periodic wrap, eta.
static bool check_sites(int X, int Y, int Z, int T, long stride) {
    const Geom g = make_geom(X, Y, Z, T, 0);
    const int L[4] = {X, Y, Z, T};
    long checked = 0;
    for (long lex = 0; lex < 2L * g.Vh; lex += stride) {
        int n[4];
        long r = lex;
        for (int mu = 0; mu < 4; ++mu) {
            n[mu] = (int)(r % L[mu]);
            r /= L[mu];
        }
        const int p = (n[0] + n[1] + n[2] + n[3]) & 1;
        const int cb = (int)(lex >> 1);
        const Site s = site_of(g, p, cb);
        if (s.cb != cb || s.x != n[0] || s.y != n[1] || s.z != n[2] || s.t != n[3]) {
            printf("site_of(%dx%dx%dx%d, p=%d, cb=%d) = (%d,%d,%d,%d), expected (%d,%d,%d,%d)\n", X, Y, Z, T, p, cb,
                   s.x, s.y, s.z, s.t, n[0], n[1], n[2], n[3]);
            return false;
        }
        for (int mu = 0; mu < 4; ++mu) {
            int e = 0;
            for (int nu = 0; nu < mu; ++nu) e += n[nu];
            const float eta = (e & 1) ? -1.0f : 1.0f;
            if (eta_sign(s, mu) != eta) {
                printf("eta_sign(mu=%d) wrong at lex %ld\n", mu, lex);
                return false;
            }
            for (int dir = -1; dir <= 1; dir += 2) {
                int m[4] = {n[0], n[1], n[2], n[3]};
                m[mu] = (n[mu] + dir + L[mu]) % L[mu];
                const long ml = m[0] + (long)X * (m[1] + (long)Y * (m[2] + (long)Z * m[3]));
                const int got = nbr(g, s, mu, dir);
                if (got != (int)(ml >> 1)) {
                    printf("nbr(%dx%dx%dx%d, lex=%ld, mu=%d, dir=%d) = %d, expected %ld\n", X, Y, Z, T, lex, mu, dir,
                           got, ml >> 1);
                    return false;
                }
            }
        }
        ++checked;
    }
    printf("sites %dx%dx%dx%d: %ld sites (every %ld-th) match\n", X, Y, Z, T, checked, stride);
    return true;
}

static bool check_remap(int nb) {
    std::vector<char> seen(nb, 0);
    for (int b = 0; b < nb; ++b) {
        const int l = remap_block(b, nb);
        if (l < 0 || l >= nb || seen[l]) {
            printf("remap_block(%d, %d) = %d is out of range or repeated\n", b, nb, l);
            return false;
        }
        seen[l] = 1;
        // consecutive hardware blocks b and b + 8 (same XCD) hold consecutive logical blocks
        if (b + 8 < nb && remap_block(b + 8, nb) != l + 1) {
            printf("remap_block(%d, %d) and remap_block(%d) are not consecutive\n", b, nb, b + 8);
            return false;
        }
    }
    return true;
}

int main() {
    if (!check_divq()) return 1;
    const int lat[][4] = {{2, 2, 2, 2}, {4, 4, 4, 4}, {2, 4, 6, 8}, {4, 4, 2, 2}, {8, 6, 4, 10}, {2, 6, 4, 2},
                          {6, 4, 8, 4},  {4, 2, 6, 2}, {12, 12, 12, 24}, {16, 16, 16, 32}, {20, 20, 20, 8}};
    for (auto& d : lat)
        if (!check_sites(d[0], d[1], d[2], d[3], 1)) return 1;
    // the workload lattices, and the largest admitted shape of the tests (V/2 just below 2^24), sampled
    if (!check_sites(20, 20, 20, 64, 1)) return 1;
    if (!check_sites(28, 28, 28, 96, 7)) return 1;
    if (!check_sites(32, 32, 32, 64, 5)) return 1;
    if (!check_sites(64, 64, 64, 126, 97)) return 1;
    if (!check_sites(2, 2, 2, 4194302, 13)) return 1;
    if (!check_sites(4194302, 2, 2, 2, 13)) return 1;
    for (int nb = 1; nb <= 20000; ++nb)
        if (!check_remap(nb)) return 1;
    const int big[] = {1000, 2000, 4000, 8192, 10976, 16384, 65536};
    for (int nb : big)
        if (!check_remap(nb)) return 1;
    printf("remap_block: permutation for nb = 1..20000 and the workload launch sizes\n");
    printf("ALL OK\n");
    return 0;
}
