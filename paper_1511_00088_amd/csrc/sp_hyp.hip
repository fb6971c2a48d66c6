// HYP smearing of the gauge links (the smoothing the solver's links receive before the solve: the paper's
// quarks are HYP-smeared, Sec. 3). Three levels of staple sums restricted to the hypercubes that contain
// the link (the hypercubic blocking of Hasenfratz and Knechtli), each sum projected back to SU(3):
//
//   level 1  lv1(mu, eta):  (1 - a3) U_mu + a3/2 * staples of U_eta around U_mu        (12 fields)
//   level 2  lv2(mu, nu):   (1 - a2) U_mu + a2/4 * sum_{rho not mu, nu} staples of lv1(rho, s) around
//                           lv1(mu, s), s the direction outside {mu, nu, rho}              (12 fields)
//   level 3  V_mu:          (1 - a1) U_mu + a1/6 * sum_{nu != mu} staples of lv2(nu, mu) around lv2(mu, nu)
//
// with staples of side S around top T in direction eta at x:
//   S(x) T(x+eta) S(x+mu)^dag + S(x-eta)^dag T(x-eta) S(x-eta+mu).
//
// Proj_SU(3)(W) maximises Re tr(X^dag W) over SU(3). Where W^dag W is close to a multiple of the identity
// and the determinant phase of W is small (the usual case for smeared links) the maximiser is computed in
// closed form as a function of W^dag W (proj_direct below). Otherwise the unitary polar factor of W comes
// from scaled Newton iteration X <- (z X + X^-dag / z) / 2, z = |det X|^(-1/3), and the same closed form
// is tried from it (proj_series); failing that, the cube root of the determinant's phase (principal
// branch) is divided out and sweeps over the three SU(2) subgroups (Cabibbo-Marinari), each taking the
// subgroup element that maximises the objective, run until a sweep moves no element by more than 1e-15.
//
// One thread per (site, field); blockIdx.y selects the field, so a wavefront covers 64 consecutive sites
// of one field. Every level is FP64. Input and output links use the natural layout [4][V][3][3] complex128
// (a link is 9 consecutive double2); the intermediate fields live in the caller's workspace as planes
// [9][V] double2 per field. All directions are periodic.
#include "sp_launch.h"

namespace sp {
namespace {

using C = Cx<double>;
using M3 = Su3<double>;

struct HypGeom {
    int L[4];       // extents X, Y, Z, T
    int stride[4];  // 1, X, XY, XYZ
    int V;
};

__device__ __forceinline__ int hop(const HypGeom& g, int s, int mu, int d) {
    const int c = (s / g.stride[mu]) % g.L[mu];
    const int c1 = c + d;
    int s1 = s + d * g.stride[mu];
    if (c1 == g.L[mu]) s1 -= g.L[mu] * g.stride[mu];
    if (c1 < 0) s1 += g.L[mu] * g.stride[mu];
    return s1;
}

// A link field: element (site s, entry j) at p[s * ss + j * ps] (double2 units).
struct LinkField {
    const double2* p;
    long ss, ps;
};

__device__ __forceinline__ M3 ld(const LinkField& f, int s) {
    M3 m;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        const double2 v = f.p[(long)s * f.ss + (long)j * f.ps];
        m.e[j / 3][j % 3] = {v.x, v.y};
    }
    return m;
}

__device__ __forceinline__ void st(double2* p, long ss, long ps, int s, const M3& m) {
#pragma unroll
    for (int j = 0; j < 9; ++j) p[(long)s * ss + (long)j * ps] = make_double2(m.e[j / 3][j % 3].re, m.e[j / 3][j % 3].im);
}

__device__ __forceinline__ C cmul(C a, C b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
// a * conj(b)
__device__ __forceinline__ C cmulc(C a, C b) { return {a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im}; }
__device__ __forceinline__ C cadd(C a, C b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ C csub(C a, C b) { return {a.re - b.re, a.im - b.im}; }

// a b
__device__ __forceinline__ M3 mul(const M3& a, const M3& b) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C s = cmul(a.e[i][0], b.e[0][j]);
            s = cadd(s, cmul(a.e[i][1], b.e[1][j]));
            r.e[i][j] = cadd(s, cmul(a.e[i][2], b.e[2][j]));
        }
    return r;
}

// a b^dag
__device__ __forceinline__ M3 mul_nd(const M3& a, const M3& b) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C s = cmulc(a.e[i][0], b.e[j][0]);
            s = cadd(s, cmulc(a.e[i][1], b.e[j][1]));
            r.e[i][j] = cadd(s, cmulc(a.e[i][2], b.e[j][2]));
        }
    return r;
}

// a^dag b
__device__ __forceinline__ M3 mul_dn(const M3& a, const M3& b) {
    M3 r;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C s = cmulc(b.e[0][j], a.e[0][i]);
            s = cadd(s, cmulc(b.e[1][j], a.e[1][i]));
            r.e[i][j] = cadd(s, cmulc(b.e[2][j], a.e[2][i]));
        }
    return r;
}

__device__ __forceinline__ void axpy(M3& w, double c, const M3& a) {
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            w.e[i][j].re += c * a.e[i][j].re;
            w.e[i][j].im += c * a.e[i][j].im;
        }
}

// w += c * [S(x) T(x+eta) S(x+mu)^dag + S(x-eta)^dag T(x-eta) S(x-eta+mu)]
__device__ __forceinline__ void add_staples(M3& w, double c, const HypGeom& g, const LinkField& S, const LinkField& T,
                                            int s, int mu, int eta) {
    const int s_pe = hop(g, s, eta, +1), s_pm = hop(g, s, mu, +1), s_me = hop(g, s, eta, -1);
    const int s_me_pm = hop(g, s_me, mu, +1);
    axpy(w, c, mul_nd(mul(ld(S, s), ld(T, s_pe)), ld(S, s_pm)));
    axpy(w, c, mul(mul_dn(ld(S, s_me), ld(T, s_me)), ld(S, s_me_pm)));
}

// rows of the cofactor matrix are cross products of the other two rows
__device__ __forceinline__ void cross(const C* a, const C* b, C* out) {
    out[0] = csub(cmul(a[1], b[2]), cmul(a[2], b[1]));
    out[1] = csub(cmul(a[2], b[0]), cmul(a[0], b[2]));
    out[2] = csub(cmul(a[0], b[1]), cmul(a[1], b[0]));
}

__device__ __forceinline__ C det3(const M3& x) {
    C c[3];
    cross(x.e[1], x.e[2], c);
    return cadd(cadd(cmul(x.e[0][0], c[0]), cmul(x.e[0][1], c[1])), cmul(x.e[0][2], c[2]));
}

// The unitary polar factor of w by Newton's iteration with determinant scaling. X^-dag = conj(cof(X)) /
// conj(det X), where the rows of cof(X) are r1 x r2, r2 x r0, r0 x r1.
__device__ __forceinline__ M3 polar_factor(const M3& w) {
    M3 x = w;
    int extra = -1;
    for (int it = 0; it < 40; ++it) {
        M3 cof;
        cross(x.e[1], x.e[2], cof.e[0]);
        cross(x.e[2], x.e[0], cof.e[1]);
        cross(x.e[0], x.e[1], cof.e[2]);
        const C d = cadd(cadd(cmul(x.e[0][0], cof.e[0][0]), cmul(x.e[0][1], cof.e[0][1])),
                         cmul(x.e[0][2], cof.e[0][2]));
        const double ad2 = d.re * d.re + d.im * d.im;
        const double z = 1.0 / cbrt(sqrt(ad2));
        const double hz = 0.5 * z, hr = 0.5 / (ad2 * z);
        // X^-dag_ij = conj(cof_ij / d) = conj(cof_ij) * d / |d|^2
        double diff = 0.0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const C q = cmulc(d, cof.e[i][j]);  // d * conj(cof_ij)
                const double nre = hz * x.e[i][j].re + hr * q.re;
                const double nim = hz * x.e[i][j].im + hr * q.im;
                diff = fmax(diff, fmax(fabs(nre - x.e[i][j].re), fabs(nim - x.e[i][j].im)));
                x.e[i][j] = {nre, nim};
            }
        // quadratic convergence: once the step is small, two more steps reach rounding level
        if (extra < 0 && diff < 1e-6) extra = 2;
        if (extra >= 0 && extra-- == 0) break;
    }
    return x;
}

__device__ __forceinline__ void su2_step(M3& x, const M3& w, int i, int j) {
    // entries (i,i), (i,j), (j,i), (j,j) of M = W X^dag
    auto m = [&](int a, int b) {
        C s = cmulc(w.e[a][0], x.e[b][0]);
        s = cadd(s, cmulc(w.e[a][1], x.e[b][1]));
        return cadd(s, cmulc(w.e[a][2], x.e[b][2]));
    };
    const C mii = m(i, i), mij = m(i, j), mji = m(j, i), mjj = m(j, j);
    // Re tr(h^dag A) over h = b0 + i b.sigma in SU(2) is 2 (b0 Re A0 + b . Re A), A = A0 + i A.sigma
    const double a0 = 0.5 * (mii.re + mjj.re);
    const double a1 = 0.5 * (mij.im + mji.im);
    const double a2 = 0.5 * (mij.re - mji.re);
    const double a3 = 0.5 * (mii.im - mjj.im);
    const double rn = 1.0 / sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3);
    const double b0 = a0 * rn, b1 = a1 * rn, b2 = a2 * rn, b3 = a3 * rn;
    const C h00 = {b0, b3}, h01 = {b2, b1}, h10 = {-b2, b1}, h11 = {b0, -b3};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const C xi = x.e[i][k], xj = x.e[j][k];
        x.e[i][k] = cadd(cmul(h00, xi), cmul(h01, xj));
        x.e[j][k] = cadd(cmul(h10, xi), cmul(h11, xj));
    }
}

// (m + m^dag) / 2
__device__ __forceinline__ void hermitize(M3& m) {
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        m.e[i][i].im = 0.0;
#pragma unroll
        for (int j = i + 1; j < 3; ++j) {
            const C a = m.e[i][j], b = m.e[j][i];
            m.e[i][j] = {0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
            m.e[j][i] = {m.e[i][j].re, -m.e[i][j].im};
        }
    }
}

// The maximiser of Re tr(X^dag W) over SU(3) without iterating, where it is safe. With W = up H (up the
// unitary polar factor, det up = e^{i phi}, H = up^dag W Hermitian positive definite) the maximiser is
// X = up exp(i Theta), Theta = asin(mu G) with G = H^-1: in the eigenbasis of H the problem separates into
// one phase theta_k per eigenvalue h_k, maximising sum h_k cos theta_k subject to sum theta_k = -phi, whose
// stationarity condition h_k sin theta_k = mu gives theta_k = asin(mu / h_k); mu follows from
// tr Theta = -phi. No eigenvectors are formed: the traces tr G^k come from Newton's identities, Theta from
// the arcsine series in mu G (terms to (mu G)^13) and exp(i Theta) from its Taylor series (to order 8), both
// as polynomials in G reduced to degree two by the characteristic polynomial.
// Used only when |mu| |G|_F <= 0.06, where the first omitted terms are below 1e-17 and the principal
// phases are the maximum; returns false otherwise, and the caller iterates instead.
__device__ __forceinline__ bool proj_series(const M3& w, const M3& up, M3& x) {
    constexpr double c[7] = {1.0, 1.0 / 6, 3.0 / 40, 5.0 / 112, 35.0 / 1152, 63.0 / 2816, 231.0 / 13312};
    const C du = det3(up);
    const double phi = atan2(du.im, du.re);
    M3 h = mul_dn(up, w);
    hermitize(h);
    M3 cof;
    cross(h.e[1], h.e[2], cof.e[0]);
    cross(h.e[2], h.e[0], cof.e[1]);
    cross(h.e[0], h.e[1], cof.e[2]);
    const double dh = h.e[0][0].re * cof.e[0][0].re - h.e[0][0].im * cof.e[0][0].im +
                      h.e[0][1].re * cof.e[0][1].re - h.e[0][1].im * cof.e[0][1].im +
                      h.e[0][2].re * cof.e[0][2].re - h.e[0][2].im * cof.e[0][2].im;  // real for Hermitian h
    if (!(dh > 0.0) || !isfinite(dh)) return false;
    const double rd = 1.0 / dh;
    M3 g;  // H^-1 = cof^T / det
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) g.e[i][j] = {cof.e[j][i].re * rd, cof.e[j][i].im * rd};
    hermitize(g);
    // power sums p_k = tr G^k: p1, p2 from the entries, then e1 p_{k-1} - e2 p_{k-2} + e3 p_{k-3}
    double p[14];
    p[1] = g.e[0][0].re + g.e[1][1].re + g.e[2][2].re;
    p[2] = 0.0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) p[2] += g.e[i][j].re * g.e[i][j].re + g.e[i][j].im * g.e[i][j].im;
    const double e1 = p[1], e2 = 0.5 * (p[1] * p[1] - p[2]), e3 = rd;
    p[3] = e1 * p[2] - e2 * p[1] + 3.0 * e3;
#pragma unroll
    for (int q = 4; q < 14; ++q) p[q] = e1 * p[q - 1] - e2 * p[q - 2] + e3 * p[q - 3];
    // tr asin(mu G) = -phi by Newton's method on the series
    double mu = -phi / p[1];
#pragma unroll
    for (int it = 0; it < 6; ++it) {
        const double m2 = mu * mu;
        double f = 0.0, df = 0.0, mp = 1.0;  // mp = mu^(2n)
#pragma unroll
        for (int n = 0; n < 7; ++n) {
            df += c[n] * (2 * n + 1) * p[2 * n + 1] * mp;
            f += c[n] * p[2 * n + 1] * mp * mu;
            mp *= m2;
        }
        mu -= (f + phi) / df;
    }
    if (!(fabs(mu) * sqrt(p[2]) <= 0.06)) return false;
    // Every power series in G reduces to a0 I + a1 G + a2 G^2 (Cayley-Hamilton: G^3 = e1 G^2 - e2 G + e3),
    // so Theta and exp(i Theta) are carried as three scalar coefficients each; G^2 is the only matrix
    // product before the last one.
    double gp[3] = {0.0, 1.0, 0.0};  // G^(2n+1)
    double th[3] = {0.0, 0.0, 0.0};  // Theta
    double mp = mu;
#pragma unroll
    for (int n = 0; n < 7; ++n) {
#pragma unroll
        for (int q = 0; q < 3; ++q) th[q] += c[n] * mp * gp[q];
#pragma unroll
        for (int rep = 0; rep < 2; ++rep) {  // times G
            const double a0 = gp[0], a1 = gp[1], a2 = gp[2];
            gp[0] = a2 * e3;
            gp[1] = a0 - a2 * e2;
            gp[2] = a1 + a2 * e1;
        }
        mp *= mu * mu;
    }
    // exp(i Theta) = 1 + i Theta (1 + i Theta / 2 (... (1 + i Theta / 8))), products reduced mod the
    // characteristic polynomial
    C ev[3] = {{1.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
    for (int q = 8; q >= 1; --q) {
        C cc[5] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
            for (int b = 0; b < 3; ++b) {  // (i th_a) ev_b
                cc[a + b].re -= th[a] * ev[b].im;
                cc[a + b].im += th[a] * ev[b].re;
            }
#pragma unroll
        for (int kk = 4; kk >= 3; --kk) {
            cc[kk - 1] = {cc[kk - 1].re + cc[kk].re * e1, cc[kk - 1].im + cc[kk].im * e1};
            cc[kk - 2] = {cc[kk - 2].re - cc[kk].re * e2, cc[kk - 2].im - cc[kk].im * e2};
            cc[kk - 3] = {cc[kk - 3].re + cc[kk].re * e3, cc[kk - 3].im + cc[kk].im * e3};
        }
        const double rq = 1.0 / q;
#pragma unroll
        for (int a = 0; a < 3; ++a) ev[a] = {cc[a].re * rq, cc[a].im * rq};
        ev[0].re += 1.0;
    }
    const M3 g2 = mul(g, g);
    M3 e;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            C s = cadd(cmul(ev[1], g.e[i][j]), cmul(ev[2], g2.e[i][j]));
            if (i == j) s = cadd(s, ev[0]);
            e.e[i][j] = s;
        }
    x = mul(up, e);
    return true;
}

// Polynomials a0 + a1 E + a2 E^2 in a traceless Hermitian 3x3 matrix E, reduced by its characteristic
// polynomial E^3 = -e2 E + e3 (e2 = -tr(E^2)/2, e3 = det E).
template <class T>
__device__ __forceinline__ void poly_mul(const T (&a)[3], const T (&b)[3], double e2, double e3, T (&r)[3]) {
    T c[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) c[q] = T(0.0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) c[i + j] = c[i + j] + a[i] * b[j];
#pragma unroll
    for (int q = 4; q >= 3; --q) {  // E^q = -e2 E^(q-2) + e3 E^(q-3)
        c[q - 2] = c[q - 2] - c[q] * e2;
        c[q - 3] = c[q - 3] + c[q] * e3;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) r[q] = c[q];
}

// complex scalar with the operators poly_mul needs
struct Z {
    double re, im;
    __device__ Z() = default;
    __device__ constexpr Z(double r) : re(r), im(0.0) {}
    __device__ constexpr Z(double r, double i) : re(r), im(i) {}
};
__device__ __forceinline__ Z operator+(Z a, Z b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Z operator-(Z a, Z b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ Z operator*(Z a, Z b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Z operator*(Z a, double s) { return {a.re * s, a.im * s}; }

// The same maximiser as proj_series, written entirely as a function of S = W^dag W: the polar factor is
// W S^-1/2 and H^-1 = S^-1/2, so X = W F(S) with F = S^-1/2 exp(i asin(mu S^-1/2)), det W = |det W| e^{i phi}.
// With s0 = tr S / 3 and E = S / s0 - I (traceless), S^-1/2 = s0^-1/2 sum_k binom(-1/2, k) E^k; all series
// are carried as coefficients of I, E, E^2, so the matrix products are S, E^2 and W F. Used when
// |E|_F <= 1/2 (60 terms of the binomial series then leave less than 1e-17) and |mu| |S^-1/2|_F <= 0.06;
// returns false otherwise.
__device__ __forceinline__ bool proj_direct(const M3& w, M3& x) {
    constexpr double c[7] = {1.0, 1.0 / 6, 3.0 / 40, 5.0 / 112, 35.0 / 1152, 63.0 / 2816, 231.0 / 13312};
    M3 s = mul_dn(w, w);
    hermitize(s);
    const double s0 = (s.e[0][0].re + s.e[1][1].re + s.e[2][2].re) * (1.0 / 3.0);
    if (!(s0 > 0.0) || !isfinite(s0)) return false;
    const double rs0 = 1.0 / s0;
    M3 e;
    double t2 = 0.0;  // tr E^2 = |E|_F^2
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            e.e[i][j] = {s.e[i][j].re * rs0 - (i == j ? 1.0 : 0.0), s.e[i][j].im * rs0};
            t2 += e.e[i][j].re * e.e[i][j].re + e.e[i][j].im * e.e[i][j].im;
        }
    if (!(t2 <= 0.25)) return false;
    const double e2 = -0.5 * t2, e3 = det3(e).re;
    // G = S^-1/2
    double g[3] = {0.0, 0.0, 0.0}, pk[3] = {1.0, 0.0, 0.0}, bk = 1.0;
#pragma unroll
    for (int kk = 0; kk < 60; ++kk) {
#pragma unroll
        for (int q = 0; q < 3; ++q) g[q] += bk * pk[q];
        const double a0 = pk[0], a1 = pk[1], a2 = pk[2];  // times E
        pk[0] = a2 * e3;
        pk[1] = a0 - a2 * e2;
        pk[2] = a1;
        bk *= -(2.0 * kk + 1.0) / (2.0 * kk + 2.0);
    }
    const double rsq = 1.0 / sqrt(s0);
#pragma unroll
    for (int q = 0; q < 3; ++q) g[q] *= rsq;
    const C dw = det3(w);
    const double phi = atan2(dw.im, dw.re);
    double g2[3];
    poly_mul(g, g, e2, e3, g2);
    auto trace = [&](const double (&a)[3]) { return 3.0 * a[0] + a[2] * t2; };
    // odd powers of G and their traces
    double gp[7][3], p[7];
#pragma unroll
    for (int q = 0; q < 3; ++q) gp[0][q] = g[q];
#pragma unroll
    for (int n = 1; n < 7; ++n) poly_mul(gp[n - 1], g2, e2, e3, gp[n]);
#pragma unroll
    for (int n = 0; n < 7; ++n) p[n] = trace(gp[n]);
    double mu = -phi / p[0];
#pragma unroll
    for (int it = 0; it < 6; ++it) {
        const double m2 = mu * mu;
        double f = 0.0, df = 0.0, mp = 1.0;
#pragma unroll
        for (int n = 0; n < 7; ++n) {
            df += c[n] * (2 * n + 1) * p[n] * mp;
            f += c[n] * p[n] * mp * mu;
            mp *= m2;
        }
        mu -= (f + phi) / df;
    }
    if (!(fabs(mu) * sqrt(trace(g2)) <= 0.06)) return false;
    double th[3] = {0.0, 0.0, 0.0}, mp = mu;
#pragma unroll
    for (int n = 0; n < 7; ++n) {
#pragma unroll
        for (int q = 0; q < 3; ++q) th[q] += c[n] * mp * gp[n][q];
        mp *= mu * mu;
    }
    const Z ith[3] = {Z(0.0, th[0]), Z(0.0, th[1]), Z(0.0, th[2])};
    Z ev[3] = {Z(1.0), Z(0.0), Z(0.0)};
#pragma unroll
    for (int q = 8; q >= 1; --q) {
        Z t[3];
        poly_mul(ith, ev, e2, e3, t);
        const double rq = 1.0 / q;
        ev[0] = t[0] * rq + Z(1.0);
        ev[1] = t[1] * rq;
        ev[2] = t[2] * rq;
    }
    const Z gz[3] = {Z(g[0]), Z(g[1]), Z(g[2])};
    Z f[3];
    poly_mul(gz, ev, e2, e3, f);
    const M3 ee = mul(e, e);
    M3 m;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            const C a = cmul({f[1].re, f[1].im}, e.e[i][j]), b = cmul({f[2].re, f[2].im}, ee.e[i][j]);
            m.e[i][j] = {a.re + b.re + (i == j ? f[0].re : 0.0), a.im + b.im + (i == j ? f[0].im : 0.0)};
        }
    x = mul(w, m);
    return true;
}

__device__ __forceinline__ M3 proj_su3(const M3& w) {
    M3 y;
    if (proj_direct(w, y)) return y;
    M3 x = polar_factor(w);
    if (proj_series(w, x, y)) return y;
    const C d = det3(x);
    const double th = -atan2(d.im, d.re) / 3.0;
    const C ph = {cos(th), sin(th)};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) x.e[i][j] = cmul(x.e[i][j], ph);
    for (int sweep = 0; sweep < 500; ++sweep) {  // nearly singular W can need hundreds
        const M3 x0 = x;
        su2_step(x, w, 0, 1);
        su2_step(x, w, 0, 2);
        su2_step(x, w, 1, 2);
        double diff2 = 0.0;  // largest |change|^2 of an element
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const double dr = x.e[i][j].re - x0.e[i][j].re, di = x.e[i][j].im - x0.e[i][j].im;
                diff2 = fmax(diff2, dr * dr + di * di);
            }
        if (diff2 <= 1e-30) break;
    }
    return x;
}

__device__ __forceinline__ int other(int a, int k) { return k < a ? k : k + 1; }  // k-th direction != a
__device__ __forceinline__ int fidx(int a, int b) { return a * 3 + (b < a ? b : b - 1); }  // field (a, b != a)

struct HypArgs {
    HypGeom g;
    const double2* U;  // natural [4][V][9] double2
    double2* lv1;      // [12][9][V]
    double2* lv2;      // [12][9][V]
    double2* out;      // natural [4][V][9]
    double a1, a2, a3;
};

__device__ __forceinline__ LinkField nat(const HypArgs& a, const double2* base, int mu) {
    return {base + (long)mu * a.g.V * 9, 9, 1};
}
__device__ __forceinline__ LinkField plane(const HypArgs& a, const double2* base, int f) {
    return {base + (long)f * a.g.V * 9, 1, a.g.V};
}

__global__ __launch_bounds__(256) void k_hyp_level1(HypArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.g.V) return;
    const int f = blockIdx.y, mu = f / 3, eta = other(mu, f % 3);
    const LinkField Um = nat(a, a.U, mu);
    M3 w = ld(Um, s);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            w.e[i][j].re *= 1.0 - a.a3;
            w.e[i][j].im *= 1.0 - a.a3;
        }
    add_staples(w, 0.5 * a.a3, a.g, nat(a, a.U, eta), Um, s, mu, eta);
    st(a.lv1 + (long)f * a.g.V * 9, 1, a.g.V, s, proj_su3(w));
}

__global__ __launch_bounds__(256) void k_hyp_level2(HypArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.g.V) return;
    const int f = blockIdx.y, mu = f / 3, nu = other(mu, f % 3);
    M3 w = ld(nat(a, a.U, mu), s);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            w.e[i][j].re *= 1.0 - a.a2;
            w.e[i][j].im *= 1.0 - a.a2;
        }
    for (int rho = 0; rho < 4; ++rho) {
        if (rho == mu || rho == nu) continue;
        const int sg = 6 - mu - nu - rho;
        add_staples(w, 0.25 * a.a2, a.g, plane(a, a.lv1, fidx(rho, sg)), plane(a, a.lv1, fidx(mu, sg)), s, mu, rho);
    }
    st(a.lv2 + (long)f * a.g.V * 9, 1, a.g.V, s, proj_su3(w));
}

__global__ __launch_bounds__(256) void k_hyp_level3(HypArgs a) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= a.g.V) return;
    const int mu = blockIdx.y;
    M3 w = ld(nat(a, a.U, mu), s);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            w.e[i][j].re *= 1.0 - a.a1;
            w.e[i][j].im *= 1.0 - a.a1;
        }
    for (int nu = 0; nu < 4; ++nu) {
        if (nu == mu) continue;
        add_staples(w, a.a1 / 6.0, a.g, plane(a, a.lv2, fidx(nu, mu)), plane(a, a.lv2, fidx(mu, nu)), s, mu, nu);
    }
    st(a.out + (long)mu * a.g.V * 9, 9, 1, s, proj_su3(w));
}

}  // namespace

size_t hyp_workspace_bytes(const Geom& g) { return 24ull * 2 * (size_t)g.Vh * 9 * sizeof(double2); }

hipError_t launch_hyp(const Geom& g, const double* links, const double alpha[3], double* out, void* ws,
                      hipStream_t s) {
    HypArgs a;
    a.g.L[0] = g.X;
    a.g.L[1] = g.Y;
    a.g.L[2] = g.Z;
    a.g.L[3] = g.T;
    a.g.stride[0] = 1;
    a.g.stride[1] = g.X;
    a.g.stride[2] = g.X * g.Y;
    a.g.stride[3] = g.X * g.Y * g.Z;
    a.g.V = 2 * g.Vh;
    a.U = (const double2*)links;
    a.lv1 = (double2*)ws;
    a.lv2 = (double2*)ws + 12L * a.g.V * 9;
    a.out = (double2*)out;
    a.a1 = alpha[0];
    a.a2 = alpha[1];
    a.a3 = alpha[2];
    const unsigned nb = (unsigned)blocks_for(a.g.V, 256);
    hipLaunchKernelGGL(k_hyp_level1, dim3(nb, 12), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e) return e;
    hipLaunchKernelGGL(k_hyp_level2, dim3(nb, 12), dim3(256), 0, s, a);
    if ((e = hipGetLastError())) return e;
    hipLaunchKernelGGL(k_hyp_level3, dim3(nb, 4), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace sp
