/* FP64 CPU oracle for the even-odd staggered CG. TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark; never by the GPU library.
 *
 * Every routine is the plain definition written out, site by site, in double precision and with
 * sequential sums. Definitions and their sources are listed in oracle.h. Pins (tests that tie this code
 * to facts outside itself):
 *   or_dslash / or_dslash_eo: anti-Hermiticity, zero parity-diagonal blocks, free-field plane-wave
 *     spectrum sum_mu sin^2 p_mu, gauge covariance under random SU(3) transforms;
 *   or_apply_A: even block of (m + D)^dag (m + D); closed-form free-field spectrum on 4^4;
 *   or_cg_solve: numpy.linalg.solve on the dense matrix of A (2^4, 4^4), FFT closed-form free-field
 *     solution, <= 5 iterations on free 4^4, gauge covariance of the solution;
 *   or_grad: central finite differences of l = Re phi^dag A^-1 phi in U, m and phi;
 *   or_full_solve: dense solve of (m + D) psi = src on 2^4.
 */
#include "oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
    int L[4];
    int64_t V;
    int bc_t;
} lattice;

static lattice make_lattice(const int32_t dims[4], int32_t bc_t) {
    lattice g;
    g.V = 1;
    for (int mu = 0; mu < 4; ++mu) {
        g.L[mu] = dims[mu];
        g.V *= dims[mu];
    }
    g.bc_t = bc_t;
    return g;
}

static int64_t lex_of(const lattice* g, const int n[4]) {
    return n[0] + (int64_t)g->L[0] * (n[1] + (int64_t)g->L[1] * (n[2] + (int64_t)g->L[2] * n[3]));
}

static void coords_of(const lattice* g, int64_t s, int n[4]) {
    for (int mu = 0; mu < 4; ++mu) {
        n[mu] = (int)(s % g->L[mu]);
        s /= g->L[mu];
    }
}

static int parity_of(const int n[4]) { return (n[0] + n[1] + n[2] + n[3]) & 1; }

/* Staggered phase eta_mu(n) = (-1)^(n_0 + ... + n_{mu-1}). */
static double eta(int mu, const int n[4]) {
    int s = 0;
    for (int nu = 0; nu < mu; ++nu) s += n[nu];
    return (s & 1) ? -1.0 : 1.0;
}

/* m = n + dir * mu-hat with periodic wrap. */
static void hop(const lattice* g, const int n[4], int mu, int dir, int m[4]) {
    for (int nu = 0; nu < 4; ++nu) m[nu] = n[nu];
    m[mu] = (n[mu] + dir + g->L[mu]) % g->L[mu];
}

/* Link U_mu(n) and its boundary sign (-1 on the last time slice when antiperiodic in t). */
static const cplx* link_at(const lattice* g, const cplx* U, int mu, const int n[4], double* sign) {
    *sign = (g->bc_t && mu == 3 && n[3] == g->L[3] - 1) ? -1.0 : 1.0;
    return U + ((int64_t)mu * g->V + lex_of(g, n)) * 9;
}

/* The colour vector of a field at site m; half fields are indexed by cb = lex >> 1. */
static const cplx* vec_at(const lattice* g, const cplx* f, int is_half, const int m[4]) {
    int64_t s = lex_of(g, m);
    return f + (is_half ? (s >> 1) : s) * 3;
}

/* (D chi)(n) = 1/2 sum_mu eta_mu(n) [U_mu(n) chi(n+mu) - U_mu(n-mu)^dag chi(n-mu)]. */
static void dslash_site(const lattice* g, const cplx* U, const cplx* chi, int is_half, const int n[4],
                        cplx out[3]) {
    for (int i = 0; i < 3; ++i) out[i] = 0;
    for (int mu = 0; mu < 4; ++mu) {
        double e = eta(mu, n);
        int m[4];
        double s;
        /* forward hop: U_mu(n) chi(n+mu) */
        hop(g, n, mu, +1, m);
        const cplx* u = link_at(g, U, mu, n, &s);
        const cplx* v = vec_at(g, chi, is_half, m);
        for (int i = 0; i < 3; ++i) {
            cplx acc = 0;
            for (int j = 0; j < 3; ++j) acc += u[3 * i + j] * v[j];
            out[i] += 0.5 * e * s * acc;
        }
        /* backward hop: U_mu(n-mu)^dag chi(n-mu) */
        hop(g, n, mu, -1, m);
        u = link_at(g, U, mu, m, &s);
        v = vec_at(g, chi, is_half, m);
        for (int i = 0; i < 3; ++i) {
            cplx acc = 0;
            for (int j = 0; j < 3; ++j) acc += conj(u[3 * j + i]) * v[j];
            out[i] -= 0.5 * e * s * acc;
        }
    }
}

void or_dslash(const int32_t dims[4], int32_t bc_t, const double* U, const double* in, double* out) {
    lattice g = make_lattice(dims, bc_t);
    for (int64_t s = 0; s < g.V; ++s) {
        int n[4];
        coords_of(&g, s, n);
        dslash_site(&g, (const cplx*)U, (const cplx*)in, 0, n, (cplx*)out + s * 3);
    }
}

void or_dslash_eo(const int32_t dims[4], int32_t bc_t, const double* U, const double* in, double* out,
                  int32_t out_parity) {
    lattice g = make_lattice(dims, bc_t);
    for (int64_t s = 0; s < g.V; ++s) {
        int n[4];
        coords_of(&g, s, n);
        if (parity_of(n) != out_parity) continue;
        dslash_site(&g, (const cplx*)U, (const cplx*)in, 1, n, (cplx*)out + (s >> 1) * 3);
    }
}

void or_dslash_eo_sites(const int32_t dims[4], int32_t bc_t, const double* U, const double* in,
                        int32_t out_parity, const int64_t* cbs, int64_t nsites, double* out) {
    lattice g = make_lattice(dims, bc_t);
    for (int64_t k = 0; k < nsites; ++k) {
        /* the lex index with this cb and parity is 2*cb or 2*cb+1 */
        int n[4];
        coords_of(&g, 2 * cbs[k], n);
        if (parity_of(n) != out_parity) coords_of(&g, 2 * cbs[k] + 1, n);
        dslash_site(&g, (const cplx*)U, (const cplx*)in, 1, n, (cplx*)out + k * 3);
    }
}

void or_apply_A(const int32_t dims[4], int32_t bc_t, const double* U, double mass, const double* x,
                double* y) {
    int64_t nh = (int64_t)dims[0] * dims[1] * dims[2] * dims[3] / 2;
    cplx* t = (cplx*)calloc((size_t)nh * 3, sizeof(cplx));
    or_dslash_eo(dims, bc_t, U, x, (double*)t, 1);  /* t_o = D_oe x_e */
    or_dslash_eo(dims, bc_t, U, (const double*)t, y, 0);  /* y_e = D_eo t_o */
    const cplx* xe = (const cplx*)x;
    cplx* ye = (cplx*)y;
    for (int64_t k = 0; k < nh * 3; ++k) ye[k] = mass * mass * xe[k] - ye[k];
    free(t);
}

/* <a, b> = sum conj(a) b, summed in order. */
static cplx dot(const cplx* a, const cplx* b, int64_t n) {
    cplx s = 0;
    for (int64_t k = 0; k < n; ++k) s += conj(a[k]) * b[k];
    return s;
}

static double norm2(const cplx* a, int64_t n) {
    double s = 0;
    for (int64_t k = 0; k < n; ++k) s += creal(a[k]) * creal(a[k]) + cimag(a[k]) * cimag(a[k]);
    return s;
}

int32_t or_cg_solve(const int32_t dims[4], int32_t bc_t, const double* U, double mass, const double* b,
                    double* x, double tol, int32_t max_iter, int32_t use_x0, int32_t* iters,
                    double* true_rel_resid) {
    int64_t n = (int64_t)dims[0] * dims[1] * dims[2] * dims[3] / 2 * 3;
    const cplx* bb = (const cplx*)b;
    cplx* xx = (cplx*)x;
    cplx* r = (cplx*)malloc((size_t)n * sizeof(cplx));
    cplx* p = (cplx*)malloc((size_t)n * sizeof(cplx));
    cplx* q = (cplx*)malloc((size_t)n * sizeof(cplx));
    int32_t status = 1, k = 0;
    double bnorm = sqrt(norm2(bb, n));

    if (!use_x0) memset(xx, 0, (size_t)n * sizeof(cplx));
    /* r = b - A x */
    or_apply_A(dims, bc_t, U, mass, x, (double*)q);
    for (int64_t i = 0; i < n; ++i) r[i] = bb[i] - q[i];
    double rho = norm2(r, n);
    if (bnorm == 0.0 || sqrt(rho) <= tol * bnorm) status = 0;
    for (int64_t i = 0; i < n; ++i) p[i] = r[i];

    while (status == 1 && k < max_iter) {
        or_apply_A(dims, bc_t, U, mass, (const double*)p, (double*)q);
        double pq = creal(dot(p, q, n));
        if (!(pq > 0.0) || !isfinite(pq)) {
            status = -6;
            break;
        }
        double alpha = rho / pq;
        for (int64_t i = 0; i < n; ++i) {
            xx[i] += alpha * p[i];
            r[i] -= alpha * q[i];
        }
        double rho_new = norm2(r, n);
        ++k;
        if (sqrt(rho_new) <= tol * bnorm) {
            /* apparent convergence: replace the iterated residual by the true one */
            or_apply_A(dims, bc_t, U, mass, x, (double*)q);
            for (int64_t i = 0; i < n; ++i) r[i] = bb[i] - q[i];
            rho_new = norm2(r, n);
            if (sqrt(rho_new) <= tol * bnorm) {
                status = 0;
                break;
            }
        }
        double beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }

    if (true_rel_resid) {
        or_apply_A(dims, bc_t, U, mass, x, (double*)q);
        for (int64_t i = 0; i < n; ++i) r[i] = bb[i] - q[i];
        *true_rel_resid = bnorm > 0 ? sqrt(norm2(r, n)) / bnorm : 0.0;
    }
    if (iters) *iters = k;
    free(r);
    free(p);
    free(q);
    return status;
}

/* out = a b^dag (3x3), out_ij = a_i conj(b_j), scaled by c and added. */
static void add_outer(cplx* out, double c, const cplx* a, const cplx* b) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) out[3 * i + j] += c * a[i] * conj(b[j]);
}

void or_grad(const int32_t dims[4], int32_t bc_t, const double* U, double mass, const double* x,
             const double* lambda, double* gamma, double* force, double* dmass) {
    lattice g = make_lattice(dims, bc_t);
    int64_t nh = g.V / 2;
    const cplx* xe = (const cplx*)x;
    const cplx* le = (const cplx*)lambda;
    cplx* yx = (cplx*)calloc((size_t)nh * 3, sizeof(cplx));
    cplx* yl = (cplx*)calloc((size_t)nh * 3, sizeof(cplx));
    or_dslash_eo(dims, bc_t, U, x, (double*)yx, 1);       /* y_x = D_oe x */
    or_dslash_eo(dims, bc_t, U, lambda, (double*)yl, 1);  /* y_l = D_oe lambda */

    cplx* G = (cplx*)gamma;
    for (int mu = 0; mu < 4; ++mu) {
        for (int64_t s = 0; s < g.V; ++s) {
            int n[4], m[4];
            double sgn;
            coords_of(&g, s, n);
            hop(&g, n, mu, +1, m);
            (void)link_at(&g, (const cplx*)U, mu, n, &sgn);
            double c = 0.5 * eta(mu, n) * sgn;
            cplx* out = G + ((int64_t)mu * g.V + s) * 9;
            for (int k = 0; k < 9; ++k) out[k] = 0;
            if (parity_of(n) == 0) {
                /* n even: lambda(n) y_x(n+mu)^dag + x(n) y_l(n+mu)^dag */
                add_outer(out, c, vec_at(&g, le, 1, n), vec_at(&g, yx, 1, m));
                add_outer(out, c, vec_at(&g, xe, 1, n), vec_at(&g, yl, 1, m));
            } else {
                /* n odd: -[y_x(n) lambda(n+mu)^dag + y_l(n) x(n+mu)^dag] */
                add_outer(out, -c, vec_at(&g, yx, 1, n), vec_at(&g, le, 1, m));
                add_outer(out, -c, vec_at(&g, yl, 1, n), vec_at(&g, xe, 1, m));
            }
        }
    }

    if (force) {
        /* F = TA(U Gamma^dag), TA(W) = (W - W^dag)/2 - tr(W - W^dag)/6 */
        const cplx* UU = (const cplx*)U;
        cplx* F = (cplx*)force;
        for (int64_t l = 0; l < 4 * g.V; ++l) {
            const cplx* u = UU + l * 9;
            const cplx* gm = G + l * 9;
            cplx w[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    cplx acc = 0;
                    for (int k = 0; k < 3; ++k) acc += u[3 * i + k] * conj(gm[3 * j + k]);
                    w[3 * i + j] = acc;
                }
            cplx tr = 0;
            for (int i = 0; i < 3; ++i) tr += w[4 * i] - conj(w[4 * i]);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) {
                    cplx v = 0.5 * (w[3 * i + j] - conj(w[3 * j + i]));
                    if (i == j) v -= tr / 6.0;
                    F[l * 9 + 3 * i + j] = v;
                }
        }
    }

    if (dmass) *dmass = -2.0 * mass * creal(dot(le, xe, nh * 3));
    free(yx);
    free(yl);
}

int32_t or_full_solve(const int32_t dims[4], int32_t bc_t, const double* U, double mass,
                      const double* src, double* psi, double tol, int32_t max_iter, int32_t* iters) {
    lattice g = make_lattice(dims, bc_t);
    int64_t nh = g.V / 2;
    const cplx* sf = (const cplx*)src;
    cplx* pf = (cplx*)psi;
    cplx* se = (cplx*)malloc((size_t)nh * 3 * sizeof(cplx));
    cplx* so = (cplx*)malloc((size_t)nh * 3 * sizeof(cplx));
    cplx* be = (cplx*)malloc((size_t)nh * 3 * sizeof(cplx));
    cplx* xe = (cplx*)calloc((size_t)nh * 3, sizeof(cplx));
    cplx* xo = (cplx*)malloc((size_t)nh * 3 * sizeof(cplx));
    /* split the source by parity */
    for (int64_t s = 0; s < g.V; ++s) {
        int n[4];
        coords_of(&g, s, n);
        cplx* dst = (parity_of(n) == 0 ? se : so) + (s >> 1) * 3;
        for (int c = 0; c < 3; ++c) dst[c] = sf[s * 3 + c];
    }
    /* b_e = m src_e - D_eo src_o */
    or_dslash_eo(dims, bc_t, U, (const double*)so, (double*)be, 0);
    for (int64_t k = 0; k < nh * 3; ++k) be[k] = mass * se[k] - be[k];
    int32_t st = or_cg_solve(dims, bc_t, U, mass, (const double*)be, (double*)xe, tol, max_iter, 0, iters,
                             NULL);
    /* psi_o = (src_o - D_oe psi_e) / m */
    or_dslash_eo(dims, bc_t, U, (const double*)xe, (double*)xo, 1);
    for (int64_t k = 0; k < nh * 3; ++k) xo[k] = (so[k] - xo[k]) / mass;
    for (int64_t s = 0; s < g.V; ++s) {
        int n[4];
        coords_of(&g, s, n);
        const cplx* srcv = (parity_of(n) == 0 ? xe : xo) + (s >> 1) * 3;
        for (int c = 0; c < 3; ++c) pf[s * 3 + c] = srcv[c];
    }
    free(se);
    free(so);
    free(be);
    free(xe);
    free(xo);
    return st;
}
