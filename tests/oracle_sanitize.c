/* Drives every oracle entry point once on small lattices so that a build with -fsanitize=address,undefined checks
 * the oracle's memory accesses and arithmetic (compiled and run by tests/test_sanitize_cpu.py). Exits non-zero if
 * a solve fails or a result is not finite; the sanitizers abort on any invalid access. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/oracle.h"

static uint64_t state = 88172645463325252ull;
static double uniform(void) { /* xorshift64, in [-1, 1) */
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) / 4503599627370496.0 - 1.0;
}

static int finite_all(const double* a, long n) {
    for (long i = 0; i < n; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

static int run(const int32_t dims[4], int32_t bc_t) {
    const long V = (long)dims[0] * dims[1] * dims[2] * dims[3];
    const long nU = 4 * V * 18, nF = V * 6, nH = V / 2 * 6;
    double* U = malloc(sizeof(double) * nU);
    double* full = malloc(sizeof(double) * nF);
    double* fout = malloc(sizeof(double) * nF);
    double* b = malloc(sizeof(double) * nH);
    double* x = malloc(sizeof(double) * nH);
    double* y = malloc(sizeof(double) * nH);
    double* lam = malloc(sizeof(double) * nH);
    double* gamma = malloc(sizeof(double) * nU);
    double* force = malloc(sizeof(double) * nU);
    /* links near the identity (the operator does not need unitary links: A stays positive definite) */
    for (long l = 0; l < 4 * V; ++l)
        for (int k = 0; k < 18; ++k) U[l * 18 + k] = (k % 8 == 0 ? 1.0 : 0.0) + 0.2 * uniform();
    for (long i = 0; i < nF; ++i) full[i] = uniform();
    for (long i = 0; i < nH; ++i) b[i] = uniform();
    int ok = 1;
    or_dslash(dims, bc_t, U, full, fout);
    ok &= finite_all(fout, nF);
    or_dslash_eo(dims, bc_t, U, b, y, 1);
    or_dslash_eo(dims, bc_t, U, b, y, 0);
    ok &= finite_all(y, nH);
    int64_t cbs[3] = {0, V / 4, V / 2 - 1};
    double ys[9 * 2];
    or_dslash_eo_sites(dims, bc_t, U, b, 1, cbs, 3, ys);
    ok &= finite_all(ys, 18);
    or_apply_A(dims, bc_t, U, 0.3, b, y);
    ok &= finite_all(y, nH);
    int32_t it = 0;
    double res = 0;
    int32_t st = or_cg_solve(dims, bc_t, U, 0.3, b, x, 1e-12, 5000, 0, &it, &res);
    ok &= st == 0 && res <= 1e-12;
    memcpy(lam, b, sizeof(double) * nH);
    st = or_cg_solve(dims, bc_t, U, 0.3, b, lam, 1e-10, 5000, 1, &it, &res); /* warm start */
    ok &= st == 0;
    double dm = 0;
    or_grad(dims, bc_t, U, 0.3, x, lam, gamma, force, &dm);
    or_grad(dims, bc_t, U, 0.3, x, lam, gamma, NULL, NULL);
    ok &= finite_all(gamma, nU) && finite_all(force, nU) && isfinite(dm);
    st = or_full_solve(dims, bc_t, U, 0.3, full, fout, 1e-11, 5000, &it);
    ok &= st == 0 && finite_all(fout, nF);
    /* iteration cap: status 1, not a crash */
    st = or_cg_solve(dims, bc_t, U, 0.01, b, x, 1e-14, 2, 0, &it, NULL);
    ok &= st == 1 && it == 2;
    printf("dims %dx%dx%dx%d bc_t %d: %s\n", dims[0], dims[1], dims[2], dims[3], bc_t, ok ? "ok" : "FAILED");
    free(U); free(full); free(fout); free(b); free(x); free(y); free(lam); free(gamma); free(force);
    return ok;
}

int main(void) {
    const int32_t lat[][4] = {{2, 2, 2, 2}, {4, 4, 4, 4}, {2, 4, 6, 8}, {6, 2, 4, 2}};
    int ok = 1;
    for (int i = 0; i < 4; ++i) {
        ok &= run(lat[i], 0);
        ok &= run(lat[i], 1);
    }
    printf(ok ? "ALL OK\n" : "FAILED\n");
    return ok ? 0 : 1;
}
