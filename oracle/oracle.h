/* FP64 CPU oracle for the even-odd staggered CG (test infrastructure only).
 *
 * This is the plain, slow, single-threaded reference that the GPU library is checked against. Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark load it; the GPU library never
 * links, includes or calls it, and the two share no source.
 *
 * The paper (Sec. 3, "CG Performance") runs a mixed-precision CG inverter for HYP-smeared staggered
 * quarks on 20^3x64 lattices but prints none of the operator's formulas. The definitions used here are
 * the standard staggered ones:
 *   (D chi)(n) = 1/2 sum_mu eta_mu(n) [ U_mu(n) chi(n+mu) - U_mu(n-mu)^dag chi(n-mu) ],
 *   eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z),
 * with D mapping even sites to odd and odd to even (D_oe, D_eo), and the even-site system
 *   A x_e = b_e,  A = m^2 - D_eo D_oe  (Hermitian positive definite for any links).
 *
 * Layout (natural, complex128 interleaved re/im):
 *   links  U[mu][lex][i][j], mu = 0..3 = x,y,z,t, lex = x + X*(y + Y*(z + Z*t));
 *   full vectors  v[lex][c];  half vectors v[cb][c], cb = lex >> 1 over sites of one parity.
 * dims = {X, Y, Z, T}, each even and >= 2. bc_t = 1 multiplies the t-links on the last time slice by -1
 * (antiperiodic in time), 0 is periodic.
 *
 * All pointers are host pointers owned by the caller. No function allocates memory that outlives the
 * call.
 */
#ifndef STAG_ORACLE_H
#define STAG_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Full-lattice staggered operator: out[V][3] = D in[V][3]. */
void or_dslash(const int32_t dims[4], int32_t bc_t, const double* U, const double* in, double* out);

/* Half operator: out (parity out_parity, [V/2][3]) = D_{p,1-p} in (parity 1-out_parity, [V/2][3]). */
void or_dslash_eo(const int32_t dims[4], int32_t bc_t, const double* U, const double* in, double* out,
                  int32_t out_parity);

/* The same half operator evaluated only at the nsites checkerboard indices cbs[] of parity out_parity;
 * out is [nsites][3]. */
void or_dslash_eo_sites(const int32_t dims[4], int32_t bc_t, const double* U, const double* in,
                        int32_t out_parity, const int64_t* cbs, int64_t nsites, double* out);

/* y_e = (m^2 - D_eo D_oe) x_e on even sites. */
void or_apply_A(const int32_t dims[4], int32_t bc_t, const double* U, double mass, const double* x,
                double* y);

/* Textbook FP64 CG on A x = b (even sites). On entry x holds the initial guess if use_x0, else it is
 * ignored and 0 is used. Stops when the true relative residual |b - A x| / |b| <= tol.
 * Returns 0 converged, 1 not converged within max_iter, -6 breakdown (Re<p,Ap> <= 0 or non-finite).
 * iters and true_rel_resid (nullable) receive the iteration count and the final true residual. */
int32_t or_cg_solve(const int32_t dims[4], int32_t bc_t, const double* U, double mass, const double* b,
                    double* x, double tol, int32_t max_iter, int32_t use_x0, int32_t* iters,
                    double* true_rel_resid);

/* Adjoint gradient of a real loss l(x), x = A^-1 b, given x and lambda = A^-1 (dl/dx):
 *   gamma[4][V][3][3] = dl/dU (complex convention dl/dRe + i dl/dIm),
 *   force[4][V][3][3] = TA(U gamma^dag) (nullable),
 *   *dmass = dl/dm = -2 m Re<lambda, x>. */
void or_grad(const int32_t dims[4], int32_t bc_t, const double* U, double mass, const double* x,
             const double* lambda, double* gamma, double* force, double* dmass);

/* Full-lattice solve (m + D) psi = eta_src via the even-odd system:
 *   b_e = m eta_e - D_eo eta_o;  A psi_e = b_e (CG to tol);  psi_o = (eta_o - D_oe psi_e) / m.
 * src and psi are full vectors [V][3]. Return code as or_cg_solve. */
int32_t or_full_solve(const int32_t dims[4], int32_t bc_t, const double* U, double mass,
                      const double* src, double* psi, double tol, int32_t max_iter, int32_t* iters);

#ifdef __cplusplus
}
#endif
#endif
