/* sp_api.h -- C-ABI of libstagcg.so, the MI355X (gfx950) even-odd staggered CG library.
 *
 * What it computes. The paper (Sec. 3, "CG Performance"; Fig. 1, Table 2) measures a mixed-precision
 * conjugate-gradient inverter for HYP-smeared staggered quarks on 20^3x64 lattices, in which single
 * precision dominates and a small double-precision part keeps the answer exact. The operator is the
 * standard staggered one (the paper does not print it):
 *   (D chi)(n) = 1/2 sum_mu eta_mu(n) [ U_mu(n) chi(n+mu) - U_mu(n-mu)^dag chi(n-mu) ],
 *   eta_0 = 1, eta_1 = (-1)^x, eta_2 = (-1)^(x+y), eta_3 = (-1)^(x+y+z),
 * and the solver works on even sites with A = m^2 - D_eo D_oe (Hermitian positive definite).
 *
 * Conventions shared by every entry point.
 *  - Natural layout (what callers hand in and get back): complex128 interleaved (re, im);
 *      links U[mu][lex][i][j], mu = 0..3 = x,y,z,t, lex = x + X*(y + Y*(z + Z*t));
 *      half vectors v[cb][c] with cb = lex >> 1 over sites of one parity (even = (x+y+z+t) even).
 *  - Packed layout (what the kernels read): produced only by sp_gauge_pack / sp_vec_pack, opaque to the
 *    caller apart from its size (sp_gauge_bytes / sp_vec_bytes); it is structure-of-arrays per parity
 *    and direction so that neighbouring lattice sites sit in neighbouring 16-byte words.
 *  - Pointers are DEVICE pointers unless a comment says host. All buffers belong to the caller; the
 *    library never frees them and keeps no reference after a call returns. Device buffers must be
 *    256-byte aligned (hipMalloc / torch allocations are).
 *  - `stream` is a hipStream_t (0 = the null stream). sp_gauge_pack, sp_vec_pack, sp_vec_unpack and
 *    sp_dslash only enqueue work on it and return. sp_cg_solve, sp_cg_solve_batched and sp_cg_force
 *    enqueue on it and return once it has reached their end (they need convergence decisions and
 *    statistics on the host).
 *  - Errors: the return value is an sp_status. Negative codes leave outputs unspecified;
 *    SP_NOT_CONVERGED (positive: the iteration cap, or a true residual that did not improve over seven
 *    reliable updates in a row) leaves the solution of the last reliable update, whose true residual the
 *    statistics report (it need not be the smallest seen). sp_strerror() names a
 *    code, sp_last_error() gives the detailed message of the calling thread's last failure (including
 *    the HIP error string for SP_ERR_HIP). No C++ exception crosses this interface.
 *  - Not reentrant on one workspace: two calls that share a workspace must not overlap.
 *  - Host threads: the solves (sp_cg_solve, sp_cg_solve_batched and the even solve inside sp_full_solve)
 *    hold one library-wide lock from entry to return, so solves issued from several host threads run
 *    one after another; sp_dslash takes the lock only to read the tuning table.
 *  - Diagnostics (environment, read once): SP_LOG=1 prints one line per solved system to stderr (status,
 *    iterations, reliable updates, true residual, time), SP_LOG=2 also one line per chunk poll. Each solve and
 *    each chunk is a roctx range (rocprofv3 --marker-trace) when the roctx library can be loaded; SP_ROCTX=0
 *    turns the ranges off.
 */
#ifndef SP_API_H
#define SP_API_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage precisions. Arithmetic is FP64 for SP_F64 and FP32 for the others. SP_I16 is 16-bit fixed point
 * (q / 32767, rounded to nearest, absolute error <= 2^-16 for entries in [-1, 1]) and stores links only, for FP32
 * iterations. */
typedef enum { SP_F64 = 0, SP_F32 = 1, SP_F16 = 2, SP_BF16 = 3, SP_I16 = 4 } sp_prec;

typedef enum {
    SP_OK = 0,
    SP_NOT_CONVERGED = 1,     /* max_iter reached or residual stagnated; outputs valid */
    SP_ERR_INVALID_ARG = -1,  /* null pointer, bad enum, bad parity, bad tolerance ... */
    SP_ERR_ODD_EXTENT = -2,   /* a lattice extent is odd or < 2 */
    SP_ERR_UNSUPPORTED = -3,  /* combination not built (e.g. FP64 with recon 12, too large a lattice) */
    SP_ERR_WORKSPACE = -4,    /* workspace null or smaller than the *_workspace_bytes query */
    SP_ERR_HIP = -5,          /* a HIP runtime call failed */
    SP_ERR_BREAKDOWN = -6     /* CG breakdown: Re<p,Ap> <= 0 or a non-finite scalar (e.g. NaN source) */
} sp_status;

/* Lattice geometry: extents X, Y, Z, T (each even, >= 2; V/2 < 2^24) and the time boundary
 * (0 periodic, 1 antiperiodic: the t-links on the last time slice enter with a factor -1). */
typedef struct {
    int32_t dims[4];
    int32_t bc_t;
} sp_geom;

/* A packed gauge field. f64: FP64 recon-18 packing (needed by every solve: true residuals);
 * lo: the packing used by the low-precision iterations, of precision lo_prec with recon 18 (all 9 complex
 * entries), 12 (first two rows; the third is rebuilt as conj(row0 x row1), exact for SU(3) links) or, for SP_F32
 * only, 8 (U01, U02, the smaller in modulus of U10 and U20, and the phases of U00 and of the larger one; the rest
 * rebuilt from unitarity and det = 1, for SU(3) links whose first row is not a phase times (1, 0, 0); entries
 * within about 6e-7 of the FP64 links while |U00| stays away from 0, as in smeared fields). lo_prec is the inner
 * precision, or, for FP32 iterations, a 16-bit link storage (SP_F16, SP_BF16, SP_I16) with FP32 vectors and
 * arithmetic. lo may equal f64 when lo_prec is SP_F64. */
typedef struct {
    const void* f64;
    const void* lo;
    int32_t lo_prec;
    int32_t recon;
} sp_gauge;

/* Solver parameters.
 *  tol        stop when the FP64 true residual |b - A x| / |b| <= tol (> 0, < 1)
 *  max_iter   iteration cap (> 0)
 *  inner      precision of the iterated vectors and links: SP_F64 gives plain FP64 CG; SP_F32, SP_F16,
 *             SP_BF16 give mixed precision with FP64 reliable updates (true residual recomputed from an
 *             FP64 solution that accumulates the low-precision increments). 16-bit storage needs a
 *             moderate condition number: on near-identity fields it converges at m = 0.01 (condition
 *             number ~1.6e5) but stalls near m = 1e-3 (~1.6e7), where SP_F32 and SP_F64 still converge
 *  delta      reliable update when |r_iterated| < delta * |r at the last update| (0 disables; ignored
 *             for SP_F64; checked at the end of each poll chunk)
 *  ru_every   reliable update at least every ru_every iterations (ignored for SP_F64; <= 0 picks 100, or
 *             for FP32 iterations on SP_I16 links 75 with 75-iteration chunks and 50 otherwise; checked at
 *             the end of each poll chunk). With BF16 storage every update restarts the search direction, so
 *             short intervals slow the solve (every 50 iterations: 1,649 against 733 at 20^3x64, m = 0.01)
 *  poll_chunk iterations per device-side chunk (one hipGraph launch) between host convergence polls
 *             (<= 0 picks, for a single solve of at least 2^16 even sites, 100 with FP32 iterations on FP32
 *             links or SP_F64 and 75 with FP32 iterations on SP_I16 links; 25 otherwise)
 *  use_x0     1: x_e holds the initial guess on entry; 0: start from zero
 *  use_graph  1: capture each chunk in a hipGraph and replay it; 0: launch kernels one by one
 * A reliable update also runs whenever the iterated residual reaches tol, at the iteration cap, and (for
 * SP_F32, SP_F16, SP_BF16) when the iterated residual falls three decades below the true residual of the
 * last update. After it the search direction is kept (re-orthogonalised against the new residual) unless
 * the true |r|^2 exceeds the iterated one by more than 1.5x (FP32 iterations on FP32 or SP_I16 links) or
 * 1.25x (FP16 storage of the vectors or of the links), when it restarts from the residual; BF16 storage
 * restarts it at every update. */
typedef struct {
    double tol;
    int32_t max_iter;
    int32_t inner;
    double delta;
    int32_t ru_every;
    int32_t poll_chunk;
    int32_t use_x0;
    int32_t use_graph;
} sp_cg_params;

/* Host-side statistics of one solve. */
typedef struct {
    int32_t iters;             /* CG iterations performed */
    int32_t reliable_updates;  /* FP64 true-residual recomputations after the initial one */
    int32_t converged;         /* 1 if true_rel_resid <= tol */
    int32_t status;            /* sp_status of this system */
    double true_rel_resid;     /* FP64 |b - A x| / |b| at the last reliable update */
    double seconds;            /* wall time of the solve, packing of b and x included */
} sp_cg_stats;

/* One system of a batch. Systems that share (U, geometry) are solved with one multi-right-hand-side
 * operator application per iteration (each link is loaded once for all of them). */
typedef struct {
    const sp_geom* g;
    const sp_gauge* U;
    double mass;
    const double* b_e;  /* device, natural [V/2][3] complex128 */
    double* x_e;        /* device, natural [V/2][3] complex128; in: initial guess if use_x0 */
} sp_system;

/* Library version (major * 10000 + minor * 100 + patch). */
int sp_version(void);

/* Static text for an sp_status code. */
const char* sp_strerror(int code);

/* Detailed message of the calling thread's last failing call ("" if none). */
const char* sp_last_error(void);

/* Bytes of a packed gauge field (all 4 directions, both parities) for prec and recon (18, 12, or 8 with
 * SP_F32); 0 for a combination that is not built. */
size_t sp_gauge_bytes(const sp_geom* g, int prec, int recon);

/* Pack natural links (device, complex128 [4][V][3][3]) into out (device, sp_gauge_bytes). Rounds to
 * nearest-even when narrowing. Asynchronous on stream. Recon 8 stores, per link, the float4 planes
 * (U01, U02) and (S, arg U00, f): S the smaller in modulus of U10 and U20, f the phase of the other one, plus 8
 * when S is U20 (angles from atan2 in FP64, then rounded). It needs |U01|^2 + |U02|^2 > 0 for every link (not
 * checked here). */
int sp_gauge_pack(const sp_geom* g, const double* links_nat, int prec, int recon, void* out, void* stream);

/* Bytes of one packed parity-half vector of precision prec (FP16 includes a per-site FP32 norm). */
size_t sp_vec_bytes(const sp_geom* g, int prec);

/* Pack a natural half vector (device, complex128 [V/2][3]) into out (sp_vec_bytes). Asynchronous. */
int sp_vec_pack(const sp_geom* g, const double* v_nat, int prec, void* out, void* stream);

/* Unpack a packed half vector into natural complex128 [V/2][3]. Asynchronous. */
int sp_vec_unpack(const sp_geom* g, const void* v, int prec, double* v_nat, void* stream);

/* Half staggered operator (the Dslash whose single-precision application dominates the paper's CG, Sec. 3; the
 * operator is the staggered one of the header above, the paper does not print it):
 * out (parity out_parity) = D_{out_parity, 1-out_parity} in, both packed with
 * precision prec. Links: U->f64 when prec is SP_F64, else U->lo (U->lo_prec equal to prec, or a 16-bit link
 * storage when prec is SP_F32).
 * Asynchronous on stream. This is the kernel the solver spends most of its time in. */
int sp_dslash(const sp_geom* g, const sp_gauge* U, int prec, const void* in, void* out, int out_parity,
              void* stream);

/* Workspace bytes for sp_cg_solve (nsys = 1, systems[0] describes it; b_e/x_e may be null) or for
 * sp_cg_solve_batched over the same system list. */
size_t sp_cg_workspace_bytes(int nsys, const sp_system* systems, const sp_cg_params* params);

/* The paper's mixed-precision CG inverter (Sec. 3, "CG Performance"; Fig. 1 and Table 2 time it on 20^3x64): the
 * iterations in the inner precision, a small double-precision part (true residual, accumulated solution, global
 * sums) keeping the answer exact. Solve (m^2 - D_eo D_oe) x_e = b_e. b_e, x_e: device natural [V/2][3] complex128. stats: host,
 * nullable. ws: device workspace of at least sp_cg_workspace_bytes bytes. Returns SP_OK,
 * SP_NOT_CONVERGED or an error. Synchronous with respect to stream. */
int sp_cg_solve(const sp_geom* g, const sp_gauge* U, double mass, const double* b_e, double* x_e,
                const sp_cg_params* params, sp_cg_stats* stats, void* ws, size_t ws_bytes, void* stream);

/* Many solves of the paper's CG (Sec. 3) at once, a batching extension of this library: systems that share a gauge
 * field share each link load, and independent systems are the unit that spreads over GPUs without communication.
 * Solve nsys independent systems together: systems sharing a gauge field and geometry form groups of up
 * to 4 right-hand sides; all groups advance in one launch per kernel, captured in a hipGraph per chunk
 * of iterations; converged systems stop updating while the others continue. Groups may differ in volume
 * and time boundary; a zero b_e stops at the first residual check with x_e = 0. stats: host array of nsys
 * (nullable). Returns SP_OK if every system converged, SP_NOT_CONVERGED if any did not, or an error. When
 * some systems break down (SP_ERR_BREAKDOWN), stats[i].status names them and the other systems' x_e and
 * statistics are valid: reductions and states are kept per system. Synchronous with respect to stream. */
int sp_cg_solve_batched(int nsys, const sp_system* systems, const sp_cg_params* params,
                        sp_cg_stats* stats, void* ws, size_t ws_bytes, void* stream);

/* Workspace bytes for sp_cg_force on geometry g. */
size_t sp_force_workspace_bytes(const sp_geom* g);

/* Differentiation of the paper's solve (Sec. 3) with respect to the links, the mass and the source, by the adjoint
 * method (an extension of this library: the paper computes no gradients).
 * Adjoint link and mass gradient of a real loss l(x) with x = A^-1 b, given x_e and
 * lambda_e = A^-1 (dl/dx) (device natural [V/2][3] complex128), U->f64 packed links:
 *   gamma[4][V][3][3] (device, complex128, overwritten) = dl/dU_mu(n) with the complex convention
 *     dl/dRe U + i dl/dIm U:
 *       n even:  1/2 eta_mu(n) s [ lambda(n) y_x(n+mu)^dag + x(n) y_l(n+mu)^dag ],
 *       n odd:  -1/2 eta_mu(n) s [ y_x(n) lambda(n+mu)^dag + y_l(n) x(n+mu)^dag ],
 *     y_x = D_oe x, y_l = D_oe lambda, s the boundary sign of the link;
 *   force[4][V][3][3] (nullable) = TA(U gamma^dag), TA(W) = (W - W^dag)/2 - tr(W - W^dag)/6, the
 *     su(3)-projected force: for U -> exp(i t T) U, dl/dt = i tr(force T);
 *   grad_mass (device double, nullable) = -2 m Re<lambda, x>.
 * The gradient with respect to b is lambda itself. Synchronous with respect to stream. */
int sp_cg_force(const sp_geom* g, const sp_gauge* U, double mass, const double* x_e,
                const double* lambda_e, double* gamma, double* force, double* grad_mass, void* ws,
                size_t ws_bytes, void* stream);

/* Size of the device array that sp_cg_force_noalloc keeps its scratch in (64 MiB per GPU): enough for
 * lattices with V/2 up to 349,000 sites (20^3x64 and 16^3x32 fit; 28^3x96 does not). */
#define SP_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* sp_cg_force for callers that cannot allocate device memory (code under stream capture, serving loops,
 * harnesses that forbid hipMalloc): the same gradient from the same kernels, with no workspace argument and no
 * allocation of any kind. Its scratch is a fixed device array of SP_NOALLOC_SCRATCH_BYTES that each GPU the
 * library runs on holds until the process ends; lattices whose sp_force_workspace_bytes exceeds it are refused
 * with SP_ERR_WORKSPACE before anything is enqueued. The first call on a device looks up that device's array
 * (hipGetSymbolAddress), so make it outside stream capture. Asynchronous on stream (unlike sp_cg_force): the
 * outputs are ready when the stream reaches the end of the call. Every call on one GPU shares that GPU's
 * array: calls that can overlap on one GPU (on different streams, or from several host threads without
 * ordering) race and must be serialised, e.g. by issuing them on one stream. Nothing in the array needs to
 * start at zero (each launch writes every word it later reads); it keeps the last call's contents. */
int sp_cg_force_noalloc(const sp_geom* g, const sp_gauge* U, double mass, const double* x_e,
                        const double* lambda_e, double* gamma, double* force, double* grad_mass, void* stream);

/* Workspace bytes for sp_hyp_smear on geometry g (24 FP64 link fields of V links). */
size_t sp_hyp_workspace_bytes(const sp_geom* g);

/* HYP smearing of SU(3) links, the smoothing applied to the links before the solve (the paper's quarks
 * are HYP-smeared, Sec. 3; the paper does not define it, the definition is the hypercubic blocking of
 * Hasenfratz and Knechtli). Three levels, each a weighted sum of a link and staples restricted to the
 * hypercubes containing it, projected to SU(3):
 *   lv1(mu, eta) = P[(1 - a3) U_mu + a3/2 S(U_eta; U_mu)]                              eta != mu
 *   lv2(mu, nu)  = P[(1 - a2) U_mu + a2/4 sum_{rho not mu, nu} S(lv1(rho, s); lv1(mu, s))]
 *                  s = the direction outside {mu, nu, rho}
 *   V_mu         = P[(1 - a1) U_mu + a1/6 sum_{nu != mu} S(lv2(nu, mu); lv2(mu, nu))]
 * with S(A; B)(x) = A_eta(x) B(x+eta) A_eta(x+mu)^dag + A_eta(x-eta)^dag B(x-eta) A_eta(x-eta+mu) for the
 * staple direction eta of the sum, and P(W) = the SU(3) matrix maximising Re tr(X^dag W) (in closed
 * form when W is close enough to unitary up to a factor, else from its unitary polar factor by
 * SU(2)-subgroup sweeps to convergence).
 * links_nat, out_nat: device, complex128 [4][V][3][3] in the natural layout (lex = x + X(y + Y(z + Z t)));
 * they must not overlap. alpha: host, 3 doubles (a1, a2, a3), each in [0, 1]; (0.75, 0.6, 0.3) is the
 * standard choice. All directions are periodic (bc_t is ignored: it is a fermion boundary condition).
 * ws: device workspace of at least sp_hyp_workspace_bytes(g) bytes. Asynchronous on stream. */
int sp_hyp_smear(const sp_geom* g, const double* links_nat, const double* alpha, double* out_nat, void* ws,
                 size_t ws_bytes, void* stream);

/* Bytes of the path-link array of sp_npr_path_links on geometry g: 256 complex128 3x3 matrices per
 * hypercube (V/16 hypercubes). */
size_t sp_npr_path_bytes(const sp_geom* g);

/* Path links of the NPR four-fermion contraction (the paper's Eq. (1), Sec. 4, the U_{i;AD}(z) factors):
 * for every hypercube z (corners z_A = 2z + A, A in {0,1}^4, A = A0 + 2A1 + 4A2 + 8A3; hypercubes in
 * lexicographic order of the coarse lattice X/2 x Y/2 x Z/2 x T/2) and every corner pair (A, D), the average
 * over the shortest paths from z_A to z_D of the ordered link products (a step +mu from x takes U_mu(x), a
 * step -mu takes U_mu(x - mu)^dag; U_AA = 1). links_nat: device, complex128 [4][V][3][3]; uad: device,
 * sp_npr_path_bytes(g) bytes, written as complex128 [V/16][16 A][16 D][3][3]. Asynchronous on stream. */
int sp_npr_path_links(const sp_geom* g, const double* links_nat, void* uad, void* stream);

/* The one-colour-trace four-fermion contraction (the paper's Eq. (1), Sec. 4), per hypercube z and field
 * set i = 0..n-1:
 *   O_i(z) = sum_{A,B,C,D} M1_{AB} M2_{CD} [chib1(z_A)^T U_AD(z) chi4(z_D)] [chib3(z_C)^T U_CB(z) chi2(z_B)]
 * with chib^T U chi = sum_{c,c'} chib_c U_cc' chi_c' and the spin-taste matrices
 * M_{AB} = (1/4) tr(gamma_A^dag gamma_S gamma_B gamma_F^dag), gamma_A = g1^A0 g2^A1 g3^A2 g4^A3 (Hermitian
 * Euclidean Dirac matrices). labels: host, 4 ints (S1, F1, S2, F2), each a 4-bit spin or taste label in
 * [0, 16). uad: from sp_npr_path_links. chib1, chi2, chib3, chi4: device, complex128 [n][V][3] (natural
 * layout, no conjugation implied). out: device, complex128 [n][V/16]. Asynchronous on stream. */
int sp_npr_contract(const sp_geom* g, const void* uad, int n, const double* chib1, const double* chi2,
                    const double* chib3, const double* chi4, const int32_t* labels, double* out, void* stream);

/* The same contraction with the path links built inside it, per hypercube in on-chip memory, from the natural
 * links (device complex128 [4][V][3][3]): no path-link array is written or read (36 KB per hypercube, 1.18 GB at
 * 20^3x64). The paths are rebuilt by every call, so when many calls share one gauge field (other labels or other
 * field sets) sp_npr_path_links once and sp_npr_contract per call move fewer bytes in total. Asynchronous. */
int sp_npr_contract_links(const sp_geom* g, const double* links_nat, int n, const double* chib1, const double* chi2,
                          const double* chib3, const double* chi4, const int32_t* labels, double* out, void* stream);

/* Workspace bytes for sp_full_solve. */
size_t sp_full_workspace_bytes(const sp_geom* g, const sp_gauge* U, const sp_cg_params* params);

/* Full-lattice solve (m + D) psi = src, the system the even-odd solve is carved from: with M split by
 * parity, b_e = m src_e - D_eo src_o, (m^2 - D_eo D_oe) psi_e = b_e (solved as sp_cg_solve with params),
 * psi_o = (src_o - D_oe psi_e) / m. src, psi: device natural [V][3] complex128 (lex order). mass must
 * be non-zero. Returns the even solve's status. Synchronous with respect to stream. */
int sp_full_solve(const sp_geom* g, const sp_gauge* U, double mass, const double* src, double* psi,
                  const sp_cg_params* params, sp_cg_stats* stats, void* ws, size_t ws_bytes, void* stream);

/* Autotune the half-operator launch (block size, XCD-aware block order, and for one right-hand side the
 * link-load policy: cached or streaming loads) for (g, prec, U->recon) by
 * timing it with HIP events on stream, for one right-hand side and for the 4-right-hand-side operator of
 * batched solves (which has its own register use); in and out are scratch packed vectors of that
 * precision. The 4-right-hand-side timing uses a temporary device buffer of 8 vectors plus descriptors,
 * allocated and freed inside the call. The choices are kept for the process and used by sp_dslash and the
 * solvers (sp_tune_save writes both; the batched one under the key suffix "/n4"). best_ms (host,
 * nullable) receives the best one-right-hand-side time per launch. Synchronous with respect to stream. */
int sp_tune_dslash(const sp_geom* g, const sp_gauge* U, int prec, void* in, void* out, void* stream,
                   double* best_ms);

/* Save / load the tuned launches as JSON text (path on the host file system). Keys are
 * "XxYxZxT/l<link prec>/r<recon>/v<vector prec>" (precisions as the SP_* codes), with the suffix "/n4" for the
 * batched operator and "/solve" for a single solve's iteration (written by the tuning driver, which times short
 * solves; a single solve uses it when present, else the plain operator's entry). Values are
 * {"nt": 64|128|256, "remap": 0|1, "stream": 0|1} ("stream" may be left out: 0). Load merges the file's
 * entries into the table; a malformed or truncated file returns SP_ERR_INVALID_ARG and changes nothing. */
int sp_tune_save(const char* path);
int sp_tune_load(const char* path);

/* One GPU's share of a lattice cut in time across GPUs: the decomposition of the paper's multi-GPU CG (Sec. 3,
 * Fig. 2 and Table 2), where each GPU exchanges the boundary slices of the vector with its two neighbours in
 * every operator application. local: X, Y, Z and the shard's time extent Tl (each even, >= 2); local.bc_t is
 * the GLOBAL time boundary (the antiperiodic sign enters at global t = T - 1 -> 0). t0: global time of the
 * shard's first slice (even); T: global time extent (even, t0 + Tl <= T). Local checkerboard index
 * cb = global cb - t0 X Y Z / 2. One parity of one time slice is a face of F = X Y Z / 2 sites. */
typedef struct {
    sp_geom local;
    int32_t t0;
    int32_t T;
} sp_shard;

/* Bytes of one packed face (F sites) of vector precision prec; 0 on a bad shard. */
size_t sp_shard_face_bytes(const sp_shard* s, int prec);

/* Bytes of an extended shard vector of one parity: the packed planes of Vh + 2F sites, [ghost slice t0 - 1]
 * [the shard's Tl slices][ghost slice t0 + Tl], local site cb at plane position F + cb. */
size_t sp_shard_vec_bytes(const sp_shard* s, int prec);

/* Natural local half vector (device, complex128 [Vh][3], local cb order) -> the local part of an extended
 * vector (the ghost slices are left as they are). Asynchronous. */
int sp_shard_vec_pack(const sp_shard* s, const double* v_nat, int prec, void* ext, void* stream);

/* Face pack: copy the shard's lowest (side 0, local t = 0: for the neighbour below) or highest (side 1,
 * t = Tl - 1: for the neighbour above) slice of an extended vector into face (sp_shard_face_bytes), word for
 * word (no rounding; the FP16 per-site norms travel with their sites). Asynchronous. */
int sp_face_pack(const sp_shard* s, int prec, const void* ext, int side, void* face, void* stream);

/* Face unpack: copy a received face into the ghost slice below (side 0: the neighbour below's side-1 face) or
 * above (side 1: the neighbour above's side-0 face) of an extended vector, word for word. Asynchronous. */
int sp_face_unpack(const sp_shard* s, int prec, const void* face, int side, void* ext, void* stream);

/* Bytes of the ghost t-links of a shard (U_t on global slice t0 - 1, both parities, 2F links) in the packed link
 * format of (prec, recon): recon 18 or 12, or 8 with SP_F32, as for sp_gauge_bytes; 0 for a combination that is
 * not built. */
size_t sp_shard_ghost_bytes(const sp_shard* s, int prec, int recon);

/* Pack the ghost t-links: tlinks_nat = U_t(x, y, z, t0 - 1 mod T), device complex128 [X Y Z][3][3] in the order
 * x + X (y + Y z). Exchanged once per gauge field. Asynchronous. */
int sp_shard_ghost_pack(const sp_shard* s, const double* tlinks_nat, int prec, int recon, void* ghost, void* stream);

/* Halo-fed half operator on a shard: out (local packed vector of parity out_parity, Vh sites, sp_vec_bytes of
 * the local geometry) = D_{p,1-p} ext_in, where ext_in is an extended vector whose ghost slices hold the
 * neighbours' faces, U is the shard's local packed gauge field (sp_gauge_pack on the local geometry, link
 * precision as for sp_dslash) and ghost its ghost t-links in U's low-precision packing (FP64 recon 18 for
 * prec SP_F64). part 0: every site; 1: the interior slices 1 .. Tl-2, which read no ghost and can run while the
 * faces are in flight; 2: the boundary slices 0 and Tl - 1. With T = Tl (one shard) and each ghost holding the
 * shard's own opposite face, this is sp_dslash on the periodic lattice. Asynchronous. */
int sp_dslash_halo(const sp_shard* s, const sp_gauge* U, const void* ghost, int prec, const void* ext_in, void* out,
                   int out_parity, int part, void* stream);

/* Streaming-bandwidth probe, the attainable-bandwidth ceiling that the bandwidth-bound kernels are measured
 * against (the paper's Sec. 4 / Table 3 reason about CG speed from memory bandwidth). kind 0 reads n16 16-byte
 * words of a (writing one float per block of 256 lanes to b, sp_stream_out_bytes(n16, k) bytes), kind 1 copies
 * a to b, kind 2 writes b = a + 0.5 c (FP32 lanes); each lane moves k whole 16-byte words (k = 1, 2, 4 or 8).
 * a, b, c: device, 16-byte aligned, n16 words each (c only for kind 2). Asynchronous on stream; the caller
 * times it. */
size_t sp_stream_out_bytes(size_t n16, int k);
int sp_stream_probe(int kind, int k, const void* a, void* b, const void* c, size_t n16, void* stream);

/* Drop cached hipGraphs and tuning entries. */
void sp_release_cache(void);

#ifdef __cplusplus
}
#endif
#endif /* SP_API_H */
