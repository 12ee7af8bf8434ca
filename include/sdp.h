/*
 * sdp.h -- C ABI of libsdp: chordal-decomposed primal ADMM for sparse SDPs on
 * one AMD Instinct MI355X (gfx950).
 *
 * Method: Zheng, Fantuzzi, Papachristodoulou, Goulart, Wynn, "Chordal
 * decomposition in operator-splitting methods for sparse semidefinite
 * programs", Algorithm 1 (ADMM for the domain-space decomposition of sparse
 * primal-form SDPs).
 *
 * The problem (the primal SDP of the Introduction, decomposed as in Section
 * "Domain-space decomposition"):
 *     minimise <C, X>  subject to  <A_i, X> = b_i (i = 1..m),
 *                                  E_k X E_k^T  PSD  for every maximal clique C_k
 * of the chordal aggregate sparsity pattern E (Theorem 1).
 *
 * Conventions shared by every entry point:
 *  - Symmetric matrices on the pattern are given by their lower-triangle
 *    coordinates (row >= col) sorted by column, then row; every diagonal
 *    entry (i, i) is present.  The pattern must equal the union of all clique
 *    pairs (a chordal graph or a chordal extension).
 *  - Cliques are 0-based vertex lists in strictly increasing order, at most
 *    128 vertices each.  In SDP_FP64, cliques of more than 96 vertices are
 *    projected by the matrix sign function (no eigenvectors), so the unrolled
 *    iterations refuse them (SDP_ERR_UNSUPPORTED).
 *  - A clique block X_k (s x s) is stored "packed": lower triangle row by
 *    row, entry (i, j), i >= j, at i*(i+1)/2 + j.
 *  - All functions return an int status: 0 = SDP_OK, >0 informational,
 *    <0 error.  No C++ exception crosses the boundary.  After a non-zero
 *    status, sdp_last_error() returns a thread-local message.
 */
#ifndef SDP_H
#define SDP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
enum {
  SDP_OK = 0,
  SDP_MAX_ITER = 1,              /* iteration limit reached before tol      */
  SDP_PRIMAL_INFEASIBLE = 2,     /* Algorithm 3: primal infeasibility certified */
  SDP_DUAL_INFEASIBLE = 3,       /* Algorithm 3: dual infeasibility certified   */
  SDP_ERR_ARG = -1,              /* bad size/pointer/ordering of an input   */
  SDP_ERR_PATTERN_UNCOVERED = -2,/* a pattern entry lies in no clique (D_jj=0) */
  SDP_ERR_OFF_PATTERN = -3,      /* a clique holds a pair not in the pattern */
  SDP_ERR_CLIQUE_ORDER = -4,     /* clique vertices not strictly increasing / out of range */
  SDP_ERR_RANK_DEFICIENT = -5,   /* A D^-1 A^T not positive definite (A_i dependent) */
  SDP_ERR_NONFINITE = -6,        /* NaN/Inf in A, b or C                    */
  SDP_ERR_UNSUPPORTED = -7,      /* clique too large for the chosen precision */
  SDP_ERR_HIP = -8,              /* a HIP runtime call failed (message has the HIP error) */
  SDP_ERR_OOM = -9               /* device allocation failed                */
};

enum { SDP_A_DENSE = 0, SDP_A_CSR = 1 };
/* precision of the PSD projections (eigensolve + rebuild); the affine step,
 * multipliers and residuals are always FP64 */
enum { SDP_FP64 = 0, SDP_FP32_EIG = 1 };
enum { SDP_DTYPE_FP64 = 0, SDP_DTYPE_FP32 = 1 };
/* which ADMM runs on the decomposed problem: Algorithm 1 (domain-space
 * decomposition of the primal form, Section 4.1), Algorithm 2 (range-space
 * decomposition of the dual form, Section 4.2) or Algorithm 3 (the
 * homogeneous self-dual embedding of the decomposed pair, Section 5) */
enum { SDP_ALG_PRIMAL = 0, SDP_ALG_DUAL = 1, SDP_ALG_HSDE = 2 };

typedef struct sdp_handle sdp_handle;   /* opaque; owns every device buffer it allocates */

/* One SDP instance.  Host memory, caller-owned, copied during sdp_setup. */
typedef struct {
  int32_t n;                    /* cone size                                   */
  int32_t m;                    /* number of equality constraints             */
  int64_t nnz_pattern;          /* number of lower pattern coordinates        */
  const int32_t *pat_row;       /* [nnz_pattern]                              */
  const int32_t *pat_col;       /* [nnz_pattern]                              */
  int32_t p;                    /* number of maximal cliques                  */
  const int32_t *clique_ptr;    /* [p+1], clique_ptr[0] = 0                   */
  const int32_t *clique_vert;   /* [clique_ptr[p]]                            */
  int32_t a_format;             /* SDP_A_DENSE: a_val is m x nnz_pattern row-major;
                                   SDP_A_CSR: a_rowptr/a_col/a_val over pattern coordinates */
  const int64_t *a_rowptr;      /* [m+1] (CSR only)                           */
  const int32_t *a_col;         /* [a_rowptr[m]] (CSR only)                   */
  const double *a_val;          /* lower-triangle values (A_i)_{row,col}      */
  const double *b;              /* [m]                                        */
  const double *c;              /* [nnz_pattern] lower-triangle values of C   */
} sdp_instance;

/* Solver options (Algorithm 1, first step: rho, eps_tol, n_max; adaptive
 * penalty parameters mu, nu of the Section "Adaptive penalty strategy"). */
typedef struct {
  double rho;                   /* initial penalty rho_0 (> 0)                */
  double tol;                   /* stop when max(eps_c, eps_lambda) <= tol    */
  int32_t max_iter;             /* n_max                                      */
  int32_t precision;            /* SDP_FP64 or SDP_FP32_EIG                   */
  int32_t adaptive_rho;         /* 0/1                                        */
  double mu, nu;                /* adaptive rule factors (>= 1)               */
  int32_t rho_period;           /* apply the rule every rho_period iterations */
  int32_t graph_chunk;          /* iterations per captured HIP graph (0: plain launches) */
  void *stream;                 /* hipStream_t to run on (NULL: the library's own stream) */
  int32_t jacobi_max_sweeps;    /* 0: default (30 for FP32, 40 for FP64)     */
  double jacobi_tol;            /* 0: default; off(A) <= tol * ||A||_F stops the sweeps */
  int32_t autotune;             /* 1: time the projection kernel variants per clique size
                                   at setup and keep the fastest (cached per process);
                                   0: smallest fitting block size */
  int32_t warm_start;           /* 1: each clique's eigen-solve starts from the eigenvector
                                   basis it ended with in the previous iteration (kept
                                   orthonormal on the device); 0: from the identity */
  int32_t algorithm;            /* SDP_ALG_PRIMAL (Algorithm 1) or SDP_ALG_DUAL (Algorithm 2:
                                   z_k = P+(v_k - lambda_k/rho), the KKT system with right-hand
                                   sides c - sum H_k^T(z_k + lambda_k/rho) and -b/rho,
                                   v_k = z_k + lambda_k/rho + H_k x, lambda_k += rho(z_k - v_k));
                                   the same factor, kernels and stopping rule) or
                                   SDP_ALG_HSDE (Algorithm 3: u_hat = (I+Q)^-1(u+v) by block
                                   elimination with the factor of I + A (I + D/2)^-1 A^T,
                                   u = P_K(u_hat - v), v += u - u_hat; stops on
                                   max(eps_p, eps_d, eps_g, eps_c) <= tol or on an
                                   infeasibility certificate; no penalty, so adaptive_rho
                                   must be 0) */
  int32_t cg_max_iter;          /* 0: the affine step solves with the cached Cholesky factor
                                   of A D^-1 A^T.  > 0 (Algorithm 1 only): no factor is
                                   formed; each iteration solves (A W D^-1 A^T) y = rhs by
                                   conjugate gradients with the Jacobi preconditioner
                                   diag(A W D^-1 A^T), started from the previous iteration's
                                   y, at most cg_max_iter steps (the iterative alternative of
                                   Section 4.1.1, for m where the m x m factor is too large;
                                   also lifts the m <= 20480 limit of sparse A) */
  double cg_tol;                /* the solve also stops once ||r||_2 <= cg_tol (1 + ||b||_2);
                                   0: always cg_max_iter steps */
  int32_t projection_method;    /* eigensolver of the clique projections: 0 the autotuner (or,
                                   with autotune = 0, the default variant) chooses, and the
                                   cliques listed under 3 take the sign function; 1 scalar parallel-order Jacobi only (FP64
                                   cliques of 97-128 still take the sign function, the only
                                   kernel for them); 2 the two-level (block) Jacobi wherever a
                                   variant for the clique size exists (blocks of 64 and more),
                                   scalar elsewhere; 3 the matrix sign function, X_k = (W + W sign(W)) / 2 (no eigenvectors, no
                                   warm start), for cliques of up to 32 vertices (in one
                                   wave's registers) and in SDP_FP64 for all cliques (larger
                                   ones with one block in LDS); the rest as with 0 */
  int32_t decouple;             /* 1 (SDP_FP32_EIG with warm_start = 1; blocks padded to 64
                                   and more; Algorithms 1-3 outside the unrolled iterations):
                                   a warm-started projection first separates the eigenspaces
                                   of the positive and the non-positive eigenvalues:
                                   simultaneous Jacobi rotations of the opposite-sign pairs of
                                   V^T W V, at most 2 refinements on the matrix cores; when
                                   the remaining opposite-sign mass is below the sweep
                                   tolerance and Gershgorin bounds certify both diagonal
                                   blocks, X is rebuilt from the positive block with no sweep;
                                   otherwise the Jacobi sweeps continue from the refined basis
                                   (and the clique skips the attempt for 4 iterations,
                                   doubling after each further failure in a row, up to 64;
                                   blocks of up to 96 with two or more failures in a row
                                   use the matrix sign function instead of sweeps while
                                   they wait).  The
                                   result is P+(W) to the sweep tolerance either way.  With
                                   projection_method = 0 those blocks then take the scalar
                                   variants (which carry the decoupling).  Ignored for FP64
                                   and smaller blocks.  0: sweeps only.  Default 1 */
} sdp_options;

/* Per-instance result. */
typedef struct {
  int32_t iters;                /* iterations executed                        */
  int32_t status;               /* SDP_OK (converged), SDP_MAX_ITER, or with
                                   Algorithm 3 SDP_PRIMAL_INFEASIBLE /
                                   SDP_DUAL_INFEASIBLE                        */
  double eps_c, eps_lambda;     /* residuals of the last iteration (Algorithm 3:
                                   eps_c = consensus residual, eps_lambda =
                                   max(eps_p, eps_d, eps_g))                   */
  double objective;             /* Algorithm 1: <C, X> = sum_j w_j c_j u_j;
                                   Algorithm 2: the dual objective b^T y;
                                   Algorithm 3: <C, X> with X = u_x / tau     */
  double rho;                   /* penalty after the last iteration (Algorithm 3: tau) */
  double eps_p, eps_d, eps_g;   /* primal/dual residuals and gap (NaN unless computed;
                                   Algorithm 3 computes them every iteration) */
  double eps_alpha;             /* PSD-completability violation (NaN unless computed) */
} sdp_result;

/* Fills *opt with defaults: rho 1, tol 1e-4, max_iter 20000, SDP_FP64,
 * adaptive off, mu 2, nu 10, rho_period 1, graph_chunk 25, own stream,
 * autotune on, warm_start on. */
void sdp_default_options(sdp_options *opt);

/* Validates `batch` instances, copies them to the device, builds the clique
 * index lists, the overlap counts D = sum_k H_k^T H_k (Section "Minimization
 * over X"), factors A D^-1 A^T = L L^T once in FP64 on the GPU and caches the
 * inverse factor, and sets X_k = Lambda_k = 0.  Instances are independent and
 * are iterated together.  On error nothing is allocated and *out is NULL. */
int sdp_setup(int32_t batch, const sdp_instance *inst, const sdp_options *opt,
              sdp_handle **out);

/* Restores the initial state (X_k = Lambda_k = 0, rho = rho_0, 0 iterations)
 * without redoing the factorisation. */
int sdp_reset(sdp_handle *h);

/* Enqueues n_steps iterations of Algorithm 1 on the handle's stream: the
 * x-update through the KKT system (OptCondMinYPrimal) with the cached factor,
 * the clique projections (XkUpdate), the multiplier update (LambdakUpdate),
 * the residuals (PrimalConsensusResidual) and the stopping test.  Instances
 * that have met the tolerance (or max_iter) stay frozen.  With res != NULL
 * (batch entries) it synchronises and fills the results; with res == NULL it
 * returns without synchronising. */
int sdp_admm_step(sdp_handle *h, int32_t n_steps, sdp_result *res);

/* Iterates until every instance meets the tolerance or max_iter (or, with
 * Algorithm 3, certifies infeasibility); fills res (batch entries).  Returns
 * SDP_MAX_ITER if an instance hit the limit, else the first infeasibility
 * status, else SDP_OK. */
int sdp_solve(sdp_handle *h, sdp_result *res);

/* Standalone PSD projection of `count` symmetric blocks (XkUpdate):
 * out_k = V diag(max(theta, 0)) V^T for in_k = V diag(theta) V^T.
 * sizes (int32[count]) and offsets (int64[count], element offsets of each
 * full s x s row-major block) are DEVICE pointers; in/out are device buffers
 * of `dtype`; every size must be <= max_size <= 128.  Blocks
 * must not overlap between in and out.  Asynchronous on `stream`.  Runs the
 * sign-function variant (sdp_projection_variant_kind = 2) of the smallest
 * block size that holds max_size: the same projection to the tolerance of
 * the Jacobi variants (1e-6 ||W||_F in FP32, 1e-14 in FP64), which
 * sdp_psd_project_variant still selects.  A block with a NaN or infinite
 * entry comes out all NaN (every variant). */
int sdp_psd_project_batched(int32_t count, int32_t max_size, const int32_t *sizes,
                            const int64_t *offsets, const void *in, void *out,
                            int32_t dtype, void *stream);

/* The projection kernel variants built for `dtype`: padded block size N and
 * threads per workgroup.  Writes up to `cap` entries and the number of
 * variants through *count (host only, no GPU work). */
int sdp_projection_variants(int32_t dtype, int32_t cap, int32_t *block_n, int32_t *threads,
                            int32_t *count);

/* The method of kernel variant `variant` of `dtype` (host only):
 *   *kind = 0  scalar parallel-order Jacobi;
 *   *kind = 1  two-level (block) Jacobi: groups of 8 indices paired
 *              round-robin, each pair's 16 x 16 problem diagonalised by one
 *              wave and applied to the block on the matrix cores;
 *   *kind = 2  matrix sign function, P+(W) = (W + W sign(W)) / 2, sign(W) by
 *              polynomial iterations on the matrix cores (k1 steps of
 *              X (3I - 3.2X^2 + 1.2X^4), then k2 of X (3I - X^2) / 2, as
 *              sdp_sign_schedule gives them).  It yields no eigenvectors: the
 *              standalone projections run it, and the solver's plans hold it
 *              only for the cliques of up to 32 vertices of Algorithms 1 and
 *              2 (projection_method 0 or 3; the one-wave variants of 16 and
 *              32), where the projection needs no eigenvectors; everything
 *              else in the solver is kind 0 or 1. */
int sdp_projection_variant_kind(int32_t dtype, int32_t variant, int32_t *kind);

/* The steps of the sign iteration for blocks of n vertices and a tolerance
 * tol relative to ||W||_F (host only): *k1 fast steps
 * X <- X (3I - 3.2X^2 + 1.2X^4) (three matrix products each) from
 * X0 = W / ||W||_F, then *k2 >= 2 Newton-Schulz steps X <- X (3I - X^2) / 2
 * (two products each), and one product for W sign(W).  The schedule is the
 * fewest products for which the error of P+(W) = (W + W sign(W)) / 2, in exact
 * arithmetic, stays within tol ||W||_F / 2 in the Frobenius norm (each
 * eigenvalue follows the scalar maps; the bound takes n - 1 eigenvalues at
 * the worst point of a fine grid).  FP32-eig's default tolerance 1e-6 gives
 * (12, 2) for n = 16; FP64's 1e-14 gives (29, 2).  Tolerances below 1e-16
 * are taken as 1e-16.  SDP_ERR_ARG if n < 1 or a pointer is NULL. */
int sdp_sign_schedule(double tol, int32_t n, int32_t *k1, int32_t *k2);

/* The variant sdp_psd_project_batched runs for blocks of up to max_size
 * (host only): the sign-function variant of the smallest block size that
 * holds max_size, the one-wave register kernel where there are several
 * (blocks of 16 and 32).  SDP_ERR_UNSUPPORTED if max_size is out of range
 * for dtype. */
int sdp_projection_default_variant(int32_t dtype, int32_t max_size, int32_t *variant);

/* sdp_psd_project_batched with an explicit kernel variant (an index into the
 * list of sdp_projection_variants); max_size must not exceed that variant's
 * N.  The result is the same projection (to the tolerance); the variants
 * differ in the method (sdp_projection_variant_kind) and in how the work is
 * spread over the workgroup. */
int sdp_psd_project_variant(int32_t variant, int32_t count, int32_t max_size,
                            const int32_t *sizes, const int64_t *offsets, const void *in,
                            void *out, int32_t dtype, void *stream);

/* Copies instance `inst`'s iterate to host memory (any pointer may be NULL):
 * u[nnz_pattern] the lower values of X; y_dual[m] = -rho*y (the dual
 * multipliers of <A_i, X> = b_i); Xk/Lk the packed clique blocks of all p
 * cliques concatenated.  With SDP_ALG_DUAL: u = -rho x (the primal matrix
 * estimate; x is the KKT variable of Algorithm 2), y_dual = y (the dual
 * variable itself), Xk = z_k, Lk = lambda_k.  With SDP_ALG_HSDE: u = u_x / tau,
 * y_dual = u_y / tau (u_x and u_y themselves -- the certificates up to scale --
 * when tau = 0), Xk = u_s, Lk = v_z.  Synchronises. */
int sdp_get_solution(sdp_handle *h, int32_t inst, double *u, double *y_dual,
                     double *Xk_packed, double *Lk_packed);

/* Overwrites instance `inst`'s clique blocks (packed, host memory) and its
 * penalty (rho > 0) -- a warm start.  With SDP_ALG_DUAL the blocks are z_k
 * and lambda_k, and the slack blocks v_k are set to z_k.  Synchronises. */
int sdp_set_state(sdp_handle *h, int32_t inst, const double *Xk_packed,
                  const double *Lk_packed, double rho);

/* Per-instance residual history of the iterations run since setup/reset:
 * eps_c, eps_lambda and the rho used (Algorithm 3: eps_c, max(eps_p, eps_d,
 * eps_g) and tau), up to `cap` entries each (any pointer may be NULL).
 * Returns the number of entries written through *count. */
int sdp_get_history(sdp_handle *h, int32_t inst, int32_t cap, double *eps_c,
                    double *eps_lambda, double *rho, int32_t *count);

/* Computes the diagnostics eps_p, eps_d, eps_g (HSDEerror, with
 * z = sum_k H_k^T lambda_k) and eps_alpha (PSD-violation) of the current
 * iterate on the GPU and stores them in res (batch entries). */
int sdp_diagnostics(sdp_handle *h, sdp_result *res);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the same
 * diagnostics as sdp_diagnostics, with the same results, but every scratch
 * vector lives in one static device array of 2^21 doubles (16 MiB) that the
 * library holds on each GPU it runs on until the process ends; the call
 * makes no hipMalloc, hipFree or other device allocation.  The handle needs
 * 3 doubles per coordinate slot, 2 per row slot and 1 per clique (slots are
 * the 64-padded counts of all instances); a larger handle returns
 * SDP_ERR_UNSUPPORTED without launching anything.  The first call on a
 * device looks up the array's address there (SDP_ERR_HIP if that fails).
 * Every call on one GPU shares the array and overwrites what the previous
 * call left (all of it is written before it is read): calls that overlap in
 * time on one GPU, from several threads or on several streams, race.
 * Synchronises the handle's stream. */
int sdp_diagnostics_noalloc(sdp_handle *h, sdp_result *res);

/* Statistics since setup/reset: total Jacobi sweeps and clique projections run. */
int sdp_get_stats(sdp_handle *h, int64_t *jacobi_sweeps, int64_t *projections);

/* The same statistics plus the number of projections since setup/reset that
 * took the matrix sign function as the fallback of a clique whose
 * decoupling certificate failed twice or more in a row (option decouple).
 * Any pointer may be NULL. */
int sdp_get_projection_stats(sdp_handle *h, int64_t *jacobi_sweeps, int64_t *projections,
                             int64_t *sign_fallbacks);

/* The projection launch plan chosen at setup: one entry per launch list, with
 * the padded block size N, the threads per workgroup NT and the number of
 * cliques it covers.  Writes up to `cap` entries (pointers may be NULL when cap
 * is 0) and the number of lists through *count. */
int sdp_projection_plan(sdp_handle *h, int32_t cap, int32_t *block_n, int32_t *threads,
                        int32_t *cliques, int32_t *count);

/* The kernel variant (index into sdp_projection_variants for the handle's
 * precision) of each launch list of sdp_projection_plan, same order. */
int sdp_projection_plan_variants(sdp_handle *h, int32_t cap, int32_t *variant, int32_t *count);

/* Times every stage of the iteration on its own: stage s is launched n_iter
 * times back to back between two HIP events on the handle's stream (stages
 * in iteration order), and ms[s] receives the mean milliseconds per launch:
 * 0 scatter (bhat), 1 A v - b (B v - L^-1 b for dense A), 2 L^-1 r, 3 L^-T y1
 * (2 and 3 only for sparse-A instances), 4 u = (bhat - A^T y)/D, 5 clique
 * projections with the multiplier update (all launch lists), 6 residual
 * reduction.  Stages 0-4 recompute the same outputs on every launch; stages 5
 * and 6 advance X_k, Lambda_k and the iteration counters n_iter times, so afterwards the state is no longer
 * an iterate of Algorithm 1 (sdp_reset or sdp_set_state before solving
 * again).  Synchronises. */
int sdp_time_stages(sdp_handle *h, int32_t n_iter, double *ms);

/* ---- differentiation of the unrolled iteration ---------------------------
 * The map (C, b) -> u_T: T iterations of Algorithm 1 from X_k = Lambda_k = 0
 * with fixed rho and no stopping test (A and the factor are held fixed).
 * The reverse sweep applies, iteration by iteration, the adjoints of the
 * multiplier update (LambdakUpdate), of the projection (XkUpdate, through the
 * derivative of the PSD projection in eigenvector divided-difference form),
 * of the gather/scatter with the entry selectors H_k and of the KKT solve
 * (OptCondMinYPrimal; self-adjoint in bhat, so one more solve with b = 0).
 * Per-instance vectors are concatenated over the batch: c and u as
 * [nnz_pattern of instance 0, instance 1, ...], b as [m_0, m_1, ...]. */

/* Replaces C and/or b of every instance (DEVICE pointers in the concatenated
 * layout above; either may be NULL).  The factor does not depend on them. */
int sdp_update_data(sdp_handle *h, const double *c, const double *b);

/* Runs the T unrolled iterations from the initial state, keeping X_k and
 * Lambda_k every ckpt_every iterations for the reverse sweep, and copies u_T
 * to u_out (DEVICE, concatenated layout; may be NULL).  Needs adaptive_rho = 0,
 * SDP_ALG_PRIMAL, the cached factor and cliques of up to 128 vertices in
 * SDP_FP32_EIG or 96 in SDP_FP64 (SDP_ERR_UNSUPPORTED otherwise).
 * Leaves the handle at iterate T.  Synchronises. */
int sdp_unrolled_forward(sdp_handle *h, int32_t T, int32_t ckpt_every, double *u_out);

/* Vector-Jacobian product of the last sdp_unrolled_forward: given the
 * cotangent u_bar of u_T, writes c_bar and b_bar (all DEVICE, concatenated
 * layout).  With euclidean = 0 the cotangents of u and c are taken w.r.t. the
 * Frobenius inner product of the symmetric matrices (off-diagonal coordinates
 * weighted by 2); with euclidean = 1 w.r.t. the plain dot product of the
 * compact vectors (what an autodiff framework uses).  Segments between
 * checkpoints are recomputed forward, storing each projection's eigenvectors
 * (FP32 in the SDP_FP32_EIG form), then reversed; the projection adjoints run
 * on the matrix cores for cliques of up to 128 vertices in FP32 and 96 in
 * FP64 (larger ones: sdp_unrolled_forward returns SDP_ERR_UNSUPPORTED).  The
 * handle's iterate is unspecified afterwards (call
 * sdp_reset before solving again).  Synchronises. */
int sdp_vjp(sdp_handle *h, const double *u_bar, double *c_bar, double *b_bar,
            int32_t euclidean);

/* Conjugate-gradient steps taken over all instances since the last reset
 * (0 when the handle uses the factor).  Synchronises. */
int sdp_cg_steps(sdp_handle *h, int64_t *steps);

/* Releases every device buffer of the handle. */
void sdp_destroy(sdp_handle *h);

/* Thread-local message of the last non-zero status ("" if none). */
const char *sdp_last_error(void);

/* ---- generic sparsity patterns (host only, no device work) -------------- */
/* A pattern that is not chordal is first replaced by a chordal extension
 * whose maximal cliques define the decomposition (Theorem 1; Section 7.1.1
 * describes this preprocessing).  The extension computed here is the filled
 * graph of a symbolic Cholesky elimination under a greedy minimum-degree
 * order (ties broken by the smaller vertex label); its maximal cliques are
 * read off that perfect elimination order.  Both are deterministic. */
typedef struct sdp_pattern sdp_pattern;   /* opaque; host memory only */

/* Builds the chordal extension of the symmetric pattern on n vertices given
 * by nnz coordinates (row[k], col[k]) in [0, n) (either triangle, duplicates
 * and diagonal entries allowed; the diagonal is always part of the result).
 * On success *out owns the result (release with sdp_pattern_destroy);
 * SDP_ERR_ARG for n <= 0, nnz < 0, NULL arrays or coordinates out of range. */
int sdp_pattern_create(int32_t n, int64_t nnz, const int32_t *row, const int32_t *col,
                       sdp_pattern **out);

/* Sizes of the result: *nnz_ext lower coordinates of the extended pattern,
 * *p maximal cliques holding *clique_total vertices in all.  Any output
 * pointer may be NULL. */
int sdp_pattern_sizes(const sdp_pattern *pat, int64_t *nnz_ext, int32_t *p,
                      int64_t *clique_total);

/* Copies the result into caller arrays (each may be NULL to skip it):
 * pat_row/pat_col [nnz_ext] the extended lower pattern in the order
 * sdp_instance expects (sorted by column, then row, every diagonal present);
 * clique_ptr [p + 1] and clique_vert [clique_total] the maximal cliques,
 * vertices increasing, cliques in lexicographic order.  With index_out
 * non-NULL, each of the nnz coordinates (row[k], col[k]) (either triangle)
 * is mapped to its position in the extended pattern (always found for a
 * coordinate of the original pattern; -1 if not in the extension). */
int sdp_pattern_get(const sdp_pattern *pat, int32_t *pat_row, int32_t *pat_col,
                    int32_t *clique_ptr, int32_t *clique_vert, int64_t nnz,
                    const int32_t *row, const int32_t *col, int64_t *index_out);

/* Releases the pattern (NULL is ignored). */
void sdp_pattern_destroy(sdp_pattern *pat);

/* ---- data scaling (host only, no device work) --------------------------- */
/* Section 7.1.3: the problem is rescaled by positive diagonal matrices on the
 * variable (preserving the cone) and on the equality constraints and by
 * positive scalars on b and C, so that the rows of A and b have norms near one
 * and the columns of A and c similar norms.  The variable scaling used here
 * is a congruence X -> S X S by one positive diagonal S over the vertices,
 * which keeps the pattern and every clique block's PSD cone:
 *     A'_i = e_i S A_i S,   b'_i = rho_b e_i b_i,   C' = sigma_c S C S.
 * The scaled instance has the same pattern, cliques and A layout, so the
 * solver runs on it unchanged; its tolerance then applies to the scaled
 * problem. */

/* Computes e [m] (row_scale), s [n] (vertex_scale), rho_b and sigma_c: iters
 * Ruiz iterations from e = s = 1, each taking ||A'_i||_F and the norm of
 * vertex v's row over all A'_i on the current scaled A and dividing e_i and
 * s_v by the square roots of those norms (zero norms leave the factor alone;
 * factors clamped to [1e-4, 1e4]); then rho_b = mean row norm / ||E b||_2 and
 * sigma_c = mean vertex norm / ||S C S||_F (denominators at least 1e-4, results
 * clamped to [1e-4, 1e4]).  The instance's cliques are not read.
 * SDP_ERR_ARG / SDP_ERR_NONFINITE on invalid data. */
int sdp_scale_compute(const sdp_instance *inst, int32_t iters, double *row_scale,
                      double *vertex_scale, double *rho_b, double *sigma_c);

/* Writes the scaled data: a_val_out in the instance's own A layout (dense
 * m x nnz_pattern, or the CSR values in a_col order), b_out [m], c_out
 * [nnz_pattern]; each may be NULL.  The scalings are the caller's (from
 * sdp_scale_compute or any positive values). */
int sdp_scale_apply(const sdp_instance *inst, const double *row_scale, const double *vertex_scale,
                    double rho_b, double sigma_c, double *a_val_out, double *b_out,
                    double *c_out);

/* Maps a solution of the scaled problem back, in place: x [nnz_pattern] (the
 * lower pattern values of X) to S X S / rho_b, y [m] to E y / sigma_c and
 * z [nnz_pattern] (of Z = C - sum y_i A_i) to S^-1 Z S^-1 / sigma_c; each may
 * be NULL.  Only n, m and the pattern of inst are read. */
int sdp_scale_recover(const sdp_instance *inst, const double *row_scale, const double *vertex_scale,
                      double rho_b, double sigma_c, double *x, double *y, double *z);

#ifdef __cplusplus
}
#endif
#endif /* SDP_H */
