// Internal declarations shared by the libsdp translation units.
//
// Device data layout (all instances of a batch concatenated):
//  * coordinate space: instance i owns `ld` consecutive slots starting at
//    coord_off (ld = nnz rounded up to a multiple of 64; padding slots have
//    D = 1, c = 0, w/D = 0 and no contributors, so they stay exactly zero).
//    Arrays: c, D, wd (= w/D), bhat, v (= wd*bhat), u, coord_inst.
//  * row space: instance i owns `ldm` slots (m rounded up to 64) from row_off.
//    Arrays: b, r (= A v - b), y1 (= L^-1 r), y (= L^-T y1).
//  * dense A: row-major m x ld per instance at a_off (zero padded).
//    CSR A: global row pointers (int64) with instance-local column indices,
//    plus a CSC copy for A^T y.
//  * factor: T = L^-1 (row-major, pitch ldm, zero above the diagonal) and its
//    transpose U = L^-T (zero below the diagonal), both at t_off.
//  * cliques: global list; packed lower blocks X, Lambda (FP64) at cl_off;
//    blk_loc maps a packed entry to its global coordinate; the contributor
//    CSR (coordinate -> packed entries, sorted by clique) drives the scatter.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define SDP_WAVE 64
// per-clique partial sums: ||X_k - H_k x||^2, ||X_k||^2, ||H_k x||^2,
// ||X_k - X_k^prev||^2, ||Lambda_k||^2 (full Frobenius), Jacobi sweeps
#define NPART 8   // (Algorithm 3 uses seven: two consensus residuals need three norms each)

struct InstDesc {
  int32_t n, m, p, a_format;
  int32_t ld;          // padded coordinate count (pitch of dense A)
  int32_t ldm;         // padded row count (pitch of T)
  int64_t nnz;
  int64_t coord_off;
  int64_t row_off;
  int64_t a_off;       // dense: element offset; csr: offset into row pointer array
  int64_t t_off;
  int64_t clique_off;  // first global clique
};

// Per-instance mutable scalars live in one struct array on the device.
struct InstState {
  double rho;
  double eps_c, eps_l;
  double total_sweeps;
  double total_sign;   // projections that took the sign-function fallback
  int32_t iter;
  int32_t done;        // 1: converged, 2: iteration limit reached,
                       // 3: primal infeasible, 4: dual infeasible (Algorithm 3)
};

// Affine step by preconditioned conjugate gradients: per-instance scalars
// of the current solve.
struct CgState {
  double rz;           // r^T z (z = r / diag(A W D^-1 A^T))
  double rn2;          // ||r||^2
  int32_t steps;       // steps taken in this iteration's solve
  int32_t done;        // 1: this iteration's solve has stopped
  int64_t total;       // steps since the last reset
};

// Algorithm 3 (homogeneous self-dual embedding): per-instance scalars.
struct HsdeState {
  double tau, kappa;   // u_tau and v_kappa
  double w2;           // tau + kappa of the current iterate (omega_2)
  double kz;           // 1 / (1 + zeta^T M^-1 zeta)
  double f;            // kz * zeta^T sigma of the current iteration
  double nrm_b, nrm_c; // ||b||, ||c|| (full-vector norms)
  double rp2, ax2, bty, ctx;   // row-space pieces of the residuals (u, not divided by tau)
  double eps_p, eps_d, eps_g;
};

struct SolverParams {
  double tol;
  double mu, nu;
  int32_t max_iter;
  int32_t adaptive;
  int32_t rho_period;
  int32_t hist_cap;    // capacity of the per-instance history ring
  int32_t no_stop;     // unrolled iterations: no stopping test, no penalty change
};

// ----------------------------------------------------------------------------
// Projection (k_project.hip)
// ----------------------------------------------------------------------------
struct ProjArgs {
  const int32_t *cl_inst;
  const int32_t *cl_size;
  const int64_t *cl_off;
  const int32_t *blk_loc;
  const double *u;
  double *X;
  double *Lam;
  double *part;        // NPART doubles per clique
  const InstState *state;
  int max_sweeps;
  double tol;
  // positive/negative decoupling of warm-started blocks: on/off, refinements
  // per attempt, iterations a clique skips it after a failed attempt, bound
  // on ||T||_F^2 for one Newton-Schulz step
  int decouple, dec_max_ref, dec_skip;
  int sign_k1, sign_k2;   // sign-function steps for cliques whose decoupling keeps failing
  double dec_tmax2;
  void *eig;              // optional: per clique V (s x N) then theta (N), precision T
  const int64_t *eig_off; // element offset of each clique's record in eig
  void *vw;               // optional: per clique N x N eigenvector basis (warm start), T
  int ns_period;          // the basis is re-orthonormalised every ns_period-th iteration
  int ns_shift;           // (of iteration + ns_shift; 0 except in the stage timing)
  const int64_t *vw_off;  // element offset of each clique's basis in vw
  // Algorithm 2 (range-space dual ADMM): X holds z_k, Lam holds lambda_k and
  // Vd the slack blocks v_k (packed lower, like X); the projection input is
  // v_k - lambda_k / rho and the multiplier update runs in launch_dual_update
  int dual;
  double *Vd;
  // Algorithm 3 (HSDE): X holds u_s, Lam holds v_z; the projection input is
  // u_hat_s - v_z with u_hat_s = (nu_s - nu_t + H sigma_x) / 2 - f M^-1 zeta_s,
  // and the epilogue also writes u_t = u_hat_t and the consensus partials
  int hsde;
  const HsdeState *hs;
  const double *h_ns, *h_nt, *h_sx, *h_ux, *h_mzs, *h_mzt;
  double *h_ut;
};

// Kernel variants (padded size N, threads NT): ids are per precision.
int projection_variant_count(int precision);
void projection_variant_info(int precision, int variant, int *N, int *NT);
// 1: two-level (block) Jacobi with 16 x 16 pair problems; 0: scalar rounds
int projection_variant_two_level(int precision, int variant);
// 0 scalar Jacobi, 1 two-level Jacobi, 2 sign function (standalone only)
int projection_variant_kind(int precision, int variant);
int projection_default_variant(int precision, int s);   // -1 if s is too large (Jacobi)
// Steps of the sign iteration for blocks of n vertices and a tolerance
// relative to ||W||_F: k1 fast steps, k2 Newton-Schulz steps (cached per
// (tol, n); thread-safe)
void sign_schedule(double tol, int n, int *k1, int *k2);
int projection_standalone_variant(int precision, int s);  // sign function where built
hipError_t fill_random_blocks(int precision, void *out, int s, int count, uint32_t seed,
                              double offdiag, hipStream_t st);
// Sets the warm-start bases of cliques [c0, c0 + count) to the identity.
hipError_t launch_identity_bases(int precision, void *vw, const int64_t *vw_off,
                                 const int32_t *cl_n, int64_t c0, int64_t count, hipStream_t st);

// Launch the ADMM projection for the cliques in `list` (all handled by one
// kernel variant).  precision: 0 = FP64, 1 = FP32.  split_ws: the list's
// workspace of split_workspace(precision, variant, count) doubles where that
// is positive and the list is the plan's only one (the sign iteration split
// over workgroups), else nullptr.
hipError_t launch_admm_projection(int precision, int variant, const int32_t *list,
                                  int count, const ProjArgs &a, hipStream_t st,
                                  double *split_ws = nullptr);
// Doubles of workspace the split sign iteration needs for `count` cliques of
// this variant; 0 where the list takes one workgroup per clique (FP32,
// blocks below 96, or enough cliques to fill the chip).
int64_t split_workspace(int precision, int variant, int count);

// Standalone batched projection of full row-major blocks.
hipError_t launch_standalone_projection(int dtype, int variant, int count,
                                        const int32_t *sizes, const int64_t *offsets,
                                        const void *in, void *out, int max_sweeps,
                                        double tol, hipStream_t st);

// Algorithm 2: v_k = z_k + lambda_k / rho + H_k x (vkEqn), lambda_k += rho
// (z_k - v_k) (MultUpdateDualSDP) and the residual partials ||z - v||^2,
// ||z||^2, ||v||^2, ||lambda||^2 of every clique (||z - z_prev||^2 and the
// sweeps come from the projection).  x is a.u.
hipError_t launch_dual_update(const ProjArgs &a, int64_t ncl, hipStream_t st);

// Minimum eigenvalue of each E_k U E_k^T (for eps_alpha; with a.dual of
// E_k (-rho x) E_k^T); FP64.
hipError_t launch_min_eig(int precision, int variant, const int32_t *list, int count,
                          const ProjArgs &a, double *lmin_out, hipStream_t st);

int projection_bucket(int precision, int s);   // N of the default variant, 0 if unsupported
int projection_max_size(int precision);

// ----------------------------------------------------------------------------
// Affine step and reductions (k_affine.hip)
// ----------------------------------------------------------------------------
struct AffineArgs {
  const InstDesc *inst;
  InstState *state;
  SolverParams params;
  // coordinate space
  const int32_t *coord_inst;
  const double *c, *D, *w;
  double *bhat, *v, *u;
  const int64_t *contrib_ptr;
  const int32_t *contrib_idx;
  const double *X, *Lam;
  int64_t ncoord;
  // rows
  const double *b;
  double *r, *y1, *y;
  // matrices
  const double *A;        // dense
  const int64_t *a_rowptr; const int32_t *a_col; const double *a_val;     // CSR
  const int64_t *a_colptr; const int32_t *a_row; const double *a_cval;    // CSC (per instance blocks)
  const double *T;        // L^-1, lower, row-major (pitch ldm)
  const double *U;        // L^-T, upper, row-major (pitch ldm)
  const double *Bm;       // B = L^-1 A for dense instances (layout of A), or NULL
  const double *bp;       // L^-1 b (row space), used with Bm
  // tiles: (inst, start) pairs
  const int32_t *row_tiles; int n_row_tiles; int rows_per_tile;
  const int32_t *col_tiles; int n_col_tiles;
  const int32_t *t_rows; int n_t_rows;      // (inst, row) per wave for T r
  const int32_t *t3_rows; int n_t3_rows;    // (inst, row) per wave for T^T y1
  const int32_t *csr_rows; int n_csr_rows;   // (inst, row) pairs for CSR instances
  const int32_t *csc_cols; int n_csc_cols;   // (inst, col-chunk) pairs for CSR instances
  // residual partials
  const double *part;
  const int64_t *inst_cl_first;               // [B+1]
  double *hist;                               // B x hist_cap x 3
  // k_scatter: number of leading workgroups (a multiple of 8, >= batch, or
  // 0) that first finish the previous iteration (residuals, stopping test)
  int32_t res_blocks;
  int batch;
  int ignore_done;                            // diagnostics: run on frozen instances too
  int dual;                                   // Algorithm 2: right-hand sides c - sum(z + lambda/rho), -b/rho
  // affine step by preconditioned conjugate gradients (cg_max_iter > 0)
  int cg_max_iter;
  CgState *cg;                                // [batch]
  const double *cg_tol2;                      // [batch] (cg_tol (1 + ||b||))^2
  const double *cg_diag;                      // rows: diag(A W D^-1 A^T)
  double *cg_g;                               // coordinates: A^T y of the last solve
  double *cg_z, *cg_p, *cg_Mp;                // rows (the residual lives in r)
  const int32_t *cg_tiles; int cg_ntiles;     // (inst, first row) per tile of rows
  const int32_t *cg_tile_first;               // [batch + 1]: an instance's tiles
  double *cg_part;                            // [3][cg_ntiles]: p^T M p, r^T z, ||r||^2
  int cg_loop;                                // products inside the solve: skip stopped instances
  int stream_nt;                              // dense passes with non-temporal loads
  int no_b;                                   // row products without the -b term
};

// Scratch of the diagnostics pass (allocated on first use).
struct DiagScratch {
  double *wu;     // ncoord: w .* u
  double *z;      // ncoord: sum_k H_k^T lambda_k
  double *aty;    // ncoord: A^T y_dual
  double *ax;     // nrow: A (w .* u) - b
  double *yd;     // nrow: y_dual = -rho y
  double *lmin;   // ncl: min eigenvalue of E_k U E_k^T
};

hipError_t launch_diagnostics(const AffineArgs &a, const DiagScratch &s,
                              const int64_t *inst_cl_first, int64_t nrow, double *out,
                              hipStream_t st);
hipError_t launch_scaled_copy(const double *src, double *dst, int64_t n, const InstState *state,
                              int inst, hipStream_t st);

hipError_t launch_iteration_affine(const AffineArgs &a, hipStream_t st);
// The affine step with conjugate gradients: scatter, r0, the solve, u.
hipError_t launch_cg_affine(const AffineArgs &a, hipStream_t st);
// Stages of that step for timing: 0 scatter, 1 r0, 2 the solve, 4 u.
hipError_t launch_cg_stage(const AffineArgs &a, int stage, hipStream_t st);
// rows of one conjugate-gradient tile
int affine_cg_tile_rows();
// diag(A W D^-1 A^T) into out (wd = w / D; rows: (inst, row) pairs)
hipError_t launch_cg_diag(const AffineArgs &a, const double *wd, const int32_t *rows, int nrows,
                          double *out, hipStream_t st);
hipError_t launch_residual_reduce(const AffineArgs &a, hipStream_t st);
hipError_t launch_affine_stage(const AffineArgs &a, int stage, hipStream_t st);
hipError_t launch_objective(const AffineArgs &a, double *obj, hipStream_t st);

// ----------------------------------------------------------------------------
// One-time factorisation (k_factor.hip)
// ----------------------------------------------------------------------------
struct FactorArgs {
  const InstDesc *inst;          // device
  int batch;
  int max_m;
  const double *A;               // dense A (or NULL)
  const int64_t *a_rowptr; const int32_t *a_col; const double *a_val;
  const int64_t *a_colptr; const int32_t *a_row; const double *a_cval;
  const double *wd;              // w/D per coordinate
  double *M;                     // work: per instance m x m (pitch ldm) at t_off
  double *T;                     // out: L^-1 at t_off
  double *U;                     // out: L^-T at t_off
  int32_t *fail;                 // per instance: 1 if a pivot <= 0
  double *Bout;                  // out: B = L^-1 A for dense instances (layout of A)
  double diag_shift;             // added to the diagonal of M before the factorisation
};

hipError_t launch_syrk_dense(const FactorArgs &f, const int32_t *tiles, int ntiles,
                             hipStream_t st);
hipError_t launch_syrk_csr(const FactorArgs &f, const int32_t *rows, int nrows, int max_ldm,
                           hipStream_t st);
hipError_t launch_cholesky_and_inverse(const FactorArgs &f, int max_nblk, hipStream_t st);
// tiles: (inst, row tile, column tile) triples over dense instances
hipError_t launch_form_b(const FactorArgs &f, const int32_t *tiles, int ntiles, hipStream_t st);

// ----------------------------------------------------------------------------
// Algorithm 3 (k_hsde.hip): the HSDE iteration around the shared kernels
// ----------------------------------------------------------------------------
struct HsdeArgs {
  const InstDesc *inst;
  InstState *state;
  HsdeState *hs;
  SolverParams params;
  int batch;
  int ignore_done;
  // coordinate space (compact lower coordinates, weights w)
  int64_t ncoord;
  const int32_t *coord_inst;
  const double *c, *w, *P;            // P = 1 + D/2
  const int64_t *contrib_ptr;
  const int32_t *contrib_idx;
  double *ux, *nx, *xp, *v, *sx, *mzx, *atmz;
  // row space
  int64_t nrow;
  const int32_t *row_inst;
  const double *b;
  double *uy, *ny, *g, *mzy, *az;
  // packed clique blocks
  int64_t npk;
  const int32_t *blk_loc;
  double *us, *vz, *ut, *ns, *nt, *mzs, *mzt;
  // wave partial sums (4 per 64 coordinates / rows), clique partials
  // (NPART per clique) and history
  double *cw_part, *rw_part;
  const double *part;
  const int64_t *inst_cl_first;
  double *hist;
};

// nu = u + v - (u_tau + v_kappa) zeta on every space (coordinates, blocks, rows)
hipError_t launch_hsde_form_nu(const HsdeArgs &h, hipStream_t st);
// x' = nu_x + H^T (nu_s + nu_t) / 2 and v = w x' / P on the coordinates
hipError_t launch_hsde_xprime(const HsdeArgs &h, const double *nx, const double *ns,
                              const double *nt, hipStream_t st);
// set-up: M^-1 zeta from the inner solve of nu = zeta, kz and the norms
hipError_t launch_hsde_setup_finish(const HsdeArgs &h, hipStream_t st);
hipError_t launch_hsde_setup_nu(const HsdeArgs &h, hipStream_t st);   // nu = zeta
// tau, kappa, u_x, u_y and the row-space residual pieces
hipError_t launch_hsde_update(const HsdeArgs &h, hipStream_t st);
// H^T v_z, the dual residual, the clique partials: residuals, stopping,
// infeasibility tests
hipError_t launch_hsde_finish(const HsdeArgs &h, hipStream_t st);
hipError_t launch_hsde_reset(const HsdeArgs &h, hipStream_t st);
hipError_t launch_hsde_solution(const HsdeArgs &h, double *x_out, double *y_out, hipStream_t st);

int affine_col_tile_width();
int affine_csc_tile_width();   // columns per workgroup of the sparse transposed product
int affine_max_rows_per_tile();

// ----------------------------------------------------------------------------
// Reverse sweep of the unrolled iteration (k_adjoint.hip)
// ----------------------------------------------------------------------------
struct AdjArgs {
  const InstDesc *inst;
  const InstState *state;
  // cliques / packed entries
  const int32_t *cl_inst, *cl_size;
  const int64_t *cl_off;
  const int32_t *blk_loc;
  const void *eig;            // (V, theta) records of the iteration being reversed
  const int64_t *eig_off;
  double *Xb, *Lb, *Ub;       // packed cotangents of X_k, Lambda_k, U_k
  int64_t npk;
  // coordinates and rows
  int64_t ncoord, nrow;
  const int32_t *coord_inst, *row_inst;
  const int64_t *contrib_ptr;
  const int32_t *contrib_idx;
  const double *w, *D;
  double *bhat_bar, *v_bar;   // input of the adjoint KKT solve
  const double *bhb;          // its output P ubar
  const double *y_bar;        // its multiplier
  const double *seed;         // cotangent of u_T in the caller's layout (or NULL)
  const int64_t *user_coord_off, *user_row_off;
  double *cbar, *bbar;        // caller's layout
  int euclid;                 // caller's cotangents are Euclidean on compact coordinates
  int batch;
};

hipError_t launch_adj_projection(int precision, int N, const int32_t *list, int count,
                                 const AdjArgs &a, hipStream_t st);
hipError_t launch_adj_scatter(const AdjArgs &a, hipStream_t st);
hipError_t launch_adj_coord_and_gather(const AdjArgs &a, hipStream_t st);
hipError_t launch_copy_user(const double *src, double *dst, const InstDesc *inst,
                            const int32_t *coord_inst, const int64_t *user_coord_off,
                            int64_t ncoord, int to_user, hipStream_t st);
hipError_t launch_copy_user_rows(const double *src, double *dst, const InstDesc *inst,
                                 const int32_t *row_inst, const int64_t *user_row_off,
                                 int64_t nrow, hipStream_t st);
int adjoint_max_bucket(int precision);   // largest padded block with a projection adjoint
