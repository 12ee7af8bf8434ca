/*
 * sdp_oracle.c -- plain CPU FP64 oracle for chordal-decomposed primal ADMM.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the GPU
 * path: the two meet only through the seeded instance generator (sdpgen).
 *
 * Paper: Zheng, Fantuzzi, Papachristodoulou, Goulart, Wynn, "Chordal
 * decomposition in operator-splitting methods for sparse semidefinite
 * programs".  What is computed, and where it comes from:
 *
 *   - Problem: the domain-space decomposition of the primal SDP (Section
 *     "Domain-space decomposition", problem (DecomposedPrimalSDP)) in the
 *     vectorised form (DecomposedPrimalVector): min <c,x> s.t. Ax = b,
 *     x_k = H_k x, x_k in S_k.
 *   - Iteration: Algorithm 1 ("ADMM for the domain-space decomposition"):
 *     x-update by the KKT system (OptCondMinYPrimal) solved by block
 *     elimination with a cached Cholesky factor of A D^-1 A^T
 *     (ADMMprimalFatorization; the two-step form (KKTflops) of the proof of
 *     Proposition 1), then the clique PSD projections (XkUpdate), then the
 *     multiplier update (LambdakUpdate), then the stopping test on
 *     eps_c and eps_lambda (PrimalConsensusResidual).
 *   - Optional adaptive penalty of the Section "Adaptive penalty strategy".
 *   - Optional affine step by preconditioned conjugate gradients, the
 *     iterative alternative to the factorisation that Section 4.1.1 names
 *     (Jacobi preconditioner, warm start from the previous multiplier).
 *   - Diagnostics eps_p, eps_d, eps_g (HSDEerror) and eps_alpha
 *     (PSD-violation), as the paper reports them for its primal solver.
 *
 * Storage.  The global variable x = vec(X) is kept on the lower-triangle
 * pattern coordinates only ("u"), because X is symmetric and every entry off
 * the chordal pattern appears in no C, A_i or H_k.  With w_j = 1 on the
 * diagonal and 2 off it, the KKT system (OptCondMinYPrimal) reads, entry by
 * entry,
 *     D_j u_j + sum_i A_ij y_i = bhat_j,          sum_j w_j A_ij u_j = b_i,
 * with bhat_j = sum_k (X_k + Lambda_k/rho)[at j] - c_j/rho and D_j the number
 * of cliques holding both endpoints of j.  Eliminating u gives
 *     (A W D^-1 A^T) y = A (W D^-1 bhat) - b,   u = D^-1 (bhat - A^T y),
 * which is (KKTflops) written on the compact coordinates; A W D^-1 A^T equals
 * the paper's A D^-1 A^T on full vectors.  Clique blocks X_k and Lambda_k are
 * kept as full s_k x s_k row-major matrices and all norms are full Frobenius
 * norms, exactly as in the vectorised problem.
 *
 * Readings where the paper is silent (the same readings the GPU path takes):
 *   initial guesses X_k = Lambda_k = 0 (x^(0) is never read); eps ratios with
 *   a zero denominator are 0 when the numerator is 0 and +inf otherwise; the
 *   adaptive rule uses eps_c as the primal and eps_lambda as the dual
 *   residual, is applied after the stopping test every rho_period iterations
 *   and never rescales Lambda (the multipliers are unscaled); the dual
 *   variable reported is y_dual = -rho * y (the KKT multiplier of Ax = b is
 *   rho*y).
 *
 * Eigen-solver: the paper projects with a library eigendecomposition.  Here
 * the symmetric eigenproblem is solved by the cyclic-by-row two-sided Jacobi
 * method with the stable 2x2 rotation of Rutishauser (Golub and Van Loan,
 * Matrix Computations, sections on the symmetric Schur decomposition and
 * cyclic Jacobi).  The PSD projection is unique, so the eigenvector basis the
 * solver returns does not matter.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Status codes: the numeric values are part of the library interface, restated
 * here (not included) so that the oracle stays independent of the GPU path. */
enum {
  ORC_OK = 0,
  ORC_MAX_ITER = 1,
  ORC_ERR_ARG = -1,
  ORC_ERR_PATTERN_UNCOVERED = -2,
  ORC_ERR_OFF_PATTERN = -3,
  ORC_ERR_CLIQUE_ORDER = -4,
  ORC_ERR_RANK_DEFICIENT = -5,
  ORC_ERR_NONFINITE = -6,
  ORC_ERR_UNSUPPORTED = -7,
};

#define ORC_MAX_CLIQUE 128

typedef struct orc_problem {
  int n, m, p;
  int64_t nnz;
  int *pat_row, *pat_col;
  int *cptr, *cvert;
  int64_t *blk_off;   /* offset of clique k's s_k*s_k block in X, Lam      */
  int *loc;           /* loc[blk_off[k] + a*s+b] = pattern index of (v_a,v_b) */
  double *D, *w;      /* overlap counts and symmetric-storage weights          */
  int a_format;       /* 0 dense m x nnz row-major, 1 CSR                     */
  int64_t *a_rowptr;
  int *a_col;
  double *a_val;
  double *b, *c;
  double *L;          /* m x m Cholesky factor (row-major, lower)              */
  /* ADMM state */
  double rho;
  double *X, *Lam, *Xprev;
  double *Vd;         /* Algorithm 2: the slack blocks v_k (X holds z_k)      */
  /* Algorithm 3 (HSDE): factor of I + A W P^-1 A^T with P = I + D/2, the
   * iterates u = (x, s, y, t, tau), v = (0, z, 0, 0, kappa) and M^-1 zeta */
  double *Lh, *hP;
  double *ux, *us, *uy, *ut, *vz, utau, kappa;
  double *mzx, *mzs, *mzy, *mzt, kz;
  double *hx, *hs, *hy, *ht, *hx2, *hs2, *hy2, *ht2;   /* work */
  double eps_p, eps_d, eps_g;
  int hsde_status;
  double *u, *y, *bhat, *r, *tmp;
  /* Affine step by preconditioned conjugate gradients instead of the cached
   * factor (the iterative alternative of Section 4.1.1): at most cg_max_iter
   * steps, stop when ||r||_2 <= cg_tol (1 + ||b||_2), Jacobi preconditioner
   * diag(A W D^-1 A^T), warm start from the previous y. */
  int cg_max_iter;    /* 0: Cholesky */
  double cg_tol;
  double *cg_diag, *cg_r, *cg_z, *cg_p, *cg_Mp, *cg_t;
  int64_t cg_steps;   /* conjugate-gradient steps taken so far */
  int64_t nblk;       /* sum s_k^2 */
  int iters;
  double eps_c, eps_l;
  /* Jacobi controls and statistics */
  int jac_max_sweeps;
  double jac_tol;
  int64_t total_sweeps;
  int max_sweeps_seen;
} orc_problem;

void orc_set_threads(int t) {
#ifdef _OPENMP
  if (t > 0) omp_set_num_threads(t);
#else
  (void)t;
#endif
}

int orc_get_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ------------------------------------------------------------------------- */
/* Symmetric eigenproblem: cyclic Jacobi                                      */
/* ------------------------------------------------------------------------- */

/* Stable symmetric 2x2 Schur rotation (c, s) that zeroes A[p][q] of
 * J^T A J with J = [[c, s], [-s, c]] acting on rows/columns p, q. */
static void sym_schur2(double app, double aqq, double apq, double *c, double *s) {
  if (apq == 0.0) { *c = 1.0; *s = 0.0; return; }
  double tau = (aqq - app) / (2.0 * apq);
  double t;
  if (fabs(tau) > 1e150) {
    t = 0.5 / tau;                     /* sqrt(1 + tau^2) would overflow */
  } else if (tau >= 0.0) {
    t = 1.0 / (tau + sqrt(1.0 + tau * tau));
  } else {
    t = -1.0 / (-tau + sqrt(1.0 + tau * tau));
  }
  *c = 1.0 / sqrt(1.0 + t * t);
  *s = t * (*c);
}

static double off_norm2(int s, const double *A) {
  double acc = 0.0;
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j)
      if (i != j) acc += A[i * s + j] * A[i * s + j];
  return acc;
}

static double frob2(int s, const double *A) {
  double acc = 0.0;
  for (int i = 0; i < s * s; ++i) acc += A[i] * A[i];
  return acc;
}

/* Eigendecomposition A = V diag(theta) V^T of a symmetric s x s matrix
 * (row-major, overwritten).  Returns the number of sweeps done. */
int orc_jacobi_eig(int s, double *A, double *V, double *theta, int max_sweeps,
                   double tol) {
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) V[i * s + j] = (i == j) ? 1.0 : 0.0;
  double nrm2 = frob2(s, A);
  int sweep = 0;
  while (sweep < max_sweeps && off_norm2(s, A) > tol * tol * nrm2) {
    for (int p = 0; p < s - 1; ++p) {
      for (int q = p + 1; q < s; ++q) {
        double c, sn;
        sym_schur2(A[p * s + p], A[q * s + q], A[p * s + q], &c, &sn);
        if (sn == 0.0) continue;
        /* A <- A J (columns p, q) */
        for (int k = 0; k < s; ++k) {
          double akp = A[k * s + p], akq = A[k * s + q];
          A[k * s + p] = c * akp - sn * akq;
          A[k * s + q] = sn * akp + c * akq;
        }
        /* A <- J^T A (rows p, q) */
        for (int k = 0; k < s; ++k) {
          double apk = A[p * s + k], aqk = A[q * s + k];
          A[p * s + k] = c * apk - sn * aqk;
          A[q * s + k] = sn * apk + c * aqk;
        }
        /* V <- V J */
        for (int k = 0; k < s; ++k) {
          double vkp = V[k * s + p], vkq = V[k * s + q];
          V[k * s + p] = c * vkp - sn * vkq;
          V[k * s + q] = sn * vkp + c * vkq;
        }
      }
    }
    ++sweep;
  }
  for (int i = 0; i < s; ++i) theta[i] = A[i * s + i];
  return sweep;
}

/* Projection onto the PSD cone (XkUpdate): X = V diag(max(theta,0)) V^T.
 * W is s x s symmetric row-major (not modified).  Optionally returns theta
 * and V.  Returns the number of Jacobi sweeps. */
int orc_psd_project(int s, const double *W, double *X, double *theta_out,
                    double *V_out, int max_sweeps, double tol) {
  double *A = (double *)malloc(sizeof(double) * s * s);
  double *V = (double *)malloc(sizeof(double) * s * s);
  double *th = (double *)malloc(sizeof(double) * (s > 0 ? s : 1));
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j)
      A[i * s + j] = 0.5 * (W[i * s + j] + W[j * s + i]);
  int sw = orc_jacobi_eig(s, A, V, th, max_sweeps, tol);
  for (int i = 0; i < s; ++i) {
    for (int j = 0; j <= i; ++j) {
      double acc = 0.0;
      for (int k = 0; k < s; ++k)
        if (th[k] > 0.0) acc += V[i * s + k] * th[k] * V[j * s + k];
      X[i * s + j] = acc;
      X[j * s + i] = acc;
    }
  }
  if (theta_out) memcpy(theta_out, th, sizeof(double) * s);
  if (V_out) memcpy(V_out, V, sizeof(double) * s * s);
  free(A); free(V); free(th);
  return sw;
}

/* ------------------------------------------------------------------------- */
/* Dense Cholesky and triangular solves (the cached factorisation)            */
/* ------------------------------------------------------------------------- */

/* M = L L^T, column by column (Cholesky-Crout).  M row-major m x m, only the
 * lower triangle is read.  Returns ORC_ERR_RANK_DEFICIENT on a non-positive
 * pivot (the paper assumes linearly independent A_i). */
int orc_cholesky(int m, const double *M, double *L) {
  memset(L, 0, sizeof(double) * (size_t)m * m);
  for (int j = 0; j < m; ++j) {
    double d = M[(size_t)j * m + j];
    for (int k = 0; k < j; ++k) d -= L[(size_t)j * m + k] * L[(size_t)j * m + k];
    if (!(d > 0.0)) return ORC_ERR_RANK_DEFICIENT;
    double ljj = sqrt(d);
    L[(size_t)j * m + j] = ljj;
#pragma omp parallel for schedule(static)
    for (int i = j + 1; i < m; ++i) {
      double acc = M[(size_t)i * m + j];
      for (int k = 0; k < j; ++k) acc -= L[(size_t)i * m + k] * L[(size_t)j * m + k];
      L[(size_t)i * m + j] = acc / ljj;
    }
  }
  return ORC_OK;
}

/* Solve L L^T y = r by forward then backward substitution. */
void orc_chol_solve(int m, const double *L, const double *r, double *y) {
  double *z = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
  for (int i = 0; i < m; ++i) {
    double acc = r[i];
    for (int k = 0; k < i; ++k) acc -= L[(size_t)i * m + k] * z[k];
    z[i] = acc / L[(size_t)i * m + i];
  }
  for (int i = m - 1; i >= 0; --i) {
    double acc = z[i];
    for (int k = i + 1; k < m; ++k) acc -= L[(size_t)k * m + i] * y[k];
    y[i] = acc / L[(size_t)i * m + i];
  }
  free(z);
}

/* ------------------------------------------------------------------------- */
/* Products with A on the compact coordinates                                 */
/* ------------------------------------------------------------------------- */

/* out_i = sum_j A_ij v_j */
static void a_times(const orc_problem *P, const double *v, double *out) {
  if (P->a_format == 0) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P->m; ++i) {
      const double *row = P->a_val + (size_t)i * P->nnz;
      double acc = 0.0;
      for (int64_t j = 0; j < P->nnz; ++j) acc += row[j] * v[j];
      out[i] = acc;
    }
  } else {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < P->m; ++i) {
      double acc = 0.0;
      for (int64_t t = P->a_rowptr[i]; t < P->a_rowptr[i + 1]; ++t)
        acc += P->a_val[t] * v[P->a_col[t]];
      out[i] = acc;
    }
  }
}

/* out_j = sum_i A_ij y_i  (rows visited in increasing i for every j) */
static void at_times(const orc_problem *P, const double *y, double *out) {
  if (P->a_format == 0) {
#pragma omp parallel for schedule(static)
    for (int64_t j = 0; j < P->nnz; ++j) {
      double acc = 0.0;
      for (int i = 0; i < P->m; ++i) acc += P->a_val[(size_t)i * P->nnz + j] * y[i];
      out[j] = acc;
    }
  } else {
    for (int64_t j = 0; j < P->nnz; ++j) out[j] = 0.0;
    for (int i = 0; i < P->m; ++i)
      for (int64_t t = P->a_rowptr[i]; t < P->a_rowptr[i + 1]; ++t)
        out[P->a_col[t]] += P->a_val[t] * y[i];
  }
}

/* M = A diag(wd) A^T (m x m, row-major, both triangles), summing over the
 * compact coordinates j in increasing order. */
static void assemble_gram(const orc_problem *P, const double *wd, double *M) {
  const int m = P->m;
  const int64_t nnz = P->nnz;
  if (P->a_format == 0) {
#pragma omp parallel for schedule(dynamic, 4)
    for (int i = 0; i < m; ++i) {
      const double *ri = P->a_val + (size_t)i * nnz;
      for (int k = 0; k <= i; ++k) {
        const double *rk = P->a_val + (size_t)k * nnz;
        double acc = 0.0;
        for (int64_t j = 0; j < nnz; ++j) acc += ri[j] * wd[j] * rk[j];
        M[(size_t)i * m + k] = acc;
        M[(size_t)k * m + i] = acc;
      }
    }
    return;
  }
  /* the same sums skipping the zero terms */
  const int64_t annz = P->a_rowptr[m];
  int64_t *cptrA = (int64_t *)calloc(nnz + 1, sizeof(int64_t));
  for (int64_t t = 0; t < annz; ++t) cptrA[P->a_col[t] + 1]++;
  for (int64_t j = 0; j < nnz; ++j) cptrA[j + 1] += cptrA[j];
  int *rowA = (int *)malloc(sizeof(int) * (annz > 0 ? annz : 1));
  double *valA = (double *)malloc(sizeof(double) * (annz > 0 ? annz : 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * nnz);
  memcpy(fill, cptrA, sizeof(int64_t) * nnz);
  for (int i = 0; i < m; ++i)
    for (int64_t t = P->a_rowptr[i]; t < P->a_rowptr[i + 1]; ++t) {
      int64_t pos = fill[P->a_col[t]]++;
      rowA[pos] = i; valA[pos] = P->a_val[t];
    }
  for (int64_t j = 0; j < nnz; ++j)
    for (int64_t s1 = cptrA[j]; s1 < cptrA[j + 1]; ++s1)
      for (int64_t s2 = cptrA[j]; s2 <= s1; ++s2) {
        int i = rowA[s1], k = rowA[s2];
        M[(size_t)i * m + k] += valA[s1] * wd[j] * valA[s2];
      }
  for (int i = 0; i < m; ++i)
    for (int k = 0; k < i; ++k) M[(size_t)k * m + i] = M[(size_t)i * m + k];
  free(cptrA); free(rowA); free(valA); free(fill);
}

/* ------------------------------------------------------------------------- */
/* Set-up (Algorithm 1, data preprocessing)                                   */
/* ------------------------------------------------------------------------- */

void orc_free(orc_problem *P) {
  if (!P) return;
  free(P->pat_row); free(P->pat_col); free(P->cptr); free(P->cvert);
  free(P->blk_off); free(P->loc); free(P->D); free(P->w);
  free(P->a_rowptr); free(P->a_col); free(P->a_val); free(P->b); free(P->c);
  free(P->L); free(P->X); free(P->Lam); free(P->Xprev); free(P->Vd);
  free(P->Lh); free(P->hP); free(P->ux); free(P->us); free(P->uy); free(P->ut); free(P->vz);
  free(P->mzx); free(P->mzs); free(P->mzy); free(P->mzt);
  free(P->hx); free(P->hs); free(P->hy); free(P->ht);
  free(P->hx2); free(P->hs2); free(P->hy2); free(P->ht2);
  free(P->u); free(P->y); free(P->bhat); free(P->r); free(P->tmp);
  free(P->cg_diag); free(P->cg_r); free(P->cg_z); free(P->cg_p); free(P->cg_Mp); free(P->cg_t);
  free(P);
}

static int finite_all(const double *v, int64_t n) {
  for (int64_t i = 0; i < n; ++i) if (!isfinite(v[i])) return 0;
  return 1;
}

/* Validate the data, build the clique index maps, D, w, and factor
 * M = A W D^-1 A^T.  All input arrays are copied. */
/* factor = 0 skips the Cholesky factor: such a problem runs Algorithm 1 only
 * with the conjugate-gradient affine step (orc_set_affine_cg first). */
int orc_create_ex(int n, int m, int64_t nnz, const int *pat_row, const int *pat_col,
                  int p, const int *clique_ptr, const int *clique_vert,
                  int a_format, const int64_t *a_rowptr, const int *a_col,
                  const double *a_val, const double *b, const double *c, int factor,
                  orc_problem **out) {
  *out = NULL;
  if (n <= 0 || m < 1 || nnz <= 0 || p <= 0 || !pat_row || !pat_col ||
      !clique_ptr || !clique_vert || !a_val || !b || !c ||
      (a_format != 0 && a_format != 1) ||
      (a_format == 1 && (!a_rowptr || !a_col)))
    return ORC_ERR_ARG;
  /* pattern: lower, in range, strictly sorted by (col, row), diagonal present */
  int ndiag = 0;
  for (int64_t j = 0; j < nnz; ++j) {
    int r = pat_row[j], cc = pat_col[j];
    if (r < 0 || r >= n || cc < 0 || cc > r) return ORC_ERR_ARG;
    if (j > 0) {
      int pr = pat_row[j - 1], pc = pat_col[j - 1];
      if (cc < pc || (cc == pc && r <= pr)) return ORC_ERR_ARG;
    }
    if (r == cc) ++ndiag;
  }
  if (ndiag != n) return ORC_ERR_ARG;
  /* cliques */
  if (clique_ptr[0] != 0) return ORC_ERR_ARG;
  for (int k = 0; k < p; ++k) {
    int s = clique_ptr[k + 1] - clique_ptr[k];
    if (s <= 0) return ORC_ERR_ARG;
  }
  for (int k = 0; k < p; ++k) {
    int s = clique_ptr[k + 1] - clique_ptr[k];
    const int *v = clique_vert + clique_ptr[k];
    for (int a = 0; a < s; ++a) {
      if (v[a] < 0 || v[a] >= n) return ORC_ERR_CLIQUE_ORDER;
      if (a > 0 && v[a] <= v[a - 1]) return ORC_ERR_CLIQUE_ORDER;
    }
  }
  for (int k = 0; k < p; ++k)
    if (clique_ptr[k + 1] - clique_ptr[k] > ORC_MAX_CLIQUE) return ORC_ERR_UNSUPPORTED;
  /* A in CSR: row pointers monotone, columns in range */
  int64_t annz = (a_format == 0) ? (int64_t)m * nnz : a_rowptr[m];
  if (a_format == 1) {
    if (a_rowptr[0] != 0) return ORC_ERR_ARG;
    for (int i = 0; i < m; ++i) if (a_rowptr[i + 1] < a_rowptr[i]) return ORC_ERR_ARG;
    for (int64_t t = 0; t < annz; ++t) if (a_col[t] < 0 || a_col[t] >= nnz) return ORC_ERR_ARG;
  }
  if (!finite_all(a_val, annz) || !finite_all(b, m) || !finite_all(c, nnz))
    return ORC_ERR_NONFINITE;

  orc_problem *P = (orc_problem *)calloc(1, sizeof(orc_problem));
  P->n = n; P->m = m; P->p = p; P->nnz = nnz;
  P->pat_row = (int *)malloc(sizeof(int) * nnz);
  P->pat_col = (int *)malloc(sizeof(int) * nnz);
  memcpy(P->pat_row, pat_row, sizeof(int) * nnz);
  memcpy(P->pat_col, pat_col, sizeof(int) * nnz);
  P->cptr = (int *)malloc(sizeof(int) * (p + 1));
  memcpy(P->cptr, clique_ptr, sizeof(int) * (p + 1));
  P->cvert = (int *)malloc(sizeof(int) * (clique_ptr[p] > 0 ? clique_ptr[p] : 1));
  memcpy(P->cvert, clique_vert, sizeof(int) * clique_ptr[p]);
  P->a_format = a_format;
  P->a_val = (double *)malloc(sizeof(double) * (annz > 0 ? annz : 1));
  memcpy(P->a_val, a_val, sizeof(double) * annz);
  if (a_format == 1) {
    P->a_rowptr = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
    memcpy(P->a_rowptr, a_rowptr, sizeof(int64_t) * (m + 1));
    P->a_col = (int *)malloc(sizeof(int) * (annz > 0 ? annz : 1));
    memcpy(P->a_col, a_col, sizeof(int) * annz);
  }
  P->b = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
  memcpy(P->b, b, sizeof(double) * m);
  P->c = (double *)malloc(sizeof(double) * nnz);
  memcpy(P->c, c, sizeof(double) * nnz);

  /* index of every lower coordinate: position table over (col, row) */
  int64_t *index = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * n);
  for (size_t t = 0; t < (size_t)n * n; ++t) index[t] = -1;
  for (int64_t j = 0; j < nnz; ++j) index[(size_t)pat_row[j] * n + pat_col[j]] = j;

  /* H_k as index lists: block entry (a, b) of clique k is pattern coordinate
   * (max(v_a, v_b), min(v_a, v_b)) -- the entry selector E_Ck of the
   * Section "Sparse matrix cones and chordal decomposition". */
  P->blk_off = (int64_t *)malloc(sizeof(int64_t) * (p + 1));
  P->blk_off[0] = 0;
  for (int k = 0; k < p; ++k) {
    int64_t s = clique_ptr[k + 1] - clique_ptr[k];
    P->blk_off[k + 1] = P->blk_off[k] + s * s;
  }
  P->nblk = P->blk_off[p];
  P->loc = (int *)malloc(sizeof(int) * P->nblk);
  int rc = ORC_OK;
  for (int k = 0; k < p && rc == ORC_OK; ++k) {
    int s = clique_ptr[k + 1] - clique_ptr[k];
    const int *v = clique_vert + clique_ptr[k];
    for (int a = 0; a < s && rc == ORC_OK; ++a)
      for (int bb = 0; bb < s; ++bb) {
        int r = v[a] > v[bb] ? v[a] : v[bb];
        int cc = v[a] > v[bb] ? v[bb] : v[a];
        int64_t j = index[(size_t)r * n + cc];
        if (j < 0) { rc = ORC_ERR_OFF_PATTERN; break; }
        P->loc[P->blk_off[k] + (int64_t)a * s + bb] = (int)j;
      }
  }
  free(index);
  if (rc != ORC_OK) { orc_free(P); return rc; }

  /* D = sum_k H_k^T H_k: per coordinate, the number of cliques covering it.
   * Counting the lower-triangle block entries (a >= b) visits each covered
   * coordinate exactly once per clique. */
  P->D = (double *)calloc(nnz, sizeof(double));
  P->w = (double *)malloc(sizeof(double) * nnz);
  for (int k = 0; k < p; ++k) {
    int s = clique_ptr[k + 1] - clique_ptr[k];
    for (int a = 0; a < s; ++a)
      for (int bb = 0; bb <= a; ++bb) P->D[P->loc[P->blk_off[k] + (int64_t)a * s + bb]] += 1.0;
  }
  for (int64_t j = 0; j < nnz; ++j) {
    if (P->D[j] == 0.0) { orc_free(P); return ORC_ERR_PATTERN_UNCOVERED; }
    P->w[j] = (pat_row[j] == pat_col[j]) ? 1.0 : 2.0;
  }

  /* M = A W D^-1 A^T (the matrix A D^-1 A^T of ADMMprimalFatorization on the
   * compact coordinates), then M = L L^T. */
  if (factor) {
    double *M = (double *)calloc((size_t)(m > 0 ? m : 1) * (m > 0 ? m : 1), sizeof(double));
    {
      double *wd = (double *)malloc(sizeof(double) * nnz);
      for (int64_t j = 0; j < nnz; ++j) wd[j] = P->w[j] / P->D[j];
      assemble_gram(P, wd, M);
      free(wd);
    }
    P->L = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (m > 0 ? m : 1));
    rc = orc_cholesky(m, M, P->L);
    free(M);
    if (rc != ORC_OK) { orc_free(P); return rc; }
  }

  P->X = (double *)calloc(P->nblk, sizeof(double));
  P->Lam = (double *)calloc(P->nblk, sizeof(double));
  P->Xprev = (double *)calloc(P->nblk, sizeof(double));
  P->Vd = (double *)calloc(P->nblk, sizeof(double));
  P->u = (double *)calloc(nnz, sizeof(double));
  P->bhat = (double *)calloc(nnz, sizeof(double));
  P->tmp = (double *)calloc(nnz, sizeof(double));
  P->y = (double *)calloc(m > 0 ? m : 1, sizeof(double));
  P->r = (double *)calloc(m > 0 ? m : 1, sizeof(double));
  P->rho = 1.0;
  P->jac_max_sweeps = 50;
  P->jac_tol = 1e-14;
  *out = P;
  return ORC_OK;
}

int orc_create(int n, int m, int64_t nnz, const int *pat_row, const int *pat_col,
               int p, const int *clique_ptr, const int *clique_vert,
               int a_format, const int64_t *a_rowptr, const int *a_col,
               const double *a_val, const double *b, const double *c,
               orc_problem **out) {
  return orc_create_ex(n, m, nnz, pat_row, pat_col, p, clique_ptr, clique_vert, a_format,
                       a_rowptr, a_col, a_val, b, c, 1, out);
}

/* Initial guesses X_k = Lambda_k = 0 and penalty rho0. */
void orc_reset(orc_problem *P, double rho0) {
  memset(P->X, 0, sizeof(double) * P->nblk);
  memset(P->Lam, 0, sizeof(double) * P->nblk);
  memset(P->Xprev, 0, sizeof(double) * P->nblk);
  memset(P->Vd, 0, sizeof(double) * P->nblk);
  memset(P->u, 0, sizeof(double) * P->nnz);
  memset(P->y, 0, sizeof(double) * (P->m > 0 ? P->m : 1));
  P->rho = rho0;
  P->iters = 0;
  P->eps_c = P->eps_l = INFINITY;
  P->total_sweeps = 0;
  P->max_sweeps_seen = 0;
  P->cg_steps = 0;
}

void orc_set_jacobi(orc_problem *P, int max_sweeps, double tol) {
  P->jac_max_sweeps = max_sweeps;
  P->jac_tol = tol;
}

/* ------------------------------------------------------------------------- */
/* One ADMM iteration (Algorithm 1)                                           */
/* ------------------------------------------------------------------------- */

/* bhat = sum_k H_k^T (x_k + lambda_k / rho) - c / rho   (right-hand side of
 * OptCondMinYPrimal).  Cliques are summed in increasing k. */
void orc_form_bhat(const orc_problem *P, const double *X, const double *Lam,
                   double rho, double *bhat) {
  for (int64_t j = 0; j < P->nnz; ++j) bhat[j] = 0.0;
  for (int k = 0; k < P->p; ++k) {
    int s = P->cptr[k + 1] - P->cptr[k];
    int64_t o = P->blk_off[k];
    for (int a = 0; a < s; ++a)
      for (int bb = 0; bb <= a; ++bb) {
        int64_t e = o + (int64_t)a * s + bb;
        bhat[P->loc[e]] += X[e] + Lam[e] / rho;
      }
  }
  for (int64_t j = 0; j < P->nnz; ++j) bhat[j] -= P->c[j] / rho;
}

/* out = A W D^-1 A^T v, without forming the matrix. */
static void gram_times(orc_problem *P, const double *v, double *out) {
  at_times(P, v, P->cg_t);
  for (int64_t j = 0; j < P->nnz; ++j) P->cg_t[j] *= P->w[j] / P->D[j];
  a_times(P, P->cg_t, out);
}

static double dot_m(int m, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < m; ++i) s += a[i] * b[i];
  return s;
}

/* Switches the affine step to preconditioned conjugate gradients (max_iter
 * > 0) or back to the cached factor (max_iter = 0).  The preconditioner is
 * the diagonal of A W D^-1 A^T: sum_j A_ij^2 w_j / D_j. */
int orc_set_affine_cg(orc_problem *P, int max_iter, double tol) {
  if (max_iter < 0 || !(tol >= 0)) return ORC_ERR_ARG;
  P->cg_max_iter = max_iter;
  P->cg_tol = tol;
  if (max_iter == 0 || P->cg_diag) return ORC_OK;
  int m = P->m > 0 ? P->m : 1;
  P->cg_diag = (double *)calloc(m, sizeof(double));
  P->cg_r = (double *)calloc(m, sizeof(double));
  P->cg_z = (double *)calloc(m, sizeof(double));
  P->cg_p = (double *)calloc(m, sizeof(double));
  P->cg_Mp = (double *)calloc(m, sizeof(double));
  P->cg_t = (double *)calloc(P->nnz, sizeof(double));
  for (int i = 0; i < P->m; ++i) {
    double s = 0.0;
    if (P->a_format == 0) {
      for (int64_t j = 0; j < P->nnz; ++j) {
        double a = P->a_val[(size_t)i * P->nnz + j];
        s += a * a * P->w[j] / P->D[j];
      }
    } else {
      for (int64_t t = P->a_rowptr[i]; t < P->a_rowptr[i + 1]; ++t)
        s += P->a_val[t] * P->a_val[t] * P->w[P->a_col[t]] / P->D[P->a_col[t]];
    }
    P->cg_diag[i] = s;
  }
  return ORC_OK;
}

/* Preconditioned conjugate gradients (Saad, Iterative Methods for Sparse
 * Linear Systems, the preconditioned CG algorithm with a left/split Jacobi
 * preconditioner) on (A W D^-1 A^T) y = rhs from the y passed in.  Before
 * every step the residual is tested: ||r||_2 <= tol_abs stops.  Optional
 * history of ||r_j||_2 (j = 0..steps).  Returns the steps taken. */
int orc_pcg(orc_problem *P, const double *rhs, double *y, int max_iter, double tol_abs,
            double *hist_rnorm) {
  const int m = P->m;
  double *r = P->cg_r, *z = P->cg_z, *p = P->cg_p, *Mp = P->cg_Mp;
  gram_times(P, y, Mp);
  for (int i = 0; i < m; ++i) r[i] = rhs[i] - Mp[i];
  for (int i = 0; i < m; ++i) z[i] = r[i] / P->cg_diag[i];
  for (int i = 0; i < m; ++i) p[i] = z[i];
  double rz = dot_m(m, r, z);
  double rn = sqrt(dot_m(m, r, r));
  if (hist_rnorm) hist_rnorm[0] = rn;
  int j = 0;
  while (j < max_iter && !(rn <= tol_abs)) {
    gram_times(P, p, Mp);
    const double alpha = rz / dot_m(m, p, Mp);
    for (int i = 0; i < m; ++i) y[i] += alpha * p[i];
    for (int i = 0; i < m; ++i) r[i] -= alpha * Mp[i];
    for (int i = 0; i < m; ++i) z[i] = r[i] / P->cg_diag[i];
    const double rz_new = dot_m(m, r, z);
    const double beta = rz_new / rz;
    for (int i = 0; i < m; ++i) p[i] = z[i] + beta * p[i];
    rz = rz_new;
    rn = sqrt(dot_m(m, r, r));
    ++j;
    if (hist_rnorm) hist_rnorm[j] = rn;
  }
  return j;
}

/* Solve the KKT system (OptCondMinYPrimal) for given bhat by block
 * elimination (KKTflops): L L^T y = A W D^-1 bhat - b, u = D^-1(bhat - A^T y). */
void orc_affine(orc_problem *P, const double *bhat, const double *bvec,
                double *u, double *y) {
  for (int64_t j = 0; j < P->nnz; ++j) P->tmp[j] = P->w[j] * bhat[j] / P->D[j];
  a_times(P, P->tmp, P->r);
  for (int i = 0; i < P->m; ++i) P->r[i] -= bvec[i];
  orc_chol_solve(P->m, P->L, P->r, y);
  at_times(P, y, P->tmp);
  for (int64_t j = 0; j < P->nnz; ++j) u[j] = (bhat[j] - P->tmp[j]) / P->D[j];
}

/* The same elimination with y from orc_pcg, started at the y of the previous
 * iteration (Algorithm 1 in conjugate-gradient mode). */
static void affine_cg(orc_problem *P, const double *bhat, const double *bvec, double *u,
                      double *y) {
  for (int64_t j = 0; j < P->nnz; ++j) P->tmp[j] = P->w[j] * bhat[j] / P->D[j];
  a_times(P, P->tmp, P->r);
  for (int i = 0; i < P->m; ++i) P->r[i] -= bvec[i];
  const double tol_abs = P->cg_tol * (1.0 + sqrt(dot_m(P->m, bvec, bvec)));
  P->cg_steps += orc_pcg(P, P->r, y, P->cg_max_iter, tol_abs, NULL);
  at_times(P, y, P->tmp);
  for (int64_t j = 0; j < P->nnz; ++j) u[j] = (bhat[j] - P->tmp[j]) / P->D[j];
}

int64_t orc_cg_steps(const orc_problem *P) { return P->cg_steps; }

/* E_k U E_k^T as a full s x s block. */
static void gather_block(const orc_problem *P, int k, const double *u, double *Uk) {
  int s = P->cptr[k + 1] - P->cptr[k];
  int64_t o = P->blk_off[k];
  for (int e = 0; e < s * s; ++e) Uk[e] = u[P->loc[o + e]];
}

static double ratio(double num, double den) {
  if (den > 0.0) return num / den;
  return (num == 0.0) ? 0.0 : INFINITY;
}

/* Runs up to max_iter iterations of Algorithm 1 from the current state.
 * Stops when max(eps_c, eps_lambda) <= tol.  Returns ORC_OK when it stopped
 * on the tolerance, ORC_MAX_ITER otherwise.  Optional per-iteration history
 * (length max_iter) of eps_c, eps_lambda and the rho used in the iteration. */
int orc_run(orc_problem *P, int max_iter, double tol, int adaptive, double mu,
            double nu, int rho_period, int *iters_done, double *hist_eps_c,
            double *hist_eps_l, double *hist_rho) {
  if (!P->L && P->cg_max_iter <= 0) return ORC_ERR_ARG;   /* no factor: CG mode only */
  int p = P->p;
  double *part = (double *)calloc((size_t)p * 5, sizeof(double));
  int *sweeps = (int *)calloc(p, sizeof(int));
  int done = 0, it;
  for (it = 0; it < max_iter; ++it) {
    double rho = P->rho;
    /* x-update */
    orc_form_bhat(P, P->X, P->Lam, rho, P->bhat);
    if (P->cg_max_iter > 0) affine_cg(P, P->bhat, P->b, P->u, P->y);
    else orc_affine(P, P->bhat, P->b, P->u, P->y);
    memcpy(P->Xprev, P->X, sizeof(double) * P->nblk);
    /* clique projections and multiplier updates (independent over k) */
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < p; ++k) {
      int s = P->cptr[k + 1] - P->cptr[k];
      int64_t o = P->blk_off[k];
      double *Uk = (double *)malloc(sizeof(double) * s * s);
      double *Wk = (double *)malloc(sizeof(double) * s * s);
      gather_block(P, k, P->u, Uk);
      for (int e = 0; e < s * s; ++e) Wk[e] = Uk[e] - P->Lam[o + e] / rho;
      sweeps[k] = orc_psd_project(s, Wk, P->X + o, NULL, NULL, P->jac_max_sweeps,
                                  P->jac_tol);
      double r_c = 0, n_x = 0, n_hx = 0, r_d = 0, n_l = 0;
      for (int e = 0; e < s * s; ++e) {
        double xk = P->X[o + e];
        P->Lam[o + e] += rho * (xk - Uk[e]);
        double dc = xk - Uk[e], dx = xk - P->Xprev[o + e], lk = P->Lam[o + e];
        r_c += dc * dc; n_x += xk * xk; n_hx += Uk[e] * Uk[e];
        r_d += dx * dx; n_l += lk * lk;
      }
      part[5 * k + 0] = r_c; part[5 * k + 1] = n_x; part[5 * k + 2] = n_hx;
      part[5 * k + 3] = r_d; part[5 * k + 4] = n_l;
      free(Uk); free(Wk);
    }
    double S[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < p; ++k) {
      for (int t = 0; t < 5; ++t) S[t] += part[5 * k + t];
      P->total_sweeps += sweeps[k];
      if (sweeps[k] > P->max_sweeps_seen) P->max_sweeps_seen = sweeps[k];
    }
    /* residuals (PrimalConsensusResidual) */
    double den_c = sqrt(S[1]) > sqrt(S[2]) ? sqrt(S[1]) : sqrt(S[2]);
    P->eps_c = ratio(sqrt(S[0]), den_c);
    P->eps_l = ratio(rho * sqrt(S[3]), sqrt(S[4]));
    if (hist_eps_c) hist_eps_c[it] = P->eps_c;
    if (hist_eps_l) hist_eps_l[it] = P->eps_l;
    if (hist_rho) hist_rho[it] = rho;
    P->iters++;
    double e = P->eps_c > P->eps_l ? P->eps_c : P->eps_l;
    if (e <= tol) { done = 1; ++it; break; }
    /* adaptive penalty */
    if (adaptive && rho_period > 0 && (P->iters % rho_period) == 0) {
      if (P->eps_c >= nu * P->eps_l) P->rho = mu * rho;
      else if (P->eps_l >= nu * P->eps_c) P->rho = rho / mu;
    }
  }
  if (iters_done) *iters_done = it;
  free(part); free(sweeps);
  return done ? ORC_OK : ORC_MAX_ITER;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 2: ADMM for the range-space decomposition of the dual-form SDP   */
/* ------------------------------------------------------------------------- */

/* Runs up to max_iter iterations of Algorithm 2 from the current state
 * (z_k in X, lambda_k in Lam, v_k in Vd, x in u, y in y).  One iteration, in
 * the order the algorithm lists its steps:
 *   z_k = P+(v_k - lambda_k / rho)                                 (zkUpdate)
 *   (x, y) from the KKT system with right-hand side
 *     c - sum_k H_k^T (z_k + lambda_k / rho) and -b / rho     (OptCondMinYDual)
 *   v_k = z_k + lambda_k / rho + H_k x                               (vkEqn)
 *   lambda_k += rho (z_k - v_k)                              (MultUpdateDualSDP)
 *   eps_c, eps_lambda as in DualConsensusResidual; stop, adaptive rho.
 * On compact coordinates the KKT system reads D_j x_j + sum_i A_ij y_i = rhs_j
 * and sum_j w_j A_ij x_j = -b_i / rho: the primal solve with other data.
 * Same return values and history as orc_run. */
int orc_run_dual(orc_problem *P, int max_iter, double tol, int adaptive, double mu,
                 double nu, int rho_period, int *iters_done, double *hist_eps_c,
                 double *hist_eps_l, double *hist_rho) {
  if (!P->L) return ORC_ERR_ARG;
  int p = P->p;
  double *part = (double *)calloc((size_t)p * 5, sizeof(double));
  int *sweeps = (int *)calloc(p, sizeof(int));
  double *bvec = (double *)malloc(sizeof(double) * (P->m > 0 ? P->m : 1));
  int done = 0, it;
  for (it = 0; it < max_iter; ++it) {
    double rho = P->rho;
    /* z-update: independent projections */
    memcpy(P->Xprev, P->X, sizeof(double) * P->nblk);
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < p; ++k) {
      int s = P->cptr[k + 1] - P->cptr[k];
      int64_t o = P->blk_off[k];
      double *Wk = (double *)malloc(sizeof(double) * s * s);
      for (int e = 0; e < s * s; ++e) Wk[e] = P->Vd[o + e] - P->Lam[o + e] / rho;
      sweeps[k] = orc_psd_project(s, Wk, P->X + o, NULL, NULL, P->jac_max_sweeps,
                                  P->jac_tol);
      free(Wk);
    }
    /* (x, y): right-hand side c - sum_k H_k^T (z_k + lambda_k / rho), summed
       over the lower entries of the blocks in increasing k */
    for (int64_t j = 0; j < P->nnz; ++j) P->bhat[j] = 0.0;
    for (int k = 0; k < p; ++k) {
      int s = P->cptr[k + 1] - P->cptr[k];
      int64_t o = P->blk_off[k];
      for (int a = 0; a < s; ++a)
        for (int bb = 0; bb <= a; ++bb) {
          int64_t e = o + (int64_t)a * s + bb;
          P->bhat[P->loc[e]] += P->X[e] + P->Lam[e] / rho;
        }
    }
    for (int64_t j = 0; j < P->nnz; ++j) P->bhat[j] = P->c[j] - P->bhat[j];
    for (int i = 0; i < P->m; ++i) bvec[i] = -P->b[i] / rho;
    orc_affine(P, P->bhat, bvec, P->u, P->y);
    /* v and lambda updates, residual partial sums */
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < p; ++k) {
      int s = P->cptr[k + 1] - P->cptr[k];
      int64_t o = P->blk_off[k];
      double r_c = 0, n_z = 0, n_v = 0, r_d = 0, n_l = 0;
      for (int e = 0; e < s * s; ++e) {
        double zk = P->X[o + e];
        double vk = zk + P->Lam[o + e] / rho + P->u[P->loc[o + e]];
        double lk = P->Lam[o + e] + rho * (zk - vk);
        P->Vd[o + e] = vk;
        P->Lam[o + e] = lk;
        double dc = zk - vk, dz = zk - P->Xprev[o + e];
        r_c += dc * dc; n_z += zk * zk; n_v += vk * vk;
        r_d += dz * dz; n_l += lk * lk;
      }
      part[5 * k + 0] = r_c; part[5 * k + 1] = n_z; part[5 * k + 2] = n_v;
      part[5 * k + 3] = r_d; part[5 * k + 4] = n_l;
    }
    double S[5] = {0, 0, 0, 0, 0};
    for (int k = 0; k < p; ++k) {
      for (int t = 0; t < 5; ++t) S[t] += part[5 * k + t];
      P->total_sweeps += sweeps[k];
      if (sweeps[k] > P->max_sweeps_seen) P->max_sweeps_seen = sweeps[k];
    }
    /* residuals (DualConsensusResidual) */
    double den_c = sqrt(S[1]) > sqrt(S[2]) ? sqrt(S[1]) : sqrt(S[2]);
    P->eps_c = ratio(sqrt(S[0]), den_c);
    P->eps_l = ratio(rho * sqrt(S[3]), sqrt(S[4]));
    if (hist_eps_c) hist_eps_c[it] = P->eps_c;
    if (hist_eps_l) hist_eps_l[it] = P->eps_l;
    if (hist_rho) hist_rho[it] = rho;
    P->iters++;
    double e = P->eps_c > P->eps_l ? P->eps_c : P->eps_l;
    if (e <= tol) { done = 1; ++it; break; }
    if (adaptive && rho_period > 0 && (P->iters % rho_period) == 0) {
      if (P->eps_c >= nu * P->eps_l) P->rho = mu * rho;
      else if (P->eps_l >= nu * P->eps_c) P->rho = rho / mu;
    }
  }
  if (iters_done) *iters_done = it;
  free(part); free(sweeps); free(bvec);
  return done ? ORC_OK : ORC_MAX_ITER;
}

/* ------------------------------------------------------------------------- */
/* Algorithm 3: ADMM for the homogeneous self-dual embedding (Section 5)      */
/* ------------------------------------------------------------------------- */
/* Vectors over the pattern are compact lower coordinates: the paper's
 * Euclidean products on vec(X) become sums weighted by w (1 on the diagonal,
 * 2 off it), A x becomes A (w .* x), and the identity stays the identity.
 * Clique blocks s, t, z are full s_k x s_k matrices (plain Frobenius
 * products). */

/* sum over the lower entries of every clique block into the coordinates:
 * the compact form of H^T applied to blocks (increasing k) */
static void h_transpose(const orc_problem *P, const double *blocks, double *out) {
  for (int64_t j = 0; j < P->nnz; ++j) out[j] = 0.0;
  for (int k = 0; k < P->p; ++k) {
    int s = P->cptr[k + 1] - P->cptr[k];
    int64_t o = P->blk_off[k];
    for (int a = 0; a < s; ++a)
      for (int bb = 0; bb <= a; ++bb) {
        int64_t e = o + (int64_t)a * s + bb;
        out[P->loc[e]] += blocks[e];
      }
  }
}

static double wdot(const orc_problem *P, const double *a, const double *b) {
  double acc = 0.0;
  for (int64_t j = 0; j < P->nnz; ++j) acc += P->w[j] * a[j] * b[j];
  return acc;
}

/* The "inner" system M sigma = nu with M = [[I, -Ahat^T], [Ahat, I]],
 * Ahat = [[A, 0], [H, -I]] (SecondBlockElimination), by the two block
 * eliminations and the matrix inversion lemma of Section 5.2.2:
 *   nu_x' = nu_x + H^T (nu_s + nu_t) / 2
 *   g     = (I + A P^-1 A^T)^-1 (A P^-1 nu_x' - nu_y)
 *   sigma_x = P^-1 (nu_x' - A^T g),  sigma_y = -g
 *   sigma_s = (nu_s - nu_t + H sigma_x) / 2,  sigma_t = sigma_s - H sigma_x + nu_t */
static void hsde_inner(orc_problem *P, const double *nx, const double *ns, const double *ny,
                       const double *nt, double *sx, double *ss, double *sy, double *st) {
  const int64_t nnz = P->nnz, nb = P->nblk;
  double *sum = (double *)malloc(sizeof(double) * nb);
  double *xp = (double *)malloc(sizeof(double) * nnz);
  double *tmp = (double *)malloc(sizeof(double) * nnz);
  double *r = (double *)malloc(sizeof(double) * (P->m > 0 ? P->m : 1));
  for (int64_t e = 0; e < nb; ++e) sum[e] = 0.5 * (ns[e] + nt[e]);
  h_transpose(P, sum, xp);
  for (int64_t j = 0; j < nnz; ++j) xp[j] += nx[j];
  for (int64_t j = 0; j < nnz; ++j) tmp[j] = P->w[j] * xp[j] / P->hP[j];
  a_times(P, tmp, r);
  for (int i = 0; i < P->m; ++i) r[i] -= ny[i];
  orc_chol_solve(P->m, P->Lh, r, sy);            /* g, stored in sy for now */
  at_times(P, sy, tmp);
  for (int64_t j = 0; j < nnz; ++j) sx[j] = (xp[j] - tmp[j]) / P->hP[j];
  for (int i = 0; i < P->m; ++i) sy[i] = -sy[i];
  for (int k = 0; k < P->p; ++k) {
    int s = P->cptr[k + 1] - P->cptr[k];
    int64_t o = P->blk_off[k];
    for (int e = 0; e < s * s; ++e) {
      const double hx = sx[P->loc[o + e]];
      ss[o + e] = 0.5 * (ns[o + e] - nt[o + e] + hx);
      st[o + e] = ss[o + e] - hx + nt[o + e];
    }
  }
  free(sum); free(xp); free(tmp); free(r);
}

/* zeta^T (x, s, y, t) with zeta = (c, 0, -b, 0) */
static double zeta_dot(const orc_problem *P, const double *x, const double *y) {
  double acc = wdot(P, P->c, x);
  for (int i = 0; i < P->m; ++i) acc -= P->b[i] * y[i];
  return acc;
}

/* Data preprocessing of Algorithm 3: factor I + A W P^-1 A^T
 * (HSDEFactorizationFinal on compact coordinates), M^-1 zeta and
 * 1 / (1 + zeta^T M^-1 zeta); u = (0, 0, 0, 0, 1), v = (0, 0, 0, 0, 1). */
int orc_hsde_setup(orc_problem *P) {
  const int m = P->m;
  const int64_t nnz = P->nnz, nb = P->nblk;
  if (!P->Lh) {
    double *wd = (double *)malloc(sizeof(double) * nnz);
    P->hP = (double *)malloc(sizeof(double) * nnz);
    for (int64_t j = 0; j < nnz; ++j) {
      P->hP[j] = 1.0 + 0.5 * P->D[j];
      wd[j] = P->w[j] / P->hP[j];
    }
    double *M = (double *)calloc((size_t)m * m, sizeof(double));
    assemble_gram(P, wd, M);
    for (int i = 0; i < m; ++i) M[(size_t)i * m + i] += 1.0;
    P->Lh = (double *)malloc(sizeof(double) * (size_t)m * m);
    int rc = orc_cholesky(m, M, P->Lh);
    free(M); free(wd);
    if (rc != ORC_OK) return rc;
    P->ux = (double *)calloc(nnz, sizeof(double)); P->us = (double *)calloc(nb, sizeof(double));
    P->uy = (double *)calloc(m, sizeof(double));   P->ut = (double *)calloc(nb, sizeof(double));
    P->vz = (double *)calloc(nb, sizeof(double));
    P->mzx = (double *)calloc(nnz, sizeof(double)); P->mzs = (double *)calloc(nb, sizeof(double));
    P->mzy = (double *)calloc(m, sizeof(double));   P->mzt = (double *)calloc(nb, sizeof(double));
    P->hx = (double *)calloc(nnz, sizeof(double)); P->hs = (double *)calloc(nb, sizeof(double));
    P->hy = (double *)calloc(m, sizeof(double));   P->ht = (double *)calloc(nb, sizeof(double));
    P->hx2 = (double *)calloc(nnz, sizeof(double)); P->hs2 = (double *)calloc(nb, sizeof(double));
    P->hy2 = (double *)calloc(m, sizeof(double));   P->ht2 = (double *)calloc(nb, sizeof(double));
    /* M^-1 zeta: nu = (c, 0, -b, 0) */
    double *zs = (double *)calloc(nb, sizeof(double));
    double *zy = (double *)malloc(sizeof(double) * m);
    for (int i = 0; i < m; ++i) zy[i] = -P->b[i];
    hsde_inner(P, P->c, zs, zy, zs, P->mzx, P->mzs, P->mzy, P->mzt);
    P->kz = 1.0 / (1.0 + zeta_dot(P, P->mzx, P->mzy));
    free(zs); free(zy);
  }
  memset(P->ux, 0, sizeof(double) * nnz); memset(P->us, 0, sizeof(double) * nb);
  memset(P->uy, 0, sizeof(double) * m);   memset(P->ut, 0, sizeof(double) * nb);
  memset(P->vz, 0, sizeof(double) * nb);
  P->utau = 1.0;
  P->kappa = 1.0;
  P->iters = 0;
  P->eps_c = P->eps_l = P->eps_p = P->eps_d = P->eps_g = INFINITY;
  P->hsde_status = ORC_MAX_ITER;
  P->total_sweeps = 0;
  P->max_sweeps_seen = 0;
  return ORC_OK;
}

static double cratio(double num, double a, double b) {
  double den = a > b ? a : b;
  if (den > 0.0) return num / den;
  return (num == 0.0) ? 0.0 : INFINITY;
}

/* Runs up to max_iter iterations of Algorithm 3 (after orc_hsde_setup):
 *   u_hat = (I + Q)^-1 (u + v)       (HsdeStep1: LinearSystem, MatrixInverseResult,
 *                                     FirstBlockElimination, hsde_inner)
 *   u = P_K(u_hat - v)               (HsdeStep2: x, y, t free, s in the PSD cones
 *                                     of the cliques, tau >= 0)
 *   v = v - u_hat + u                (HsdeStep3; only z and kappa are nonzero)
 * then, with tau > 0, the residuals HSDEerror and the consensus residual
 * (the larger of PrimalConsensusResidual on (s, H x) and DualConsensusResidual
 * on (z, t)); with tau = 0 the two infeasibility tests of Infeasibility.
 * Returns ORC_OK (solved), 2 (primal infeasible), 3 (dual infeasible) or
 * ORC_MAX_ITER.  Optional histories of max(eps_p, eps_d, eps_g) and eps_c. */
int orc_run_hsde(orc_problem *P, int max_iter, double tol, int *iters_done, double *hist_e,
                 double *hist_c) {
  const int m = P->m, p = P->p;
  const int64_t nnz = P->nnz, nb = P->nblk;
  double nb2 = 0.0, nc2 = wdot(P, P->c, P->c);
  for (int i = 0; i < m; ++i) nb2 += P->b[i] * P->b[i];
  const double nrm_b = sqrt(nb2), nrm_c = sqrt(nc2);
  double *hxs = (double *)malloc(sizeof(double) * nb);
  double *ax = (double *)malloc(sizeof(double) * (m > 0 ? m : 1));
  double *aty = (double *)malloc(sizeof(double) * nnz);
  double *zc = (double *)malloc(sizeof(double) * nnz);
  double *tmp = (double *)malloc(sizeof(double) * nnz);
  int *sweeps = (int *)calloc(p, sizeof(int));
  int status = ORC_MAX_ITER, it;
  for (it = 0; it < max_iter; ++it) {
    /* omega = u + v; nu = omega_1 - omega_2 zeta */
    const double w2 = P->utau + P->kappa;
    for (int64_t j = 0; j < nnz; ++j) P->hx[j] = P->ux[j] - w2 * P->c[j];
    for (int64_t e = 0; e < nb; ++e) P->hs[e] = P->us[e] + P->vz[e];
    for (int i = 0; i < m; ++i) P->hy[i] = P->uy[i] + w2 * P->b[i];
    memcpy(P->ht, P->ut, sizeof(double) * nb);
    /* sigma = M^-1 nu; u_hat_1 = sigma - M^-1 zeta (zeta^T sigma) / (1 + zeta^T M^-1 zeta) */
    hsde_inner(P, P->hx, P->hs, P->hy, P->ht, P->hx2, P->hs2, P->hy2, P->ht2);
    const double f = P->kz * zeta_dot(P, P->hx2, P->hy2);
    for (int64_t j = 0; j < nnz; ++j) P->hx2[j] -= f * P->mzx[j];
    for (int64_t e = 0; e < nb; ++e) { P->hs2[e] -= f * P->mzs[e]; P->ht2[e] -= f * P->mzt[e]; }
    for (int i = 0; i < m; ++i) P->hy2[i] -= f * P->mzy[i];
    const double uhat_tau = w2 + zeta_dot(P, P->hx2, P->hy2);
    /* u = P_K(u_hat - v), v = v - u_hat + u */
    memcpy(P->ux, P->hx2, sizeof(double) * nnz);
    memcpy(P->uy, P->hy2, sizeof(double) * m);
    memcpy(P->ut, P->ht2, sizeof(double) * nb);
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < p; ++k) {
      int s = P->cptr[k + 1] - P->cptr[k];
      int64_t o = P->blk_off[k];
      double *Wk = (double *)malloc(sizeof(double) * s * s);
      for (int e = 0; e < s * s; ++e) Wk[e] = P->hs2[o + e] - P->vz[o + e];
      sweeps[k] = orc_psd_project(s, Wk, P->us + o, NULL, NULL, P->jac_max_sweeps, P->jac_tol);
      for (int e = 0; e < s * s; ++e) P->vz[o + e] += P->us[o + e] - P->hs2[o + e];
      free(Wk);
    }
    const double tau_new = uhat_tau - P->kappa > 0.0 ? uhat_tau - P->kappa : 0.0;
    P->kappa += tau_new - uhat_tau;
    P->utau = tau_new;
    for (int k = 0; k < p; ++k) {
      P->total_sweeps += sweeps[k];
      if (sweeps[k] > P->max_sweeps_seen) P->max_sweeps_seen = sweeps[k];
    }
    P->iters++;
    /* stopping conditions */
    double crit;
    for (int64_t j = 0; j < nnz; ++j) tmp[j] = P->w[j] * P->ux[j];
    a_times(P, tmp, ax);                       /* A u_x */
    h_transpose(P, P->vz, zc);                 /* H^T v_z */
    at_times(P, P->uy, aty);                   /* A^T u_y */
    if (P->utau > 0.0) {
      const double tau = P->utau;
      double rp = 0.0, rd = 0.0;
      for (int i = 0; i < m; ++i) { double d = ax[i] / tau - P->b[i]; rp += d * d; }
      for (int64_t j = 0; j < nnz; ++j) {
        double d = (aty[j] + zc[j]) / tau - P->c[j];
        rd += P->w[j] * d * d;
      }
      const double ctx = wdot(P, P->c, P->ux) / tau;
      double bty = 0.0;
      for (int i = 0; i < m; ++i) bty += P->b[i] * P->uy[i];
      bty /= tau;
      P->eps_p = sqrt(rp) / (1.0 + nrm_b);
      P->eps_d = sqrt(rd) / (1.0 + nrm_c);
      P->eps_g = fabs(ctx - bty) / (1.0 + fabs(ctx) + fabs(bty));
      /* consensus residuals on (s, H x) and (z, t) */
      double pc = 0, ns2 = 0, nh2 = 0, dc = 0, nz2 = 0, nt2 = 0;
      for (int k = 0; k < p; ++k) {
        int s = P->cptr[k + 1] - P->cptr[k];
        int64_t o = P->blk_off[k];
        for (int e = 0; e < s * s; ++e) {
          const double hx = P->ux[P->loc[o + e]];
          const double a1 = P->us[o + e] - hx, a2 = P->vz[o + e] - P->ut[o + e];
          pc += a1 * a1; ns2 += P->us[o + e] * P->us[o + e]; nh2 += hx * hx;
          dc += a2 * a2; nz2 += P->vz[o + e] * P->vz[o + e]; nt2 += P->ut[o + e] * P->ut[o + e];
        }
      }
      const double c1 = cratio(sqrt(pc), sqrt(ns2), sqrt(nh2));
      const double c2 = cratio(sqrt(dc), sqrt(nz2), sqrt(nt2));
      P->eps_c = c1 > c2 ? c1 : c2;
      crit = P->eps_p;
      if (P->eps_d > crit) crit = P->eps_d;
      if (P->eps_g > crit) crit = P->eps_g;
      if (hist_e) hist_e[it] = crit;
      if (hist_c) hist_c[it] = P->eps_c;
      if (P->eps_c > crit) crit = P->eps_c;
      if (crit <= tol) { status = ORC_OK; ++it; break; }
    } else {
      if (hist_e) hist_e[it] = INFINITY;
      if (hist_c) hist_c[it] = INFINITY;
      /* Infeasibility: ||A^T u_y + H^T v_z|| - (b^T u_y / ||b||) tol <= 0 certifies
         primal infeasibility, ||A u_x|| + (c^T u_x / ||c||) tol <= 0 dual infeasibility */
      double r1 = 0.0, r2 = 0.0, bty = 0.0;
      for (int i = 0; i < m; ++i) { r1 += ax[i] * ax[i]; bty += P->b[i] * P->uy[i]; }
      for (int64_t j = 0; j < nnz; ++j) {
        double d = aty[j] + zc[j];
        r2 += P->w[j] * d * d;
      }
      const double ctx = wdot(P, P->c, P->ux);
      const double tp = sqrt(r2) - (nrm_b > 0 ? bty / nrm_b : 0.0) * tol;
      const double td = sqrt(r1) + (nrm_c > 0 ? ctx / nrm_c : 0.0) * tol;
      if (tp <= 0.0 && bty > 0.0) { status = 2; ++it; break; }
      if (td <= 0.0 && ctx < 0.0) { status = 3; ++it; break; }
    }
  }
  P->hsde_status = status;
  if (iters_done) *iters_done = it;
  free(hxs); free(ax); free(aty); free(zc); free(tmp); free(sweeps);
  return status;
}

/* Accessors of the Algorithm 3 iterate: x = u_x / tau, y = u_y / tau (or the
 * raw u_x, u_y when tau = 0), out = (tau, kappa, eps_p, eps_d, eps_g, eps_c). */
void orc_hsde_get(const orc_problem *P, double *x, double *y, double *s_blocks,
                  double *z_blocks, double *t_blocks, double *out) {
  const double sc = P->utau > 0.0 ? 1.0 / P->utau : 1.0;
  if (x) for (int64_t j = 0; j < P->nnz; ++j) x[j] = P->ux[j] * sc;
  if (y) for (int i = 0; i < P->m; ++i) y[i] = P->uy[i] * sc;
  if (s_blocks) memcpy(s_blocks, P->us, sizeof(double) * P->nblk);
  if (z_blocks) memcpy(z_blocks, P->vz, sizeof(double) * P->nblk);
  if (t_blocks) memcpy(t_blocks, P->ut, sizeof(double) * P->nblk);
  if (out) {
    out[0] = P->utau; out[1] = P->kappa; out[2] = P->eps_p; out[3] = P->eps_d;
    out[4] = P->eps_g; out[5] = P->eps_c;
  }
}

/* One-step access for tests: M^-1 zeta and the inner solve. */
void orc_hsde_inner(orc_problem *P, const double *nx, const double *ns, const double *ny,
                    const double *nt, double *sx, double *ss, double *sy, double *st) {
  hsde_inner(P, nx, ns, ny, nt, sx, ss, sy, st);
}

void orc_hsde_set(orc_problem *P, const double *ux, const double *us, const double *uy,
                  const double *ut, const double *vz, double utau, double kappa) {
  memcpy(P->ux, ux, sizeof(double) * P->nnz);
  memcpy(P->us, us, sizeof(double) * P->nblk);
  memcpy(P->uy, uy, sizeof(double) * P->m);
  memcpy(P->ut, ut, sizeof(double) * P->nblk);
  memcpy(P->vz, vz, sizeof(double) * P->nblk);
  P->utau = utau;
  P->kappa = kappa;
}

void orc_hsde_raw(const orc_problem *P, double *ux, double *uy) {
  if (ux) memcpy(ux, P->ux, sizeof(double) * P->nnz);
  if (uy) memcpy(uy, P->uy, sizeof(double) * P->m);
}

/* Dual objective b^T y of the current iterate of Algorithm 2. */
double orc_dual_objective(const orc_problem *P) {
  double acc = 0.0;
  for (int i = 0; i < P->m; ++i) acc += P->b[i] * P->y[i];
  return acc;
}

void orc_get_vd(const orc_problem *P, double *V) { memcpy(V, P->Vd, sizeof(double) * P->nblk); }
void orc_set_vd(orc_problem *P, const double *V) { memcpy(P->Vd, V, sizeof(double) * P->nblk); }

/* ------------------------------------------------------------------------- */
/* Accessors and diagnostics                                                 */
/* ------------------------------------------------------------------------- */

int64_t orc_nblk(const orc_problem *P) { return P->nblk; }
double orc_rho(const orc_problem *P) { return P->rho; }
int orc_iters(const orc_problem *P) { return P->iters; }
double orc_eps_c(const orc_problem *P) { return P->eps_c; }
double orc_eps_l(const orc_problem *P) { return P->eps_l; }
int64_t orc_total_sweeps(const orc_problem *P) { return P->total_sweeps; }
int orc_max_sweeps_seen(const orc_problem *P) { return P->max_sweeps_seen; }

void orc_get_u(const orc_problem *P, double *u) { memcpy(u, P->u, sizeof(double) * P->nnz); }
void orc_get_y(const orc_problem *P, double *y) { memcpy(y, P->y, sizeof(double) * P->m); }
void orc_get_D(const orc_problem *P, double *D) { memcpy(D, P->D, sizeof(double) * P->nnz); }
void orc_get_L(const orc_problem *P, double *L) {
  memcpy(L, P->L, sizeof(double) * (size_t)P->m * P->m);
}
void orc_get_blocks(const orc_problem *P, double *X, double *Lam) {
  if (X) memcpy(X, P->X, sizeof(double) * P->nblk);
  if (Lam) memcpy(Lam, P->Lam, sizeof(double) * P->nblk);
}
void orc_set_blocks(orc_problem *P, const double *X, const double *Lam) {
  if (X) memcpy(P->X, X, sizeof(double) * P->nblk);
  if (Lam) memcpy(P->Lam, Lam, sizeof(double) * P->nblk);
}
void orc_set_rho(orc_problem *P, double rho) { P->rho = rho; }

/* W_k = E_k U E_k^T - Lambda_k/rho for the current state, blocks concatenated
 * (the inputs of the projections of the next iteration). */
void orc_next_w(orc_problem *P, double *W) {
  orc_form_bhat(P, P->X, P->Lam, P->rho, P->bhat);
  double *u = (double *)malloc(sizeof(double) * P->nnz);
  double *y = (double *)malloc(sizeof(double) * (P->m > 0 ? P->m : 1));
  orc_affine(P, P->bhat, P->b, u, y);
  for (int k = 0; k < P->p; ++k) {
    int s = P->cptr[k + 1] - P->cptr[k];
    int64_t o = P->blk_off[k];
    gather_block(P, k, u, W + o);
    for (int e = 0; e < s * s; ++e) W[o + e] -= P->Lam[o + e] / P->rho;
  }
  free(u); free(y);
}

/* <C, X> on the compact coordinates: sum_j w_j c_j u_j. */
double orc_objective(const orc_problem *P) {
  double acc = 0.0;
  for (int64_t j = 0; j < P->nnz; ++j) acc += P->w[j] * P->c[j] * P->u[j];
  return acc;
}

/* Diagnostics of the current iterate: out[0] = eps_p, out[1] = eps_d,
 * out[2] = eps_g (HSDEerror with x = u, y_dual = -rho*y and
 * z = sum_k H_k^T lambda_k), out[3] = eps_alpha (PSD-violation),
 * out[4] = objective <C,X>, out[5] = b^T y_dual.  Norms of symmetric
 * matrices are full (off-diagonal entries weighted by 2). */
void orc_diagnostics(orc_problem *P, double *out) {
  int m = P->m;
  int64_t nnz = P->nnz;
  double *ax = (double *)calloc(m > 0 ? m : 1, sizeof(double));
  double *tmp = (double *)calloc(nnz, sizeof(double));
  double *z = (double *)calloc(nnz, sizeof(double));
  double *yd = (double *)calloc(m > 0 ? m : 1, sizeof(double));
  for (int64_t j = 0; j < nnz; ++j) tmp[j] = P->w[j] * P->u[j];
  a_times(P, tmp, ax);
  double np = 0, nb = 0;
  for (int i = 0; i < m; ++i) { double d = ax[i] - P->b[i]; np += d * d; nb += P->b[i] * P->b[i]; }
  for (int i = 0; i < m; ++i) yd[i] = -P->rho * P->y[i];
  for (int k = 0; k < P->p; ++k) {
    int s = P->cptr[k + 1] - P->cptr[k];
    int64_t o = P->blk_off[k];
    for (int a = 0; a < s; ++a)
      for (int bb = 0; bb <= a; ++bb) z[P->loc[o + (int64_t)a * s + bb]] += P->Lam[o + (int64_t)a * s + bb];
  }
  at_times(P, yd, tmp);
  double nd = 0, nc = 0, ctx = 0, bty = 0, nx = 0;
  for (int64_t j = 0; j < nnz; ++j) {
    double d = tmp[j] + z[j] - P->c[j];
    nd += P->w[j] * d * d;
    nc += P->w[j] * P->c[j] * P->c[j];
    ctx += P->w[j] * P->c[j] * P->u[j];
    nx += P->w[j] * P->u[j] * P->u[j];
  }
  for (int i = 0; i < m; ++i) bty += P->b[i] * yd[i];
  double lmin = 0.0;
  for (int k = 0; k < P->p; ++k) {
    int s = P->cptr[k + 1] - P->cptr[k];
    double *Uk = (double *)malloc(sizeof(double) * s * s);
    double *V = (double *)malloc(sizeof(double) * s * s);
    double *th = (double *)malloc(sizeof(double) * s);
    gather_block(P, k, P->u, Uk);
    orc_jacobi_eig(s, Uk, V, th, P->jac_max_sweeps, P->jac_tol);
    for (int i = 0; i < s; ++i) if (th[i] < lmin) lmin = th[i];
    free(Uk); free(V); free(th);
  }
  out[0] = sqrt(np) / (1.0 + sqrt(nb));
  out[1] = sqrt(nd) / (1.0 + sqrt(nc));
  out[2] = fabs(ctx - bty) / (1.0 + fabs(ctx) + fabs(bty));
  out[3] = (-lmin) / (1.0 + sqrt(nx));
  out[4] = ctx;
  out[5] = bty;
  free(ax); free(tmp); free(z); free(yd);
}

/* E_k U E_k^T for every clique (blocks concatenated, full s_k x s_k). */
void orc_gather_blocks(const orc_problem *P, const double *u, double *blocks) {
  for (int k = 0; k < P->p; ++k) gather_block(P, k, u, blocks + P->blk_off[k]);
}

/* ------------------------------------------------------------------------- */
/* Reverse mode of the unrolled iteration (differentiation w.r.t. C and b)    */
/* ------------------------------------------------------------------------- */

/* Derivative of the PSD projection at W = V diag(theta) V^T applied to a
 * symmetric direction G (Daleckii-Krein):  D P+(W)[G] = V (Gam o (V^T G V)) V^T
 * with Gam_ij = (max(th_i,0) - max(th_j,0)) / (th_i - th_j) when the signs
 * differ, 1 when both are positive and 0 when both are <= 0.  The map is
 * self-adjoint, so it is also the vector-Jacobian product. */
void orc_psd_project_derivative(int s, const double *V, const double *th, const double *G,
                                double *out) {
  double *T1 = (double *)calloc((size_t)s * s, sizeof(double));
  double *T2 = (double *)calloc((size_t)s * s, sizeof(double));
  /* T1 = V^T G */
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (int k = 0; k < s; ++k) acc += V[k * s + i] * G[k * s + j];
      T1[i * s + j] = acc;
    }
  /* T2 = (T1 V) o Gam */
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (int k = 0; k < s; ++k) acc += T1[i * s + k] * V[k * s + j];
      double gam;
      if (th[i] > 0.0 && th[j] > 0.0) gam = 1.0;
      else if (!(th[i] > 0.0) && !(th[j] > 0.0)) gam = 0.0;
      else gam = ((th[i] > 0 ? th[i] : 0.0) - (th[j] > 0 ? th[j] : 0.0)) / (th[i] - th[j]);
      T2[i * s + j] = acc * gam;
    }
  /* T1 = V T2 */
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (int k = 0; k < s; ++k) acc += V[i * s + k] * T2[k * s + j];
      T1[i * s + j] = acc;
    }
  /* out = T1 V^T */
  for (int i = 0; i < s; ++i)
    for (int j = 0; j < s; ++j) {
      double acc = 0.0;
      for (int k = 0; k < s; ++k) acc += T1[i * s + k] * V[j * s + k];
      out[i * s + j] = acc;
    }
  free(T1);
  free(T2);
}

/* T iterations of Algorithm 1 from X_k = Lambda_k = 0 with fixed rho (no
 * stopping test), then the vector-Jacobian product of u_T.  Cotangents of
 * symmetric-matrix quantities (u, c) are taken w.r.t. the Frobenius inner
 * product, <x, x'> = sum_j w_j x_j x'_j on the compact coordinates; the
 * cotangent of b is Euclidean.  Given ubar it returns u_T, cbar and bbar.
 *
 * Forward, per iteration: bhat = sum_k H_k^T (X_k + L_k/rho) - c/rho;
 * (u, y) from the KKT system; U_k = H_k u; W_k = U_k - L_k/rho;
 * X_k' = P+(W_k); L_k' = L_k + rho (X_k' - U_k).  The reverse sweep takes
 * these steps backwards; the affine map u = P bhat + Q b is self-adjoint in
 * bhat for the Frobenius product, so its VJP is one more KKT solve with
 * b = 0, whose multiplier is the cotangent of b. */
int orc_unrolled_vjp(orc_problem *P, int T, double rho, const double *ubar, double *u_T,
                     double *cbar, double *bbar) {
  const int p = P->p;
  const int64_t nnz = P->nnz, nb = P->nblk;
  orc_reset(P, rho);
  double *Vst = (double *)malloc(sizeof(double) * (size_t)T * nb);
  int64_t nth = 0;
  for (int k = 0; k < p; ++k) nth += P->cptr[k + 1] - P->cptr[k];
  double *thst = (double *)malloc(sizeof(double) * (size_t)T * nth);
  int64_t *thoff = (int64_t *)malloc(sizeof(int64_t) * (p + 1));
  thoff[0] = 0;
  for (int k = 0; k < p; ++k) thoff[k + 1] = thoff[k] + (P->cptr[k + 1] - P->cptr[k]);
  double *zero_b = (double *)calloc(P->m > 0 ? P->m : 1, sizeof(double));
  /* forward */
  for (int t = 0; t < T; ++t) {
    orc_form_bhat(P, P->X, P->Lam, rho, P->bhat);
    orc_affine(P, P->bhat, P->b, P->u, P->y);
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < p; ++k) {
      int s = P->cptr[k + 1] - P->cptr[k];
      int64_t o = P->blk_off[k];
      double *Uk = (double *)malloc(sizeof(double) * s * s);
      double *Wk = (double *)malloc(sizeof(double) * s * s);
      gather_block(P, k, P->u, Uk);
      for (int e = 0; e < s * s; ++e) Wk[e] = Uk[e] - P->Lam[o + e] / rho;
      orc_psd_project(s, Wk, P->X + o, thst + (size_t)t * nth + thoff[k],
                      Vst + (size_t)t * nb + o, P->jac_max_sweeps, P->jac_tol);
      for (int e = 0; e < s * s; ++e) P->Lam[o + e] += rho * (P->X[o + e] - Uk[e]);
      free(Uk); free(Wk);
    }
  }
  memcpy(u_T, P->u, sizeof(double) * nnz);
  /* reverse */
  double *Xb = (double *)calloc(nb, sizeof(double));
  double *Lb = (double *)calloc(nb, sizeof(double));
  double *Ub = (double *)calloc(nb, sizeof(double));
  double *ub = (double *)malloc(sizeof(double) * nnz);
  double *bhb = (double *)malloc(sizeof(double) * nnz);
  double *yb = (double *)calloc(P->m > 0 ? P->m : 1, sizeof(double));
  for (int64_t j = 0; j < nnz; ++j) cbar[j] = 0.0;
  for (int i = 0; i < P->m; ++i) bbar[i] = 0.0;
  for (int t = T - 1; t >= 0; --t) {
    /* steps 6', 5', 4' for every clique (zero cotangents at t = T-1) */
#pragma omp parallel for schedule(dynamic, 1)
    for (int k = 0; k < p; ++k) {
      int s = P->cptr[k + 1] - P->cptr[k];
      int64_t o = P->blk_off[k];
      double *G = (double *)malloc(sizeof(double) * s * s);
      double *Wb = (double *)malloc(sizeof(double) * s * s);
      for (int e = 0; e < s * s; ++e) {
        G[e] = Xb[o + e] + rho * Lb[o + e];   /* cotangent of X_k' */
        Ub[o + e] = -rho * Lb[o + e];
      }
      orc_psd_project_derivative(s, Vst + (size_t)t * nb + o,
                                 thst + (size_t)t * nth + thoff[k], G, Wb);
      for (int e = 0; e < s * s; ++e) {
        Ub[o + e] += Wb[e];
        Lb[o + e] -= Wb[e] / rho;
      }
      free(G); free(Wb);
    }
    /* step 3': ubar of this iteration's u (the adjoint of the gather) */
    for (int64_t j = 0; j < nnz; ++j) ub[j] = (t == T - 1) ? ubar[j] : 0.0;
    for (int k = 0; k < p; ++k) {
      int s = P->cptr[k + 1] - P->cptr[k];
      int64_t o = P->blk_off[k];
      for (int e = 0; e < s * s; ++e) {
        int64_t j = P->loc[o + e];
        ub[j] += Ub[o + e] / P->w[j];
      }
    }
    /* step 2': one KKT solve with b = 0 */
    orc_affine(P, ub, zero_b, bhb, yb);
    for (int i = 0; i < P->m; ++i) bbar[i] += yb[i];
    /* step 1': the adjoint of bhat = sum H_k^T (X_k + L_k/rho) - c/rho */
    for (int64_t j = 0; j < nnz; ++j) cbar[j] -= bhb[j] / rho;
    for (int k = 0; k < p; ++k) {
      int s = P->cptr[k + 1] - P->cptr[k];
      int64_t o = P->blk_off[k];
      for (int e = 0; e < s * s; ++e) {
        double g = bhb[P->loc[o + e]];
        Xb[o + e] = g;
        Lb[o + e] += g / rho;
      }
    }
  }
  free(Vst); free(thst); free(thoff); free(zero_b);
  free(Xb); free(Lb); free(Ub); free(ub); free(bhb); free(yb);
  return ORC_OK;
}

/* Replace C and b of the problem (A and the factor are unchanged). */
void orc_set_cb(orc_problem *P, const double *c, const double *b) {
  if (c) memcpy(P->c, c, sizeof(double) * P->nnz);
  if (b) memcpy(P->b, b, sizeof(double) * P->m);
}
