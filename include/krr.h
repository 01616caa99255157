/*
 * krr.h -- C ABI of the MI355X (gfx950) random-features-preconditioned kernel ridge
 * regression library (libkrr.so).
 *
 * Method: Avron, Clarkson, Woodruff, "Faster Kernel Ridge Regression Using Sketching
 * and Preconditioning" (arXiv 1611.03220). The library solves Eq. 1,
 *     (K + lambda I_n) c = y,   K_ij = exp(-||x_i - x_j||^2 / (2 sigma^2))   (Sec. 6),
 * by PCG (Alg. 1) with the preconditioner Z Z^T + lambda_p I_n built from random
 * Fourier features Z = sqrt(2/s) cos(X W + b) (Sec. 2.2) and applied through its
 * Woodbury form lambda_p^{-1} (I - U^T U), U = C^{-1} Z^T, C C^T = Z^T Z + lambda_p I_s
 * (Sec. 3.1; Alg. 1). The kernel matrix is never stored: every product
 * recomputes it tile by tile from X.
 *
 * Conventions shared by every entry point
 *   - All array arguments are DEVICE pointers (HIP global memory) owned by the caller,
 *     except those documented as host pointers. Matrices are row-major with an explicit
 *     leading dimension (elements between consecutive rows, >= the row length).
 *   - Points X are FP32 (n x d). Right-hand sides, solutions and kernel-product operands
 *     are FP64. Features Z and the preconditioner factor U^T are FP32.
 *   - `stream` is a hipStream_t (NULL = the null stream). Work is enqueued on it.
 *   - No entry point allocates device memory. Scratch space is the caller's `ws` buffer
 *     (device, 256-byte aligned) of at least krr_workspace_bytes(...) bytes; the library
 *     does not keep a reference to it after the call returns.
 *   - Every call returns a krr_status. On failure the outputs are undefined unless stated
 *     otherwise, and krr_last_error() describes the failure. No exception or abort
 *     crosses the ABI.
 *   - Calls are thread-safe as long as concurrent calls use distinct workspaces.
 */
#ifndef KRR_H
#define KRR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum krr_status {
  KRR_OK = 0,
  KRR_E_ARG = 1,        /* invalid argument: null pointer, bad size or stride, lambda <= 0,
                           sigma <= 0, s >= n, tol <= 0 (the paper assumes lambda > 0, s < n,
                           epsilon > 0: Sec. 2.1, Sec. 3.1, Alg. 1) */
  KRR_E_NOT_SPD = 2,    /* Z^T Z + lambda_p I not numerically positive definite (info set) */
  KRR_E_NO_CONV = 3,    /* PCG reached max_iter; alpha holds the last iterate, report filled */
  KRR_E_BREAKDOWN = 4,  /* non-finite data or <p, A p> <= 0 in some column; that column frozen */
  KRR_E_HIP = 5,        /* a HIP runtime call failed */
  KRR_E_WORKSPACE = 6   /* ws is NULL, misaligned or smaller than krr_workspace_bytes() */
} krr_status;

/* Arithmetic of the kernel product K V (Sec. 3.1: the dominant per-iteration cost). */
typedef enum krr_prec {
  KRR_PREC_FP64 = 0,   /* FP64-class distances, FP64 exp, FP64 sums ("plain FP64 path"):
                          for d <= 128 the inner products are exact integer sums of the rows
                          in 46-bit fixed point (relative to each row's largest coordinate),
                          computed on int8 MFMA; for larger d FP64 products of the FP32
                          coordinates */
  KRR_PREC_F16X3 = 1,  /* distances on MFMA from FP16 hi+lo splits of the (power-of-two
                          scaled) points, 3 products hi*hi + hi*lo + lo*hi, FP32 accumulate;
                          FP32 exp2; FP32 products with V, FP64 sums across tiles (default) */
  KRR_PREC_BF16X3 = 2  /* as F16X3 with BF16 hi+lo splits (16 instead of 22 mantissa bits) */
} krr_prec;

/* Operation codes for krr_workspace_bytes. */
typedef enum krr_op {
  KRR_OP_FEATURES = 0,
  KRR_OP_PRECOND_FACTOR = 1,
  KRR_OP_KERNEL_MATMAT = 2,
  KRR_OP_PCG_SOLVE = 3,
  KRR_OP_GRAD = 4,
  KRR_OP_PRECOND_APPLY = 5,
  KRR_OP_DSIGMA_INNER = 6
} krr_op;

/*
 * krr_workspace_bytes -- size of the device workspace an operation needs.
 *   op   : a krr_op code.
 *   n1   : points (rows) of the operation; n2: columns of a cross kernel product
 *          (KRR_OP_KERNEL_MATMAT; pass n2 = n1 otherwise).
 *   d, s, m : dimension, feature count, right-hand sides (0 where not used).
 *   prec : a krr_prec (kernel-product arithmetic).
 * Returns 0 for an unknown op.
 */
size_t krr_workspace_bytes(int32_t op, int64_t n1, int64_t n2, int64_t d, int64_t s, int64_t m,
                           int32_t prec);

/* Thread-local description of the last failure on this thread ("" if none). */
const char* krr_last_error(void);

/* Library version string. */
const char* krr_version(void);

/*
 * krr_features -- random Fourier features, the feature map of Alg. 1 (Sec. 2.2):
 *     Z[i, l] = sqrt(2/s) * cos( sum_k X[i, k] W[k, l] + b[l] ).
 * The scale is sqrt(2/s) (not the printed s^{-1/2}): with it E[z(x)^T z(y)] = k(x, y).
 *   X  : n x d FP32, leading dimension ldx >= d.
 *   W  : d x s FP32 row-major (leading dimension s); columns w_l ~ N(0, sigma^-2 I) drawn by
 *        the caller.
 *   b  : s FP32 offsets in [0, 2 pi), drawn by the caller.
 *   Z  : n x s FP32 output, leading dimension ldz >= s.
 * The product X W runs on MFMA from FP16 hi+lo splits (power-of-two scaled, three
 * products, FP32 accumulate); cos is the accurate FP32 cosine. Asynchronous on `stream`.
 * Errors: KRR_E_ARG, KRR_E_WORKSPACE.
 */
krr_status krr_features(const float* X, int64_t n, int64_t d, int64_t ldx, const float* W,
                        const float* b, int64_t s, float* Z, int64_t ldz, void* ws,
                        size_t ws_bytes, void* stream);

/*
 * krr_precond_factor -- preconditioner set-up of Alg. 1 (Woodbury form, Sec. 3.1):
 *     G = Z^T Z + lambda_p I_s,  C C^T = G (C lower, FP64),  Ut = Z C^{-T}  (= U^T, n x s).
 * Then (Z Z^T + lambda_p I)^{-1} v = (v - Ut (Ut^T v)) / lambda_p.
 *   Z   : n x s FP32, leading dimension ldz >= s (s < n).
 *   lambda_p : > 0 (Alg. 1 uses lambda_p = lambda; Table 2 varies it).
 *   C   : s x s FP64 output, row-major, leading dimension s; lower triangle is the factor,
 *         the strict upper triangle is set to zero.
 *   Ut  : n x s FP32 output, leading dimension ldu >= s: row i is (C^{-1} z_i)^T.
 *   info: HOST pointer; 0 on success, else the 1-based index of the first non-positive
 *         pivot (then KRR_E_NOT_SPD is returned and C, Ut are undefined).
 * The Gram product runs on MFMA from FP16 hi+lo splits with FP64 sums; the Cholesky and
 * the triangular inverse run in FP64; Ut is formed by one GEMM with C^{-1} (GEMM instead
 * of per-iteration triangular solves, as Sec. 3.1 argues). Synchronises `stream`.
 */
krr_status krr_precond_factor(const float* Z, int64_t n, int64_t s, int64_t ldz, double lambda_p,
                              double* C, float* Ut, int64_t ldu, void* ws, size_t ws_bytes,
                              int64_t* info, void* stream);

/*
 * krr_precond_apply -- the preconditioner step of the PCG in Alg. 1, in the Woodbury form of
 * Sec. 3.1:  Zout = (Z Z^T + lambda_p I)^{-1} R = (R - Ut (Ut^T R)) / lambda_p.
 *   Ut : n x s FP32 from krr_precond_factor (ldu >= s), s < n.
 *   R  : n x m FP64 (ldr >= m);  Zout: n x m FP64 (ldz >= m), must not alias R.
 *   lambda_p : > 0, the value Ut was built with.
 * Two streaming passes over Ut with FP64 accumulation (workspace: krr_workspace_bytes with
 * KRR_OP_PRECOND_APPLY, n1 = n, s, m). Asynchronous on `stream`. Errors: KRR_E_ARG,
 * KRR_E_WORKSPACE.
 */
krr_status krr_precond_apply(const float* Ut, int64_t n, int64_t s, int64_t ldu, double lambda_p,
                             const double* R, int64_t m, int64_t ldr, double* Zout, int64_t ldz,
                             void* ws, size_t ws_bytes, void* stream);

/*
 * krr_kernel_matmat -- matrix-free kernel product (the per-iteration product of the PCG in
 * Alg. 1; Sec. 3.1 cost discussion):
 *     OUT[i, :] = sum_j k(x1_i, x2_j) V[j, :] + shift * V[i, :],
 * with k the Gaussian kernel of Sec. 6, or, with deriv = 1, its sigma-derivative
 * dk/dsigma = k * ||x1_i - x2_j||^2 / sigma^3.
 *   X1 : n1 x d FP32 (ldx1 >= d);  X2 : n2 x d FP32 (ldx2 >= d).
 *   V  : n2 x m FP64 (ldv >= m);   OUT: n1 x m FP64 (ldo >= m), must not alias V.
 *   shift : requires n1 == n2 when non-zero (square case: shift = lambda gives (K + lambda I) V).
 *   prec  : a krr_prec. Squared distances are not clamped at zero: where rounding leaves one
 *           slightly negative (coincident points), k comes out slightly above 1, within the
 *           product's error bound; a NaN coordinate propagates to every output it meets.
 * Asynchronous on `stream`. Errors: KRR_E_ARG, KRR_E_WORKSPACE.
 */
krr_status krr_kernel_matmat(const float* X1, int64_t n1, int64_t ldx1, const float* X2, int64_t n2,
                             int64_t ldx2, int64_t d, double sigma, double shift, const double* V,
                             int64_t m, int64_t ldv, double* OUT, int64_t ldo, int32_t deriv,
                             int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* Options of krr_pcg_solve (zero-initialise, then set what you need; see krr_pcg_defaults). */
typedef struct krr_pcg_opts {
  double tol;            /* stop when ||y_j - A c_j|| <= tol ||y_j|| for every column j (Sec. 6),
                            tracked on the recursive residual */
  int32_t max_iter;      /* iteration cap (the paper's ablation uses 1000) */
  int32_t prec;          /* krr_prec of the kernel products */
  int32_t use_precond;   /* 1: preconditioner from Ut (Alg. 1); 0: plain CG (Table 4 baseline) */
  int32_t check_every;   /* read the convergence count back to the host every k iterations */
  double lambda_p;       /* regulariser Ut was built with; <= 0 means lambda */
  int32_t true_residual; /* 1: at exit, compute the FP64 true residual per column */
  int32_t refine;        /* max outer refinement steps driven by the FP64 true residual
                            (0 = none); each step solves A delta = y - A c by PCG */
  int32_t warm_start;    /* 0: start from zero as in Thm. 1 (alpha's input is ignored);
                            1: start from the alpha passed in (resume a saved iterate) */
} krr_pcg_opts;

/* Report of krr_pcg_solve. Host arrays may be NULL; when given they hold m entries. */
typedef struct krr_pcg_report {
  int32_t iters;           /* PCG iterations (summed over refinement steps) */
  int32_t converged_cols;  /* columns meeting tol on the recursive residual */
  int32_t breakdown_cols;  /* columns frozen by breakdown */
  int32_t refine_steps;    /* outer refinement steps taken */
  double* relres_rec;      /* host[m]: recursive ||r_j|| / ||y_j|| at exit */
  double* relres_true;     /* host[m]: FP64 ||y_j - (K + lambda I) c_j|| / ||y_j|| (if requested) */
  double* history;         /* host[history_cap]: max relative recursive residual at each check */
  int32_t history_cap;
  int32_t history_len;
  int32_t matmat_calls;    /* kernel products in the solve precision (iterations, warm start) */
  double matmat_ms;        /* summed device time of those products (HIP events on `stream`);
                              the FP64 true-residual products are not included */
} krr_pcg_report;

/* Fill `o` with the defaults: tol 1e-6, max_iter 1000, F16X3, preconditioned, check every
 * iteration, lambda_p = lambda, true residual on, no refinement, zero start. */
void krr_pcg_defaults(krr_pcg_opts* o);

/*
 * krr_pcg_solve -- the solve of Alg. 1: (K + lambda I_n) alpha = Y by PCG with the
 * preconditioner (Z Z^T + lambda_p I)^{-1} = (I - Ut Ut^T) / lambda_p, one independent
 * PCG recurrence per right-hand side (columns freeze once converged; Sec. 6).
 *   X     : n x d FP32 (ldx >= d).   sigma > 0, lambda > 0.
 *   Ut, s, ldu : output of krr_precond_factor (ignored when opts->use_precond == 0).
 *   Y     : n x m FP64 right-hand sides (ldy >= m).
 *   alpha : n x m FP64 (lda >= m). On entry the starting point when opts->warm_start is 1
 *           (else ignored: the iteration starts from zero as in Thm. 1); on exit the
 *           solution.
 *   opts  : HOST pointer (NULL = defaults).  rep: HOST pointer (may be NULL).
 * CG scalars (inner products, step lengths) and the iterates x, r are FP64; the kernel
 * product uses opts->prec. Synchronises `stream`. Errors: KRR_E_ARG, KRR_E_WORKSPACE,
 * KRR_E_NO_CONV (alpha holds the last iterate, report filled), KRR_E_BREAKDOWN.
 */
krr_status krr_pcg_solve(const float* X, int64_t n, int64_t d, int64_t ldx, double sigma,
                         double lambda, const float* Ut, int64_t s, int64_t ldu, const double* Y,
                         int64_t ldy, double* alpha, int64_t lda, int64_t m,
                         const krr_pcg_opts* opts, krr_pcg_report* rep, void* ws, size_t ws_bytes,
                         void* stream);

/*
 * krr_grad -- hyper-parameter gradients of a loss through the solve of Eq. 1 (adjoint
 * method). Given alpha = A^{-1} Y and the adjoint abar = A^{-1} Gbar (A = K + lambda I):
 *     dL_dsigma  = - sum_ij <abar_i, alpha_j> dk(x_i, x_j)/dsigma   (= -<abar, (dK/dsigma) alpha>)
 *     dL_dlambda = - <abar, alpha>.
 *   X : n x d FP32 (ldx >= d).  alpha, abar : n x m FP64 (leading dimension ld >= m).
 *   dL_dsigma, dL_dlambda : HOST pointers.
 * The sigma term is one matrix-free product with dK/dsigma (krr_kernel_matmat, deriv = 1)
 * followed by an FP64 inner product. Synchronises `stream`.
 */
krr_status krr_grad(const float* X, int64_t n, int64_t d, int64_t ldx, double sigma,
                    const double* alpha, const double* abar, int64_t m, int64_t ld,
                    double* dL_dsigma, double* dL_dlambda, int32_t prec, void* ws, size_t ws_bytes,
                    void* stream);

/*
 * krr_kernel_dsigma_inner -- the direct sigma-term of a loss that reads a kernel product
 * (the validation prediction of a differentiated solve):
 *     out = <G, (dK(X1, X2)/dsigma) V> = sum_ij dk(x1_i, x2_j)/dsigma <G[i, :], V[j, :]>,
 * with dk/dsigma = k * ||x1_i - x2_j||^2 / sigma^3 (the Sec. 6 Gaussian kernel differentiated
 * in sigma). It is the term of dL/dsigma that does not pass through the solve; krr_grad
 * gives the term that does.
 *   X1 : n1 x d FP32 (ldx1 >= d);  X2 : n2 x d FP32 (ldx2 >= d).
 *   V  : n2 x m FP64 (ldv >= m);   G  : n1 x m FP64 (ldg >= m).
 *   out : HOST pointer, receives the FP64 sum.
 *   prec : a krr_prec for the dK/dsigma product (FP64 recommended: the two sigma-terms of a
 *          validation loss nearly cancel).
 * One matrix-free dK/dsigma product (as krr_kernel_matmat with deriv = 1) and an FP64 inner
 * product with G summed in a fixed order (deterministic). Workspace: krr_workspace_bytes with
 * KRR_OP_DSIGMA_INNER (n1, n2, d, 0, m, prec). Synchronises `stream`. Errors: KRR_E_ARG,
 * KRR_E_WORKSPACE.
 */
krr_status krr_kernel_dsigma_inner(const float* X1, int64_t n1, int64_t ldx1, const float* X2,
                                   int64_t n2, int64_t ldx2, int64_t d, double sigma,
                                   const double* V, int64_t m, int64_t ldv, const double* G,
                                   int64_t ldg, double* out, int32_t prec, void* ws,
                                   size_t ws_bytes, void* stream);

/*
 * krr_kernel_matmat_noalloc -- krr_kernel_matmat without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same arguments, semantics, arithmetic and kernels as
 * krr_kernel_matmat, minus ws / ws_bytes.
 * Scratch space: a fixed device array of KRR_NOALLOC_SCRATCH_BYTES inside the library, one
 * per GPU, created when the library's code is loaded on that GPU and held until the process
 * ends; the call itself allocates nothing. Problems whose krr_workspace_bytes(
 * KRR_OP_KERNEL_MATMAT, n1, n2, d, 0, m, prec) exceeds that size are rejected with
 * KRR_E_WORKSPACE (for example F16X3, d <= 128, m <= 16 fits up to about n1 = n2 = 16384).
 * Every call on one GPU shares that GPU's array and leaves its contents behind (nothing in it
 * needs to start at zero): calls that overlap on one GPU, from different streams or threads,
 * race on it and must be serialised by the caller. Asynchronous on `stream`. Errors:
 * KRR_E_ARG, KRR_E_WORKSPACE (too large), KRR_E_HIP (the scratch address lookup failed).
 */
#define KRR_NOALLOC_SCRATCH_BYTES (64ll << 20)
krr_status krr_kernel_matmat_noalloc(const float* X1, int64_t n1, int64_t ldx1, const float* X2,
                                     int64_t n2, int64_t ldx2, int64_t d, double sigma,
                                     double shift, const double* V, int64_t m, int64_t ldv,
                                     double* OUT, int64_t ldo, int32_t deriv, int32_t prec,
                                     void* stream);

/* ----------------------------------------------------------------------------------------
 * Batched solves: many independent problems in one plan. Every iteration runs ONE persistent
 * kernel-product launch over a work queue of (problem, 128-row block, column range) items for
 * all problems at once, plus batched CG and preconditioner kernels; the iteration is captured
 * once in a hipGraph and replayed until every column of every problem has converged. The
 * work-item granularity is chosen by timing candidates when the plan is created.
 * Products use KRR_PREC_F16X3. The plan owns device memory (allocated at creation, freed by
 * krr_batch_plan_destroy); krr_batch_solve allocates nothing.
 */
#define KRR_BATCH_MAX_M 16

/* One problem of a batch; all arrays are device memory owned by the caller and must stay
 * valid for the plan's lifetime (the plan keeps the pointers). */
typedef struct krr_batch_problem {
  const float* X;      /* n x d FP32 points (ldx >= d) */
  int64_t n, d, ldx;
  double sigma;        /* > 0 */
  double lambda;       /* > 0 */
  double lambda_p;     /* preconditioner regulariser Ut was built with; <= 0 means lambda */
  const float* Ut;     /* krr_precond_factor output (n x s, ldu), or NULL for plain CG */
  int64_t s, ldu;
  const double* Y;     /* n x m right-hand sides (ldy >= m) */
  int64_t ldy;
  double* alpha;       /* n x m solution (lda >= m); written by krr_batch_solve */
  int64_t lda;
  int64_t m;           /* 1 <= m <= KRR_BATCH_MAX_M */
} krr_batch_problem;

typedef struct krr_batch_plan krr_batch_plan;

typedef struct krr_batch_report {
  int32_t iters;           /* replayed iterations, over all refinement solves */
  int32_t converged_cols;  /* over all problems */
  int32_t breakdown_cols;
  int32_t refine_steps;    /* batched FP64-residual refinement steps (opts->refine) */
  double* relres_rec;      /* host[count * KRR_BATCH_MAX_M] or NULL: problem p column c at
                              p * KRR_BATCH_MAX_M + c (recursive residual) */
  double* relres_true;     /* same layout, FP64 true residual (opts->true_residual) or NULL */
  int32_t* col_iters;      /* same layout or NULL: iterations of each column's first solve */
  double product_ms;       /* device time of one batched kernel product (autotuned) */
  double iteration_ms;     /* average device time of one replayed iteration graph */
  int32_t tiles_per_item;  /* autotuned work-item size, in 64-column tiles */
  int32_t work_items;      /* items in the persistent product's queue */
} krr_batch_report;

/*
 * krr_batch_plan_create -- prepare `count` problems (Eq. 1 each, solved as in Alg. 1) for
 * batched PCG: validates them, prepares points, builds the work queues, autotunes the
 * product's work-item size and captures one iteration in a hipGraph. The points are
 * prepared here: a plan serves later changes of Y, Ut contents or alpha's memory, not of X
 * or sigma. opts: HOST pointer (NULL = defaults; opts->prec must be KRR_PREC_F16X3;
 * use_precond = 0 ignores every Ut; refine > 0 adds up to that many refinement steps, each
 * a batched solve of A delta = Y - A alpha for the columns whose FP64 true residual is
 * still above tol; lambda_p and warm_start are not used: each problem carries its own
 * lambda_p). The plan owns its device memory (about
 * 5 * 8 * sum(n_p) * M bytes of vectors, where M is the widest m_p, plus the prepared points
 * and the product partials). Synchronises `stream`. Errors: KRR_E_ARG, KRR_E_HIP.
 */
krr_status krr_batch_plan_create(const krr_batch_problem* probs, int32_t count,
                                 const krr_pcg_opts* opts, krr_batch_plan** plan, void* stream);

/*
 * krr_batch_solve -- run the plan: zero start (Thm. 1), replay the iteration graph until all
 * problems meet opts->tol on every column or opts->max_iter, write each problem's alpha.
 * rep: HOST pointer (may be NULL). Synchronises `stream`. Errors: KRR_E_ARG, KRR_E_HIP,
 * KRR_E_NO_CONV, KRR_E_BREAKDOWN (alpha written in every case).
 */
krr_status krr_batch_solve(krr_batch_plan* plan, krr_batch_report* rep, void* stream);

/* Free everything the plan owns (NULL is ignored). */
void krr_batch_plan_destroy(krr_batch_plan* plan);

#ifdef __cplusplus
}
#endif
#endif /* KRR_H */
