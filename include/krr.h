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
  KRR_OP_DSIGMA_INNER = 6,
  KRR_OP_GAUSSIAN_PROJECT = 7,  /* n1 = n, d = s2 (input width), s = s3 (output width) */
  KRR_OP_PRECOND_TEST = 8,      /* n1 = n, d, s (candidate width), prec */
  KRR_OP_ADAPTIVE_FEATURES = 9, /* n1 = n, d, s = s_max, prec */
  KRR_OP_AUTOTUNE = 10          /* n1 = n, d, m, prec */
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
 *           With KRR_PREC_F16X3 and d + 2 past a multiple of 32 (d = 31, 32, 63, 64, 95, 96)
 *           the squared norms are added to the exponent in FP32 after the split inner
 *           products instead of through two extra operand columns.
 * When X1 and X2 are the same array (same pointer, n1 == n2, ldx1 == ldx2) the product is
 * K(X, X) V and K is symmetric: with KRR_PREC_F16X3, d > 126 and passes of up to 16
 * columns, each off-diagonal pair of 128-row blocks is formed once and serves both
 * triangles (the transposed contributions are summed exactly in 64-bit fixed point, so
 * repeated calls give identical results). The workspace size (KRR_OP_KERNEL_MATMAT) covers
 * this case whenever n1 == n2.
 * Asynchronous on `stream`. Errors: KRR_E_ARG, KRR_E_WORKSPACE.
 */
krr_status krr_kernel_matmat(const float* X1, int64_t n1, int64_t ldx1, const float* X2, int64_t n2,
                             int64_t ldx2, int64_t d, double sigma, double shift, const double* V,
                             int64_t m, int64_t ldv, double* OUT, int64_t ldo, int32_t deriv,
                             int32_t prec, void* ws, size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------------------
 * Set-up of many problems at once (features and factor of Alg. 1 for each, e.g. before a
 * batched solve). The features and Gram matrices are spread over up to
 * KRR_SETUP_MAX_STREAMS internal streams (default priority), largest problem first to the
 * least loaded stream. The factor of one problem alone is a chain of short, latency-bound
 * kernels (the blocked Cholesky and the doubling inverse), so the FP64 factors of all
 * problems then advance together on `stream`: one launch per 64-column step (and per
 * doubling level) covers every problem that still has that step. C and Ut = Z C^{-T} are
 * formed on the streams again, and all pivots are checked once at the end. Results are
 * bit for bit those of krr_features and krr_precond_factor per problem.
 */
#define KRR_SETUP_MAX_STREAMS 4

typedef struct krr_setup_problem {
  const float* X;            /* n x d FP32 points (ldx >= d), DEVICE */
  int64_t n, d, ldx;
  const float* W;            /* d x s FP32 random Fourier feature draw (leading dimension s) */
  const float* b;            /* s FP32 offsets */
  int64_t s;                 /* 1 <= s < n */
  double lambda_p;           /* > 0 */
  float* Z;                  /* n x s FP32 features, written (ldz >= s) */
  int64_t ldz;
  double* C;                 /* s x s FP64 factor, written (as krr_precond_factor) */
  float* Ut;                 /* n x s FP32, written (ldu >= s) */
  int64_t ldu;
  int64_t info;              /* written: 0, or the failing pivot + 1 */
} krr_setup_problem;

/* Workspace of krr_setup_many: one slot (the largest problem's features, or its factor's
 * operand splits and Gram partials) per stream, every problem's FP64 factor storage (about
 * 20 s_pad^2 bytes, s_pad = s rounded up to 64), pivot flags and launch descriptors.
 * Returns 0 when a problem's sizes are invalid (krr_setup_many then names it). */
size_t krr_setup_many_workspace_bytes(const krr_setup_problem* probs, int32_t count,
                                      int32_t nstreams);

/*
 * krr_setup_many -- krr_features then krr_precond_factor for each of `count` problems (HOST
 * array; each problem's info is written back), on min(nstreams, KRR_SETUP_MAX_STREAMS)
 * internal streams that start after the work already queued on `stream`; `stream` waits for
 * them and is synchronised before the call returns. Same arithmetic as the two single calls.
 * Errors: KRR_E_ARG (checked for every problem before any device work), KRR_E_WORKSPACE,
 * KRR_E_NOT_SPD (the first failing problem named in krr_last_error; every info is set),
 * KRR_E_HIP.
 */
krr_status krr_setup_many(krr_setup_problem* probs, int32_t count, int32_t nstreams, void* ws,
                          size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------------------
 * Kernel descriptor. The Gaussian kernel k(x, z) = exp(-||x - z||^2 / (2 sigma^2)) and the
 * polynomial kernel k(x, z) = (gamma x^T z + c)^q are the two kernels of the paper's
 * experiments (Sec. 6); the homogeneous polynomial kernel (gamma = 1, c = 0) is the kernel
 * of Sec. 2.2 and Thm. 1. The *_k entry points take it; the others are the Gaussian case.
 */
typedef enum krr_kernel_kind {
  KRR_KERNEL_GAUSSIAN = 0,
  KRR_KERNEL_POLYNOMIAL = 1
} krr_kernel_kind;

#define KRR_POLY_MAX_DEGREE 16

typedef struct krr_kernel {
  int32_t kind;     /* krr_kernel_kind */
  int32_t degree;   /* polynomial: q, 1 <= q <= KRR_POLY_MAX_DEGREE */
  double sigma;     /* Gaussian: bandwidth, > 0 */
  double gamma;     /* polynomial: scale, finite, >= 0 */
  double coef0;     /* polynomial: offset c, finite, >= 0 */
} krr_kernel;

/*
 * krr_kernel_matmat_k -- krr_kernel_matmat for a kernel descriptor. For the polynomial
 * kernel the F16X3 product forms gamma <x_i, x_j> + c on MFMA from FP16 hi+lo splits of
 * augmented rows [sqrt(gamma/T) x, sqrt(c/T)] (T the even power of two at or above
 * gamma max ||x||^2 + c, so the scaled value lies in [-1, 1]), raises it to q in FP32, splits
 * it into FP16 hi+lo for the MFMA product with V and multiplies the FP64 partial sums by T^q;
 * KRR_PREC_FP64 forms <x_i, x_j> exactly as for the Gaussian kernel and (gamma g + c)^q in
 * FP64. deriv must be 0 and prec must not be KRR_PREC_BF16X3 for the polynomial kernel.
 * Other arguments, workspace (krr_workspace_bytes with KRR_OP_KERNEL_MATMAT) and errors as
 * krr_kernel_matmat.
 */
krr_status krr_kernel_matmat_k(const krr_kernel* kernel, const float* X1, int64_t n1, int64_t ldx1,
                               const float* X2, int64_t n2, int64_t ldx2, int64_t d, double shift,
                               const double* V, int64_t m, int64_t ldv, double* OUT, int64_t ldo,
                               int32_t deriv, int32_t prec, void* ws, size_t ws_bytes,
                               void* stream);

/*
 * krr_tensorsketch -- TensorSketch features for the polynomial kernel (gamma x^T z + c)^q
 * (Sec. 2.2; the feature map of Thm. 1): each point is augmented to
 * x' = [sqrt(gamma) x, sqrt(c)] (one constant feature, the remark after Thm. 1) and mapped to
 *     Z[i, :] = IFFT( prod_{k<q} FFT( CountSketch_k(x'_i) ) ),
 * CountSketch_k(x')[b] = sum over j with hash[k][j] = b of sign[k][j] x'_j, which equals the
 * TensorSketch matrix (hash H = sum_k h_k(i_k) mod s, sign G = prod_k g_k(i_k)) applied to the
 * degree-q monomials of x', so E[Z Z^T] = K over random hashes and signs.
 *   X    : n x d FP32 (ldx >= d).
 *   gamma, coef0 : >= 0;  degree : q, 1 <= q <= KRR_POLY_MAX_DEGREE.
 *   hash : q x (d + 1) int32, row-major, DEVICE; values are taken modulo s; column d hashes
 *          the constant feature. Drawn by the caller (fully random tables satisfy the
 *          3-wise independence the definition asks for).
 *   sign : q x (d + 1) FP32 of +1 / -1, DEVICE, drawn by the caller.
 *   s    : a power of two, 2 <= s <= KRR_TENSORSKETCH_MAX_S.
 *   Z    : n x s FP32 output (ldz >= s).
 * One 256-thread block per point: the CountSketches are scattered into LDS, transformed by a
 * radix-2 FFT in LDS (FP32, accurate twiddles), multiplied, and transformed back. No
 * workspace. Asynchronous on `stream`. Errors: KRR_E_ARG.
 */
#define KRR_TENSORSKETCH_MAX_S 8192
krr_status krr_tensorsketch(const float* X, int64_t n, int64_t d, int64_t ldx, double gamma,
                            double coef0, int32_t degree, const int32_t* hash, const float* sign,
                            int64_t s, float* Z, int64_t ldz, void* stream);

/* ----------------------------------------------------------------------------------------
 * Multiple-level sketching (Sec. 4, Alg. 2): a first-level sketch Z_1 (n x s_1: random
 * Fourier features or TensorSketch) is compressed to Z_2 = Z_1 S_2^T by an SRHT, then to
 * Z_3 = s_3^{-1/2} Z_2 S_3^T by a Gaussian projection; krr_precond_factor(Z_3, lambda) then
 * gives the preconditioner Z_3 Z_3^T + lambda I of Alg. 2 (Thm. 3: O(s_lambda log s_lambda)
 * columns suffice after the SRHT).
 */
#define KRR_SRHT_MAX_S1 16384

/*
 * krr_srht -- Z2 = Z1 S^T for the subsampled randomized Walsh-Hadamard transform of Def. 2,
 *     S = s2^{-1/2} P H D  (s2 x s1),
 * D = diag(signs), H the +-1 Walsh-Hadamard matrix (H_m = [[H, H], [H, -H]]), P the rows
 * `sample` of the identity. A width s1 that is not a power of two is zero-padded to the next
 * power of two p (zero columns of Z1 do not change Z1 Z1^T); then H is p x p.
 *   Z1     : n x s1 FP32 (ldz1 >= s1);  p <= KRR_SRHT_MAX_S1.
 *   signs  : s1 FP32 of +1 / -1, DEVICE, drawn by the caller.
 *   sample : s2 int32 coordinates in [0, p) (taken modulo p), DEVICE, drawn by the caller
 *            (uniformly, without replacement, for Thm. 3's setting).
 *   Z2     : n x s2 FP32 output (ldz2 >= s2), 1 <= s2 <= p.
 * One 256-thread block per row: the signed row in LDS, the fast transform in place (log2 p
 * butterfly stages, FP32), a gather of the sampled coordinates. No workspace. Asynchronous on
 * `stream`. Errors: KRR_E_ARG.
 */
krr_status krr_srht(const float* Z1, int64_t n, int64_t s1, int64_t ldz1, const float* signs,
                    const int32_t* sample, int64_t s2, float* Z2, int64_t ldz2, void* stream);

/*
 * krr_gaussian_project -- Z3 = s3^{-1/2} Z2 S3^T, the dense third level of Alg. 2.
 *   Z2 : n x s2 FP32 (ldz2 >= s2).   S3 : s3 x s2 FP32 row-major, entries N(0, 1) drawn by
 *   the caller.   Z3 : n x s3 FP32 output (ldz3 >= s3).
 * One MFMA GEMM from FP16 hi+lo splits of both operands (three products, FP32 accumulate).
 * Workspace: krr_workspace_bytes(KRR_OP_GAUSSIAN_PROJECT, n, n, s2, s3, 0, KRR_PREC_F16X3).
 * Asynchronous on `stream`. Errors: KRR_E_ARG, KRR_E_WORKSPACE.
 */
krr_status krr_gaussian_project(const float* Z2, int64_t n, int64_t s2, int64_t ldz2,
                                const float* S3, int64_t s3, float* Z3, int64_t ldz3, void* ws,
                                size_t ws_bytes, void* stream);

/* ----------------------------------------------------------------------------------------
 * Adaptive sketch size (Sec. 5, Thm. 4). For a candidate sketch Z (n x s) let P project on the
 * eigenvectors of Z Z^T whose eigenvalues exceed 0.05 lambda. Thm. 4: if
 *   (1) ||(I - P) K (I - P)||_2 <= 0.1 lambda, and
 *   (2) ||V^T P x||^2 = (1 +- 0.1) ||Z^T P x||^2 for all x (K = V V^T),
 * then Z Z^T + lambda I is as good a preconditioner as Thm. 1 guarantees. The test below
 * estimates both sides by power iteration, as the paper suggests for condition 1; for
 * condition 2 (whose test the paper leaves open) it estimates the extreme eigenvalues of
 * W U^T K U W on range(P) (U the eigenvectors, W = diag(eigenvalue^-1/2)), which are the
 * extremes of that ratio. The adaptive driver doubles s until the test passes.
 */
typedef struct krr_precond_test_report {
  double cond1;           /* Rayleigh-quotient estimate of ||(I - P) K (I - P)||_2 (from below) */
  double ratio_lo;        /* estimate of the smallest ratio ||V^T P x||^2 / ||Z^T P x||^2 */
  double ratio_hi;        /* estimate of the largest ratio */
  int32_t rank;           /* dim range(P) */
  int32_t passed;         /* cond1 <= 0.1 lambda and 0.9 <= ratio_lo, ratio_hi <= 1.1 */
  int32_t power_iters;    /* iterations of each power iteration */
  int32_t jacobi_sweeps;  /* sweeps of the eigen-decomposition of Z^T Z */
} krr_precond_test_report;

/*
 * krr_precond_test -- the Thm. 4 test of a candidate sketch.
 *   kernel : the kernel of K (krr_kernel).  X : n x d FP32 (ldx >= d).
 *   Z      : n x s FP32 candidate (ldz >= s), 1 <= s < n.   lambda > 0.
 *   power_iters : iterations of each power iteration (>= 1; 30-50 is typical).
 *   prec   : arithmetic of the kernel products (a krr_prec).
 *   rep    : HOST pointer, filled.
 * Steps: Z^T Z + 5e-6 lambda I (split MFMA Gram, FP64 Cholesky C), eigen-decomposition of
 * C C^T by one-sided Jacobi rotations on the rows of C (FP64), U = Z V_k diag(e_k^-1/2) for
 * the eigenvalues above 0.05 lambda (split MFMA GEMM), then power iterations whose products
 * are matrix-free kernel products, Woodbury-type projections (I - U U^T) and GEMVs with U.
 * Workspace: krr_workspace_bytes(KRR_OP_PRECOND_TEST, n, n, d, s, 0, prec). Synchronises
 * `stream`. Errors: KRR_E_ARG, KRR_E_WORKSPACE, KRR_E_NOT_SPD (non-finite Z).
 */
krr_status krr_precond_test(const krr_kernel* kernel, const float* X, int64_t n, int64_t d,
                            int64_t ldx, const float* Z, int64_t s, int64_t ldz, double lambda,
                            int32_t power_iters, int32_t prec, krr_precond_test_report* rep,
                            void* ws, size_t ws_bytes, void* stream);

/*
 * krr_adaptive_features -- Sec. 5: starting from s = s0 features, form Z, run
 * krr_precond_test, and double s until the test passes or 2 s would exceed s_max.
 *   Gaussian kernel: W (d x s_max FP32, row-major) and b (s_max) are one random Fourier
 *     feature draw; the sketch of size s uses its first s columns (iid, so a valid draw of s
 *     features), scaled by sqrt(2/s).
 *   Polynomial kernel: hash, sign (degree x (d + 1), as krr_tensorsketch) with hash values in
 *     [0, s_max); size s takes them modulo s (s0 and every doubling must be powers of two
 *     <= KRR_TENSORSKETCH_MAX_S).
 *   Z       : n x s_max FP32 buffer (ldz >= s_max); on return its first *s_out columns hold
 *             the accepted sketch (the last one tried when none passed).
 *   s_out   : HOST, the chosen s.   history: HOST array of history_cap reports (may be NULL),
 *   history_len: HOST, the number of sizes tried.
 * Workspace: krr_workspace_bytes(KRR_OP_ADAPTIVE_FEATURES, n, n, d, s_max, 0, prec).
 * Synchronises `stream`. Errors: as krr_precond_test, KRR_E_ARG for a missing draw.
 */
krr_status krr_adaptive_features(const krr_kernel* kernel, const float* X, int64_t n, int64_t d,
                                 int64_t ldx, double lambda, const float* W, const float* b,
                                 const int32_t* hash, const float* sign, int64_t s0,
                                 int64_t s_max, float* Z, int64_t ldz, int64_t* s_out,
                                 krr_precond_test_report* history, int32_t history_cap,
                                 int32_t* history_len, int32_t power_iters, int32_t prec, void* ws,
                                 size_t ws_bytes, void* stream);

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
 * krr_pcg_solve_k -- krr_pcg_solve for a kernel descriptor: PCG on (K + lambda I) alpha = Y
 * with K from `kernel` (Gaussian or polynomial), the preconditioner from Ut (for the
 * polynomial kernel, built from krr_tensorsketch features as in Thm. 1), the same options,
 * report, workspace (KRR_OP_PCG_SOLVE) and errors. The polynomial kernel needs opts->prec
 * F16X3 or FP64; its FP64 true residual uses the FP64 product.
 */
krr_status krr_pcg_solve_k(const krr_kernel* kernel, const float* X, int64_t n, int64_t d,
                           int64_t ldx, double lambda, const float* Ut, int64_t s, int64_t ldu,
                           const double* Y, int64_t ldy, double* alpha, int64_t lda, int64_t m,
                           const krr_pcg_opts* opts, krr_pcg_report* rep, void* ws,
                           size_t ws_bytes, void* stream);

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
 * Autotuning of the kernel products. Launch choices (column splits of the product, and for
 * large d the right-hand-side pass width) are found by timing candidates on the device and
 * kept in a process-wide table keyed by (precision, padded width, ceil log2 m, floor log2 n);
 * every later product of that shape (krr_kernel_matmat*, krr_pcg_solve*, krr_grad, ...) uses
 * them. With the environment variable KRR_TUNE_CACHE set to a file path, the table is read
 * from it at first use and written back after every tuning; entries of another architecture
 * or another build of the kernels (krr_tune_digest) are ignored. Different split counts sum
 * the partial products in a different (still fixed) order, so a tuned product may differ from
 * the untuned one by rounding, within the product's error bound.
 */
typedef struct krr_tune_report {
  int32_t candidates;          /* launch choices timed */
  int32_t default_nsplit, default_pass_width;
  int32_t nsplit, pass_width;  /* the choice stored in the table */
  double default_ms, best_ms;  /* device time of one product: rule vs stored choice */
} krr_tune_report;

/*
 * krr_autotune_matmat -- time the candidate launch choices of the square product K(X, X) V
 * (m synthetic right-hand sides) and store the fastest (the rule's own choice unless a
 * candidate is at least 3 % faster).
 * Workspace: krr_workspace_bytes(KRR_OP_AUTOTUNE, n, n, d, 0, m, prec). rep: HOST pointer.
 * Synchronises `stream`. Errors: KRR_E_ARG, KRR_E_WORKSPACE, KRR_E_HIP.
 */
krr_status krr_autotune_matmat(const krr_kernel* kernel, const float* X, int64_t n, int64_t d,
                               int64_t ldx, int64_t m, int32_t prec, krr_tune_report* rep,
                               void* ws, size_t ws_bytes, void* stream);

/* Host-side tuning table: write it to / read it from `path` (1 on success, 0 otherwise; a file
 * of another architecture or build reads as 0 entries), drop every entry, count the entries,
 * and the digest of the kernel sources this library was built from. */
int32_t krr_tune_cache_save(const char* path);
int32_t krr_tune_cache_load(const char* path);
void krr_tune_cache_clear(void);
int32_t krr_tune_cache_size(void);
const char* krr_tune_digest(void);

/* ----------------------------------------------------------------------------------------
 * Batched solves: many independent problems in one plan. Every iteration runs ONE persistent
 * kernel-product launch over a work queue of (problem, 128-row block, column range) items for
 * all problems at once, plus batched CG and preconditioner kernels; opts->check_every
 * iterations (at most KRR_BATCH_MAX_GROUP) are captured once in a hipGraph, which is replayed
 * until every column of every problem has converged, with one host read of the active count
 * per replay (iterations therefore run in groups of check_every: a converged column is left
 * unchanged by the rest of its group, and max_iter is reached rounded up to a multiple of
 * check_every). The product's work items run the register-resident small-d body for
 * d <= 128 (operands round_up(d, 32) wide, the exponent's norm terms added in FP32 in its
 * epilogue) and the LDS-streamed body above; the work-item granularity is chosen by timing
 * candidates when the plan is created.
 * Products use KRR_PREC_F16X3. The plan owns device memory (allocated at creation, freed by
 * krr_batch_plan_destroy); krr_batch_solve allocates nothing.
 */
#define KRR_BATCH_MAX_M 16
#define KRR_BATCH_MAX_GROUP 16  /* iterations per replayed graph (opts->check_every cap) */

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
 * product's work-item size and captures opts->check_every iterations in a hipGraph. The points are
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
