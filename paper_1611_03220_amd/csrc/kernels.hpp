// Internal launcher declarations of libkrr (not part of the C ABI).
#pragma once
#include <algorithm>
#include "../../include/krr.h"
#include "common.hpp"

namespace krr {

template <typename T> struct MixedPoints {
  const T* hi;
  const T* lo;
  int64_t n;      // valid rows (arrays hold round_up(n, ROW_PAD) rows)
  int64_t Kp;     // padded augmented width (multiple of 32)
  const float* qinv2;  // device kernel parameters: 1/q^2, then (polynomial rows) log2 of the
                       // output multiplier and the degree
  const float* nrm = nullptr;  // Gaussian rows without the two norm columns: -q^2 c nu per
                               // row, added to the exponent in the product's epilogue
};

struct F64Points {
  const double* nu;  // rows_pad, FP64 squared norms
  int64_t n;
  int64_t dp;        // multiple of 8 (<= 128) or of 32
  const float* Xf = nullptr;  // rows_pad x dp FP32 coordinates (dp > 128)
  const int8_t* S = nullptr;  // int8 slices (d <= 128): rows_pad x OZ_SLICES x oz_kp(d)
  const double* scale = nullptr;  // rows_pad: 2^(e_i - 46) of the slices
  int64_t d = 0;
};

struct SplitOperand {
  const _Float16* hi;
  const _Float16* lo;
  int64_t ld;          // elements per row (the padded contraction length)
  const float* amax;   // device max |entry| of the unsplit operand (scale source)
};

struct CGScalars {
  double *ynorm, *rnorm, *rho, *alpha, *beta;
  int *active, *broken, *col_iters, *count;
};

enum { EPI_PART64 = 0, EPI_F32 = 1, EPI_COS = 2 };

// prep.hip
hipError_t fill_f32(float* p, int64_t count, float v, hipStream_t st);
hipError_t fill_f64(double* p, int64_t count, double v, hipStream_t st);
hipError_t fill_i32(int* p, int64_t count, int v, hipStream_t st);
hipError_t fill2d_f64(double* p, int64_t ld, int64_t rows, int64_t cols, double v, hipStream_t st);
hipError_t point_stats(const float* X, int64_t n, int64_t d, int64_t ldx, float* stats,
                       hipStream_t st);
// What the augmented rows of the mixed products encode (see prep.hip).
struct RowSpec {
  int poly = 0;        // 0: Gaussian kernel, 1: polynomial kernel
  int deg = 1;         // polynomial degree
  double c2 = 0.0;     // Gaussian: log2(e) / (2 sigma^2)
  double gamma = 0.0;  // polynomial scale
  double coef0 = 0.0;  // polynomial offset
};
template <typename T>
hipError_t prep_points(const float* X, int64_t n, int64_t d, int64_t ldx, int64_t rows_pad,
                       int64_t Kp, const RowSpec& rs, const float* stats, int side, int pshift,
                       T* hi, T* lo, float* kpar, hipStream_t st, float* nrm = nullptr);
hipError_t vec_split_t(float* V, int64_t n, int64_t m, int64_t ldv, int64_t rows_pad, int64_t mpad,
                       float* colmax, int pshift, bool packed, _Float16* hi, _Float16* lo,
                       float* vscale, hipStream_t st);
hipError_t prep_points_i8(const float* X, int64_t n, int64_t d, int64_t ldx, int64_t rows_pad,
                          int8_t* S, double* scale, double* nu, hipStream_t st);
hipError_t prep_points_f64x(const float* X, int64_t n, int64_t d, int64_t ldx, int64_t rows_pad,
                            int64_t dp, float* X32, double* nu, hipStream_t st);
hipError_t vec_to_f32(const double* V, int64_t n, int64_t m, int64_t ldv, int64_t rows_pad,
                      int64_t ldo, float* out, hipStream_t st);
hipError_t vec_pad_f64(const double* V, int64_t n, int64_t m, int64_t ldv, int64_t rows_pad,
                       int64_t ldo, double* out, hipStream_t st);
template <typename S>
hipError_t absmax(const S* src, int64_t rows, int64_t cols, int64_t ld, float* amax,
                  hipStream_t st);
template <typename S, typename T>
hipError_t split_operand(const S* src, int64_t rows, int64_t cols, int64_t ld, const float* amax,
                         int transpose, int64_t out_rows, int64_t out_cols, T* hi, T* lo,
                         hipStream_t st);

// matmat.hip
struct SplitRhs {          // right-hand sides prepared for the MFMA accumulation
  const _Float16* hi;      // [mpad][rows_pad] V^T, scaled per column
  const _Float16* lo;
  const float* vscale;     // [mpad] 1 / (column scale * 2^pshift)
  int64_t rows_pad, mpad;
  bool packed = false;     // m <= 8: rows 0..7 of hi hold the high parts, rows 8..15 the low
};
// Exponent shift of the MFMA-accumulate products. Folding a shift into the augmented
// contraction makes the FP32 accumulator carry log2 k + shift, whose rounding is relative
// to the shift; measured, that raised the solve's residual floor, so no shift is applied:
// k in (0, 1] is split directly (absolute error <= 2^-25 where k is below FP16's normal range).
constexpr int PSHIFT = 0;
// Epilogues of the fused kernel products (the value formed from each pair's inner product)
constexpr int KV_GAUSS = 0;   // Gaussian kernel (Sec. 6)
constexpr int KV_DSIGMA = 1;  // its sigma-derivative
constexpr int KV_POLY = 2;    // polynomial kernel (gamma x^T z + c)^q (Sec. 6, Thm. 1)
// Polynomial kernel value in FP64 from the inner product g = <x_i, x_j>: (gamma g + c)^deg.
struct PolyF64 {
  double gamma = 0.0, coef0 = 0.0;
  int deg = 1;
  __device__ inline double value(double g) const {
    const double t = fma(gamma, g, coef0);
    double p = t;
    for (int e = 1; e < deg; ++e) p *= t;
    return p;
  }
};
// Column-side accumulator of the symmetric large-d product K(X, X) V: 64-bit fixed-point
// sums (value times 2^F, two's complement) and per-row flags of non-finite contributions
// (bit c: column c). Each holds rows_pad rows; the product clears what it uses.
struct SymBuf {
  unsigned long long* fx;  // [rows_pad][ldfx]
  unsigned* flag;          // [rows_pad]
  int64_t ldfx;            // >= the pass's V^T rows (16)
};
struct SymOut {            // what the symmetric kernel receives
  unsigned long long* fx = nullptr;
  unsigned* flag = nullptr;
  int64_t ldfx = 0;
  float fxs = 1.0f;        // 2^F
  int nsplit = 1;
  int64_t nrb = 0;         // 128-row blocks
};
// OUT partial sums of K(A, B) V (or dK/dsigma, or the polynomial kernel) on MFMA. With sym
// (square products only: A and B prepared from the same points), large-d passes of up to
// 16 columns form each off-diagonal tile pair once and use it for both triangles.
hipError_t matmat_f16pv(const MixedPoints<_Float16>& A, const MixedPoints<_Float16>& B,
                        const SplitRhs& V, int64_t m, int epi, float dscale, double* part,
                        int64_t ldp, int64_t part_stride, int nsplit, hipStream_t st,
                        const SymBuf* sym = nullptr);
template <typename T>
hipError_t matmat_mixed(const MixedPoints<T>& A, const MixedPoints<T>& B, const float* Vf,
                        int64_t ldvf, int64_t m, bool deriv, float dscale, double* part,
                        int64_t ldp, int64_t part_stride, int nsplit, hipStream_t st);
// Column-side accumulator of the symmetric FP64 large-d product (two-word 64-bit fixed
// point, rows_pad x 16 each, per-row non-finite flags, and 16 per-column maxima of |V|).
struct F64SymBuf {
  unsigned long long *fh, *fl;
  unsigned* flag;
  unsigned long long* vmax;
};
// FP64 kernel product. With sym (square products: A and B the same points), a large-d
// Gaussian product of at most 16 columns forms each off-diagonal block pair once.
hipError_t matmat_f64(const F64Points& A, const F64Points& B, const double* V, int64_t ldv,
                      int64_t m, int epi, double c, double dscale, const PolyF64& pk,
                      double* part, int64_t ldp, int64_t part_stride, int nsplit,
                      hipStream_t st, const F64SymBuf* sym = nullptr);
template <typename VS>
hipError_t matmat_finalize(const double* part, int64_t part_stride, int nsplit, int64_t n,
                           int64_t m, int64_t ldp, double shift, const VS* Vs, int64_t ldvs,
                           double* out, int64_t ldo, hipStream_t st);

// batched kernel product (matmat.hip)
struct BatchInst {          // one problem of a batch, prepared for the F16X3 product
  const _Float16 *Ahi, *Alo, *Bhi, *Blo;   // rows padded to ROW_PAD, Kp wide
  const float* nrm;                        // Kp <= 128: the norm terms of the exponent
                                           // (rows_pad), added in the epilogue
  const _Float16 *Vth, *Vtl;              // [16][ldvt] split V^T
  const float* vscale;                     // [16]
  const float* qinv2;                      // device scalar
  double* part;                            // partial sums [nsplit][rows_pad][ldp]
  int64_t n, m, ldvt, ldp, part_stride;
  int Kp;
};
struct BatchItem {          // a 128-row block of one problem against one column range
  int inst;
  int tiles_per_split;
  int64_t rb, split;
};
// items[list[0 .. *nlist)] are the live work items (batch_compact_live)
hipError_t matmat_batch(const BatchItem* items, const int* list, const int* nlist,
                        const BatchInst* inst, int* counter, bool packed, int grid,
                        hipStream_t st);
hipError_t batch_compact_live(const BatchItem* items, int nitems, const int* live, int* chunk_cnt,
                              int* list, int* count, hipStream_t st);

// gemm.hip
hipError_t gemm_nt_f16x3(const SplitOperand& A, const SplitOperand& B, int64_t M, int64_t N,
                         int64_t K, int nsplit, int epi, int lower_only, int tri_b, double alpha,
                         double* out64, int64_t out64_stride, float* out32, int64_t ldc,
                         const float* bias, float amp, hipStream_t st);
hipError_t dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t sai,
                 int64_t sak, int64_t bA, const double* B, int64_t sbk, int64_t sbj, int64_t bB,
                 double beta, double* C, int64_t ldc, int64_t bC, int batch, int lower_only,
                 hipStream_t st);
// One product of a grouped FP64 GEMM launch (device memory): C = beta C + alpha A B with
// A(i, k) = A[i*sai + k*sak], B(k, j) = B[k*sbk + j*sbj], C(i, j) = C[i*ldc + j].
struct DgemmProblem {
  const double* A;
  const double* B;
  double* C;
  int64_t sai, sak, sbk, sbj, ldc;
  int64_t M, N, K;
  double alpha, beta;
  int lower_only;
};
// `count` products of at most max_m x max_n outputs each in one launch
hipError_t dgemm_grouped(const DgemmProblem* probs, int count, int64_t max_m, int64_t max_n,
                         hipStream_t st);

// chol.hip
hipError_t cholesky_blocked(double* G, int64_t s_pad, double* Cinv, int* info, hipStream_t st);
// One factor of a grouped Cholesky (device memory): G (s_pad x s_pad, factored in place),
// Cinv (its inverted diagonal 64 x 64 blocks are written), the pivot flag.
struct FactorMember {
  double* G;
  double* Cinv;
  int* info;
  int64_t s_pad;
};
// Column block k0 of every member whose s_pad exceeds k0: diagonal factor, then the panel
// below it (rows up to max_rest); members with nothing left return at once.
hipError_t cholesky_step_grouped(const FactorMember* mem, int count, int64_t k0, int64_t max_rest,
                                 hipStream_t st);
// Inverses of every member's diagonal 64 x 64 blocks (max_s_pad the largest order).
hipError_t diag_inverse_grouped(const FactorMember* mem, int count, int64_t max_s_pad,
                                hipStream_t st);
hipError_t tri_inverse_doubling(const double* C, int64_t s_pad, double* Cinv, double* tmp,
                                hipStream_t st);
hipError_t gram_finalize(const double* part, int nsplit, int64_t s, int64_t ldp, int64_t pstride,
                         double lambda_p, int64_t s_pad, double* G, hipStream_t st);
hipError_t copy_lower(const double* a, int64_t lda, int64_t s, double* C, hipStream_t st);

// cg.hip
template <typename TA, typename TB>
hipError_t dot_partial(const TA* a, int64_t lda, const TB* b, int64_t ldb, int64_t n, int64_t m,
                       double* part, int nblk, hipStream_t st);
hipError_t cg_init_scalars(const double* part_yy, const double* part_rr, const double* part_rz,
                           int nblk, int64_t m, double tol, CGScalars& S, hipStream_t st);
hipError_t cg_alpha(const double* part_pq, int nblk, int64_t m, CGScalars& S, hipStream_t st);
hipError_t cg_conv(const double* part_rr, int nblk, int64_t m, double tol, int it, CGScalars& S,
                   double* hist_slot, hipStream_t st);
hipError_t cg_beta(const double* part_rz, const double* part_rr, int nblk, int64_t m,
                   CGScalars& S, hipStream_t st);
template <typename TP>
hipError_t cg_update_xr(double* x, int64_t ldx, double* r, const TP* p, int64_t ldp,
                        const double* q, const double* alpha, int64_t n, int64_t m,
                        double* part_rr, int nblk, hipStream_t st);
hipError_t cg_update_p(const double* z, double* p, float* pf, int64_t ldpf, const double* beta,
                       const int* active, int init, int64_t n, int64_t m, hipStream_t st);
hipError_t residual_from(const double* y, int64_t ldy, const double* ax, int64_t n, int64_t m,
                         double* r, hipStream_t st);
hipError_t copy2d(const double* a, int64_t lda, double* b, int64_t ldb, int64_t n, int64_t m,
                  hipStream_t st);
hipError_t add2d(const double* a, int64_t lda, double* b, int64_t ldb, int64_t n, int64_t m,
                 hipStream_t st);
hipError_t precond_apply(const float* Ut, int64_t ldu, int64_t n, int64_t s, int64_t m,
                         double lambda_p, const double* r, double* z, double* part, int nchunk,
                         double* T, hipStream_t st);

// tsketch.hip: TensorSketch features of the augmented points [sqrt(gamma) x, sqrt(c)]
// (hash q x (d + 1) in [0, s), sign q x (d + 1) of +-1), s = 2^logs <= 8192.
hipError_t tensor_sketch(const float* X, int64_t n, int64_t d, int64_t ldx, double gamma,
                         double coef0, int q, const int* hash, const float* sign, int logs,
                         float* Z, int64_t ldz, hipStream_t st);

// srht.hip: Z2 = Z1 S^T for the SRHT S = s2^{-1/2} P H D (rows of Z1 zero-padded to a power
// of two <= 16384; sample holds s2 coordinates of the padded width).
hipError_t srht_rows(const float* Z1, int64_t n, int64_t s1, int64_t ldz1, const float* signs,
                     const int* sample, int64_t s2, float* Z2, int64_t ldz2, hipStream_t st);

// jacobi.hip: eigen-decomposition of C C^T by one-sided Jacobi on the rows of C (A in: C,
// out: rotated rows; Vt: eigenvectors as rows; ev: eigenvalues), and the small kernels of the
// preconditioner test.
hipError_t jacobi_eig(double* A, int s, double* Vt, double* ev, unsigned long long* off,
                      double tol, int max_sweeps, int* sweeps, hipStream_t st);
hipError_t gather_scaled_rows(const double* Vt, int s, const int* idx, const double* scale, int k,
                              float* Bk, hipStream_t st);
constexpr int GEMV_PARTS_MAX = 128;
hipError_t gemv_t(const float* U, int64_t ldu, int64_t n, int k, const double* r, const double* w,
                  double* y, double* part, hipStream_t st);
hipError_t gemv_n(const float* U, int64_t ldu, int64_t n, int k, const double* x, const double* w,
                  double* r, hipStream_t st);
hipError_t hash_fill(double* v, int64_t n, uint64_t seed, hipStream_t st);
hipError_t axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                 hipStream_t st);
hipError_t f32_to_f64_2d(const float* a, int64_t n, int64_t cols, int64_t lda, double* out,
                         hipStream_t st);

// tune.cpp: launch choices of the kernel products found by timing (0 = the default rule)
struct TuneChoice {
  int nsplit = 0;       // column splits of the product
  int pass_width = 0;   // right-hand-side columns per pass (large d)
  double ms_default = 0.0, ms_best = 0.0;
};
bool tune_lookup(int prec, int kind, int64_t Kp, int64_t m, int64_t n, TuneChoice* out);
void tune_store(int prec, int kind, int64_t Kp, int64_t m, int64_t n, const TuneChoice& c);
const char* tune_digest();

// Record `msg` as the calling thread's krr_last_error() text and return `code` (entry points
// defined outside the main ABI source report through it).
krr_status report_error(krr_status code, const char* msg);

}  // namespace krr
