// FP64 Cholesky of G = Z^T Z + lambda_p I and the inverse of its factor (Sec. 3.1).
//
// Blocked right-looking factorisation with 64 x 64 diagonal blocks: one wave factors
// the diagonal block with its rows in registers; the panel below is solved against it (one
// thread per panel row); the trailing lower triangle gets an FP64 rank-64 update. The
// inverses of all diagonal blocks are then formed at once, one workgroup per block, and
// the full inverse C^{-1} is assembled from them by recursive doubling,
// inv([A 0; B D]) = [A^-1 0; -D^-1 B A^-1  D^-1], with batched FP64 GEMMs. The matrix
// order is padded to a multiple of 64 with an identity block, which leaves the leading
// factor and its inverse unchanged; the last block of a doubling level may be short.
#include "kernels.hpp"

namespace krr {

constexpr int NB = 64;

// Factor the diagonal block at (k0, k0) of A (lda) in place (lower; strict upper zeroed).
// One wave: lane r keeps row r of the block in registers. Column j: the pivot W[j][j] is
// read from lane j (readlane); every lane scales its entry W[r][j] by 1 / sqrt(W[j][j])
// (below the diagonal this is L[r][j], on it L[j][j] to within an ulp) and publishes it
// in LDS; every row then subtracts L[r][j] L[c][j] from its entries c > j. Values
// above the diagonal of a row are never used for its lower part, and col[c] is read only
// for c > j, so the steps need no lane-dependent selects. Within one wave the LDS write
// is seen by the reads that follow it, so no barrier is needed; the column steps are
// unrolled at compile time, so register indices are constants.
// *info receives the 1-based global index of the first non-positive (or non-finite) pivot
// if it is still 0.
__device__ __forceinline__ double lane_value(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}

// Column steps J, J + 1, ... of the diagonal factorisation (compile-time J, so register
// indices are constants and the update touches only the columns after J).
template <int J>
__device__ __forceinline__ void potrf_steps(double (&w)[NB], double* col, int r,
                                            int& first_bad) {
  if constexpr (J < NB) {
    const double dj = lane_value(w[J], J);
    if (first_bad == 0 && (!(dj > 0.0) || !(dj < INFINITY))) first_bad = J + 1;
    const double inv = 1.0 / sqrt(dj);
    const double lrj = w[J] * inv;
    w[J] = lrj;
    col[r] = lrj;
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int c = J + 1; c < NB; ++c) w[c] = fma(-lrj, col[c], w[c]);
    __builtin_amdgcn_wave_barrier();
    potrf_steps<J + 1>(w, col, r, first_bad);
  }
}

__device__ __forceinline__ void potrf_diag_body(double* __restrict__ A, int64_t lda, int64_t k0,
                                                int* __restrict__ info, double* col) {
  const int r = threadIdx.x;
  double w[NB];  // the whole row; entries above the diagonal (stale) are never used, and
                 // loading them keeps lane-dependent masks out of the steps
#pragma unroll
  for (int c = 0; c < NB; ++c) w[c] = A[(k0 + r) * lda + k0 + c];
  int first_bad = 0;
  potrf_steps<0>(w, col, r, first_bad);
  if (r == 0 && first_bad != 0 && *info == 0) *info = (int)(k0 + first_bad);
#pragma unroll
  for (int c = 0; c < NB; ++c) A[(k0 + r) * lda + k0 + c] = c <= r ? w[c] : 0.0;
}

__global__ __launch_bounds__(64, 2) void potrf_diag_kernel(double* __restrict__ A, int64_t lda,
                                                        int64_t k0, int* __restrict__ info) {
  __shared__ double col[NB];
  potrf_diag_body(A, lda, k0, info, col);
}

// member blockIdx.x of a grouped factor
__global__ __launch_bounds__(64, 2) void potrf_diag_grouped_kernel(const FactorMember* __restrict__ mem,
                                                                int64_t k0) {
  const FactorMember f = mem[blockIdx.x];
  if (k0 >= f.s_pad) return;
  __shared__ double col[NB];
  potrf_diag_body(f.G, f.s_pad, k0, f.info, col);
}

// Forward substitution against the 64 x 64 lower factor held in LDS (Ls, reciprocal
// diagonal in dinv): x[j] = (b[j] - sum_{k<j} Ls[j][k] x[k]) dinv[j]. Every thread reads the
// same Ls entries (broadcasts); the loops are unrolled so x stays in registers.
__device__ __forceinline__ void lower_solve64(const double (*Ls)[NB + 1], const double* dinv,
                                              double (&x)[NB]) {
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    double acc = x[j];
#pragma unroll
    for (int k = 0; k < j; ++k) acc = fma(-Ls[j][k], x[k], acc);
    x[j] = acc * dinv[j];
  }
}

// Panel below the diagonal block k0: P <- P L^{-T} (row i of P solves x L^T = p_i), one
// thread per row, L staged in LDS.
__device__ __forceinline__ void trsm_panel_body(double* __restrict__ G, int64_t ld, int64_t k0,
                                                int64_t rows, double (&Ls)[NB][NB + 1],
                                                double* dinv) {
  for (int e = threadIdx.x; e < NB * NB; e += 256) Ls[e / NB][e % NB] = G[(k0 + e / NB) * ld + k0 + e % NB];
  __syncthreads();
  if (threadIdx.x < NB) dinv[threadIdx.x] = 1.0 / Ls[threadIdx.x][threadIdx.x];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= rows) return;
  double* p = G + (k0 + NB + i) * ld + k0;
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = p[j];
  lower_solve64(Ls, dinv, x);
#pragma unroll
  for (int j = 0; j < NB; ++j) p[j] = x[j];
}

__global__ __launch_bounds__(256) void trsm_panel_kernel(double* __restrict__ G, int64_t ld,
                                                         int64_t k0, int64_t rows) {
  __shared__ double Ls[NB][NB + 1];
  __shared__ double dinv[NB];
  trsm_panel_body(G, ld, k0, rows, Ls, dinv);
}

// member blockIdx.y of a grouped factor; blocks past its panel return before any barrier
__global__ __launch_bounds__(256) void trsm_panel_grouped_kernel(const FactorMember* __restrict__ mem,
                                                                 int64_t k0) {
  const FactorMember f = mem[blockIdx.y];
  const int64_t rows = f.s_pad - k0 - NB;
  if ((int64_t)blockIdx.x * 256 >= rows) return;
  __shared__ double Ls[NB][NB + 1];
  __shared__ double dinv[NB];
  trsm_panel_body(f.G, f.s_pad, k0, rows, Ls, dinv);
}

// Inverse of the diagonal 64 x 64 block at k0 of the factor, written to the same position of
// Cinv: thread c solves L x = e_c for column c of the inverse (one block per diagonal block).
__device__ __forceinline__ void diag_inverse_body(const double* __restrict__ G, int64_t ld,
                                                  double* __restrict__ Cinv, int64_t k0,
                                                  double (&Ls)[NB][NB + 1], double* dinv) {
  for (int e = threadIdx.x; e < NB * NB; e += 64) Ls[e / NB][e % NB] = G[(k0 + e / NB) * ld + k0 + e % NB];
  __syncthreads();
  dinv[threadIdx.x] = 1.0 / Ls[threadIdx.x][threadIdx.x];
  __syncthreads();
  const int c = threadIdx.x;
  double x[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) x[j] = j == c ? 1.0 : 0.0;
  lower_solve64(Ls, dinv, x);
#pragma unroll
  for (int j = 0; j < NB; ++j) Cinv[(k0 + j) * ld + k0 + c] = x[j];
}

__global__ __launch_bounds__(64) void diag_inverse_kernel(const double* __restrict__ G,
                                                          int64_t ld, double* __restrict__ Cinv) {
  __shared__ double Ls[NB][NB + 1];
  __shared__ double dinv[NB];
  diag_inverse_body(G, ld, Cinv, (int64_t)blockIdx.x * NB, Ls, dinv);
}

// block blockIdx.x of member blockIdx.y of a grouped factor
__global__ __launch_bounds__(64) void diag_inverse_grouped_kernel(const FactorMember* __restrict__ mem) {
  const FactorMember f = mem[blockIdx.y];
  const int64_t k0 = (int64_t)blockIdx.x * NB;
  if (k0 >= f.s_pad) return;
  __shared__ double Ls[NB][NB + 1];
  __shared__ double dinv[NB];
  diag_inverse_body(f.G, f.s_pad, f.Cinv, k0, Ls, dinv);
}

// G (s_pad x s_pad, lower part used) -> C in place; Cinv diagonal blocks filled.
hipError_t cholesky_blocked(double* G, int64_t s_pad, double* Cinv, int* info, hipStream_t st) {
  for (int64_t k0 = 0; k0 < s_pad; k0 += NB) {
    potrf_diag_kernel<<<1, NB, 0, st>>>(G, s_pad, k0, info);
    KRR_LAUNCH_CHECK();
    const int64_t rest = s_pad - k0 - NB;
    if (rest <= 0) break;
    trsm_panel_kernel<<<ceil_div(rest, 256), 256, 0, st>>>(G, s_pad, k0, rest);
    KRR_LAUNCH_CHECK();
    double* panel = G + (k0 + NB) * s_pad + k0;
    // trailing lower triangle <- trailing - panel * panel^T
    hipError_t e = dgemm(rest, rest, NB, -1.0, panel, s_pad, 1, 0, panel, 1, s_pad, 0, 1.0,
                         G + (k0 + NB) * s_pad + k0 + NB, s_pad, 0, 1, 1, st);
    if (e != hipSuccess) return e;
  }
  diag_inverse_kernel<<<s_pad / NB, 64, 0, st>>>(G, s_pad, Cinv);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t cholesky_step_grouped(const FactorMember* mem, int count, int64_t k0, int64_t max_rest,
                                 hipStream_t st) {
  if (count <= 0) return hipSuccess;
  potrf_diag_grouped_kernel<<<count, NB, 0, st>>>(mem, k0);
  KRR_LAUNCH_CHECK();
  if (max_rest > 0) {
    trsm_panel_grouped_kernel<<<dim3(ceil_div(max_rest, 256), count), 256, 0, st>>>(mem, k0);
    KRR_LAUNCH_CHECK();
  }
  return hipSuccess;
}

hipError_t diag_inverse_grouped(const FactorMember* mem, int count, int64_t max_s_pad,
                                hipStream_t st) {
  if (count <= 0 || max_s_pad <= 0) return hipSuccess;
  diag_inverse_grouped_kernel<<<dim3(ceil_div(max_s_pad, NB), count), 64, 0, st>>>(mem);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// Off-diagonal blocks of C^{-1} by recursive doubling; Cinv holds the inverted diagonal
// 64 x 64 blocks on entry, s_pad is a multiple of 64, tmp needs s_pad * s_pad / 2 doubles.
// Level b joins the aligned blocks [2pb, 2pb + b) and [2pb + b, min(2pb + 2b, s_pad)), both
// already inverted by the levels before it (the second may be shorter than b, or absent at
// the end, where the first block carries over unchanged). The full pairs of a level go
// through one batched GEMM pair; a short second block gets a GEMM pair of its own.
hipError_t tri_inverse_doubling(const double* C, int64_t s_pad, double* Cinv, double* tmp,
                                hipStream_t st) {
  if (s_pad % NB) return hipErrorInvalidValue;
  for (int64_t b = NB; b < s_pad; b *= 2) {
    const int full = (int)(s_pad / (2 * b));
    const int64_t pair_stride = 2 * b * s_pad + 2 * b;  // element offset between pairs
    hipError_t e;
    if (full > 0) {
      // T_p = B_p * Ainv_p, B_p = C[o2:o2+b, o1:o1+b], Ainv_p = Cinv[o1:o1+b, o1:o1+b]
      e = dgemm(b, b, b, 1.0, C + b * s_pad, s_pad, 1, pair_stride, Cinv, s_pad, 1, pair_stride,
                0.0, tmp, b, b * b, full, 0, st);
      if (e != hipSuccess) return e;
      // X_p = -Dinv_p * T_p -> Cinv[o2:o2+b, o1:o1+b]
      e = dgemm(b, b, b, -1.0, Cinv + b * s_pad + b, s_pad, 1, pair_stride, tmp, b, 1, b * b,
                0.0, Cinv + b * s_pad, s_pad, pair_stride, full, 0, st);
      if (e != hipSuccess) return e;
    }
    const int64_t o1 = 2 * b * full, o2 = o1 + b, m2 = s_pad - o2;  // short pair, if any
    if (m2 > 0) {
      e = dgemm(m2, b, b, 1.0, C + o2 * s_pad + o1, s_pad, 1, 0, Cinv + o1 * s_pad + o1, s_pad,
                1, 0, 0.0, tmp, b, 0, 1, 0, st);
      if (e != hipSuccess) return e;
      e = dgemm(m2, b, m2, -1.0, Cinv + o2 * s_pad + o2, s_pad, 1, 0, tmp, b, 1, 0, 0.0,
                Cinv + o2 * s_pad + o1, s_pad, 0, 1, 0, st);
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

// Gram reduction: G[i][j] = sum_s part[s][i][j] for the lower triangle (i >= j, i, j < s),
// mirrored; + lambda_p on the diagonal; identity on the padded diagonal; zero elsewhere.
// 32 x 32 tiles: the block of a tile on or below the diagonal reads that lower source
// tile of every split once (coalesced rows), sums the splits in order, and writes the tile
// and, through LDS, its mirror above the diagonal; in a diagonal tile the entries above
// the diagonal take their lower mirror. Blocks of tiles above the diagonal return.
constexpr int GF_T = 32;
__global__ __launch_bounds__(256) void gram_finalize_kernel(const double* __restrict__ part,
                                                            int nsplit, int64_t s, int64_t ldp,
                                                            int64_t pstride, double lambda_p,
                                                            int64_t s_pad,
                                                            double* __restrict__ G) {
  const int64_t bi = blockIdx.y, bj = blockIdx.x;
  if (bj > bi) return;
  __shared__ double t[GF_T][GF_T + 1];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t i0 = bi * GF_T, j0 = bj * GF_T;
  for (int yy = ty; yy < GF_T; yy += 8) {
    const int64_t i = i0 + yy, j = j0 + tx;
    double v = 0.0;
    if (i < s && j < s)
      for (int k = 0; k < nsplit; ++k) v += part[k * pstride + i * ldp + j];
    t[yy][tx] = v;
  }
  __syncthreads();
  for (int yy = ty; yy < GF_T; yy += 8) {
    const int64_t i = i0 + yy, j = j0 + tx;
    double v = (bi == bj && tx > yy) ? t[tx][yy] : t[yy][tx];
    if (i >= s || j >= s) v = i == j ? 1.0 : 0.0;
    else if (i == j) v += lambda_p;
    G[i * s_pad + j] = v;
  }
  if (bi != bj) {
    for (int yy = ty; yy < GF_T; yy += 8) {
      const int64_t r = j0 + yy, c = i0 + tx;  // mirror entry (r, c) = source (c, r)
      G[r * s_pad + c] = (r < s && c < s) ? t[tx][yy] : 0.0;
    }
  }
}

hipError_t gram_finalize(const double* part, int nsplit, int64_t s, int64_t ldp, int64_t pstride,
                         double lambda_p, int64_t s_pad, double* G, hipStream_t st) {
  if (s_pad % GF_T) return hipErrorInvalidValue;
  dim3 grid(s_pad / GF_T, s_pad / GF_T);
  gram_finalize_kernel<<<grid, 256, 0, st>>>(part, nsplit, s, ldp, pstride, lambda_p, s_pad, G);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// Copy the leading s x s lower triangle of a (ld) into C (ld s), zeroing the upper part.
__global__ void copy_lower_kernel(const double* __restrict__ a, int64_t lda, int64_t s,
                                  double* __restrict__ C) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s * s) return;
  const int64_t i = e / s, j = e % s;
  C[e] = j <= i ? a[i * lda + j] : 0.0;
}

hipError_t copy_lower(const double* a, int64_t lda, int64_t s, double* C, hipStream_t st) {
  copy_lower_kernel<<<ceil_div(s * s, 256), 256, 0, st>>>(a, lda, s, C);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace krr
