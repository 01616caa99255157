// FP64 Cholesky of G = Z^T Z + lambda_p I and the inverse of its factor (step a3).
//
// Blocked right-looking factorisation with 64 x 64 diagonal blocks: one workgroup factors
// the diagonal block in LDS and also inverts it; the panel below is multiplied by that
// inverse (a GEMM instead of a triangular solve); the trailing lower triangle gets an
// FP64 rank-64 update. The full inverse C^{-1} is then assembled by recursive doubling,
// inv([A 0; B D]) = [A^-1 0; -D^-1 B A^-1  D^-1], with batched FP64 GEMMs. The matrix
// order is padded to 64 * 2^k with an identity block, which leaves the leading factor
// and its inverse unchanged.
#include "kernels.hpp"

namespace krr {

constexpr int NB = 64;

// Factor the diagonal block at (k0, k0) of A (lda) in place (lower, strict upper zeroed)
// and write its inverse into Ainv (same offsets, ld lda_inv). One wave: lane r owns row r.
// *info receives the 1-based global index of the first non-positive (or non-finite) pivot
// if it is still 0.
__global__ __launch_bounds__(64) void potrf_diag_kernel(double* __restrict__ A, int64_t lda,
                                                        int64_t k0, double* __restrict__ Ainv,
                                                        int64_t ldi, int* __restrict__ info) {
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  const int r = threadIdx.x;
  for (int i = 0; i < NB; ++i) L[i][r] = (r <= i) ? A[(k0 + i) * lda + k0 + r] : 0.0;
  __syncthreads();
  for (int j = 0; j < NB; ++j) {
    const double dj = L[j][j];
    if (r == 0 && (!(dj > 0.0) || !(dj < INFINITY)) && *info == 0) *info = (int)(k0 + j + 1);
    const double ljj = sqrt(dj);
    double lrj = 0.0;
    if (r > j) {
      lrj = L[r][j] / ljj;
      L[r][j] = lrj;
    }
    __syncthreads();
    if (r == j) L[j][j] = ljj;
    if (r > j)
      for (int c = j + 1; c <= r; ++c) L[r][c] -= lrj * L[c][j];
    __syncthreads();
  }
  // inverse of the lower triangular block: lane c computes column c by forward substitution
  {
    const int c = r;
    for (int i = 0; i < NB; ++i) {
      if (i < c) { X[i][c] = 0.0; continue; }
      double sacc = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) sacc -= L[i][k] * X[k][c];
      X[i][c] = sacc / L[i][i];
    }
  }
  __syncthreads();
  for (int i = 0; i < NB; ++i) {
    A[(k0 + i) * lda + k0 + r] = L[i][r];
    Ainv[(k0 + i) * ldi + k0 + r] = X[i][r];
  }
}

// G (s_pad x s_pad, lower part used) -> C in place; Cinv diagonal blocks filled.
hipError_t cholesky_blocked(double* G, int64_t s_pad, double* Cinv, int* info, hipStream_t st) {
  for (int64_t k0 = 0; k0 < s_pad; k0 += NB) {
    potrf_diag_kernel<<<1, 64, 0, st>>>(G, s_pad, k0, Cinv, s_pad, info);
    KRR_LAUNCH_CHECK();
    const int64_t rest = s_pad - k0 - NB;
    if (rest <= 0) break;
    double* panel = G + (k0 + NB) * s_pad + k0;
    const double* linv = Cinv + k0 * s_pad + k0;
    // panel <- panel * Linv^T   (B(k, j) = Linv[j][k])
    hipError_t e = dgemm(rest, NB, NB, 1.0, panel, s_pad, 1, 0, linv, 1, s_pad, 0, 0.0, panel,
                         s_pad, 0, 1, 0, st);
    if (e != hipSuccess) return e;
    // trailing lower triangle <- trailing - panel * panel^T
    e = dgemm(rest, rest, NB, -1.0, panel, s_pad, 1, 0, panel, 1, s_pad, 0, 1.0,
              G + (k0 + NB) * s_pad + k0 + NB, s_pad, 0, 1, 1, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Off-diagonal blocks of C^{-1} by recursive doubling; Cinv holds the inverted diagonal
// 64 x 64 blocks on entry. tmp needs s_pad * s_pad / 2 doubles. s_pad = 64 * 2^k.
hipError_t tri_inverse_doubling(const double* C, int64_t s_pad, double* Cinv, double* tmp,
                                hipStream_t st) {
  for (int64_t b = NB; b < s_pad; b *= 2) {
    const int pairs = (int)(s_pad / (2 * b));
    const int64_t pair_stride = 2 * b * s_pad + 2 * b;  // element offset between pairs
    // T_p = B_p * Ainv_p, B_p = C[o2:o2+b, o1:o1+b], Ainv_p = Cinv[o1:o1+b, o1:o1+b]
    hipError_t e = dgemm(b, b, b, 1.0, C + b * s_pad, s_pad, 1, pair_stride, Cinv, s_pad, 1,
                         pair_stride, 0.0, tmp, b, b * b, pairs, 0, st);
    if (e != hipSuccess) return e;
    // X_p = -Dinv_p * T_p -> Cinv[o2:o2+b, o1:o1+b]
    e = dgemm(b, b, b, -1.0, Cinv + b * s_pad + b, s_pad, 1, pair_stride, tmp, b, 1, b * b, 0.0,
              Cinv + b * s_pad, s_pad, pair_stride, pairs, 0, st);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Gram reduction: G[i][j] = sum_s part[s][i][j] for the lower triangle (i >= j, i, j < s),
// mirrored; + lambda_p on the diagonal; identity on the padded diagonal; zero elsewhere.
__global__ void gram_finalize_kernel(const double* __restrict__ part, int nsplit, int64_t s,
                                     int64_t ldp, int64_t pstride, double lambda_p, int64_t s_pad,
                                     double* __restrict__ G) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s_pad * s_pad) return;
  const int64_t i = e / s_pad, j = e % s_pad;
  double v = 0.0;
  if (i < s && j < s) {
    const int64_t a = i >= j ? i : j, b = i >= j ? j : i;  // lower triangle entry
    for (int k = 0; k < nsplit; ++k) v += part[k * pstride + a * ldp + b];
    if (i == j) v += lambda_p;
  } else if (i == j) {
    v = 1.0;
  }
  G[e] = v;
}

hipError_t gram_finalize(const double* part, int nsplit, int64_t s, int64_t ldp, int64_t pstride,
                         double lambda_p, int64_t s_pad, double* G, hipStream_t st) {
  gram_finalize_kernel<<<ceil_div(s_pad * s_pad, 256), 256, 0, st>>>(part, nsplit, s, ldp,
                                                                      pstride, lambda_p, s_pad, G);
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
