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
// and write its inverse into Ainv (same offsets, ld lda_inv). 256 threads.
// Factor: right-looking in LDS; per column j one thread takes the pivot, the column below it
// is scaled, and the trailing lower triangle takes the rank-1 update (4 threads per row).
// Inverse: X = L^{-1} row by row, X[i][c] = (delta_ic - sum_{c<=k<i} L[i][k] X[k][c]) / L[i][i]
// with the columns c in parallel and the k-sum split over 4 thread groups.
// *info receives the 1-based global index of the first non-positive (or non-finite) pivot
// if it is still 0.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ A, int64_t lda,
                                                         int64_t k0, double* __restrict__ Ainv,
                                                         int64_t ldi, int* __restrict__ info) {
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  __shared__ double part[4][NB];
  __shared__ int bad;
  const int t = threadIdx.x;
  if (t == 0) bad = 0;
  for (int e = t; e < NB * NB; e += 256) {
    const int i = e / NB, c = e % NB;
    L[i][c] = (c <= i) ? A[(k0 + i) * lda + k0 + c] : 0.0;
  }
  __syncthreads();
  const int row = t >> 2, sub = t & 3;
  for (int j = 0; j < NB; ++j) {
    if (t == 0) {
      const double dj = L[j][j];
      if (!(dj > 0.0) || !(dj < INFINITY)) {
        if (!bad && *info == 0) *info = (int)(k0 + j + 1);
        bad = 1;
      }
      L[j][j] = sqrt(dj);
    }
    __syncthreads();
    const double ljj = L[j][j];
    if (t > j && t < NB) L[t][j] /= ljj;
    __syncthreads();
    // trailing update of rows r > j, columns j < c <= r
    const int r = j + 1 + row;
    if (r < NB) {
      const double lrj = L[r][j];
      for (int c = j + 1 + sub; c <= r; c += 4) L[r][c] -= lrj * L[c][j];
    }
    __syncthreads();
  }
  // inverse of the lower triangular factor
  const int c = t & 63, q = t >> 6;
  for (int i = 0; i < NB; ++i) {
    double acc = 0.0;
    if (c < i)
      for (int k = c + q; k < i; k += 4) acc += L[i][k] * X[k][c];
    part[q][c] = acc;
    __syncthreads();
    if (q == 0) {
      double v;
      if (c > i) v = 0.0;
      else if (c == i) v = 1.0 / L[i][i];
      else v = -(part[0][c] + part[1][c] + part[2][c] + part[3][c]) / L[i][i];
      X[i][c] = v;
    }
    __syncthreads();
  }
  for (int e = t; e < NB * NB; e += 256) {
    const int i = e / NB, cc = e % NB;
    A[(k0 + i) * lda + k0 + cc] = cc <= i ? L[i][cc] : 0.0;
    Ainv[(k0 + i) * ldi + k0 + cc] = X[i][cc];
  }
}

// G (s_pad x s_pad, lower part used) -> C in place; Cinv diagonal blocks filled.
hipError_t cholesky_blocked(double* G, int64_t s_pad, double* Cinv, int* info, hipStream_t st) {
  for (int64_t k0 = 0; k0 < s_pad; k0 += NB) {
    potrf_diag_kernel<<<1, 256, 0, st>>>(G, s_pad, k0, Cinv, s_pad, info);
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
