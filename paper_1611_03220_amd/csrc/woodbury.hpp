// Woodbury apply of the random-features preconditioner (Sec. 3.1):
//   z = (ZZ^T + lambda_p I)^{-1} r = (r - Ut (Ut^T r)) / lambda_p,   Ut = Z C^{-T} (n x s, FP32).
// Two streaming passes over Ut, each reading it once from HBM; FP64 accumulation.
// Device bodies shared by the single-problem and the batched launches.
#pragma once
#include "common.hpp"

namespace krr {

// Pass 1: T partial over rows [i0, i1) for one feature column k (one thread per k; the
// threads of a block read consecutive k, so every row read is one contiguous segment).
// The rows of r are the same for every lane, so they come through scalar loads.
// out[k * ldo + c] = sum_{i in [i0, i1)} Ut[i][k] r[i][c], c < MC.
template <int MC>
__device__ __forceinline__ void woodbury_tpart(const float* __restrict__ Ut, int64_t ldu,
                                               int64_t s, const double* __restrict__ r,
                                               int64_t ldr, int64_t i0, int64_t i1, int64_t k,
                                               double* __restrict__ out, int64_t ldo) {
  double acc[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) acc[c] = 0.0;
  const bool kin = k < s;
  const float* up = Ut + (kin ? k : 0);
  int64_t i = i0;
  for (; i + 4 <= i1; i += 4) {
    float u[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float t = up[kin ? (i + j) * ldu : 0];
      u[j] = kin ? t : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const double uj = (double)u[j];
      const double* rr = r + (i + j) * ldr;
#pragma unroll
      for (int c = 0; c < MC; ++c) acc[c] = fma(uj, rr[c], acc[c]);
    }
  }
  for (; i < i1; ++i) {
    const float t = up[kin ? i * ldu : 0];
    const double uj = kin ? (double)t : 0.0;
    const double* rr = r + i * ldr;
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[c] = fma(uj, rr[c], acc[c]);
  }
  if (kin) {
#pragma unroll
    for (int c = 0; c < MC; ++c) out[k * ldo + c] = acc[c];
  }
}

// Pass 2 for one block of 64 rows [i0, i0 + 64) (rows >= iend masked) with 256 threads:
// wave w covers the feature range [w kq, (w + 1) kq) in chunks of 32; lane l owns row i0 + l.
// Each wave stages its 64 x 32 chunk of Ut in its own LDS tile (rows of 33 floats: the
// row-wise reads of the lanes hit distinct banks), T values are wave-uniform (scalar loads).
// The four waves' partial sums meet in LDS; wave 0 writes
//   z[i][c] = (r[i][c] - sum_k Ut[i][k] T[k][c]) * inv_lp,   c < MC.
// smem: at least 4 * 64 * 33 floats and 4 * 64 * MC doubles.
constexpr int WB_CH = 32;
template <int MC>
__device__ __forceinline__ void woodbury_z(const float* __restrict__ Ut, int64_t ldu, int64_t s,
                                           const double* __restrict__ T, int64_t ldt,
                                           const double* __restrict__ r, int64_t ldr,
                                           double inv_lp, double* __restrict__ z, int64_t ldz,
                                           int64_t i0, int64_t iend, float* __restrict__ smem) {
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  float* su = smem + w * 64 * (WB_CH + 1);
  const int64_t kq = round_up(ceil_div(s, 4), WB_CH);
  const int64_t kb0 = w * kq;
  const int nch = (int)(kq / WB_CH);
  double acc[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) acc[c] = 0.0;
  // loader: lane l reads column l % 32 of rows l / 32 + 2 j (j < 32)
  const int lc = lane & 31, lr = lane >> 5;
  for (int ch = 0; ch < nch; ++ch) {
    const int64_t kb = kb0 + (int64_t)ch * WB_CH;
    const bool kin = kb + lc < s;
    float v[32];
    const float* ub = Ut + (kin ? kb + lc : 0);
    if (i0 + 64 <= iend && kb + WB_CH <= s) {  // whole tile in range (wave-uniform)
      const float* up = ub + (i0 + lr) * ldu;
#pragma unroll
      for (int j = 0; j < 32; ++j) v[j] = up[2 * j * ldu];
    } else {
#pragma unroll
      for (int j = 0; j < 32; ++j) {
        // masked lanes read the (valid) first element and drop it
        const int64_t row = i0 + lr + 2 * j;
        const bool ok = kin && row < iend;
        const float t = ub[ok ? row * ldu : 0];
        v[j] = ok ? t : 0.0f;
      }
    }
    __syncthreads();  // previous chunk fully consumed
#pragma unroll
    for (int j = 0; j < 32; ++j) su[(lr + 2 * j) * (WB_CH + 1) + lc] = v[j];
    __syncthreads();
    if (kb < s) {
      const int kend = s - kb < WB_CH ? (int)(s - kb) : WB_CH;
      const double* Tk = T + kb * ldt;
      if (kend == WB_CH) {
#pragma unroll 8
        for (int kk = 0; kk < WB_CH; ++kk) {
          const double u = (double)su[lane * (WB_CH + 1) + kk];
#pragma unroll
          for (int c = 0; c < MC; ++c) acc[c] = fma(u, Tk[kk * ldt + c], acc[c]);
        }
      } else {
        for (int kk = 0; kk < kend; ++kk) {
          const double u = (double)su[lane * (WB_CH + 1) + kk];
#pragma unroll
          for (int c = 0; c < MC; ++c) acc[c] = fma(u, Tk[kk * ldt + c], acc[c]);
        }
      }
    }
  }
  __syncthreads();
  double* red = reinterpret_cast<double*>(smem);  // [4][64][MC]
#pragma unroll
  for (int c = 0; c < MC; ++c) red[(w * 64 + lane) * MC + c] = acc[c];
  __syncthreads();
  if (w == 0) {
    const int64_t i = i0 + lane;
    if (i < iend) {
#pragma unroll
      for (int c = 0; c < MC; ++c) {
        const double t = red[lane * MC + c] + red[(64 + lane) * MC + c] +
                         red[(128 + lane) * MC + c] + red[(192 + lane) * MC + c];
        z[i * ldz + c] = (r[i * ldr + c] - t) * inv_lp;
      }
    }
  }
}

// LDS floats needed by woodbury_z for MC columns
constexpr int woodbury_z_smem_floats(int MC) {
  return 4 * 64 * (WB_CH + 1) > 4 * 64 * MC * 2 ? 4 * 64 * (WB_CH + 1) : 4 * 64 * MC * 2;
}

}  // namespace krr
