// Woodbury apply of the random-features preconditioner (Sec. 3.1):
//   z = (ZZ^T + lambda_p I)^{-1} r = (r - Ut (Ut^T r)) / lambda_p,   Ut = Z C^{-T} (n x s, FP32).
// Two streaming passes over Ut, each reading it once from HBM; FP64 accumulation.
// Device bodies shared by the single-problem and the batched launches.
#pragma once
#include <type_traits>

#include "common.hpp"

namespace krr {

// Pass 1: T partial over rows [i0, i1) for feature columns k0 .. k0 + KPT - 1 (consecutive
// threads take consecutive column groups, so every row read is one contiguous segment; KPT
// columns per thread and sixteen rows per step keep enough loads in flight to stream Ut).
// All threads of the block call it with the same rows: the rows of r are staged in LDS
// (sr: at least WB_RB * MC doubles) in rounds of WB_RB and read back as broadcasts.
// out[k * ldo + c] = sum_{i in [i0, i1)} Ut[i][k] r[i][c], c < MC.
constexpr int WB_RB = 128;  // rows of r staged per round
template <int MC, int KPT>
__device__ __forceinline__ void woodbury_tpart(const float* __restrict__ Ut, int64_t ldu,
                                               int64_t s, const double* __restrict__ r,
                                               int64_t ldr, int64_t i0, int64_t i1, int64_t k0,
                                               double* __restrict__ out, int64_t ldo,
                                               double* __restrict__ sr) {
  constexpr int RU = 16;  // rows per step
  double acc[KPT][MC];
#pragma unroll
  for (int q = 0; q < KPT; ++q)
#pragma unroll
    for (int c = 0; c < MC; ++c) acc[q][c] = 0.0;
  bool kin[KPT];
#pragma unroll
  for (int q = 0; q < KPT; ++q) kin[q] = k0 + q < s;
  // vector loads when the whole group is in range and aligned (ldu and k0 multiples of KPT)
  const bool vec = KPT > 1 && k0 + KPT <= s && (ldu % KPT) == 0 &&
                   (reinterpret_cast<uintptr_t>(Ut) % (4 * KPT)) == 0;
  const float* up = Ut + (kin[0] ? k0 : 0);
  // rows [ib, ib + nr) of one round; VEC selects float2 loads (uniform per thread)
  auto rows = [&](auto vec_tag, int64_t ib, int nr) __attribute__((always_inline)) {
    constexpr bool VEC = decltype(vec_tag)::value;
    auto load = [&](int64_t i, float (&u)[KPT]) __attribute__((always_inline)) {
      if (VEC) {
        const float2 t = *reinterpret_cast<const float2*>(up + i * ldu);
        u[0] = t.x;
        u[KPT - 1] = t.y;
      } else {
#pragma unroll
        for (int q = 0; q < KPT; ++q) {
          const float t = Ut[kin[q] ? i * ldu + k0 + q : 0];
          u[q] = kin[q] ? t : 0.0f;
        }
      }
    };
    int j0 = 0;
    for (; j0 + RU <= nr; j0 += RU) {
      float u[RU][KPT];
#pragma unroll
      for (int j = 0; j < RU; ++j) load(ib + j0 + j, u[j]);
#pragma unroll
      for (int j = 0; j < RU; ++j) {
        const double* rr = sr + (j0 + j) * MC;
#pragma unroll
        for (int c = 0; c < MC; ++c) {
          const double rc = rr[c];
#pragma unroll
          for (int q = 0; q < KPT; ++q) acc[q][c] = fma((double)u[j][q], rc, acc[q][c]);
        }
      }
    }
    for (; j0 < nr; ++j0) {
      float u[KPT];
      load(ib + j0, u);
      const double* rr = sr + j0 * MC;
#pragma unroll
      for (int c = 0; c < MC; ++c)
#pragma unroll
        for (int q = 0; q < KPT; ++q) acc[q][c] = fma((double)u[q], rr[c], acc[q][c]);
    }
  };
  for (int64_t ib = i0; ib < i1; ib += WB_RB) {
    const int nr = (int)(i1 - ib < WB_RB ? i1 - ib : WB_RB);
    __syncthreads();  // the previous round's reads of sr are done
    for (int e = threadIdx.x; e < nr * MC; e += blockDim.x) sr[e] = r[(ib + e / MC) * ldr + e % MC];
    __syncthreads();
    if (KPT > 1 && vec) rows(std::true_type{}, ib, nr);
    else rows(std::false_type{}, ib, nr);
  }
#pragma unroll
  for (int q = 0; q < KPT; ++q)
    if (kin[q]) {
#pragma unroll
      for (int c = 0; c < MC; ++c) out[(k0 + q) * ldo + c] = acc[q][c];
    }
}

// columns per thread of the first pass for MC right-hand sides
constexpr int woodbury_kpt(int MC) { return MC <= 8 ? 2 : 1; }

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
