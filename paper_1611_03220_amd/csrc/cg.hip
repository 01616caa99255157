// PCG vector work: per-column FP64 inner products, step lengths,
// iterate updates, convergence masks, and the Woodbury preconditioner apply
//   z = (r - Ut (Ut^T r)) / lambda_p     (Sec. 3.1).
// Reductions are two-pass and deterministic: each block writes one partial per column;
// consumers sum the partials in block order.
#include "kernels.hpp"
#include "woodbury.hpp"

namespace krr {

constexpr int RB = 256;  // threads per reduction block

// Block-level column sums of f(i, c) over rows [r0, r1), written to part[blockIdx.x*m + c].
// Thread t handles column t % m and rows offset by t / m (256 / m rows in flight).
template <typename F>
__device__ inline void colwise_block_sum(F f, int64_t r0, int64_t r1, int64_t m,
                                         double* __restrict__ part, double* sh) {
  const int tid = threadIdx.x;
  for (int64_t cbase = 0; cbase < m; cbase += RB) {
    const int64_t mc = m - cbase < RB ? m - cbase : RB;
    const int rows_in_flight = (int)(RB / mc);
    double acc = 0.0;
    const int64_t c = cbase + tid % mc;
    const int ro = tid / (int)mc;
    if (ro < rows_in_flight)
      for (int64_t i = r0 + ro; i < r1; i += rows_in_flight) acc += f(i, c);
    sh[tid] = (ro < rows_in_flight) ? acc : 0.0;
    __syncthreads();
    if (tid < mc) {
      double s = 0.0;
      for (int k = 0; k < rows_in_flight; ++k) s += sh[k * mc + tid];
      part[(int64_t)blockIdx.x * m + cbase + tid] = s;
    }
    __syncthreads();
  }
}

__device__ inline void row_range(int64_t n, int64_t& r0, int64_t& r1) {
  const int64_t per = ceil_div(n, gridDim.x);
  r0 = (int64_t)blockIdx.x * per;
  r1 = r0 + per < n ? r0 + per : n;
}

// part[b][c] = sum_{i in block b} a[i][c] * b[i][c]
template <typename TA, typename TB>
__global__ __launch_bounds__(RB) void dot_partial_kernel(const TA* __restrict__ a, int64_t lda,
                                                         const TB* __restrict__ b, int64_t ldb,
                                                         int64_t n, int64_t m,
                                                         double* __restrict__ part) {
  __shared__ double sh[RB];
  int64_t r0, r1;
  row_range(n, r0, r1);
  colwise_block_sum([&](int64_t i, int64_t c) { return (double)a[i * lda + c] * (double)b[i * ldb + c]; },
                    r0, r1, m, part, sh);
}

template <typename TA, typename TB>
hipError_t dot_partial(const TA* a, int64_t lda, const TB* b, int64_t ldb, int64_t n, int64_t m,
                       double* part, int nblk, hipStream_t st) {
  dot_partial_kernel<TA, TB><<<nblk, RB, 0, st>>>(a, lda, b, ldb, n, m, part);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
template hipError_t dot_partial<double, double>(const double*, int64_t, const double*, int64_t,
                                                int64_t, int64_t, double*, int, hipStream_t);
template hipError_t dot_partial<float, double>(const float*, int64_t, const double*, int64_t,
                                               int64_t, int64_t, double*, int, hipStream_t);

// Sum of the nblk block partials of column c by one wave (lane-strided, then a shuffle
// tree): a fixed order, so the result is deterministic. Lane 0 holds the sum used.
__device__ inline double sum_parts(const double* part, int nblk, int64_t m, int64_t c) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int b = lane; b < nblk; b += 64) s += part[(int64_t)b * m + c];
  return wave_sum(s);
}

// ---------------------------------------------------------------- scalar kernels
// One block of 256 threads; wave w handles columns w, w + 4, ...; lane 0 decides and writes.
// Initial state: ynorm = ||y||, rnorm = ||r0||; active if finite and rnorm > tol * ynorm,
// broken if non-finite; rho = <r0, z0> (from part_rz) for active columns.
__global__ __launch_bounds__(256) void cg_init_scalars_kernel(
    const double* part_yy, const double* part_rr, const double* part_rz, int nblk, int64_t m,
    double tol, double* ynorm, double* rnorm, double* rho, int* active, int* broken,
    int* col_iters, int* count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t c = w; c < m; c += 4) {
    const double yn = sqrt(sum_parts(part_yy, nblk, m, c));
    const double rn = sqrt(sum_parts(part_rr, nblk, m, c));
    const double rz = part_rz ? sum_parts(part_rz, nblk, m, c) : rn * rn;
    if (lane == 0) {
      const bool bad = !isfinite(yn) || !isfinite(rn) || !isfinite(rz);
      const bool act = !bad && rn > tol * yn;
      ynorm[c] = yn;
      rnorm[c] = rn;
      rho[c] = rz;
      active[c] = act ? 1 : 0;
      broken[c] = bad ? 1 : 0;
      col_iters[c] = 0;
      if (act) atomicAdd(&cnt, 1);
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) *count = cnt;
}

// alpha_c = rho_c / <p, Ap>_c for active columns; curvature <= 0 or non-finite -> breakdown.
__global__ __launch_bounds__(256) void cg_alpha_kernel(const double* part_pq, int nblk, int64_t m,
                                                       const double* rho, int* active,
                                                       int* broken, double* alpha) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t c = w; c < m; c += 4) {
    if (!active[c]) {  // wave-uniform
      if (lane == 0) alpha[c] = 0.0;
      continue;
    }
    const double pq = sum_parts(part_pq, nblk, m, c);
    if (lane == 0) {
      double a = 0.0;
      if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rho[c])) {
        active[c] = 0;
        broken[c] = 1;
      } else {
        a = rho[c] / pq;
      }
      alpha[c] = a;
    }
  }
}

// ||r|| and convergence: active columns with ||r|| <= tol ||y|| are frozen.
__global__ __launch_bounds__(256) void cg_conv_kernel(const double* part_rr, int nblk, int64_t m,
                                                      double tol, const double* ynorm,
                                                      double* rnorm, int* active, int* broken,
                                                      int* col_iters, int it, int* count,
                                                      double* hist_slot) {
  __shared__ int cnt;
  __shared__ double worst;
  if (threadIdx.x == 0) { cnt = 0; worst = 0.0; }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t c = w; c < m; c += 4) {
    if (!active[c]) continue;  // wave-uniform
    const double rn = sqrt(sum_parts(part_rr, nblk, m, c));
    if (lane == 0) {
      rnorm[c] = rn;
      col_iters[c] = it;
      if (!isfinite(rn)) {
        active[c] = 0;
        broken[c] = 1;
      } else if (rn <= tol * ynorm[c]) {
        active[c] = 0;
      } else {
        atomicAdd(&cnt, 1);
      }
      const double rel = ynorm[c] > 0.0 ? rn / ynorm[c] : 0.0;
      if (isfinite(rel)) atomicMax(reinterpret_cast<unsigned long long*>(&worst),
                                   (unsigned long long)__double_as_longlong(rel));
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    *count = cnt;
    if (hist_slot) *hist_slot = worst;
  }
}

// beta = rho_new / rho for active columns; rho <- rho_new. Non-finite -> breakdown.
__global__ __launch_bounds__(256) void cg_beta_kernel(const double* part_rz, const double* part_rr,
                                                      int nblk, int64_t m, double* rho,
                                                      int* active, int* broken, double* beta) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t c = w; c < m; c += 4) {
    if (!active[c]) {  // wave-uniform
      if (lane == 0) beta[c] = 0.0;
      continue;
    }
    const double rn = part_rz ? sum_parts(part_rz, nblk, m, c) : sum_parts(part_rr, nblk, m, c);
    if (lane == 0) {
      double bt = 0.0;
      if (!isfinite(rn) || rho[c] == 0.0) {
        active[c] = 0;
        broken[c] = 1;
      } else {
        bt = rn / rho[c];
        rho[c] = rn;
      }
      beta[c] = bt;
    }
  }
}

hipError_t cg_init_scalars(const double* part_yy, const double* part_rr, const double* part_rz,
                           int nblk, int64_t m, double tol, CGScalars& S, hipStream_t st) {
  cg_init_scalars_kernel<<<1, 256, 0, st>>>(part_yy, part_rr, part_rz, nblk, m, tol, S.ynorm,
                                            S.rnorm, S.rho, S.active, S.broken, S.col_iters,
                                            S.count);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
hipError_t cg_alpha(const double* part_pq, int nblk, int64_t m, CGScalars& S, hipStream_t st) {
  cg_alpha_kernel<<<1, 256, 0, st>>>(part_pq, nblk, m, S.rho, S.active, S.broken, S.alpha);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
hipError_t cg_conv(const double* part_rr, int nblk, int64_t m, double tol, int it, CGScalars& S,
                   double* hist_slot, hipStream_t st) {
  cg_conv_kernel<<<1, 256, 0, st>>>(part_rr, nblk, m, tol, S.ynorm, S.rnorm, S.active, S.broken,
                                    S.col_iters, it, S.count, hist_slot);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
hipError_t cg_beta(const double* part_rz, const double* part_rr, int nblk, int64_t m,
                   CGScalars& S, hipStream_t st) {
  cg_beta_kernel<<<1, 256, 0, st>>>(part_rz, part_rr, nblk, m, S.rho, S.active, S.broken, S.beta);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// ---------------------------------------------------------------- vector updates
// x += alpha p~, r -= alpha q (active columns only, alpha = 0 otherwise); part_rr partials.
template <typename TP>
__global__ __launch_bounds__(RB) void cg_update_xr_kernel(double* __restrict__ x, int64_t ldx,
                                                          double* __restrict__ r,
                                                          const TP* __restrict__ p, int64_t ldp,
                                                          const double* __restrict__ q,
                                                          const double* __restrict__ alpha,
                                                          int64_t n, int64_t m,
                                                          double* __restrict__ part_rr) {
  __shared__ double sh[RB];
  int64_t r0, r1;
  row_range(n, r0, r1);
  colwise_block_sum(
      [&](int64_t i, int64_t c) {
        const double a = alpha[c];
        double rv = r[i * m + c];
        if (a != 0.0) {
          x[i * ldx + c] += a * (double)p[i * ldp + c];
          rv -= a * q[i * m + c];
          r[i * m + c] = rv;
        }
        return rv * rv;
      },
      r0, r1, m, part_rr, sh);
}

template <typename TP>
hipError_t cg_update_xr(double* x, int64_t ldx, double* r, const TP* p, int64_t ldp,
                        const double* q, const double* alpha, int64_t n, int64_t m,
                        double* part_rr, int nblk, hipStream_t st) {
  cg_update_xr_kernel<TP><<<nblk, RB, 0, st>>>(x, ldx, r, p, ldp, q, alpha, n, m, part_rr);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
template hipError_t cg_update_xr<double>(double*, int64_t, double*, const double*, int64_t,
                                         const double*, const double*, int64_t, int64_t, double*,
                                         int, hipStream_t);
template hipError_t cg_update_xr<float>(double*, int64_t, double*, const float*, int64_t,
                                        const double*, const double*, int64_t, int64_t, double*,
                                        int, hipStream_t);

// p = z + beta p for active columns (first call: beta = 0 and all columns set: init = 1);
// pf (FP32 copy used by the mixed kernel product, row stride ldpf) refreshed when given.
__global__ void cg_update_p_kernel(const double* __restrict__ z, double* __restrict__ p,
                                   float* __restrict__ pf, int64_t ldpf,
                                   const double* __restrict__ beta, const int* __restrict__ active,
                                   int init, int64_t n, int64_t m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e / m, c = e % m;
  double v;
  if (init) {
    v = z[e];
  } else if (active[c]) {
    v = z[e] + beta[c] * p[e];
  } else {
    return;
  }
  p[e] = v;
  if (pf) pf[i * ldpf + c] = (float)v;
}

hipError_t cg_update_p(const double* z, double* p, float* pf, int64_t ldpf, const double* beta,
                       const int* active, int init, int64_t n, int64_t m, hipStream_t st) {
  cg_update_p_kernel<<<ceil_div(n * m, 256), 256, 0, st>>>(z, p, pf, ldpf, beta, active, init, n,
                                                           m);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// r = y - (Ax) (warm start), FP64, n x m contiguous r; y with ldy.
__global__ void sub_kernel(const double* __restrict__ y, int64_t ldy, const double* __restrict__ ax,
                           int64_t n, int64_t m, double* __restrict__ r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e / m, c = e % m;
  r[e] = y[i * ldy + c] - (ax ? ax[e] : 0.0);
}

hipError_t residual_from(const double* y, int64_t ldy, const double* ax, int64_t n, int64_t m,
                         double* r, hipStream_t st) {
  sub_kernel<<<ceil_div(n * m, 256), 256, 0, st>>>(y, ldy, ax, n, m, r);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// Copy an n x m block between strided FP64 arrays.
__global__ void copy2d_kernel(const double* __restrict__ a, int64_t lda, double* __restrict__ b,
                              int64_t ldb, int64_t n, int64_t m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e / m, c = e % m;
  b[i * ldb + c] = a[i * lda + c];
}
hipError_t copy2d(const double* a, int64_t lda, double* b, int64_t ldb, int64_t n, int64_t m,
                  hipStream_t st) {
  if (n * m == 0) return hipSuccess;
  copy2d_kernel<<<ceil_div(n * m, 256), 256, 0, st>>>(a, lda, b, ldb, n, m);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// b += a (strided FP64)
__global__ void axpy2d_kernel(const double* __restrict__ a, int64_t lda, double* __restrict__ b,
                              int64_t ldb, int64_t n, int64_t m) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e / m, c = e % m;
  b[i * ldb + c] += a[i * lda + c];
}
hipError_t add2d(const double* a, int64_t lda, double* b, int64_t ldb, int64_t n, int64_t m,
                 hipStream_t st) {
  if (n * m == 0) return hipSuccess;
  axpy2d_kernel<<<ceil_div(n * m, 256), 256, 0, st>>>(a, lda, b, ldb, n, m);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// ---------------------------------------------------------- preconditioner apply
// Pass 1 (T partials over row chunks) and pass 2 (z) of the Woodbury apply; the device
// bodies are shared with the batched solve. m columns run in passes of at most PC_M.
constexpr int PC_M = 16;
template <int MC>
__global__ __launch_bounds__(256) void precond_t_partial_kernel(
    const float* __restrict__ Ut, int64_t ldu, const double* __restrict__ r, int64_t n, int64_t s,
    int64_t m, int c0, int64_t rows_per_chunk, double* __restrict__ part) {
  constexpr int KPT = woodbury_kpt(MC);
  __shared__ double sr[WB_RB * MC];
  const int64_t k0 = ((int64_t)blockIdx.x * 256 + threadIdx.x) * KPT;
  const int64_t i0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t i1 = i0 + rows_per_chunk < n ? i0 + rows_per_chunk : n;
  woodbury_tpart<MC, KPT>(Ut, ldu, s, r + c0, m, i0, i1, k0,
                          part + (int64_t)blockIdx.y * s * m + c0, m, sr);
}

// T[k][c] = sum_chunk part[chunk][k][c]
__global__ void precond_t_reduce_kernel(const double* __restrict__ part, int nchunk, int64_t s,
                                        int64_t m, double* __restrict__ T) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= s * m) return;
  // four interleaved partial sums (independent loads in flight), combined in a fixed order
  const int64_t st = s * m;
  double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
  int b = 0;
  for (; b + 4 <= nchunk; b += 4) {
    v0 += part[(int64_t)b * st + e];
    v1 += part[(int64_t)(b + 1) * st + e];
    v2 += part[(int64_t)(b + 2) * st + e];
    v3 += part[(int64_t)(b + 3) * st + e];
  }
  for (; b < nchunk; ++b) v0 += part[(int64_t)b * st + e];
  T[e] = (v0 + v1) + (v2 + v3);
}

// Pass 2: z[i][c] = (r[i][c] - sum_k Ut[i][k] T[k][c]) / lambda_p for 64-row blocks.
template <int MC>
__global__ __launch_bounds__(256) void precond_z_kernel(const float* __restrict__ Ut, int64_t ldu,
                                                        const double* __restrict__ T,
                                                        const double* __restrict__ r, int64_t n,
                                                        int64_t s, int64_t m, int c0,
                                                        double inv_lp, double* __restrict__ z) {
  __shared__ __attribute__((aligned(16))) float smem[woodbury_z_smem_floats(MC)];
  woodbury_z<MC>(Ut, ldu, s, T + c0, m, r + c0, m, inv_lp, z + c0, m, (int64_t)blockIdx.x * 64, n,
                 smem);
}

hipError_t precond_apply(const float* Ut, int64_t ldu, int64_t n, int64_t s, int64_t m,
                         double lambda_p, const double* r, double* z, double* part, int nchunk,
                         double* T, hipStream_t st) {
  const int64_t rows_per_chunk = ceil_div(n, nchunk);
  for (int64_t c0 = 0; c0 < m; c0 += PC_M) {
    const int mc = (int)std::min<int64_t>(PC_M, m - c0);
    dim3 g1(ceil_div(s, 256 * (mc <= 8 ? 2 : 1)), nchunk);  // 256 threads x woodbury_kpt(mc)
    switch (mc) {
#define KRR_PC(N)                                                                            \
  case N:                                                                                    \
    precond_t_partial_kernel<N><<<g1, 256, 0, st>>>(Ut, ldu, r, n, s, m, (int)c0,            \
                                                    rows_per_chunk, part);                   \
    break;
      KRR_PC(1) KRR_PC(2) KRR_PC(3) KRR_PC(4) KRR_PC(5) KRR_PC(6) KRR_PC(7) KRR_PC(8)
      KRR_PC(9) KRR_PC(10) KRR_PC(11) KRR_PC(12) KRR_PC(13) KRR_PC(14) KRR_PC(15) KRR_PC(16)
#undef KRR_PC
    }
    KRR_LAUNCH_CHECK();
  }
  precond_t_reduce_kernel<<<ceil_div(s * m, 256), 256, 0, st>>>(part, nchunk, s, m, T);
  KRR_LAUNCH_CHECK();
  for (int64_t c0 = 0; c0 < m; c0 += PC_M) {
    const int mc = (int)std::min<int64_t>(PC_M, m - c0);
    switch (mc) {
#define KRR_PZ(N)                                                                           \
  case N:                                                                                   \
    precond_z_kernel<N><<<ceil_div(n, 64), 256, 0, st>>>(Ut, ldu, T, r, n, s, m, (int)c0,   \
                                                         1.0 / lambda_p, z);                \
    break;
      KRR_PZ(1) KRR_PZ(2) KRR_PZ(3) KRR_PZ(4) KRR_PZ(5) KRR_PZ(6) KRR_PZ(7) KRR_PZ(8)
      KRR_PZ(9) KRR_PZ(10) KRR_PZ(11) KRR_PZ(12) KRR_PZ(13) KRR_PZ(14) KRR_PZ(15) KRR_PZ(16)
#undef KRR_PZ
    }
    KRR_LAUNCH_CHECK();
  }
  return hipSuccess;
}

}  // namespace krr
