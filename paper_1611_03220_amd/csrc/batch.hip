// Batched PCG vector work: many independent problems packed row-wise.
// Problem p owns packed rows [off_p, off_p + n_p) (offsets are multiples of ROW_PAD) and M
// columns (p's own m_p <= M; extra columns carry zero right-hand sides and stay inactive).
// Per-(problem, column) scalars live at index p * M + c. Reductions are two-pass and
// deterministic: reduction items (problem, 1024-row chunk) write partials, scalar kernels sum
// a problem's partials in item order.
#include "batch.hpp"
#include "woodbury.hpp"

namespace krr {

__device__ inline int row_to_inst(const int* __restrict__ row_inst, int64_t row) {
  return row_inst[row];
}

// partial[item][c] = sum over the item's rows of a[row][c] * b[row][c]
template <typename TA, typename TB>
__global__ __launch_bounds__(256) void batch_dot_kernel(const TA* __restrict__ a,
                                                        const TB* __restrict__ b, int M,
                                                        const RedItem* __restrict__ items,
                                                        const int* __restrict__ live,
                                                        double* __restrict__ part) {
  const RedItem it = items[blockIdx.x];
  if (!live[it.inst]) return;
  __shared__ double sh[256];
  const int tid = threadIdx.x;
  const int rif = 256 / M;
  const int ro = tid / M, c = tid % M;
  double acc = 0.0;
  if (ro < rif)
    for (int64_t row = it.r0 + ro; row < it.r1; row += rif)
      acc += (double)a[row * M + c] * (double)b[row * M + c];
  sh[tid] = ro < rif ? acc : 0.0;
  __syncthreads();
  if (tid < M) {
    double s = 0.0;
    for (int k = 0; k < rif; ++k) s += sh[k * M + tid];
    part[(int64_t)blockIdx.x * M + tid] = s;
  }
}

template <typename TA, typename TB>
hipError_t batch_dot(const TA* a, const TB* b, int M, const RedItem* items, int nitems,
                     const int* live, double* part, hipStream_t st) {
  batch_dot_kernel<TA, TB><<<nitems, 256, 0, st>>>(a, b, M, items, live, part);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
template hipError_t batch_dot<double, double>(const double*, const double*, int, const RedItem*,
                                              int, const int*, double*, hipStream_t);
template hipError_t batch_dot<float, double>(const float*, const double*, int, const RedItem*,
                                             int, const int*, double*, hipStream_t);

__device__ inline double inst_sum(const double* part, const BatchMeta& P, int M, int c) {
  double s = 0.0;
  for (int k = P.red_begin; k < P.red_end; ++k) s += part[(int64_t)k * M + c];
  return s;
}

// ---------------------------------------------------------------- scalars
__global__ void batch_init_kernel(const BatchMeta* __restrict__ meta, int count, int M,
                                  const double* part_yy, const double* part_rz,
                                  BatchScalars S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) { *S.count = 0; *S.iter = 0; }
  if (e >= count * M) return;
  const int p = e / M, c = e % M;
  const BatchMeta P = meta[p];
  const double yn = sqrt(inst_sum(part_yy, P, M, c));
  const double rz = part_rz ? inst_sum(part_rz, P, M, c) : yn * yn;
  const bool bad = !isfinite(yn) || !isfinite(rz);
  const bool act = c < P.m && !bad && yn > 0.0 && S.tol[e] < 1.0;
  S.ynorm[e] = yn;
  S.rnorm[e] = yn;
  S.rho[e] = rz;
  S.active[e] = act ? 1 : 0;
  S.broken[e] = (c < P.m && bad) ? 1 : 0;
  S.col_iters[e] = 0;
}

__global__ void batch_count_kernel(int n, const int* __restrict__ active, int* count) {
  __shared__ int cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  for (int e = threadIdx.x; e < n; e += blockDim.x)
    if (active[e]) atomicAdd(&cnt, 1);
  __syncthreads();
  if (threadIdx.x == 0) *count = cnt;
}

__global__ void batch_alpha_kernel(const BatchMeta* __restrict__ meta, int count, int M,
                                   const double* part_pq, BatchScalars S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) *S.count = 0;
  if (e >= count * M) return;
  double a = 0.0;
  if (S.active[e]) {
    const double pq = inst_sum(part_pq, meta[e / M], M, e % M);
    if (!(pq > 0.0) || !isfinite(pq) || !isfinite(S.rho[e])) {
      S.active[e] = 0;
      S.broken[e] = 1;
    } else {
      a = S.rho[e] / pq;
    }
  }
  S.alpha[e] = a;
}

__global__ void batch_conv_kernel(const BatchMeta* __restrict__ meta, int count, int M,
                                  const double* part_rr, BatchScalars S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int it = *S.iter + 1;
  if (e < count * M && S.active[e]) {
    const double rn = sqrt(inst_sum(part_rr, meta[e / M], M, e % M));
    S.rnorm[e] = rn;
    S.col_iters[e] = it;
    if (!isfinite(rn)) {
      S.active[e] = 0;
      S.broken[e] = 1;
    } else if (rn <= S.tol[e] * S.ynorm[e]) {
      S.active[e] = 0;
    } else {
      atomicAdd(S.count, 1);
    }
  }
}

__global__ void batch_beta_kernel(const BatchMeta* __restrict__ meta, int count, int M,
                                  const double* part_rz, const double* part_rr, BatchScalars S) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e == 0) *S.iter += 1;
  if (e >= count * M) return;
  double bt = 0.0;
  if (S.active[e]) {
    const BatchMeta P = meta[e / M];
    const double rn = P.has_u ? inst_sum(part_rz, P, M, e % M) : inst_sum(part_rr, P, M, e % M);
    if (!isfinite(rn) || S.rho[e] == 0.0) {
      S.active[e] = 0;
      S.broken[e] = 1;
    } else {
      bt = rn / S.rho[e];
      S.rho[e] = rn;
    }
  }
  S.beta[e] = bt;
}

// live[p] = 1 while any column of problem p is active
__global__ void batch_live_kernel(int count, int M, const int* __restrict__ active,
                                  int* __restrict__ live) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= count) return;
  int any = 0;
  for (int c = 0; c < M; ++c) any |= active[p * M + c];
  live[p] = any;
}

static inline int sgrid(int n) { return (n + 255) / 256; }

hipError_t batch_init_scalars(const BatchMeta* meta, int count, int M, const double* part_yy,
                              const double* part_rz, BatchScalars& S, hipStream_t st) {
  batch_init_kernel<<<sgrid(count * M), 256, 0, st>>>(meta, count, M, part_yy, part_rz, S);
  KRR_LAUNCH_CHECK();
  batch_count_kernel<<<1, 256, 0, st>>>(count * M, S.active, S.count);
  KRR_LAUNCH_CHECK();
  batch_live_kernel<<<sgrid(count), 256, 0, st>>>(count, M, S.active, S.live);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
hipError_t batch_alpha(const BatchMeta* meta, int count, int M, const double* part_pq,
                       BatchScalars& S, hipStream_t st) {
  batch_alpha_kernel<<<sgrid(count * M), 256, 0, st>>>(meta, count, M, part_pq, S);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
hipError_t batch_conv(const BatchMeta* meta, int count, int M, const double* part_rr,
                      BatchScalars& S, hipStream_t st) {
  batch_conv_kernel<<<sgrid(count * M), 256, 0, st>>>(meta, count, M, part_rr, S);
  KRR_LAUNCH_CHECK();
  batch_live_kernel<<<sgrid(count), 256, 0, st>>>(count, M, S.active, S.live);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
hipError_t batch_beta(const BatchMeta* meta, int count, int M, const double* part_rz,
                      const double* part_rr, BatchScalars& S, hipStream_t st) {
  batch_beta_kernel<<<sgrid(count * M), 256, 0, st>>>(meta, count, M, part_rz, part_rr, S);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// ---------------------------------------------------------------- vectors
// q[row][c] = sum_split part_p[split][lr][c] + lambda_p * pf[row][c] (zero on padding rows)
__global__ void batch_finalize_kernel(const BatchMeta* __restrict__ meta,
                                      const int* __restrict__ row_inst,
                                      const int* __restrict__ live, int64_t nrows, int M,
                                      const float* __restrict__ pf, double* __restrict__ q) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrows * M) return;
  const int64_t row = e / M;
  const int c = (int)(e % M);
  const int p = row_to_inst(row_inst, row);
  if (!live[p]) return;
  const BatchMeta P = meta[p];
  const int64_t lr = row - P.off;
  double v = 0.0;
  if (lr < P.n) {
    for (int k = 0; k < P.nsplit; ++k) v += P.part[k * P.part_stride + lr * M + c];
    v += P.lambda * (double)pf[e];
  }
  q[e] = v;
}

hipError_t batch_finalize(const BatchMeta* meta, const int* row_inst, const int* live,
                          int64_t nrows, int M, const float* pf, double* q, hipStream_t st) {
  batch_finalize_kernel<<<ceil_div(nrows * M, 256), 256, 0, st>>>(meta, row_inst, live, nrows, M,
                                                                  pf, q);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// x += alpha pf, r -= alpha q per (problem, column), then ||r||^2 partials per reduction item
__global__ void batch_update_xr_kernel(const int* __restrict__ row_inst, int64_t nrows, int M,
                                       const double* __restrict__ alpha, const float* __restrict__ pf,
                                       const double* __restrict__ q, double* __restrict__ x,
                                       double* __restrict__ r) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrows * M) return;
  const int p = row_to_inst(row_inst, e / M);
  const double a = alpha[p * M + (int)(e % M)];
  if (a != 0.0) {
    x[e] += a * (double)pf[e];
    r[e] -= a * q[e];
  }
}

hipError_t batch_update_xr(const int* row_inst, int64_t nrows, int M, const double* alpha,
                           const float* pf, const double* q, double* x, double* r,
                           hipStream_t st) {
  batch_update_xr_kernel<<<ceil_div(nrows * M, 256), 256, 0, st>>>(row_inst, nrows, M, alpha, pf,
                                                                   q, x, r);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// p = z + beta p for active (problem, column); init: p = z everywhere. pf = (float)p.
__global__ void batch_update_p_kernel(const int* __restrict__ row_inst, int64_t nrows, int M,
                                      const double* __restrict__ beta, const int* __restrict__ active,
                                      int init, const double* __restrict__ z, double* __restrict__ p,
                                      float* __restrict__ pf) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrows * M) return;
  const int k = row_to_inst(row_inst, e / M) * M + (int)(e % M);
  double v;
  if (init) v = z[e];
  else if (active[k]) v = z[e] + beta[k] * p[e];
  else return;
  p[e] = v;
  pf[e] = (float)v;
}

hipError_t batch_update_p(const int* row_inst, int64_t nrows, int M, const double* beta,
                          const int* active, int init, const double* z, double* p, float* pf,
                          hipStream_t st) {
  batch_update_p_kernel<<<ceil_div(nrows * M, 256), 256, 0, st>>>(row_inst, nrows, M, beta, active,
                                                                  init, z, p, pf);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// ------------------------------------------------------- V^T split for the batch product
// colmax[p * 16 + c] = max |pf| over problem p's rows (reduction items), atomic max.
__global__ __launch_bounds__(256) void batch_colmax_kernel(const float* __restrict__ pf, int M,
                                                           const RedItem* __restrict__ items,
                                                           const int* __restrict__ live,
                                                           float* __restrict__ colmax) {
  const RedItem it = items[blockIdx.x];
  if (!live[it.inst]) return;
  __shared__ float sh[256];
  const int tid = threadIdx.x;
  const int rif = 256 / M;
  const int ro = tid / M, c = tid % M;
  float mx = 0.0f;
  if (ro < rif)
    for (int64_t row = it.r0 + ro; row < it.r1; row += rif) mx = fmaxf(mx, fabsf(pf[row * M + c]));
  sh[tid] = ro < rif ? mx : 0.0f;
  __syncthreads();
  if (tid < M) {
    float v = 0.0f;
    for (int k = 0; k < rif; ++k) v = fmaxf(v, sh[k * M + tid]);
    atomic_max_pos(&colmax[it.inst * 16 + tid], v);
  }
}

// Vt[c][row] = split(q_pc pf[row][c]) for c < 16 (zero beyond M and on padding rows);
// pf <- the value the split represents; vscale[p * 16 + c] = 1 / q_pc. 32-row tiles never
// straddle problems (offsets are multiples of ROW_PAD). Packed (M <= 8): row c < 8 of hi
// holds the high part of column c, row c + 8 its low part, and lo is not written.
__global__ __launch_bounds__(256) void batch_split_kernel(const int* __restrict__ row_inst,
                                                          const BatchMeta* __restrict__ meta,
                                                          const int* __restrict__ live,
                                                          int64_t nrows, int M,
                                                          float* __restrict__ pf,
                                                          const float* __restrict__ colmax,
                                                          _Float16* __restrict__ hi,
                                                          _Float16* __restrict__ lo,
                                                          float* __restrict__ vscale,
                                                          int packed) {
  __shared__ float tile[32][17];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t r0 = (int64_t)blockIdx.x * 32;
  const int p = row_to_inst(row_inst, r0);
  if (!live[p]) return;
  const BatchMeta P = meta[p];
  for (int e = threadIdx.x; e < 32 * 16; e += 256) {
    const int rr = e / 16, c = e % 16;
    const int64_t row = r0 + rr;
    tile[rr][c] = (c < M && row - P.off < P.n) ? pf[row * M + c] : 0.0f;
  }
  __syncthreads();
  for (int c = ty; c < 16; c += 8) {
    const int cv = packed ? (c & 7) : c;  // source column
    const bool low_row = packed && c >= 8;
    const float qv = cv < M ? split_scale(colmax[p * 16 + cv]) : 1.0f;
    const int64_t row = r0 + tx;
    const float v = tile[tx][cv] * qv;
    _Float16 h, l;
    Elem<_Float16>::split(v, h, l);
    if (packed) {
      hi[(int64_t)c * nrows + row] = low_row ? l : h;
    } else {
      hi[(int64_t)c * nrows + row] = h;
      lo[(int64_t)c * nrows + row] = l;
    }
    if (low_row) {
      if (row == P.off) vscale[p * 16 + c] = 0.0f;
      continue;
    }
    if (c < M && row - P.off < P.n) pf[row * M + c] = ((float)h + (float)l) / qv;
    if (row == P.off) vscale[p * 16 + c] = c < M ? 1.0f / qv : 0.0f;
  }
}

hipError_t batch_split_v(const int* row_inst, const BatchMeta* meta, const int* live, int count,
                         int64_t nrows, int M, float* pf, const RedItem* items, int nitems,
                         float* colmax, _Float16* hi, _Float16* lo, float* vscale, bool packed,
                         hipStream_t st) {
  if (packed && M > 8) return hipErrorInvalidValue;
  hipError_t e = fill_f32(colmax, (int64_t)count * 16, 0.0f, st);
  if (e != hipSuccess) return e;
  batch_colmax_kernel<<<nitems, 256, 0, st>>>(pf, M, items, live, colmax);
  KRR_LAUNCH_CHECK();
  batch_split_kernel<<<ceil_div(nrows, 32), 256, 0, st>>>(row_inst, meta, live, nrows, M, pf,
                                                          colmax, hi, lo, vscale, packed ? 1 : 0);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// --------------------------------------------------------- batched preconditioner
// Pass 1: item (problem, 256 feature columns, row chunk): part[item chunk][k][c] for c < M.
template <int MC>
__global__ __launch_bounds__(256) void batch_t_partial_kernel(const PCItem* __restrict__ items,
                                                              const BatchMeta* __restrict__ meta,
                                                              const int* __restrict__ live,
                                                              const double* __restrict__ r,
                                                              double* __restrict__ part) {
  __shared__ double sr[WB_RB * MC];
  const PCItem it = items[blockIdx.x];
  if (!live[it.inst]) return;  // uniform per block
  const BatchMeta P = meta[it.inst];
  woodbury_tpart<MC, 1>(P.Ut, P.ldu, P.s, r + P.off * MC, MC, it.i0, it.i1, it.k0 + threadIdx.x,
                        part + it.part_off + (int64_t)it.chunk * P.s * 16, 16, sr);
}

// T_p[k][c] = sum over chunks (c < M); blockIdx.y = problem
__global__ void batch_t_reduce_kernel(const BatchMeta* __restrict__ meta,
                                      const int* __restrict__ live, int M,
                                      const double* __restrict__ part, double* __restrict__ T) {
  const int p = blockIdx.y;
  if (!live[p]) return;
  const BatchMeta P = meta[p];
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (!P.has_u || e >= P.s * 16 || (int)(e % 16) >= M) return;
  double v = 0.0;
  for (int k = 0; k < P.pc_chunks; ++k) v += part[P.pc_part_off + (int64_t)k * P.s * 16 + e];
  T[P.t_off + e] = v;
}

// Pass 2: item (problem, 64-row block): z = (r - Ut T) / lambda_p, or z = r without Ut
template <int MC>
__global__ __launch_bounds__(256) void batch_z_kernel(const ZItem* __restrict__ items,
                                                      const BatchMeta* __restrict__ meta,
                                                      const int* __restrict__ live,
                                                      const double* __restrict__ T,
                                                      const double* __restrict__ r,
                                                      double* __restrict__ z) {
  __shared__ __attribute__((aligned(16))) float smem[woodbury_z_smem_floats(MC)];
  const ZItem it = items[blockIdx.x];
  if (!live[it.inst]) return;
  const BatchMeta P = meta[it.inst];
  const double* rp = r + P.off * MC;
  double* zp = z + P.off * MC;
  if (P.has_u) {
    woodbury_z<MC>(P.Ut, P.ldu, P.s, T + P.t_off, 16, rp, MC, P.inv_lp, zp, MC, it.i0, P.n, smem);
  } else {
    for (int e = threadIdx.x; e < 64 * MC; e += 256) {
      const int64_t i = it.i0 + e / MC;
      if (i < P.n) zp[i * MC + e % MC] = rp[i * MC + e % MC];
    }
  }
}

hipError_t batch_precond(const BatchMeta* meta, int count, const PCItem* pitems, int npitems,
                         const ZItem* zitems, int nzitems, int64_t smax, const int* live,
                         const double* r, int M, double* part, double* T, double* z,
                         hipStream_t st) {
  switch (M) {
#define KRR_BP(N)                                                                            \
  case N:                                                                                    \
    if (npitems > 0) {                                                                       \
      batch_t_partial_kernel<N><<<npitems, 256, 0, st>>>(pitems, meta, live, r, part);       \
      KRR_LAUNCH_CHECK();                                                                    \
      dim3 g(ceil_div(smax * 16, 256), count);                                               \
      batch_t_reduce_kernel<<<g, 256, 0, st>>>(meta, live, M, part, T);                      \
      KRR_LAUNCH_CHECK();                                                                    \
    }                                                                                        \
    batch_z_kernel<N><<<nzitems, 256, 0, st>>>(zitems, meta, live, T, r, z);                 \
    KRR_LAUNCH_CHECK();                                                                      \
    return hipSuccess;
    KRR_BP(1) KRR_BP(2) KRR_BP(3) KRR_BP(4) KRR_BP(5) KRR_BP(6) KRR_BP(7) KRR_BP(8)
    KRR_BP(9) KRR_BP(10) KRR_BP(11) KRR_BP(12) KRR_BP(13) KRR_BP(14) KRR_BP(15) KRR_BP(16)
#undef KRR_BP
  }
  return hipErrorInvalidValue;
}

// packed <-> per-problem copies (rows < n_p, columns < m_p; padding zero on pack)
__global__ void batch_pack_kernel(const int* __restrict__ row_inst,
                                  const BatchMeta* __restrict__ meta, int64_t nrows, int M,
                                  int mode, double* __restrict__ packed) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrows * M) return;
  const int64_t row = e / M;
  const int c = (int)(e % M);
  const BatchMeta P = meta[row_to_inst(row_inst, row)];
  const int64_t lr = row - P.off;
  const bool in = lr < P.n && c < P.m;
  if (mode == BATCH_PACK_IN) packed[e] = in ? P.ext_in[lr * P.ld_in + c] : 0.0;
  else if (in && mode == BATCH_UNPACK_ADD) P.ext_out[lr * P.ld_out + c] += packed[e];
  else if (in) P.ext_out[lr * P.ld_out + c] = packed[e];
}

hipError_t batch_pack(const int* row_inst, const BatchMeta* meta, int64_t nrows, int M,
                      int mode, double* packed, hipStream_t st) {
  batch_pack_kernel<<<ceil_div(nrows * M, 256), 256, 0, st>>>(row_inst, meta, nrows, M, mode,
                                                              packed);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// ------------------------------------------------------ live work-item compaction
// The product's work queue keeps only the items of problems that still have an active
// column, in the queue's own (cost-sorted) order: pass 1 counts the live items of each chunk
// of BC_CHUNK items, pass 2 gives every chunk its offset (the sum of the counts before it) and
// writes its live item indices in order with a block-wide scan. The product kernel then
// walks `count` entries instead of skipping converged problems' items one by one.
constexpr int BC_CHUNK = 256;
__global__ __launch_bounds__(BC_CHUNK) void batch_count_live_kernel(
    const BatchItem* __restrict__ items, int nitems, const int* __restrict__ live,
    int* __restrict__ chunk_cnt) {
  __shared__ int red[4];
  const int i = blockIdx.x * BC_CHUNK + threadIdx.x;
  const int f = (i < nitems && live[items[i].inst]) ? 1 : 0;
  const int w = wave_sum(f);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) chunk_cnt[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}
__global__ __launch_bounds__(BC_CHUNK) void batch_write_live_kernel(
    const BatchItem* __restrict__ items, int nitems, const int* __restrict__ live,
    const int* __restrict__ chunk_cnt, int* __restrict__ list, int* __restrict__ count) {
  __shared__ int base, wsum[4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  if (tid == 0) {
    int b = 0;
    for (int c = 0; c < (int)blockIdx.x; ++c) b += chunk_cnt[c];
    base = b;
    if (blockIdx.x == gridDim.x - 1) *count = b + chunk_cnt[blockIdx.x];
  }
  const int i = blockIdx.x * BC_CHUNK + tid;
  const int f = (i < nitems && live[items[i].inst]) ? 1 : 0;
  // inclusive scan within the wave, then across the four waves
  int x = f;
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(x, o, 64);
    if (lane >= o) x += y;
  }
  if (lane == 63) wsum[w] = x;
  __syncthreads();
  int pre = 0;
  for (int k = 0; k < w; ++k) pre += wsum[k];
  if (f) list[base + pre + x - 1] = i;
}
hipError_t batch_compact_live(const BatchItem* items, int nitems, const int* live, int* chunk_cnt,
                              int* list, int* count, hipStream_t st) {
  const int nb = (int)ceil_div(nitems, BC_CHUNK);
  if (nb <= 0) return fill_i32(count, 1, 0, st);
  batch_count_live_kernel<<<nb, BC_CHUNK, 0, st>>>(items, nitems, live, chunk_cnt);
  KRR_LAUNCH_CHECK();
  batch_write_live_kernel<<<nb, BC_CHUNK, 0, st>>>(items, nitems, live, chunk_cnt, list, count);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace krr
