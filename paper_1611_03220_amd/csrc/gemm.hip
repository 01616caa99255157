// Dense products of the set-up (random features and preconditioner factor):
//   * gemm_nt_f16x3: C[M x N] = s * sum_k A[i, k] B[j, k] on MFMA from FP16 hi/lo splits
//     (three products), FP32 accumulate within a k split, with epilogues
//       EPI_PART64 : FP64 partial per k split (Gram Z^T Z; summed in fixed order later)
//       EPI_F32    : FP32 store (Ut = Z C^{-T})
//       EPI_COS    : amp * cos(C + b[j]) (random Fourier features, Sec. 2.2)
//   * dgemm: FP64 C = beta C + alpha op(A) op(B) with general strides (Cholesky trailing
//     updates and the triangular inverse).
#include "kernels.hpp"

namespace krr {

constexpr int G_BM = GEMM_TILE, G_BN = GEMM_TILE, G_BK = 32;

// Block: 128 x 128 output tile, 4 waves in 2 x 2, each wave 64 x 64 (4 x 4 MFMA blocks of
// 16 x 16); k steps of 32 (one MFMA k). Operand tiles (hi and lo of A and B, 128 rows x 32
// halves) are double-buffered in LDS; rows are 64 bytes whose four 16-byte pieces are XOR-
// swizzled with (row >> 1) & 3, so the 16 rows x 4 pieces of a fragment read hit distinct
// banks. Global loads for the next step are issued before the MFMAs of the current one.
// Operand rows are padded to a multiple of 128 and k to a multiple of 32 (zero padding).
template <int EPI>
__global__ __launch_bounds__(256, 2) void gemm_nt_f16x3_kernel(
    const _Float16* __restrict__ Ahi, const _Float16* __restrict__ Alo, int64_t lda,
    const _Float16* __restrict__ Bhi, const _Float16* __restrict__ Blo, int64_t ldb, int64_t M,
    int64_t N, int64_t K, int64_t k_per_split, int lower_only, int tri_b,
    const float* __restrict__ qa, const float* __restrict__ qb, double alpha,
    double* __restrict__ out64, int64_t out64_stride, float* __restrict__ out32, int64_t ldc,
    const float* __restrict__ bias, float amp) {
  // XCD-aware order: workgroups go round-robin to the 8 XCDs (linear id mod 8), so the
  // linear ids are remapped to give each XCD one contiguous run of tiles (row-major, the
  // k split outermost); its L2 then serves the operand rows that neighbouring tiles share.
  const int64_t gx = gridDim.x, gy = gridDim.y, total = gx * gy * (int64_t)gridDim.z;
  int64_t lin = blockIdx.x + gx * (blockIdx.y + gy * (int64_t)blockIdx.z);
  if (total % 8 == 0) lin = (lin % 8) * (total / 8) + lin / 8;
  const int64_t bj = lin % gx, bi = (lin / gx) % gy, bz = lin / (gx * gy);
  if (lower_only && bj > bi) return;
  constexpr int TILE = G_BM * G_BK;  // halves per operand tile
  __shared__ __attribute__((aligned(16))) _Float16 smem[2][4][TILE];  // [buf][Ah, Al, Bh, Bl]
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lg = lane >> 4;
  const int wr = w >> 1, wc = w & 1;
  const int64_t row0 = bi * G_BM, col0 = bj * G_BN;
  const int64_t k_begin = bz * k_per_split;
  int64_t k_end = k_begin + k_per_split < K ? k_begin + k_per_split : K;
  if (tri_b) {  // B lower triangular in (j, k): entries with k > j vanish
    const int64_t kmax = round_up(col0 + G_BN, G_BK);
    if (k_end > kmax) k_end = kmax;
  }
  f32x4 acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};

  // loader: 128 rows x 4 pieces = 512 pieces per operand; thread takes rows tid/4, tid/4 + 64
  const int lr0 = tid >> 2, lp = tid & 3;
  const int lr1 = lr0 + 64;
  const int so0 = lr0 * G_BK + ((lp ^ ((lr0 >> 1) & 3)) * 8);
  const int so1 = lr1 * G_BK + ((lp ^ ((lr1 >> 1) & 3)) * 8);
  u32x4 ra[4], rb[4];  // [Ah0, Ah1, Al0, Al1], [Bh0, Bh1, Bl0, Bl1]
  auto gload = [&](int64_t k0) __attribute__((always_inline)) {
    const int64_t a0 = (row0 + lr0) * lda + k0 + lp * 8, a1 = (row0 + lr1) * lda + k0 + lp * 8;
    const int64_t b0 = (col0 + lr0) * ldb + k0 + lp * 8, b1 = (col0 + lr1) * ldb + k0 + lp * 8;
    ra[0] = *reinterpret_cast<const u32x4*>(Ahi + a0);
    ra[1] = *reinterpret_cast<const u32x4*>(Ahi + a1);
    ra[2] = *reinterpret_cast<const u32x4*>(Alo + a0);
    ra[3] = *reinterpret_cast<const u32x4*>(Alo + a1);
    rb[0] = *reinterpret_cast<const u32x4*>(Bhi + b0);
    rb[1] = *reinterpret_cast<const u32x4*>(Bhi + b1);
    rb[2] = *reinterpret_cast<const u32x4*>(Blo + b0);
    rb[3] = *reinterpret_cast<const u32x4*>(Blo + b1);
  };
  auto lstore = [&](int buf) __attribute__((always_inline)) {
    *reinterpret_cast<u32x4*>(&smem[buf][0][so0]) = ra[0];
    *reinterpret_cast<u32x4*>(&smem[buf][0][so1]) = ra[1];
    *reinterpret_cast<u32x4*>(&smem[buf][1][so0]) = ra[2];
    *reinterpret_cast<u32x4*>(&smem[buf][1][so1]) = ra[3];
    *reinterpret_cast<u32x4*>(&smem[buf][2][so0]) = rb[0];
    *reinterpret_cast<u32x4*>(&smem[buf][2][so1]) = rb[1];
    *reinterpret_cast<u32x4*>(&smem[buf][3][so0]) = rb[2];
    *reinterpret_cast<u32x4*>(&smem[buf][3][so1]) = rb[3];
  };
  // fragment piece of row r (lane group lg reads k = 8 lg .. 8 lg + 7)
  auto frag = [&](int buf, int op, int r) __attribute__((always_inline)) {
    return *reinterpret_cast<const half8*>(&smem[buf][op][r * G_BK + ((lg ^ ((r >> 1) & 3)) * 8)]);
  };
  if (k_begin < k_end) {
    gload(k_begin);
    lstore(0);
  }
  wait_vmem_all();  // no load pending at the loop's entry on any path (precise waits inside)
  __syncthreads();
  int buf = 0;
  for (int64_t k0 = k_begin; k0 < k_end; k0 += G_BK) {
    const bool more = k0 + G_BK < k_end;
    if (more) gload(k0 + G_BK);
    half8 bh[4], bl[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int c = 64 * wc + 16 * b + li;
      bh[b] = frag(buf, 2, c);
      bl[b] = frag(buf, 3, c);
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const int r = 64 * wr + 16 * a + li;
      const half8 ah = frag(buf, 0, r), al = frag(buf, 1, r);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[b], acc[a][b], 0, 0, 0);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[b], acc[a][b], 0, 0, 0);
      }
    }
    if (more) lstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  const float sa = split_scale(*qa), sb = split_scale(*qb);
  const double scale = alpha / ((double)sa * (double)sb);
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = row0 + 64 * wr + 16 * a + 4 * lg + r;
        const int64_t j = col0 + 64 * wc + 16 * b + li;
        if (i < M && j < N) {
          const double v = (double)acc[a][b][r] * scale;
          if (EPI == EPI_PART64) out64[bz * out64_stride + i * ldc + j] = v;
          else if (EPI == EPI_F32) out32[i * ldc + j] = (float)v;
          else out32[i * ldc + j] = amp * cosf((float)v + bias[j]);
        }
      }
}

hipError_t gemm_nt_f16x3(const SplitOperand& A, const SplitOperand& B, int64_t M, int64_t N,
                         int64_t K, int nsplit, int epi, int lower_only, int tri_b, double alpha,
                         double* out64, int64_t out64_stride, float* out32, int64_t ldc,
                         const float* bias, float amp, hipStream_t st) {
  if (K % G_BK) return hipErrorInvalidValue;
  const int64_t kps = round_up(ceil_div(K, nsplit), G_BK);
  dim3 grid(ceil_div(N, G_BN), ceil_div(M, G_BM), nsplit);
#define KRR_G(E)                                                                               \
  gemm_nt_f16x3_kernel<E><<<grid, 256, 0, st>>>(A.hi, A.lo, A.ld, B.hi, B.lo, B.ld, M, N, K,   \
                                                kps, lower_only, tri_b, A.amax, B.amax, alpha,  \
                                                out64, out64_stride, out32, ldc, bias, amp)
  if (epi == EPI_PART64) KRR_G(EPI_PART64);
  else if (epi == EPI_F32) KRR_G(EPI_F32);
  else KRR_G(EPI_COS);
#undef KRR_G
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// ------------------------------------------------------------------- FP64 GEMM
// C[i, j] = beta C[i, j] + alpha sum_k A(i, k) B(k, j), A(i, k) = A[i*sai + k*sak],
// B(k, j) = B[k*sbk + j*sbj]; batched over blockIdx.z with element strides bA, bB, bC.
// 64 x 64 tile, k chunks of 64 (one load round trip for the rank-64 Cholesky updates: all
// loads of a chunk are issued before any is used), each thread 4 x 4 outputs. lower_only
// skips tiles that lie strictly above the block diagonal and entries with j > i.
constexpr int D_BK = 64;
// One 64 x 64 output tile (bi, bj) of one product; sA and sB are the block's LDS tiles.
__device__ __forceinline__ void dgemm_tile(int64_t bi, int64_t bj, int64_t M, int64_t N,
                                           int64_t K, double alpha, const double* __restrict__ A,
                                           int64_t sai, int64_t sak,
                                           const double* __restrict__ B, int64_t sbk,
                                           int64_t sbj, double beta, double* __restrict__ C,
                                           int64_t ldc, int lower_only,
                                           double (&sA)[D_BK][64 + 1],
                                           double (&sB)[D_BK][64 + 1]) {
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int64_t row0 = bi * 64, col0 = bj * 64;
  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[r][q] = 0.0;
  constexpr int EPT = 64 * D_BK / 256;  // elements of each operand tile per thread
  // element e of a tile: consecutive threads along the unit-stride index
  auto a_pos = [&](int e, int& rr, int& kk) __attribute__((always_inline)) {
    if (sak == 1) { rr = e / D_BK; kk = e % D_BK; } else { kk = e / 64; rr = e % 64; }
  };
  auto b_pos = [&](int e, int& cc, int& kk) __attribute__((always_inline)) {
    if (sbk == 1) { cc = e / D_BK; kk = e % D_BK; } else { kk = e / 64; cc = e % 64; }
  };
  for (int64_t k0 = 0; k0 < K; k0 += D_BK) {
    // out-of-range elements load a valid element and are zeroed at the LDS store (a select
    // right after each load would wait for it)
    double va[EPT], vb[EPT];
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      int rr, kk, cc, k2;
      a_pos(tid + 256 * u, rr, kk);
      b_pos(tid + 256 * u, cc, k2);
      const int64_t gi = row0 + rr, gk = k0 + kk, gj = col0 + cc, gk2 = k0 + k2;
      va[u] = A[(gi < M && gk < K) ? gi * sai + gk * sak : 0];
      vb[u] = B[(gj < N && gk2 < K) ? gk2 * sbk + gj * sbj : 0];
    }
#pragma unroll
    for (int u = 0; u < EPT; ++u) {
      int rr, kk, cc, k2;
      a_pos(tid + 256 * u, rr, kk);
      b_pos(tid + 256 * u, cc, k2);
      sA[kk][rr] = (row0 + rr < M && k0 + kk < K) ? va[u] : 0.0;
      sB[k2][cc] = (col0 + cc < N && k0 + k2 < K) ? vb[u] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < D_BK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = sA[kk][ty * 4 + r];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = sB[kk][tx + 16 * q];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[r][q] = fma(a[r], b[q], acc[r][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t i = row0 + ty * 4 + r, j = col0 + tx + 16 * q;
      if (i < M && j < N && (!lower_only || j <= i)) {
        const double prev = beta != 0.0 ? C[i * ldc + j] : 0.0;
        C[i * ldc + j] = beta * prev + alpha * acc[r][q];
      }
    }
}

__global__ __launch_bounds__(256) void dgemm_kernel(int64_t M, int64_t N, int64_t K,
                                                    double alpha, const double* __restrict__ A,
                                                    int64_t sai, int64_t sak, int64_t bA,
                                                    const double* __restrict__ B, int64_t sbk,
                                                    int64_t sbj, int64_t bB, double beta,
                                                    double* __restrict__ C, int64_t ldc,
                                                    int64_t bC, int lower_only) {
  const int64_t bi = blockIdx.y, bj = blockIdx.x;
  if (lower_only && bj > bi) return;
  __shared__ double sA[D_BK][64 + 1];
  __shared__ double sB[D_BK][64 + 1];
  dgemm_tile(bi, bj, M, N, K, alpha, A + (int64_t)blockIdx.z * bA, sai, sak,
             B + (int64_t)blockIdx.z * bB, sbk, sbj, beta, C + (int64_t)blockIdx.z * bC, ldc,
             lower_only, sA, sB);
}

// Products of different shapes in one launch: blockIdx.z selects the product, blocks
// outside its tile range return.
__global__ __launch_bounds__(256) void dgemm_grouped_kernel(const DgemmProblem* __restrict__ probs) {
  const DgemmProblem p = probs[blockIdx.z];
  const int64_t bi = blockIdx.y, bj = blockIdx.x;
  if (bi * 64 >= p.M || bj * 64 >= p.N || (p.lower_only && bj > bi)) return;
  __shared__ double sA[D_BK][64 + 1];
  __shared__ double sB[D_BK][64 + 1];
  dgemm_tile(bi, bj, p.M, p.N, p.K, p.alpha, p.A, p.sai, p.sak, p.B, p.sbk, p.sbj, p.beta, p.C,
             p.ldc, p.lower_only, sA, sB);
}

hipError_t dgemm(int64_t M, int64_t N, int64_t K, double alpha, const double* A, int64_t sai,
                 int64_t sak, int64_t bA, const double* B, int64_t sbk, int64_t sbj, int64_t bB,
                 double beta, double* C, int64_t ldc, int64_t bC, int batch, int lower_only,
                 hipStream_t st) {
  if (M <= 0 || N <= 0 || batch <= 0) return hipSuccess;
  dim3 grid(ceil_div(N, 64), ceil_div(M, 64), batch);
  dgemm_kernel<<<grid, 256, 0, st>>>(M, N, K, alpha, A, sai, sak, bA, B, sbk, sbj, bB, beta, C,
                                     ldc, bC, lower_only);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t dgemm_grouped(const DgemmProblem* probs, int count, int64_t max_m, int64_t max_n,
                         hipStream_t st) {
  if (count <= 0 || max_m <= 0 || max_n <= 0) return hipSuccess;
  dim3 grid(ceil_div(max_n, 64), ceil_div(max_m, 64), count);
  dgemm_grouped_kernel<<<grid, 256, 0, st>>>(probs);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace krr
