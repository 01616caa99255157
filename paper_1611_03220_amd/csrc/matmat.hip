// Matrix-free Gaussian kernel products: OUT = K(X1, X2) V.
//
// Mixed kernel (F16X3 / BF16X3): each 64-thread wave owns 16 output rows i; the block
// (4 waves, 64 rows) sweeps a range of 64-column tiles j. Per 16x16 (i, j) block, three
// 16x16x32 MFMAs per 32-wide k step form <a_i, b_j> = q^2 log2 k_ij from hi/lo splits
// (lo*hi, hi*lo, hi*hi). The epilogue is VALU: log2 k = min(S / q^2, 0), k = exp2(log2 k)
// (times -log2 k / (c sigma^3) for dk/dsigma), then k * V[j, c] accumulated in FP32 over
// FLUSH tiles and added into FP64 accumulators (cross-tile sums in FP64). The row operands
// a_i live in registers for the whole sweep; b_j tiles and V rows are double-buffered
// through LDS.
//
// MFMA 16x16x32 lane layout (gfx950): A operand lane l holds A[l%16][8(l/16)+t], B operand
// B[8(l/16)+t][l%16], result C[4(l/16)+r][l%16], t = 0..7, r = 0..3.
#include "kernels.hpp"

namespace krr {

constexpr int MM_BM = 64;   // rows per block (4 waves x 16)
constexpr int MM_BN = 64;   // columns per tile
constexpr int MM_FLUSH = 4; // tiles between FP32 -> FP64 flushes (16 terms per lane)
typedef unsigned int u32x4v __attribute__((ext_vector_type(4)));

template <typename T, int KS, int MC, bool DERIV>
__global__ __launch_bounds__(256) void matmat_mixed_kernel(
    const T* __restrict__ Ahi, const T* __restrict__ Alo, const T* __restrict__ Bhi,
    const T* __restrict__ Blo, const float* __restrict__ Vf, int64_t ldvf, int64_t n1,
    int64_t n2, int c0, const float* __restrict__ qinv2_ptr, float dscale,
    double* __restrict__ part, int64_t ldp, int64_t part_stride, int tiles_per_split) {
  typedef typename Elem<T>::vec8 vec8;
  constexpr int KP = KS * 32;
  constexpr int LDS_K = KP + 8;  // padded row (halves) to spread LDS banks
  constexpr int CHUNKS = MM_BN * KP / 8;  // 16-byte chunks per operand tile
  constexpr int CPT = (CHUNKS + 255) / 256;
  constexpr int VEL = MM_BN * MC;  // V floats per tile
  constexpr int VPT = (VEL + 255) / 256;

  __shared__ __attribute__((aligned(16))) T sBh[2][MM_BN * LDS_K];
  __shared__ __attribute__((aligned(16))) T sBl[2][MM_BN * LDS_K];
  __shared__ float sV[2][MM_BN * MC];

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * MM_BM + 16 * w;
  const int64_t ntiles = ceil_div(n2, MM_BN);
  const int64_t t_begin = (int64_t)blockIdx.y * tiles_per_split;
  const int64_t t_end = t_begin + tiles_per_split < ntiles ? t_begin + tiles_per_split : ntiles;
  const float qinv2 = *qinv2_ptr;

  // row operands in registers
  vec8 ah[KS], al[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int64_t off = (i0 + li) * KP + ks * 32 + 8 * lg;
    ah[ks] = *reinterpret_cast<const vec8*>(Ahi + off);
    al[ks] = *reinterpret_cast<const vec8*>(Alo + off);
  }

  float acc[4][MC];
  double acc64[4][MC];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < MC; ++c) { acc[r][c] = 0.0f; acc64[r][c] = 0.0; }

  u32x4v rh[CPT], rl[CPT];
  float rv[VPT];
  auto gload = [&](int64_t t) {
    const int64_t j0 = t * MM_BN;
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int ch = tid + 256 * u;
      if (ch < CHUNKS) {
        const int row = ch / (KP / 8), col8 = ch % (KP / 8);
        const int64_t off = (j0 + row) * KP + col8 * 8;
        rh[u] = *reinterpret_cast<const u32x4v*>(Bhi + off);
        rl[u] = *reinterpret_cast<const u32x4v*>(Blo + off);
      }
    }
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int e = tid + 256 * u;
      if (e < VEL) {
        const int row = e / MC, c = e % MC;
        rv[u] = (j0 + row < n2) ? Vf[(j0 + row) * ldvf + c0 + c] : 0.0f;
      }
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
      const int ch = tid + 256 * u;
      if (ch < CHUNKS) {
        const int row = ch / (KP / 8), col8 = ch % (KP / 8);
        *reinterpret_cast<u32x4v*>(&sBh[buf][row * LDS_K + col8 * 8]) = rh[u];
        *reinterpret_cast<u32x4v*>(&sBl[buf][row * LDS_K + col8 * 8]) = rl[u];
      }
    }
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int e = tid + 256 * u;
      if (e < VEL) sV[buf][e] = rv[u];
    }
  };

  if (t_begin < t_end) {
    gload(t_begin);
    lstore(0);
  }
  __syncthreads();
  int since_flush = 0;
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int buf = (int)((t - t_begin) & 1);
    if (t + 1 < t_end) gload(t + 1);
#pragma unroll
    for (int jb = 0; jb < MM_BN / 16; ++jb) {
      f32x4 S = {0.0f, 0.0f, 0.0f, 0.0f};
      const T* bh = &sBh[buf][(16 * jb + li) * LDS_K + 8 * lg];
      const T* bl = &sBl[buf][(16 * jb + li) * LDS_K + 8 * lg];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        const vec8 bhv = *reinterpret_cast<const vec8*>(bh + ks * 32);
        const vec8 blv = *reinterpret_cast<const vec8*>(bl + ks * 32);
        S = Elem<T>::mfma(al[ks], bhv, S);
        S = Elem<T>::mfma(ah[ks], blv, S);
        S = Elem<T>::mfma(ah[ks], bhv, S);
      }
      float v[MC];
#pragma unroll
      for (int c = 0; c < MC; ++c) v[c] = sV[buf][(16 * jb + li) * MC + c];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float l2 = fminf(S[r] * qinv2, 0.0f);
        float p = __builtin_amdgcn_exp2f(l2);
        if (DERIV) p = p * (-l2) * dscale;
#pragma unroll
        for (int c = 0; c < MC; ++c) acc[r][c] = fmaf(p, v[c], acc[r][c]);
      }
    }
    if (++since_flush == MM_FLUSH) {
      since_flush = 0;
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < MC; ++c) { acc64[r][c] += (double)acc[r][c]; acc[r][c] = 0.0f; }
    }
    if (t + 1 < t_end) lstore(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      double s = acc64[r][c] + (double)acc[r][c];
      // lanes sharing lg hold the same rows and different j: reduce over lane bits 0..3
      for (int o = 1; o < 16; o <<= 1) s += __shfl_xor(s, o, 64);
      acc64[r][c] = s;
    }
  double* pout = part + (int64_t)blockIdx.y * part_stride;
#pragma unroll
  for (int c = 0; c < MC; ++c) {
    if (li == c) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + 4 * lg + r;
        if (i < n1) pout[i * ldp + c0 + c] = acc64[r][c];
      }
    }
  }
}

template <typename T, int KS, int MC>
static hipError_t launch_mixed_mc(const MixedPoints<T>& A, const MixedPoints<T>& B,
                                  const float* Vf, int64_t ldvf, int c0, bool deriv, float dscale,
                                  double* part, int64_t ldp, int64_t part_stride, int nsplit,
                                  int tiles_per_split, hipStream_t st) {
  dim3 grid(ceil_div(A.n, MM_BM), nsplit);
  if (deriv)
    matmat_mixed_kernel<T, KS, MC, true><<<grid, 256, 0, st>>>(
        A.hi, A.lo, B.hi, B.lo, Vf, ldvf, A.n, B.n, c0, A.qinv2, dscale, part, ldp, part_stride,
        tiles_per_split);
  else
    matmat_mixed_kernel<T, KS, MC, false><<<grid, 256, 0, st>>>(
        A.hi, A.lo, B.hi, B.lo, Vf, ldvf, A.n, B.n, c0, A.qinv2, dscale, part, ldp, part_stride,
        tiles_per_split);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

template <typename T, int KS>
static hipError_t launch_mixed_ks(const MixedPoints<T>& A, const MixedPoints<T>& B,
                                  const float* Vf, int64_t ldvf, int64_t m, bool deriv,
                                  float dscale, double* part, int64_t ldp, int64_t part_stride,
                                  int nsplit, int tiles_per_split, hipStream_t st) {
  for (int64_t c0 = 0; c0 < m; c0 += 8) {
    const int mc = (int)std::min<int64_t>(8, m - c0);
    hipError_t e;
    switch (mc) {
#define KRR_MC(N)                                                                              \
  case N:                                                                                      \
    e = launch_mixed_mc<T, KS, N>(A, B, Vf, ldvf, (int)c0, deriv, dscale, part, ldp,           \
                                  part_stride, nsplit, tiles_per_split, st);                   \
    break;
      KRR_MC(1) KRR_MC(2) KRR_MC(3) KRR_MC(4) KRR_MC(5) KRR_MC(6) KRR_MC(7) KRR_MC(8)
#undef KRR_MC
      default: return hipErrorInvalidValue;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t matmat_mixed(const MixedPoints<T>& A, const MixedPoints<T>& B, const float* Vf,
                        int64_t ldvf, int64_t m, bool deriv, float dscale, double* part,
                        int64_t ldp, int64_t part_stride, int nsplit, hipStream_t st) {
  if (A.Kp != B.Kp) return hipErrorInvalidValue;
  const int64_t ntiles = ceil_div(B.n, MM_BN);
  const int tps = (int)ceil_div(ntiles, nsplit);
  switch (A.Kp / 32) {
#define KRR_KS(N)                                                                             \
  case N:                                                                                     \
    return launch_mixed_ks<T, N>(A, B, Vf, ldvf, m, deriv, dscale, part, ldp, part_stride,    \
                                 nsplit, tps, st);
    KRR_KS(1) KRR_KS(2) KRR_KS(3) KRR_KS(4) KRR_KS(5) KRR_KS(6) KRR_KS(7) KRR_KS(8)
#undef KRR_KS
    default: return hipErrorInvalidValue;
  }
}
template hipError_t matmat_mixed<_Float16>(const MixedPoints<_Float16>&,
                                           const MixedPoints<_Float16>&, const float*, int64_t,
                                           int64_t, bool, float, double*, int64_t, int64_t, int,
                                           hipStream_t);
template hipError_t matmat_mixed<__bf16>(const MixedPoints<__bf16>&, const MixedPoints<__bf16>&,
                                         const float*, int64_t, int64_t, bool, float, double*,
                                         int64_t, int64_t, int, hipStream_t);

// ----------------------------------------------- F16X3 kernel with MFMA accumulation
// Same product as above, with the accumulation over j on MFMA too. Each wave owns 32 rows
// (two 16-row blocks) and reads 32-column halves ("j-pairs") of the 64-column tile:
//   S^T[j][i] = <b_j, a_i> on MFMA with the column operand b_j (from LDS) as A and the
//   row operand a_i (registers) as B, so lane l holds S^T[4(l/16)+r][l%16]: row i = l%16
//   and four consecutive j -- the A-operand layout of the next product once two 16-column
//   blocks are concatenated along k;
//   P = exp2(S / q^2) = k, split into FP16 hi + lo (both rounded to nearest: the error is
//   unbiased), multiplied on MFMA with the FP16 hi/lo split of V^T (three products; two
//   when m <= 8 and both halves of V^T share one operand), FP32
//   accumulate, FP64 sums every MM2_FLUSH tiles.
// The distance products of the second j-pair are issued before the first j-pair's
// epilogue so one wave's MFMA and VALU work overlap. LDS tiles are XOR-swizzled (no
// padding, no bank conflicts on the fragment reads). When q = 1 (operands already in
// FP16's comfortable range) the kernel skips the 1/q^2 scaling: a uniform branch at entry
// selects that instantiation of the body.
// Kernel value of the fused epilogue from l = <a_i, b_j> / q^2 of the augmented rows:
//   KV_GAUSS   l = log2 k(x_i, x_j) (Gaussian rows):       k = 2^l;
//   KV_DSIGMA  same rows:                                   dk/dsigma = k (-l) dscale;
//   KV_POLY    l = (gamma <x_i, x_j> + c) / t_max (polynomial rows, |l| <= 1):
//               k / t_max^deg = l^deg (the output is multiplied back by pmul = t_max^deg).
template <int EPI>
__device__ __forceinline__ float epi_value(float l, float dscale, int deg) {
  if (EPI == KV_POLY) {
    // the degree is uniform across the launch: the common degrees take straight-line code
    if (deg == 3) return l * l * l;
    if (deg == 2) return l * l;
    float p = l;
    for (int e = 1; e < deg; ++e) p *= l;
    return p;
  }
  float p = __builtin_amdgcn_exp2f(l);
  if (EPI == KV_DSIGMA) p *= -l * dscale;
  return p;
}
// Degree and output multiplier of the polynomial epilogue from the kernel parameters that
// follow 1/q^2 on the device: kp[1] = log2 of the multiplier, kp[2] = degree.
template <int EPI>
__device__ __forceinline__ void epi_params(const float* kp, int& deg, double& pmul) {
  deg = EPI == KV_POLY ? (int)kp[2] : 1;
  pmul = EPI == KV_POLY ? ldexp(1.0, (int)kp[1]) : 1.0;
}

constexpr int MM2_BM = 128;   // rows per block (4 waves x 32)
constexpr int MM2_FLUSH = 2;  // tiles between FP32 -> FP64 flushes
typedef _Float16 half4 __attribute__((ext_vector_type(4)));
typedef _Float16 half2v __attribute__((ext_vector_type(2)));
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// Low parts of a split pair: (rn16(pa - h.x), rn16(pb - h.y)), each one mixed-precision FMA
// rounding straight to FP16 into its half of the result (pa - h.x is exact in FP32, so this
// equals rounding the FP32 difference).
__device__ inline half2v split_lo2(half2v h, float pa, float pb) {
  half2v r;
  asm("v_fma_mixlo_f16 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]\n\t"
      "v_fma_mixhi_f16 %0, %1, -1.0, %3 op_sel:[1,0,0] op_sel_hi:[1,0,0]"
      : "=&v"(r)
      : "v"(h), "v"(pa), "v"(pb));
  return r;
}

// LDS position (halves) of V^T[c][j] in a 64-column tile, j a multiple of 4. Within each
// 32-column group, j = 16 b + 4 g + r sits at 8 g + 4 b + r: the eight values lane group g
// feeds to the P V MFMA (the k order of the P fragment) form one 16-byte piece. The eight
// pieces of row c are XOR-swizzled with (c >> 1) & 7, so the 16 rows of a fragment read
// spread over all banks.
// Rows of TN = 128 columns have 16 pieces, swizzled with c & 15 instead.
template <int TN = MM_BN>
__device__ inline int vswz(int c) {
  return TN == 64 ? ((c >> 1) & 7) : (c & 15);
}
template <int TN = MM_BN>
__device__ inline int vpos(int c, int j) {
  const int J = j & 31;
  const int p = (j & ~31) + 8 * ((J & 15) >> 2) + 4 * (J >> 4);
  return c * TN + (((p >> 3) ^ vswz<TN>(c)) << 3) + (p & 7);
}
// the piece lane group g reads for 32-column group jp of row c
template <int TN = MM_BN>
__device__ inline int vfrag(int c, int jp, int g) {
  return c * TN + (((4 * jp + g) ^ vswz<TN>(c)) << 3);
}

// Packed right-hand sides (m <= 8): the 16 columns of the P V product hold P V_hi in
// columns 0..7 and P V_lo in columns 8..15 (P's hi and lo parts both multiply the one
// operand: two MFMAs instead of three, and the lo x lo term is included); lane li < 8 adds
// lane li + 8 of its 16-lane row to finish column li.
template <int NCT>
__device__ inline void pack_combine(double (&acc64)[2][NCT][4]) {
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc64[ib][0][r] += __shfl_down(acc64[ib][0][r], 8, 16);
}

template <int KS, int NCT, bool PACK, bool NE = false>
struct PVSmem {
  static constexpr int KP = KS * 32;
  _Float16 Bh[2][MM_BN * KP];
  _Float16 Bl[2][MM_BN * KP];
  _Float16 Vh[2][NCT * 16 * MM_BN];
  _Float16 Vl[2][PACK ? 8 : NCT * 16 * MM_BN];  // unused with packed V^T
  float Nb[2][NE ? MM_BN : 4];                  // norm terms of the column tile
};

// NE (norms in the epilogue): the operands hold only the scaled coordinates (Kp >= d
// instead of d + 2) and the exponent is completed in FP32 as S + (nA_i + nB_j), with the
// row terms in registers and the column terms staged with their tile.
template <int KS, int NCT, bool UNIT, int EPI, bool PACK, bool NE = false>
__device__ __forceinline__ void f16pv_body(
    PVSmem<KS, NCT, PACK, NE>& sm, const _Float16* __restrict__ Ahi,
    const _Float16* __restrict__ Alo, const _Float16* __restrict__ Bhi,
    const _Float16* __restrict__ Blo, const _Float16* __restrict__ Vth,
    const _Float16* __restrict__ Vtl, const float* __restrict__ vscale, int64_t ldvt, int64_t n1,
    int64_t n2, int64_t m, float qinv2, float dscale, int deg, double pmul,
    double* __restrict__ part, int64_t ldp, int64_t part_stride, int tiles_per_split, int64_t rb,
    int64_t split, const float* __restrict__ nA = nullptr, const float* __restrict__ nB = nullptr) {
  constexpr int KP = KS * 32;
  constexpr int CPR = KP / 8;                 // 16-byte chunks per B row
  constexpr int SWZ = (KS == 1 || KS == 3) ? 3 : 7;
  constexpr int BCH = MM_BN * CPR;
  constexpr int BCPT = (BCH + 255) / 256;
  constexpr int VR = NCT * 16;
  constexpr int VCH = VR * MM_BN / 8;
  constexpr int VCPT = (VCH + 255) / 256;

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t i0 = rb * MM2_BM + 32 * w;
  const int64_t ntiles = ceil_div(n2, MM_BN);
  const int64_t t_begin = split * tiles_per_split;
  const int64_t t_end = t_begin + tiles_per_split < ntiles ? t_begin + tiles_per_split : ntiles;

  half8 ah[2][KS], al[2][KS];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int64_t off = (i0 + 16 * ib + li) * KP + ks * 32 + 8 * lg;
      ah[ib][ks] = *reinterpret_cast<const half8*>(Ahi + off);
      al[ib][ks] = *reinterpret_cast<const half8*>(Alo + off);
    }

  float na[2] = {0.0f, 0.0f};  // NE: row terms (rows are padded, so always in range)
  if constexpr (NE) {
    na[0] = nA[i0 + li];
    na[1] = nA[i0 + 16 + li];
  }

  f32x4 acc[2][NCT];
  double acc64[2][NCT][4];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      acc[ib][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[ib][ct][r] = 0.0;
    }

  // per-thread global sources (advance by one tile per step) and LDS destinations.
  // B tiles have 8 KP chunks of 16 bytes (a multiple of 256: every thread loads BCPT);
  // V^T tiles have 128 NCT chunks (threads below VCH load one each).
  static_assert(BCH % 256 == 0 && VCPT == 1, "tile shape");
  const _Float16* gbh = Bhi + (t_begin * MM_BN) * KP;
  const _Float16* gbl = Blo + (t_begin * MM_BN) * KP;
  static_assert(BCPT <= 4, "at most four B chunks per thread");
  int gbo[4] = {0, 0, 0, 0}, sbo[4] = {0, 0, 0, 0};
  // constant indices only (keeps the per-thread arrays in registers)
#define KRR_PV_INIT(u)                                                     \
  if (u < BCPT) {                                                          \
    const int ch = tid + 256 * u;                                          \
    const int row = ch / CPR, col = ch % CPR;                              \
    gbo[u] = row * KP + col * 8;                                           \
    sbo[u] = row * KP + ((col ^ (row & SWZ)) * 8);                         \
  }
  KRR_PV_INIT(0) KRR_PV_INIT(1) KRR_PV_INIT(2) KRR_PV_INIT(3)
#undef KRR_PV_INIT
  static_assert(!PACK || NCT == 1, "packed right-hand sides use one 16-row operand");
  const bool vload = tid < VCH;
  const int vch = vload ? tid : 0;
  const int vc = vch / (MM_BN / 8), vj8 = vch % (MM_BN / 8);
  const _Float16* gvh = Vth + (int64_t)vc * ldvt + t_begin * MM_BN + vj8 * 8;
  const _Float16* gvl = Vtl + (int64_t)vc * ldvt + t_begin * MM_BN + vj8 * 8;
  // 8-byte units of a V^T row are swizzled by the row index (16 units per row)
  const int svo0 = vpos(vc, 8 * vj8);
  const int svo1 = vpos(vc, 8 * vj8 + 4);
  // prefetch registers as native vectors in named variables (an array of HIP's uint4
  // struct is left in scratch memory by the compiler)
  u32x4 rbh0 = {}, rbh1 = {}, rbh2 = {}, rbh3 = {}, rbl0 = {}, rbl1 = {}, rbl2 = {}, rbl3 = {};
  u32x4 rvh = {}, rvl = {};
  // NE: the tile's 64 column terms, one 16-byte piece for each of threads 0..15
  u32x4 rnb = {};
  const bool nload = NE && tid < MM_BN / 4;
  int64_t nbo = t_begin * MM_BN + 4 * (tid & (MM_BN / 4 - 1));
#define KRR_PV_LD(u)                                                       \
  if (u < BCPT) {                                                          \
    rbh##u = *reinterpret_cast<const u32x4*>(gbh + gbo[u]);                \
    rbl##u = *reinterpret_cast<const u32x4*>(gbl + gbo[u]);                \
  }
#define KRR_PV_ST(u, b)                                                    \
  if (u < BCPT) {                                                          \
    *reinterpret_cast<u32x4*>(&sm.Bh[b][sbo[u]]) = rbh##u;                 \
    *reinterpret_cast<u32x4*>(&sm.Bl[b][sbo[u]]) = rbl##u;                 \
  }
  // distance products of j-pair jp (tile columns 32 jp .. 32 jp + 31)
  auto dist = [&](int buf, int jp, f32x4 (&S)[2][2]) __attribute__((always_inline)) {
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      half8 bh[2], bl[2];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        const int row = 32 * jp + 16 * jb + li;
        const int o = row * KP + (((4 * ks + lg) ^ (row & SWZ)) * 8);
        bh[jb] = *reinterpret_cast<const half8*>(&sm.Bh[buf][o]);
        bl[jb] = *reinterpret_cast<const half8*>(&sm.Bl[buf][o]);
      }
      // four independent accumulation chains, small terms first
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
          const f32x4 c0 = ks == 0 ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : S[jb][ib];
          S[jb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bl[jb], ah[ib][ks], c0, 0, 0, 0);
        }
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
          S[jb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bh[jb], al[ib][ks], S[jb][ib], 0, 0, 0);
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
          S[jb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bh[jb], ah[ib][ks], S[jb][ib], 0, 0, 0);
    }
  };
  // exp2, split and accumulate j-pair jp on MFMA
  auto epi = [&](int buf, int jp, const f32x4 (&S)[2][2]) __attribute__((always_inline)) {
    half8 vh[NCT], vl[NCT];
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int u = vfrag(16 * ct + li, jp, lg);
      vh[ct] = *reinterpret_cast<const half8*>(&sm.Vh[buf][u]);
      if (!PACK) vl[ct] = *reinterpret_cast<const half8*>(&sm.Vl[buf][u]);
    }
    f32x4 nb[2] = {f32x4{0.0f, 0.0f, 0.0f, 0.0f}, f32x4{0.0f, 0.0f, 0.0f, 0.0f}};
    if constexpr (NE) {
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
        nb[jb] = *reinterpret_cast<const f32x4*>(&sm.Nb[buf][32 * jp + 16 * jb + 4 * lg]);
    }
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) {
      half8 ph, pl;
#pragma unroll
      for (int jb = 0; jb < 2; ++jb)
#pragma unroll
        for (int r = 0; r < 4; r += 2) {
          float l2a = S[jb][ib][r], l2b = S[jb][ib][r + 1];
          if constexpr (NE) {
            l2a += na[ib] + nb[jb][r];
            l2b += na[ib] + nb[jb][r + 1];
          }
          if (!UNIT) { l2a *= qinv2; l2b *= qinv2; }
          const float pa = epi_value<EPI>(l2a, dscale, deg);
          const float pb = epi_value<EPI>(l2b, dscale, deg);
          // round-to-nearest split: |(hi + lo) - p| <= 2^-22 |p| (2^-25 absolute below the
          // FP16 normal range), unbiased
          const half2v h = half2v{(_Float16)pa, (_Float16)pb};
          const half2v l = split_lo2(h, pa, pb);
          ph[4 * jb + r] = h[0];
          ph[4 * jb + r + 1] = h[1];
          pl[4 * jb + r] = l[0];
          pl[4 * jb + r + 1] = l[1];
        }
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        acc[ib][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(pl, vh[ct], acc[ib][ct], 0, 0, 0);
        if (!PACK)
          acc[ib][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ph, vl[ct], acc[ib][ct], 0, 0, 0);
        acc[ib][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ph, vh[ct], acc[ib][ct], 0, 0, 0);
      }
    }
  };

  if (t_begin < t_end) {
    KRR_PV_LD(0) KRR_PV_LD(1) KRR_PV_LD(2) KRR_PV_LD(3)
    gbh += MM_BN * KP;
    gbl += MM_BN * KP;
    if (vload) {
      rvh = *reinterpret_cast<const u32x4*>(gvh);
      if (!PACK) rvl = *reinterpret_cast<const u32x4*>(gvl);
    }
    gvh += MM_BN;
    gvl += MM_BN;
    if (nload) rnb = *reinterpret_cast<const u32x4*>(nB + nbo);
    nbo += MM_BN;
    KRR_PV_ST(0, 0) KRR_PV_ST(1, 0) KRR_PV_ST(2, 0) KRR_PV_ST(3, 0)
    if (nload) *reinterpret_cast<u32x4*>(&sm.Nb[0][4 * tid]) = rnb;
    if (vload) {
      *reinterpret_cast<u32x2*>(&sm.Vh[0][svo0]) = u32x2{rvh.x, rvh.y};
      *reinterpret_cast<u32x2*>(&sm.Vh[0][svo1]) = u32x2{rvh.z, rvh.w};
      if (!PACK) {
        *reinterpret_cast<u32x2*>(&sm.Vl[0][svo0]) = u32x2{rvl.x, rvl.y};
        *reinterpret_cast<u32x2*>(&sm.Vl[0][svo1]) = u32x2{rvl.z, rvl.w};
      }
    }
  }
  // Every global load issued so far (the row operand above all) completes here, on every
  // path: otherwise the loop inherits them as pending, and the compiler's wait counts
  // inside the loop become conservative enough to stall the distance MFMAs on the next
  // tile's prefetch.
  wait_vmem_all();
  __syncthreads();
  int since_flush = 0;
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int buf = (int)((t - t_begin) & 1);
    const bool more = t + 1 < t_end;
    if (more) {
    KRR_PV_LD(0) KRR_PV_LD(1) KRR_PV_LD(2) KRR_PV_LD(3)
    gbh += MM_BN * KP;
    gbl += MM_BN * KP;
    if (vload) {
      rvh = *reinterpret_cast<const u32x4*>(gvh);
      if (!PACK) rvl = *reinterpret_cast<const u32x4*>(gvl);
    }
    gvh += MM_BN;
    gvl += MM_BN;
    if (nload) rnb = *reinterpret_cast<const u32x4*>(nB + nbo);
    nbo += MM_BN;
    }
    f32x4 S0[2][2];
    // raised wave priority while issuing the distance MFMAs lets the waves of a SIMD
    // alternate between MFMA-heavy and VALU-heavy phases
#pragma unroll
    for (int jp = 0; jp < 2; ++jp) {
      __builtin_amdgcn_s_setprio(1);
      dist(buf, jp, S0);
      __builtin_amdgcn_s_setprio(0);
      epi(buf, jp, S0);
    }
    if (++since_flush == MM2_FLUSH || t + 1 == t_end) {
      since_flush = 0;
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[ib][ct][r] += (double)acc[ib][ct][r];
          acc[ib][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
        }
    }
    if (more) {
    KRR_PV_ST(0, buf ^ 1) KRR_PV_ST(1, buf ^ 1) KRR_PV_ST(2, buf ^ 1) KRR_PV_ST(3, buf ^ 1)
    if (nload) *reinterpret_cast<u32x4*>(&sm.Nb[buf ^ 1][4 * tid]) = rnb;
    if (vload) {
      *reinterpret_cast<u32x2*>(&sm.Vh[buf ^ 1][svo0]) = u32x2{rvh.x, rvh.y};
      *reinterpret_cast<u32x2*>(&sm.Vh[buf ^ 1][svo1]) = u32x2{rvh.z, rvh.w};
      if (!PACK) {
        *reinterpret_cast<u32x2*>(&sm.Vl[buf ^ 1][svo0]) = u32x2{rvl.x, rvl.y};
        *reinterpret_cast<u32x2*>(&sm.Vl[buf ^ 1][svo1]) = u32x2{rvl.z, rvl.w};
      }
    }
    }
    __syncthreads();
  }
#undef KRR_PV_LD
#undef KRR_PV_ST
  // lane holds OUT[i0 + 16 ib + 4 lg + r][16 ct + li]
  if (PACK) pack_combine<NCT>(acc64);
  double* pout = part + split * part_stride;
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const int64_t c = 16 * ct + li;
    if (c < m && (!PACK || li < 8)) {
      const double vs = (double)vscale[c] * pmul;
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t i = i0 + 16 * ib + 4 * lg + r;
          if (i < n1) pout[i * ldp + c] = acc64[ib][ct][r] * vs;
        }
    }
  }
}

template <int KS, int NCT, int EPI, bool PACK, bool NE = false>
__global__ __launch_bounds__(256, (NCT == 1 && KS <= 2) ? (NE ? 3 : 4) : 2) void matmat_f16pv_kernel(
    const _Float16* __restrict__ Ahi, const _Float16* __restrict__ Alo,
    const _Float16* __restrict__ Bhi, const _Float16* __restrict__ Blo,
    const _Float16* __restrict__ Vth, const _Float16* __restrict__ Vtl,
    const float* __restrict__ vscale, int64_t ldvt, int64_t n1, int64_t n2, int64_t m,
    const float* __restrict__ qinv2_ptr, float dscale, double* __restrict__ part, int64_t ldp,
    int64_t part_stride, int tiles_per_split, const float* __restrict__ nA,
    const float* __restrict__ nB) {
  __shared__ __attribute__((aligned(16))) PVSmem<KS, NCT, PACK, NE> sm;
  const float qinv2 = qinv2_ptr[0];
  int deg;
  double pmul;
  epi_params<EPI>(qinv2_ptr, deg, pmul);
  if (qinv2 == 1.0f)
    f16pv_body<KS, NCT, true, EPI, PACK, NE>(sm, Ahi, Alo, Bhi, Blo, Vth, Vtl, vscale, ldvt, n1,
                                             n2, m, qinv2, dscale, deg, pmul, part, ldp,
                                             part_stride, tiles_per_split, blockIdx.x,
                                             blockIdx.y, nA, nB);
  else
    f16pv_body<KS, NCT, false, EPI, PACK, NE>(sm, Ahi, Alo, Bhi, Blo, Vth, Vtl, vscale, ldvt, n1,
                                              n2, m, qinv2, dscale, deg, pmul, part, ldp,
                                              part_stride, tiles_per_split, blockIdx.x,
                                              blockIdx.y, nA, nB);
}

// Large-d variant: the row operands no longer fit in registers, so both operands stream
// through LDS in 32-wide k chunks. Block: 128 rows (4 waves x 32) against column tiles of
// TN = 16 NJB columns; per tile, KC = Kp/32 chunk steps accumulate S^T for the wave's
// NJB x 2 blocks of 16 x 16, then the same epilogue as above (exp2, FP16 hi/lo split, MFMA
// accumulation against V^T). Wider tiles re-stream the row operand less often: its chunks
// are read once per column tile. Chunk rows are 64 bytes whose 16-byte pieces are
// XOR-swizzled with (row >> 1) & 3 so fragment reads are conflict-free.
//
// Symmetric mode (SYM, the square product K(X, X) V with TN = 128): K is symmetric, so
// only the tile pairs (I, J) with J >= I of the 128-row blocks are formed. A block owns a
// pair of row blocks (p, nrb - 1 - p), whose two tile lists together hold nrb + 1 tiles,
// and takes one of nsplit equal parts of their concatenation. The row side P_IJ V_J is
// accumulated as above; an off-diagonal pair also yields the column side P_IJ^T V_I for the
// rows of J: P is transposed per 16 x 16 block by an MFMA against a 0/1 selection matrix
// (exact: FP16 values times one), multiplied by the register-resident V_I^T on MFMA, the
// four waves' partial sums (over their 32 rows of I) are added through the LDS buffer of
// the stage not in use, and the result goes to the column-side accumulator as 64-bit
// fixed-point atomic adds (exact, so the total does not depend on the order of the adds).
//
// WM row waves per block (4, or 8 for the symmetric kernel: 256-row blocks, one block per CU,
// a quarter fewer operand bytes per MFMA flop than 128-row blocks); the symmetric kernel's
// partial sums of waves 6 and 7 need an extra 16 KB LDS area beyond the free stage.
constexpr int BD_BM = 128;
template <int NCT, int NJB, int WM = 4>
constexpr int bigd_smem_halves() {
  return 2 * 2 * (32 * WM) * 32 + 2 * 2 * (16 * NJB) * 32 + 2 * 2 * NCT * 16 * (16 * NJB) +
         (WM == 8 ? 2 * (16 * NJB) * 16 * 2 : 0);
}
template <int NCT, bool UNIT, int EPI, int NJB, bool PACK, bool SYM = false, int WM = 4>
__device__ __forceinline__ void f16pv_bigd_body(
    _Float16* __restrict__ smem, const _Float16* __restrict__ Ahi, const _Float16* __restrict__ Alo,
    const _Float16* __restrict__ Bhi, const _Float16* __restrict__ Blo,
    const _Float16* __restrict__ Vth, const _Float16* __restrict__ Vtl,
    const float* __restrict__ vscale, int64_t ldvt, int64_t n1, int64_t n2, int64_t m, int KP,
    float qinv2, float dscale, int deg, double pmul, double* __restrict__ part, int64_t ldp,
    int64_t part_stride, int tiles_per_split, int64_t rb, int64_t split,
    const SymOut& so = SymOut{}) {
  constexpr int TN = 16 * NJB;
  constexpr int NT = 64 * WM;                // threads
  constexpr int BMR = 32 * WM;               // rows per block
  constexpr int RT = BMR / TN;               // column tiles per row block (symmetric mode)
  constexpr int BPT = TN * 4 / NT;           // B chunk pieces per thread
  constexpr int VR = NCT * 16;
  constexpr int VCH = VR * TN / 8;           // V^T pieces per tile
  constexpr int VPT = (VCH + NT - 1) / NT;
  // wide V^T tiles (more than two pieces per thread) are loaded one piece per thread with
  // each of the first VPT chunks of the tile instead of all with the first
  constexpr bool VSPREAD = VPT > 2;
  constexpr int FLUSH = TN >= 128 ? 1 : MM2_FLUSH;  // flush every 128 columns
  static_assert(BPT >= 1 && BPT <= 2 && (VPT <= 2 || (VSPREAD && !PACK && !SYM)), "tile shape");
  static_assert(!PACK || NCT == 1, "packed right-hand sides use one 16-row operand");
  static_assert(!SYM || (TN == 128 && NCT == 1), "symmetric mode: 128-column tiles, NCT = 1");
  static_assert(WM == 4 || (WM == 8 && SYM), "256-row blocks in symmetric mode only");
  // LDS layout (halves): A[2][2][BMR*32], B[2][2][TN*32], V[2][2][VR*TN] (+ X[2 TN 16 floats])
  _Float16* sA = smem;
  _Float16* sB = sA + 2 * 2 * BMR * 32;
  _Float16* sV = sB + 2 * 2 * TN * 32;
  _Float16* sX = sV + 2 * 2 * VR * TN;
  auto A_at = [&](int buf, int hl) { return sA + (buf * 2 + hl) * BMR * 32; };
  auto B_at = [&](int buf, int hl) { return sB + (buf * 2 + hl) * TN * 32; };
  auto V_at = [&](int buf, int hl) { return sV + (buf * 2 + hl) * VR * TN; };

  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t ntiles = ceil_div(n2, TN);
  const int KC = KP / 32;
  // Work list: items t = 0 .. count-1, each a (row block, column tile) pair. Items below nA
  // belong to row block rbA with tile jA + t, the rest to rbB with tile jB + (t - nA).
  int64_t rbA = rb, rbB = rb, jA = 0, jB = 0;
  int nA = 0, count = 0;
  if (SYM) {
    rbB = so.nrb - 1 - rb;
    const int64_t len1 = ntiles - RT * rbA;
    const int64_t len2 = rbB > rbA ? ntiles - RT * rbB : 0;
    const int64_t L = len1 + len2;
    const int64_t b0 = split * L / so.nsplit, b1 = (split + 1) * L / so.nsplit;
    count = (int)(b1 - b0);
    const int64_t na = len1 - b0;
    nA = na < 0 ? 0 : na > count ? count : (int)na;
    jA = RT * rbA + b0;
    jB = RT * rbB + (b0 + nA - len1);
  } else {
    const int64_t t_begin = split * tiles_per_split;
    const int64_t t_end = t_begin + tiles_per_split < ntiles ? t_begin + tiles_per_split : ntiles;
    count = t_end > t_begin ? (int)(t_end - t_begin) : 0;
    nA = count;
    jA = t_begin;
  }
  auto item_rb = [&](int t) __attribute__((always_inline)) { return t < nA ? rbA : rbB; };
  auto item_j = [&](int t) __attribute__((always_inline)) { return t < nA ? jA + t : jB + (t - nA); };
  const int nsteps = count * KC;

  f32x4 acc[2][NCT];
  double acc64[2][NCT][4];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      acc[ib][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[ib][ct][r] = 0.0;
    }
  f32x4 S[NJB][2];

  // V_I^T as the A operand of the column-side product: lane (c = li, g) holds V^T[c][i] for
  // i = 32 w + 16 b + 4 g + r at position 4 b + r (the k order of the transposed P)
  half8 vIh[NCT], vIl[NCT];
  auto load_vI = [&](int64_t I) __attribute__((always_inline)) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int64_t o = (int64_t)(16 * ct + li) * ldvt + I * BMR + 32 * w + 4 * lg;
      const u32x2 a = *reinterpret_cast<const u32x2*>(Vth + o);
      const u32x2 b = *reinterpret_cast<const u32x2*>(Vth + o + 16);
      vIh[ct] = __builtin_bit_cast(half8, u32x4{a.x, a.y, b.x, b.y});
      if (!PACK) {
        const u32x2 c = *reinterpret_cast<const u32x2*>(Vtl + o);
        const u32x2 d = *reinterpret_cast<const u32x2*>(Vtl + o + 16);
        vIl[ct] = __builtin_bit_cast(half8, u32x4{c.x, c.y, d.x, d.y});
      }
    }
  };
  // 0/1 selection operand of the transposing MFMA: lane (col li, k group g) holds
  // E[4 g + r][li] = (4 g + r == li)
  half4 esel;
#pragma unroll
  for (int r = 0; r < 4; ++r) esel[r] = (_Float16)(4 * lg + r == li ? 1.0f : 0.0f);
  if (SYM && count > 0) load_vI(item_rb(0));

  // chunk loaders: A rows of the item's row block + tid/4 and + NT/4; B rows j0 + tid/4
  // (+ 64 when TN = 128 and NT = 256)
  const int arow0 = tid >> 2, arow1 = arow0 + NT / 4, acol = tid & 3;
  const int sa0 = arow0 * 32 + ((acol ^ ((arow0 >> 1) & 3)) * 8);
  const int sa1 = arow1 * 32 + ((acol ^ ((arow1 >> 1) & 3)) * 8);
  const int brow1 = arow0 + 64;
  const int sb1 = brow1 * 32 + ((acol ^ ((brow1 >> 1) & 3)) * 8);
  // V^T pieces: piece e = tid + NT u covers row e / (TN / 8), columns 8 (e % (TN / 8)) ..
  // Threads past the last piece load a duplicate and do not store it.
  const bool vld0 = tid < VCH, vld1 = VPT > 1 && tid + NT < VCH;
  const int ve0 = tid % VCH, ve1 = (tid + NT) % VCH;
  const int vc0 = ve0 / (TN / 8), vj0 = ve0 % (TN / 8);
  const int vc1 = ve1 / (TN / 8), vj1 = ve1 % (TN / 8);
  const int svo00 = vpos<TN>(vc0, 8 * vj0), svo01 = vpos<TN>(vc0, 8 * vj0 + 4);
  const int svo10 = vpos<TN>(vc1, 8 * vj1), svo11 = vpos<TN>(vc1, 8 * vj1 + 4);
  // two register sets: the chunk two steps ahead is loaded while the next one waits to be
  // stored, so global loads have about one and a half steps to arrive. With UNIFORM every
  // step issues the chunk loads (past the last step the last chunk again; the V^T tile
  // only with the first chunk of a tile): the compiler's wait counts then let the newer
  // set stay in flight while the older one is stored. Measured: faster for two column
  // tiles of V (NCT = 2), slower for one, which keeps the loads of the final steps
  // conditional.
  constexpr bool UNIFORM = NCT > 1 || NJB < 8;
  // one register set where the epilogue's registers leave no room for two (symmetric mode,
  // wide passes): the next chunk is loaded at the start of a step and stored at its end
  constexpr bool ONESET = SYM || VSPREAD;
  struct Regs {
    u32x4 ra0h, ra0l, ra1h, ra1l, rb0h, rb0l, rb1h, rb1l, rv0h, rv0l, rv1h, rv1l;
  };
  Regs R0 = {}, R1 = {};
  // position of a step: item (relative to the block's first) and k chunk, advanced one step
  // at a time (no division in the loop)
  struct Pos {
    int t, kc;
  };
  auto advance = [&](Pos& p) __attribute__((always_inline)) {
    if (++p.kc == KC) {
      p.kc = 0;
      ++p.t;
    }
  };
  auto gload = [&](const Pos& p, Regs& R) __attribute__((always_inline)) {
    const int64_t t = item_j(p.t);
    const int64_t blk_i0 = item_rb(p.t) * BMR;
    const int kc = p.kc;
    const int64_t ko = (int64_t)kc * 32 + acol * 8;
    R.ra0h = *reinterpret_cast<const u32x4*>(Ahi + (blk_i0 + arow0) * KP + ko);
    R.ra0l = *reinterpret_cast<const u32x4*>(Alo + (blk_i0 + arow0) * KP + ko);
    R.ra1h = *reinterpret_cast<const u32x4*>(Ahi + (blk_i0 + arow1) * KP + ko);
    R.ra1l = *reinterpret_cast<const u32x4*>(Alo + (blk_i0 + arow1) * KP + ko);
    R.rb0h = *reinterpret_cast<const u32x4*>(Bhi + (t * TN + arow0) * KP + ko);
    R.rb0l = *reinterpret_cast<const u32x4*>(Blo + (t * TN + arow0) * KP + ko);
    if (BPT > 1) {
      R.rb1h = *reinterpret_cast<const u32x4*>(Bhi + (t * TN + brow1) * KP + ko);
      R.rb1l = *reinterpret_cast<const u32x4*>(Blo + (t * TN + brow1) * KP + ko);
    }
    if (VSPREAD) {
      // piece tid + NT kc of the tile (VCH is a multiple of NT)
      if (kc < VPT) {
        const int e = tid + NT * kc;
        const int64_t o = (int64_t)(e / (TN / 8)) * ldvt + t * TN + (e % (TN / 8)) * 8;
        R.rv0h = *reinterpret_cast<const u32x4*>(Vth + o);
        R.rv0l = *reinterpret_cast<const u32x4*>(Vtl + o);
      }
    } else if (kc == 0) {
      R.rv0h = *reinterpret_cast<const u32x4*>(Vth + (int64_t)vc0 * ldvt + t * TN + vj0 * 8);
      if (!PACK)
        R.rv0l = *reinterpret_cast<const u32x4*>(Vtl + (int64_t)vc0 * ldvt + t * TN + vj0 * 8);
      if (VPT > 1) {
        R.rv1h = *reinterpret_cast<const u32x4*>(Vth + (int64_t)vc1 * ldvt + t * TN + vj1 * 8);
        if (!PACK)
          R.rv1l = *reinterpret_cast<const u32x4*>(Vtl + (int64_t)vc1 * ldvt + t * TN + vj1 * 8);
      }
    }
  };
  auto lstore = [&](int q, const Pos& p, const Regs& R) __attribute__((always_inline)) {
    const int buf = q & 1;
    const int kc = p.kc;
    *reinterpret_cast<u32x4*>(A_at(buf, 0) + sa0) = R.ra0h;
    *reinterpret_cast<u32x4*>(A_at(buf, 1) + sa0) = R.ra0l;
    *reinterpret_cast<u32x4*>(A_at(buf, 0) + sa1) = R.ra1h;
    *reinterpret_cast<u32x4*>(A_at(buf, 1) + sa1) = R.ra1l;
    *reinterpret_cast<u32x4*>(B_at(buf, 0) + sa0) = R.rb0h;
    *reinterpret_cast<u32x4*>(B_at(buf, 1) + sa0) = R.rb0l;
    if (BPT > 1) {
      *reinterpret_cast<u32x4*>(B_at(buf, 0) + sb1) = R.rb1h;
      *reinterpret_cast<u32x4*>(B_at(buf, 1) + sb1) = R.rb1l;
    }
    if (VSPREAD) {
      if (kc < VPT) {
        const int vb = p.t & 1;
        const int e = tid + NT * kc;
        const int vc = e / (TN / 8), vj = e % (TN / 8);
        const int o0 = vpos<TN>(vc, 8 * vj), o1 = vpos<TN>(vc, 8 * vj + 4);
        *reinterpret_cast<u32x2*>(V_at(vb, 0) + o0) = u32x2{R.rv0h.x, R.rv0h.y};
        *reinterpret_cast<u32x2*>(V_at(vb, 0) + o1) = u32x2{R.rv0h.z, R.rv0h.w};
        *reinterpret_cast<u32x2*>(V_at(vb, 1) + o0) = u32x2{R.rv0l.x, R.rv0l.y};
        *reinterpret_cast<u32x2*>(V_at(vb, 1) + o1) = u32x2{R.rv0l.z, R.rv0l.w};
      }
    } else if (kc == 0) {
      const int vb = p.t & 1;
      if (vld0) {
        *reinterpret_cast<u32x2*>(V_at(vb, 0) + svo00) = u32x2{R.rv0h.x, R.rv0h.y};
        *reinterpret_cast<u32x2*>(V_at(vb, 0) + svo01) = u32x2{R.rv0h.z, R.rv0h.w};
        if (!PACK) {
          *reinterpret_cast<u32x2*>(V_at(vb, 1) + svo00) = u32x2{R.rv0l.x, R.rv0l.y};
          *reinterpret_cast<u32x2*>(V_at(vb, 1) + svo01) = u32x2{R.rv0l.z, R.rv0l.w};
        }
      }
      if (vld1) {
        *reinterpret_cast<u32x2*>(V_at(vb, 0) + svo10) = u32x2{R.rv1h.x, R.rv1h.y};
        *reinterpret_cast<u32x2*>(V_at(vb, 0) + svo11) = u32x2{R.rv1h.z, R.rv1h.w};
        if (!PACK) {
          *reinterpret_cast<u32x2*>(V_at(vb, 1) + svo10) = u32x2{R.rv1l.x, R.rv1l.y};
          *reinterpret_cast<u32x2*>(V_at(vb, 1) + svo11) = u32x2{R.rv1l.z, R.rv1l.w};
        }
      }
    }
  };
  // row-side output of row block I: lane holds OUT[I * 128 + 32 w + 16 ib + 4 lg + r][16 ct + li]
  double* pout = part + split * part_stride;
  auto write_rows = [&](int64_t I, bool zero) __attribute__((always_inline)) {
    const int64_t i0 = I * BMR + 32 * w;
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int64_t c = 16 * ct + li;
      if (c < m && (!PACK || li < 8)) {
        const double vs = (double)vscale[c] * pmul;
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = i0 + 16 * ib + 4 * lg + r;
            if (i < n1) pout[i * ldp + c] = zero ? 0.0 : acc64[ib][ct][r] * vs;
          }
      }
    }
  };

  // pc, pn, pg: positions of steps q, q + 1 and min(q + 2, nsteps - 1)
  Pos pc{0, 0}, pn{0, 0}, pg{0, 0};
  if (nsteps > 0) {
    gload(pc, R0);
    lstore(0, pc, R0);
    if (nsteps > 1) advance(pn);
    if (!ONESET) {
      gload(pn, R0);
      pg = pn;
      if (nsteps > 2) advance(pg);
    }
  }
  // complete the prologue's loads once here, so the loop does not inherit them as pending
  // (that makes the compiler wait for every outstanding load at the top of each step)
  wait_vmem_all();
  __syncthreads();
  int since_flush = 0;
  auto compute = [&](int q, const Pos& p) __attribute__((always_inline)) {
    const int buf = q & 1;
    const int kc = p.kc;
    // fragments of this chunk: rows of the wave (B operand) and the tile's columns (A operand)
    half8 ah[2], al[2];
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) {
      const int row = 32 * w + 16 * ib + li;
      const int o = row * 32 + ((lg ^ ((row >> 1) & 3)) * 8);
      ah[ib] = *reinterpret_cast<const half8*>(A_at(buf, 0) + o);
      al[ib] = *reinterpret_cast<const half8*>(A_at(buf, 1) + o);
    }
#pragma unroll
    for (int jb = 0; jb < NJB; ++jb) {
      const int row = 16 * jb + li;
      const int o = row * 32 + ((lg ^ ((row >> 1) & 3)) * 8);
      const half8 bh = *reinterpret_cast<const half8*>(B_at(buf, 0) + o);
      const half8 bl = *reinterpret_cast<const half8*>(B_at(buf, 1) + o);
#pragma unroll
      for (int ib = 0; ib < 2; ++ib) {
        const f32x4 c0 = kc == 0 ? f32x4{0.0f, 0.0f, 0.0f, 0.0f} : S[jb][ib];
        f32x4 v = __builtin_amdgcn_mfma_f32_16x16x32_f16(bl, ah[ib], c0, 0, 0, 0);
        v = __builtin_amdgcn_mfma_f32_16x16x32_f16(bh, al[ib], v, 0, 0, 0);
        S[jb][ib] = __builtin_amdgcn_mfma_f32_16x16x32_f16(bh, ah[ib], v, 0, 0, 0);
      }
    }
  };
  // epilogue of a tile (after the chunk kc = KC - 1)
  auto epilogue = [&](int q, const Pos& p) __attribute__((always_inline)) {
    const int buf = q & 1;
    {
      const int vb = p.t & 1;
      const int64_t I = item_rb(p.t), J = item_j(p.t);
      // right of row block I's diagonal block (uniform over the block)
      const bool col = SYM && J >= RT * (I + 1);
      // column-side partial sums of wave ww: [128 columns j][16 columns c] FP32 in the LDS
      // stage the next chunk is stored to after the epilogue (free until then): waves
      // 0 .. 2 WM/4 - 1 in its A part, the next two in its B part, waves 6 and 7 (WM = 8) in
      // the extra area
      constexpr int CW = 16 * NCT;
      auto red_at = [&](int ww) __attribute__((always_inline)) {
        constexpr int NA = WM / 2;  // waves in the A part
        _Float16* base = ww < NA ? A_at(buf ^ 1, 0) : ww < NA + 2 ? B_at(buf ^ 1, 0) : sX;
        const int k = ww < NA ? ww : ww < NA + 2 ? ww - NA : ww - NA - 2;
        return reinterpret_cast<float*>(base) + k * TN * CW;
      };
#pragma unroll
      for (int jp = 0; jp < NJB / 2; ++jp) {
        // V^T fragments of all column tiles up front, or (wide passes) one tile at a time
        constexpr int NVF = VSPREAD ? 1 : NCT;
        half8 vh[NVF], vl[NVF];
        if (!VSPREAD) {
#pragma unroll
          for (int ct = 0; ct < NVF; ++ct) {
            const int u = vfrag<TN>(16 * ct + li, jp, lg);
            vh[ct] = *reinterpret_cast<const half8*>(V_at(vb, 0) + u);
            if (!PACK) vl[ct] = *reinterpret_cast<const half8*>(V_at(vb, 1) + u);
          }
        }
        half8 ph[2], pl[2];
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
#pragma unroll
          for (int jj = 0; jj < 2; ++jj)
#pragma unroll
            for (int r = 0; r < 4; r += 2) {
              float l2a = S[2 * jp + jj][ib][r], l2b = S[2 * jp + jj][ib][r + 1];
              if (!UNIT) { l2a *= qinv2; l2b *= qinv2; }
              const float pa = epi_value<EPI>(l2a, dscale, deg);
              const float pb = epi_value<EPI>(l2b, dscale, deg);
              const half2v h = half2v{(_Float16)pa, (_Float16)pb};
              const half2v l = split_lo2(h, pa, pb);
              ph[ib][4 * jj + r] = h[0];
              ph[ib][4 * jj + r + 1] = h[1];
              pl[ib][4 * jj + r] = l[0];
              pl[ib][4 * jj + r + 1] = l[1];
            }
          if (!VSPREAD) {
#pragma unroll
            for (int ct = 0; ct < NVF; ++ct) {
              acc[ib][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(pl[ib], vh[ct], acc[ib][ct], 0, 0, 0);
              if (!PACK)
                acc[ib][ct] =
                    __builtin_amdgcn_mfma_f32_16x16x32_f16(ph[ib], vl[ct], acc[ib][ct], 0, 0, 0);
              acc[ib][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ph[ib], vh[ct], acc[ib][ct], 0, 0, 0);
            }
          }
        }
        if (VSPREAD) {
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
            const int u = vfrag<TN>(16 * ct + li, jp, lg);
            const half8 wh = *reinterpret_cast<const half8*>(V_at(vb, 0) + u);
            const half8 wl = *reinterpret_cast<const half8*>(V_at(vb, 1) + u);
#pragma unroll
            for (int ib = 0; ib < 2; ++ib) {
              acc[ib][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(pl[ib], wh, acc[ib][ct], 0, 0, 0);
              acc[ib][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ph[ib], wl, acc[ib][ct], 0, 0, 0);
              acc[ib][ct] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ph[ib], wh, acc[ib][ct], 0, 0, 0);
            }
          }
        }
        if (col) {
#pragma unroll
          for (int jj = 0; jj < 2; ++jj) {
            // transpose the 32 x 16 block (rows of the wave, columns 16 jb ..): lane (j = li,
            // g) gets P[32 w + 16 b + 4 g + r][16 jb + li] at position 4 b + r
            half8 th, tl;
#pragma unroll
            for (int ib = 0; ib < 2; ++ib) {
              const half4 a_h = half4{ph[ib][4 * jj], ph[ib][4 * jj + 1], ph[ib][4 * jj + 2],
                                      ph[ib][4 * jj + 3]};
              const half4 a_l = half4{pl[ib][4 * jj], pl[ib][4 * jj + 1], pl[ib][4 * jj + 2],
                                      pl[ib][4 * jj + 3]};
              const f32x4 z = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
              const f32x4 xh = __builtin_amdgcn_mfma_f32_16x16x16f16(a_h, esel, z, 0, 0, 0);
              const f32x4 xl = __builtin_amdgcn_mfma_f32_16x16x16f16(a_l, esel, z, 0, 0, 0);
#pragma unroll
              for (int r = 0; r < 4; ++r) {
                th[4 * ib + r] = (_Float16)xh[r];
                tl[4 * ib + r] = (_Float16)xl[r];
              }
            }
            const int jb = 2 * jp + jj;
            float* red = red_at(w);
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct) {
              // D[c][j] = sum_i V_I^T[c][i] P[i][j] over the wave's 32 rows i
              f32x4 d = __builtin_amdgcn_mfma_f32_16x16x32_f16(vIh[ct], tl, f32x4{0.0f, 0.0f, 0.0f, 0.0f}, 0, 0, 0);
              if (!PACK) d = __builtin_amdgcn_mfma_f32_16x16x32_f16(vIl[ct], th, d, 0, 0, 0);
              d = __builtin_amdgcn_mfma_f32_16x16x32_f16(vIh[ct], th, d, 0, 0, 0);
              // lane (j = li, g) holds D[4 g + r][16 jb + li]
              *reinterpret_cast<f32x4*>(red + (16 * jb + li) * CW + 16 * ct + 4 * lg) = d;
            }
          }
        }
      }
      const bool switch_rb = SYM && p.t == nA - 1 && nA < count;
      if (++since_flush == FLUSH || q + 1 == nsteps || switch_rb) {
        since_flush = 0;
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[ib][ct][r] += (double)acc[ib][ct][r];
            acc[ib][ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
          }
      }
      if (switch_rb) {
        // the first row block of the pair is done: write it and start on the second
        if (PACK) pack_combine<NCT>(acc64);
        write_rows(rbA, false);
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[ib][ct][r] = 0.0;
        load_vI(rbB);
      }
      if (col) {
        __syncthreads();
        // wave w finishes columns TN/WM w .. TN/WM (w + 1) - 1: the WM waves' partials added
        // in a fixed order, then one fixed-point atomic add per (row, column)
        constexpr int JW = TN / WM;
        const int mv = PACK ? (m < 8 ? (int)m : 8) : (m < CW ? (int)m : CW);
#pragma unroll 1
        for (int u = 0; u < JW * CW / 64; ++u) {
          const int e = u * 64 + lane;
          const int jj = e / CW, c = e % CW;
          const int j = JW * w + jj;
          if (c < mv) {
            float s = 0.0f;
#pragma unroll
            for (int ww = 0; ww < WM; ++ww) {
              const float* rr = red_at(ww) + j * CW;
              s += PACK ? rr[c] + rr[c + 8] : rr[c];
            }
            const int64_t row = J * TN + j;
            if (__builtin_isfinite(s))
              atomicAdd(so.fx + row * so.ldfx + c,
                        (unsigned long long)(long long)__builtin_rintf(s * so.fxs));
            else
              atomicOr(so.flag + row, 1u << c);
          }
        }
        __syncthreads();
      }
    }
  };
  auto step = [&](int q, const Regs& hold, Regs& spare) __attribute__((always_inline)) {
    if (UNIFORM || q + 2 < nsteps) gload(pg, spare);
    compute(q, pc);
    if (pc.kc == KC - 1) epilogue(q, pc);
    if (q + 1 < nsteps) lstore(q + 1, pn, hold);
    __syncthreads();
    advance(pc);
    advance(pn);
    if (q + 3 < nsteps) advance(pg);
  };
  if (ONESET) {
    for (int q = 0; q < nsteps; ++q) {
      const bool more = q + 1 < nsteps;
      if (more) gload(pn, R0);
      compute(q, pc);
      if (pc.kc == KC - 1) epilogue(q, pc);
      if (more) lstore(q + 1, pn, R0);
      __syncthreads();
      advance(pc);
      advance(pn);
    }
  } else {
    for (int q = 0; q < nsteps; q += 2) {
      step(q, R0, R1);
      if (q + 1 < nsteps) step(q + 1, R1, R0);
    }
  }
  if (PACK) pack_combine<NCT>(acc64);
  if (SYM) {
    const bool hasA = nA > 0, hasB = nA < count;
    write_rows(hasB ? rbB : rbA, false);
    // a row block of the pair with no item in this part still gets its (zero) partial sums
    if (!hasA && hasB) write_rows(rbA, true);
    if (!hasB && rbB != rbA) write_rows(rbB, true);
  } else {
    write_rows(rb, false);
  }
}

// column tiles of the large-d single-problem product (the batched product keeps 64, and so
// does the 64-column pass, NCT = 4, whose accumulators leave no registers for wider tiles)
constexpr int BD_NJB = 8;
constexpr int BD_TN = 16 * BD_NJB;
constexpr int bd_njb(int nct) { return nct >= 4 ? 4 : BD_NJB; }
// grouped launch: BD_GROUP column splits, row blocks padded to a multiple of 8 BD_GROUP
constexpr int BD_GROUP = 8;

template <int NCT, int EPI, bool PACK, bool SYM, int WM = 4>
__global__ __launch_bounds__(64 * WM, (NCT >= 4 || WM == 8) ? 1 : 2) void matmat_f16pv_bigd_kernel(
    const _Float16* __restrict__ Ahi, const _Float16* __restrict__ Alo,
    const _Float16* __restrict__ Bhi, const _Float16* __restrict__ Blo,
    const _Float16* __restrict__ Vth, const _Float16* __restrict__ Vtl,
    const float* __restrict__ vscale, int64_t ldvt, int64_t n1, int64_t n2, int64_t m, int KP,
    const float* __restrict__ qinv2_ptr, float dscale, double* __restrict__ part, int64_t ldp,
    int64_t part_stride, int tiles_per_split, int grouped, int64_t nunits, SymOut so) {
  constexpr int NJB = bd_njb(NCT);
  // row units per XCD group: the blocks one XCD holds at once (two per CU for 128-row blocks,
  // one for 256-row blocks) over BD_GROUP splits
  constexpr int GU = WM == 8 ? BD_GROUP / 2 : BD_GROUP;
  __shared__ __attribute__((aligned(16))) _Float16 smem[bigd_smem_halves<NCT, NJB, WM>()];
  int64_t rb = blockIdx.x, sp = blockIdx.y;
  if (grouped) {
    // 1-D grid of (row unit, split) pairs with BD_GROUP splits, ordered so that the blocks
    // one XCD runs together (workgroups go round-robin to the 8 XCDs) form groups of
    // GU row units x BD_GROUP splits: each group shares its row operand chunks and its
    // column tiles in that XCD's L2 instead of streaming them per block. A row unit is a
    // 128-row block, or in symmetric mode a pair of row blocks.
    const int64_t b = blockIdx.x, x = b % 8, t = b / 8;
    const int64_t gid = (t / (GU * BD_GROUP)) * 8 + x, u = t % (GU * BD_GROUP);
    rb = gid * GU + u / BD_GROUP;
    sp = u % BD_GROUP;
    if (rb >= nunits) return;  // padding block
  }
  const float qinv2 = qinv2_ptr[0];
  int deg;
  double pmul;
  epi_params<EPI>(qinv2_ptr, deg, pmul);
  if (qinv2 == 1.0f)
    f16pv_bigd_body<NCT, true, EPI, NJB, PACK, SYM, WM>(smem, Ahi, Alo, Bhi, Blo, Vth, Vtl, vscale,
                                                   ldvt, n1, n2, m, KP, qinv2, dscale, deg, pmul,
                                                   part, ldp, part_stride, tiles_per_split, rb,
                                                   sp, so);
  else
    f16pv_bigd_body<NCT, false, EPI, NJB, PACK, SYM, WM>(smem, Ahi, Alo, Bhi, Blo, Vth, Vtl, vscale,
                                                    ldvt, n1, n2, m, KP, qinv2, dscale, deg, pmul,
                                                    part, ldp, part_stride, tiles_per_split, rb,
                                                    sp, so);
}

// Adds the column side of a symmetric product to split 0 of the partial sums:
// part[i][c] += fx[i][c] 2^-F vscale[c] pmul (NaN where a contribution was not finite).
__global__ __launch_bounds__(256) void sym_fold_kernel(const unsigned long long* __restrict__ fx,
                                                       const unsigned* __restrict__ flag,
                                                       int64_t ldfx, int64_t n, int64_t mc,
                                                       double inv_fxs,
                                                       const float* __restrict__ vscale,
                                                       const float* __restrict__ kpar, int epi,
                                                       double* __restrict__ part, int64_t ldp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * mc) return;
  const int64_t i = e / mc, c = e % mc;
  const double pmul = epi == KV_POLY ? ldexp(1.0, (int)kpar[1]) : 1.0;
  double v = (double)(long long)fx[i * ldfx + c] * inv_fxs;
  if ((flag[i] >> c) & 1u) v = __builtin_nan("");
  part[i * ldp + c] += v * ((double)vscale[c] * pmul);
}

// Column side of a symmetric product: clear the accumulator and flags, fix the fixed-point
// scale 2^F from a bound on any column-side total (n terms of |P| <= pmax: exp2 of a
// non-positive value up to rounding, a power of a value in [-1, 1], or x 2^-x dscale <=
// 0.531 dscale, times |V'| <= SPLIT_TARGET, kept below 2^62).
hipError_t sym_begin(const SymBuf& sym, int64_t n, int64_t rows_pad, int epi, float dscale,
                     int nsplit, int64_t nrb, SymOut& so, double& inv_fxs, hipStream_t st) {
  const double pmax = epi == KV_DSIGMA ? 0.54 * std::fabs((double)dscale) : 2.0;
  const double bound = (double)n * std::max(pmax, 1e-30) * SPLIT_TARGET;
  const int F = (int)std::floor(62.0 - std::log2(bound));
  so.fx = sym.fx;
  so.flag = sym.flag;
  so.ldfx = sym.ldfx;
  so.fxs = std::ldexp(1.0f, F);
  so.nsplit = nsplit;
  so.nrb = nrb;
  inv_fxs = std::ldexp(1.0, -F);
  hipError_t e = fill_f64(reinterpret_cast<double*>(so.fx), rows_pad * so.ldfx, 0.0, st);
  if (e == hipSuccess) e = fill_i32(reinterpret_cast<int*>(so.flag), rows_pad, 0, st);
  return e;
}
hipError_t sym_end(const SymOut& so, double inv_fxs, int64_t n, int64_t m, const SplitRhs& V,
                   const float* kpar, int epi, double* part, int64_t ldp, hipStream_t st) {
  const int64_t mc = V.packed ? std::min<int64_t>(m, 8) : m;
  sym_fold_kernel<<<(unsigned)ceil_div(n * mc, 256), 256, 0, st>>>(
      so.fx, so.flag, so.ldfx, n, mc, inv_fxs, V.vscale, kpar, epi, part, ldp);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

hipError_t matmat_f16pv(const MixedPoints<_Float16>& A, const MixedPoints<_Float16>& B,
                        const SplitRhs& V, int64_t m, int epi, float dscale, double* part,
                        int64_t ldp, int64_t part_stride, int nsplit, hipStream_t st,
                        const SymBuf* sym) {
  if (epi != KV_GAUSS && epi != KV_DSIGMA && epi != KV_POLY) return hipErrorInvalidValue;
  if (A.Kp != B.Kp || V.mpad < round_up(m, 16)) return hipErrorInvalidValue;
  // passes of up to 32 columns (for large d 64, NCT = 4, or 160, NCT = 10)
  if (A.Kp > 128 ? !(V.mpad <= 32 || V.mpad == 64 || V.mpad == 160) : V.mpad > 32)
    return hipErrorInvalidValue;
  if (V.packed && (m > 8 || V.mpad != 16)) return hipErrorInvalidValue;
  // norm terms in the epilogue: Gaussian products of the register-resident kernel only
  if ((A.nrm != nullptr) != (B.nrm != nullptr) || (A.nrm && (A.Kp > 128 || epi == KV_POLY)))
    return hipErrorInvalidValue;
  if (part_stride < round_up(A.n, MM2_BM) * ldp) return hipErrorInvalidValue;
  const int64_t ntiles = ceil_div(B.n, MM_BN);
  const int tps = (int)ceil_div(ntiles, nsplit);
  dim3 grid(ceil_div(A.n, MM2_BM), nsplit);
  const int nct = (int)(V.mpad / 16);
  // symmetric products: large d, one 16-column tile, the same points on both sides
  const bool symm = sym && A.Kp > 128 && nct == 1 && A.n == B.n;
  if (symm && (sym->ldfx < V.mpad || V.rows_pad < round_up(A.n, MM2_BM)))
    return hipErrorInvalidValue;
  const int64_t nrb = ceil_div(A.n, MM2_BM);
  SymOut so;
  double inv_fxs = 1.0;
  if (symm) {
    hipError_t e = sym_begin(*sym, A.n, V.rows_pad, epi, dscale, nsplit, nrb, so, inv_fxs, st);
    if (e != hipSuccess) return e;
  }
  if (A.Kp > 128) {
    const int kp = (int)A.Kp;
    const int tps = (int)ceil_div(ceil_div(B.n, 16 * bd_njb(nct)), nsplit);
    // symmetric products on 256-row blocks (8 waves) when the rows are padded for them
    const bool rows256 = symm && V.rows_pad >= round_up(A.n, 2 * BD_BM);
    if (rows256) so.nrb = ceil_div(A.n, 2 * BD_BM);
    const int64_t nunits = symm ? (so.nrb + 1) / 2 : nrb;
    const int gu = rows256 ? BD_GROUP / 2 : BD_GROUP;
    const int grouped = nsplit == BD_GROUP && nunits >= 8 * gu ? 1 : 0;
    grid = grouped ? dim3((unsigned)(round_up(nunits, 8 * gu) * BD_GROUP), 1)
                   : dim3((unsigned)nunits, nsplit);
#define KRR_BD(NCT_, D_, P_, S_, WM_)                                                            \
  matmat_f16pv_bigd_kernel<NCT_, D_, P_, S_, WM_><<<grid, 64 * WM_, 0, st>>>(                    \
      A.hi, A.lo, B.hi, B.lo, V.hi, V.lo, V.vscale, V.rows_pad, A.n, B.n, m, kp, A.qinv2, dscale, \
      part, ldp, part_stride, tps, grouped, nunits, so)
#define KRR_BD_EPI(NCT_, P_, S_, WM_)                          \
  if (epi == KV_DSIGMA) KRR_BD(NCT_, KV_DSIGMA, P_, S_, WM_);  \
  else if (epi == KV_POLY) KRR_BD(NCT_, KV_POLY, P_, S_, WM_); \
  else KRR_BD(NCT_, KV_GAUSS, P_, S_, WM_);
    if (rows256) {
      if (V.packed) {
        KRR_BD_EPI(1, true, true, 8)
      } else {
        KRR_BD_EPI(1, false, true, 8)
      }
    } else if (symm) {
      if (V.packed) {
        KRR_BD_EPI(1, true, true, 4)
      } else {
        KRR_BD_EPI(1, false, true, 4)
      }
    } else if (nct == 1 && V.packed) {
      KRR_BD_EPI(1, true, false, 4)
    } else if (nct == 1) {
      KRR_BD_EPI(1, false, false, 4)
    } else if (nct == 2) {
      KRR_BD_EPI(2, false, false, 4)
    } else if (nct == 4) {
      KRR_BD_EPI(4, false, false, 4)
    } else {
      KRR_BD_EPI(10, false, false, 4)
    }
#undef KRR_BD_EPI
#undef KRR_BD
    KRR_LAUNCH_CHECK();
    return symm ? sym_end(so, inv_fxs, A.n, m, V, A.qinv2, epi, part, ldp, st) : hipSuccess;
  }
#define KRR_PV1(KS_, NCT_, E_, PK_, NE_)                                                      \
  matmat_f16pv_kernel<KS_, NCT_, E_, PK_, NE_><<<grid, 256, 0, st>>>(                         \
      A.hi, A.lo, B.hi, B.lo, V.hi, V.lo, V.vscale, V.rows_pad, A.n, B.n, m, A.qinv2, dscale,  \
      part, ldp, part_stride, tps, A.nrm, B.nrm)
#define KRR_PV(KS_, NCT_, PK_)                                                                \
  if (A.Kp == KS_ * 32 && nct == NCT_ && V.packed == PK_) {                                   \
    if (A.nrm) {                                                                              \
      if (epi == KV_DSIGMA) KRR_PV1(KS_, NCT_, KV_DSIGMA, PK_, true);                        \
      else KRR_PV1(KS_, NCT_, KV_GAUSS, PK_, true);                                          \
    } else if (epi == KV_DSIGMA) KRR_PV1(KS_, NCT_, KV_DSIGMA, PK_, false);                  \
    else if (epi == KV_POLY) KRR_PV1(KS_, NCT_, KV_POLY, PK_, false);                        \
    else KRR_PV1(KS_, NCT_, KV_GAUSS, PK_, false);                                           \
    KRR_LAUNCH_CHECK();                                                                       \
    return hipSuccess;                                                                        \
  }
  KRR_PV(1, 1, true) KRR_PV(2, 1, true) KRR_PV(3, 1, true) KRR_PV(4, 1, true)
  KRR_PV(1, 1, false) KRR_PV(2, 1, false) KRR_PV(3, 1, false) KRR_PV(4, 1, false)
  KRR_PV(1, 2, false) KRR_PV(2, 2, false) KRR_PV(3, 2, false) KRR_PV(4, 2, false)
#undef KRR_PV
#undef KRR_PV1
  return hipErrorInvalidValue;
}

// ------------------------------------------------------- batched persistent kernel
// One launch serves many independent problems: blocks take work items (instance, 128-row
// block, column split) from an atomic counter until the list is exhausted, and run on each
// the body its feature width calls for: the register-resident small-d body (Kp <= 128, the
// row operands in registers, 64-column tiles of the other side through LDS) or the large-d
// body (both operands through LDS). Items are ordered largest first; items of a problem
// whose columns have all converged (live[inst] == 0) are skipped.
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int BATCH_SMEM_BYTES =
    cmax(cmax(2 * bigd_smem_halves<1, 4>(), (int)sizeof(PVSmem<4, 1, true, true>)),
         (int)sizeof(PVSmem<4, 1, false, true>));
__global__ __launch_bounds__(256, 2) void matmat_batch_kernel(const BatchItem* __restrict__ items,
                                                              const int* __restrict__ list,
                                                              const int* __restrict__ nlist,
                                                              const BatchInst* __restrict__ inst,
                                                              int* __restrict__ counter,
                                                              int packed) {
  __shared__ __attribute__((aligned(16))) unsigned char smem[BATCH_SMEM_BYTES];
  __shared__ int cur;
  const int nitems = *nlist;  // live items only (batch_compact_live)
  for (;;) {
    if (threadIdx.x == 0) cur = atomicAdd(counter, 1);
    __syncthreads();
    const int it = cur;
    __syncthreads();
    if (it >= nitems) break;  // uniform: every wave of the block leaves together
    const BatchItem wi = items[list[it]];
    const BatchInst I = inst[wi.inst];
    const float qinv2 = *I.qinv2;
    if (I.Kp <= 128) {
#define KRR_BATCH_SMALL(KS, U, PK)                                                          \
  f16pv_body<KS, 1, U, KV_GAUSS, PK, true>(*reinterpret_cast<PVSmem<KS, 1, PK, true>*>(smem), \
                                           I.Ahi, I.Alo, I.Bhi, I.Blo, I.Vth, I.Vtl, I.vscale,  \
                                           I.ldvt, I.n, I.n, I.m, qinv2, 0.0f, 1, 1.0, I.part,  \
                                           I.ldp, I.part_stride, wi.tiles_per_split, wi.rb,     \
                                           wi.split, I.nrm, I.nrm)
#define KRR_BATCH_KS(U, PK)                                      switch (I.Kp) {                                                  case 32: KRR_BATCH_SMALL(1, U, PK); break;                     case 64: KRR_BATCH_SMALL(2, U, PK); break;                     case 96: KRR_BATCH_SMALL(3, U, PK); break;                     default: KRR_BATCH_SMALL(4, U, PK); break;                   }
      if (packed) {
        if (qinv2 == 1.0f) { KRR_BATCH_KS(true, true) }
        else { KRR_BATCH_KS(false, true) }
      } else {
        if (qinv2 == 1.0f) { KRR_BATCH_KS(true, false) }
        else { KRR_BATCH_KS(false, false) }
      }
#undef KRR_BATCH_KS
#undef KRR_BATCH_SMALL
    } else {
      _Float16* sh = reinterpret_cast<_Float16*>(smem);
#define KRR_BATCH_BODY(U, PK)                                                                      f16pv_bigd_body<1, U, KV_GAUSS, 4, PK>(sh, I.Ahi, I.Alo, I.Bhi, I.Blo, I.Vth, I.Vtl,                                                    I.vscale, I.ldvt, I.n, I.n, I.m, I.Kp, qinv2, 0.0f, 1,                                            1.0, I.part, I.ldp, I.part_stride, wi.tiles_per_split,                                            wi.rb, wi.split)
      if (packed) {
        if (qinv2 == 1.0f) KRR_BATCH_BODY(true, true);
        else KRR_BATCH_BODY(false, true);
      } else {
        if (qinv2 == 1.0f) KRR_BATCH_BODY(true, false);
        else KRR_BATCH_BODY(false, false);
      }
#undef KRR_BATCH_BODY
    }
    __syncthreads();
  }
}

hipError_t matmat_batch(const BatchItem* items, const int* list, const int* nlist,
                        const BatchInst* inst, int* counter, bool packed, int grid,
                        hipStream_t st) {
  hipError_t e = fill_i32(counter, 1, 0, st);
  if (e != hipSuccess) return e;
  matmat_batch_kernel<<<grid, 256, 0, st>>>(items, list, nlist, inst, counter, packed ? 1 : 0);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// ------------------------------------------------------------------- FP64 path
// FP64 MFMA (16x16x4) lane layout (gfx950): A operand lane l holds A[l%16][l/16], B operand
// B[l/16][l%16], result register r holds C[l/16 + 4r][l%16].
typedef double d4v __attribute__((ext_vector_type(4)));

// e^{-x} for x >= 0 in FP64 with a 256-entry table T[j] = 2^{-j/256} (EXP_TAB entries in
// LDS): with y = 256 x log2(e), k = rint(y) and r = k/256 - x log2(e) in [-1/512, 1/512],
// e^{-x} = 2^{-(k >> 8)} T[k & 255] e^{r ln 2}. k is rounded by adding 1.5 * 2^52 (its low
// word is then k in two's complement, |k| < 2^31) and u = r ln 2 = k (ln 2 / 256) - x is
// formed with ln 2 / 256 split in two (the high part has 34 bits, so k times it is exact
// for k < 2^19); the last factor is a degree-4 Taylor polynomial (truncation below 4e-17).
// x is clamped at 745.2, where e^{-x} is below half the smallest subnormal; a NaN passes
// through. A slightly negative x (rounding of a zero distance) takes the same steps.
constexpr int EXP_TAB = 256;
__device__ inline double exp_neg_tab(double x, const double* __restrict__ T) {
  const double xc = x > 745.2 ? 745.2 : x;
  const double sh = fma(xc, 369.3299304675746, 6755399441055744.0);  // 1.5 * 2^52
  const int k = __double2loint(sh);
  const double kf = sh - 6755399441055744.0;
  const double u = fma(kf, 6.327543041662719e-14, fma(kf, 0.002707606173999011, -xc));
  double q = fma(u, 1.0 / 24.0, 1.0 / 6.0);
  q = fma(u, q, 0.5);
  q = fma(u, q, 1.0);
  q = fma(u, q, 1.0);
  return ldexp(T[k & (EXP_TAB - 1)] * q, -(k >> 8));
}

// Large-d FP64 product (dp > 128, multiple of 32): both point sets stream through LDS in
// 32-wide k chunks as FP32 coordinates (exact copies of X), converted to FP64 for the 16x16x4
// FP64 MFMA, so every product x_ik x_jk is exact and the sums are FP64. Block: 128 rows (4
// waves x 32) against 64-column tiles; per tile the wave accumulates G^T for its 4 x 2 blocks
// of 16 x 16, then D = nu_i + nu_j - 2 G, k = exp(-D c) (FP64, table-driven) and
// OUT[i][:] += sum_j k V[j][:] on FP64 MFMA. The V tile of a column tile is written to LDS at
// the tile's first chunk and read at its last (at least one barrier in between; the previous
// tile's readers have passed a barrier), so it needs one buffer.
constexpr int F64B_TJ = 64;
constexpr int F64B_LK = 33;  // padded LDS row of a chunk (floats)
// Column side of the symmetric FP64 product (SYM, K(X, X) V with one 16-column tile): each
// off-diagonal (128-row block, 64-column tile) pair gives P^T V_I for the rows of the tile,
// P transposed per 16 x 16 block by four FP64 MFMAs against 0/1 selection operands (exact)
// and multiplied by V_I^T on FP64 MFMA, each wave's sums over its 32 rows added to a
// two-word fixed-point accumulator: h = rint(v 2^F1) (exact remainder since |h| < 2^52),
// l = rint((v - h 2^-F1) 2^F2). F1 and F2 come from column c's largest finite |V|
// (f64sym_scales, also used by the fold) so that neither word's total can overflow; the
// represented sum is accurate to far below an FP64 ulp of the largest contribution, and
// integer adds make it independent of the order of the atomics.
struct F64SymOut {
  unsigned long long *fh = nullptr, *fl = nullptr;  // [rows_pad][16]
  unsigned* flag = nullptr;                          // [rows_pad]
  const unsigned long long* vmax = nullptr;          // [16] bits of max finite |V[:, c]|
  double pmax = 2.0;                                 // bound on |P|
  int nsplit = 1;
  int64_t nrb = 0;                                   // 128-row blocks
};
__device__ __forceinline__ void f64sym_scales(const F64SymOut& so, int cc, int& F1, int& F2) {
  const double vmax = fmax(__longlong_as_double((long long)so.vmax[cc]), 0x1.0p-900);
  const int lk = 64 - __builtin_clzll((unsigned long long)(4 * so.nrb));  // > log2 K
  int eb;
  frexp(32.0 * so.pmax * vmax, &eb);  // 32 |P| |V| < 2^eb: one wave's contribution
  F1 = (62 - lk < 52 ? 62 - lk : 52) - eb - 1;
  F2 = F1 + (61 - lk < 50 ? 61 - lk : 50);
}
// bits of max finite |V[i][c]| per column c < m (m <= 16), into vmax[16] (cleared before):
// non-negative doubles order like their bit patterns
__global__ __launch_bounds__(256) void f64_colmax_kernel(const double* __restrict__ V,
                                                         int64_t n, int64_t m, int64_t ldv,
                                                         unsigned long long* __restrict__ vmax) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  const int c = tid & 15;  // 16 columns x 16 row lanes per block
  double mx = 0.0;
  if (c < m)
    for (int64_t i = (int64_t)blockIdx.x * 16 + (tid >> 4); i < n; i += (int64_t)gridDim.x * 16) {
      const double a = fabs(V[i * ldv + c]);
      if (a <= 1.7976931348623157e308) mx = fmax(mx, a);  // finite only
    }
  red[tid] = mx;
  __syncthreads();
  for (int o = 128; o >= 16; o >>= 1) {
    if (tid < o) red[tid] = fmax(red[tid], red[tid + o]);
    __syncthreads();
  }
  if (tid < 16 && tid < m) atomicMax(vmax + tid, (unsigned long long)__double_as_longlong(red[tid]));
}
template <int NCT, bool SYM = false>
__global__ __launch_bounds__(256, NCT >= 4 ? 1 : 2) void matmat_f64big_kernel(
    const float* __restrict__ Xa, const double* __restrict__ nua, const float* __restrict__ Xb,
    const double* __restrict__ nub, const double* __restrict__ V, int64_t ldv, int64_t n1,
    int64_t n2, int64_t m, int c0, int dp, double c, int epi, double dscale, PolyF64 pk,
    double* __restrict__ part, int64_t ldp, int64_t part_stride, int tiles_per_split,
    F64SymOut so) {
  constexpr int VC = 16 * NCT;
  constexpr int LV = VC + 1;
  static_assert(!SYM || NCT == 1, "symmetric FP64 product: one 16-column tile");
  __shared__ float sR[2][128 * F64B_LK];
  __shared__ float sC[2][F64B_TJ * F64B_LK];
  __shared__ double sV[F64B_TJ * LV];
  __shared__ double sN[F64B_TJ];
  __shared__ double sE[EXP_TAB];
  __shared__ double sVI[SYM ? 4 * 32 * 16 : 1];  // V_I per wave: [32 rows][16 columns]
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t ntiles = ceil_div(n2, F64B_TJ);
  const int KC = dp / 32;
  // work list: item t < nA is tile jA + t of row block rbA, the rest tile jB + (t - nA) of
  // rbB (symmetric mode: the pair (p, nrb - 1 - p), row block I starting at tile 2 I)
  int64_t rbA = blockIdx.x, rbB = blockIdx.x, jA = 0, jB = 0;
  int nA = 0, count = 0;
  if (SYM) {
    rbB = so.nrb - 1 - rbA;
    const int64_t len1 = ntiles - 2 * rbA;
    const int64_t len2 = rbB > rbA ? ntiles - 2 * rbB : 0;
    const int64_t L = len1 + len2;
    const int64_t b0 = (int64_t)blockIdx.y * L / so.nsplit;
    const int64_t b1 = ((int64_t)blockIdx.y + 1) * L / so.nsplit;
    count = (int)(b1 - b0);
    const int64_t na = len1 - b0;
    nA = na < 0 ? 0 : na > count ? count : (int)na;
    jA = 2 * rbA + b0;
    jB = 2 * rbB + (b0 + nA - len1);
  } else {
    const int64_t t_begin = (int64_t)blockIdx.y * tiles_per_split;
    const int64_t t_end = t_begin + tiles_per_split < ntiles ? t_begin + tiles_per_split : ntiles;
    count = t_end > t_begin ? (int)(t_end - t_begin) : 0;
    nA = count;
    jA = t_begin;
  }
  auto item_rb = [&](int t) __attribute__((always_inline)) { return t < nA ? rbA : rbB; };
  auto item_j = [&](int t) __attribute__((always_inline)) { return t < nA ? jA + t : jB + (t - nA); };
  const int64_t nsteps = (int64_t)count * KC;
  for (int e = tid; e < EXP_TAB; e += 256) sE[e] = exp2(-(double)e / EXP_TAB);

  double nui[2];
  // V_I for the column-side MFMA, in the wave's own LDS rows: sVI[w][x][c] = V[I 128 + 32 w
  // + x][c0 + c] (zero past n or m); only this wave writes and reads its rows
  auto load_rows = [&](int64_t I) __attribute__((always_inline)) {
#pragma unroll
    for (int ib = 0; ib < 2; ++ib) nui[ib] = nua[I * 128 + 32 * w + 16 * ib + li];
    if (SYM) {
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int x = 16 * ib + lg + 4 * r;
          const int64_t i = I * 128 + 32 * w + x;
          sVI[(32 * w + x) * 16 + li] = (i < n2 && c0 + li < m) ? V[i * ldv + c0 + li] : 0.0;
        }
    }
  };
  load_rows(item_rb(0));
  d4v g[4][2], acc[2][NCT];
#pragma unroll
  for (int ib = 0; ib < 2; ++ib)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) acc[ib][ct] = d4v{0.0, 0.0, 0.0, 0.0};

  // loaders: row chunk 128 x 32 floats (4 float4 per thread), column chunk 64 x 32 (2),
  // V tile 64 x VC doubles (VU per thread) and nu of the tile's columns at each tile's first
  // chunk; a wide V tile (160 columns) comes in VU / UPS slices of UPS values per thread with
  // the tile's first chunks, each stored at the start of the next step (the last at chunk 3,
  // so a barrier separates it from the reads at the last chunk whenever KC >= 5)
  constexpr int VU = F64B_TJ * VC / 256;
  constexpr int UPS = VU > 16 ? 10 : VU;
  static_assert(VU % UPS == 0 && VU / UPS <= 4, "V tile slices");
  const int lrow = tid >> 3, lc4 = (tid & 7) * 4;
  float4 rr[4], rc[2];
  double rv[UPS];
  double rn = 0.0;
  auto gload = [&](int64_t q) __attribute__((always_inline)) {
    const int tq = (int)(q / KC);
    const int64_t t = item_j(tq);
    const int64_t blk_i0 = item_rb(tq) * 128;
    const int kc = (int)(q % KC);
    const int64_t ko = (int64_t)kc * 32 + lc4;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      rr[u] = *reinterpret_cast<const float4*>(Xa + (blk_i0 + lrow + 32 * u) * dp + ko);
#pragma unroll
    for (int u = 0; u < 2; ++u)
      rc[u] = *reinterpret_cast<const float4*>(Xb + (t * F64B_TJ + lrow + 32 * u) * dp + ko);
    if (kc < VU / UPS) {
#pragma unroll
      for (int u = 0; u < UPS; ++u) {
        const int e = tid + 256 * (kc * UPS + u), r = e / VC, cc = e % VC;
        const int64_t j = t * F64B_TJ + r;
        rv[u] = (j < n2 && c0 + cc < m) ? V[j * ldv + c0 + cc] : 0.0;
      }
    }
    if (kc == 0 && tid < F64B_TJ) rn = nub[t * F64B_TJ + tid];
  };
  auto lstore = [&](int64_t q) __attribute__((always_inline)) {
    const int buf = (int)(q & 1);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      float* d = &sR[buf][(lrow + 32 * u) * F64B_LK + lc4];
      d[0] = rr[u].x; d[1] = rr[u].y; d[2] = rr[u].z; d[3] = rr[u].w;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      float* d = &sC[buf][(lrow + 32 * u) * F64B_LK + lc4];
      d[0] = rc[u].x; d[1] = rc[u].y; d[2] = rc[u].z; d[3] = rc[u].w;
    }
  };
  auto vstore = [&](int kc) __attribute__((always_inline)) {
#pragma unroll
    for (int u = 0; u < UPS; ++u) {
      const int e = tid + 256 * (kc * UPS + u);
      sV[(e / VC) * LV + e % VC] = rv[u];
    }
    if (kc == 0 && tid < F64B_TJ) sN[tid] = rn;
  };
  // writes of the row side of row block I: lane holds OUT[I 128 + 32 w + 16 ib + lg + 4 r]
  double* pout = part + (int64_t)blockIdx.y * part_stride;
  auto write_rows = [&](int64_t I, bool zero) __attribute__((always_inline)) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct) {
      const int64_t cc = c0 + 16 * ct + li;
      if (cc < m) {
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int64_t i = I * 128 + 32 * w + 16 * ib + lg + 4 * r;
            if (i < n1) pout[i * ldp + cc] = zero ? 0.0 : acc[ib][ct][r];
          }
      }
    }
  };

  if (nsteps > 0) {
    gload(0);
    lstore(0);
  }
  __syncthreads();
  for (int64_t q = 0; q < nsteps; ++q) {
    const int buf = (int)(q & 1);
    const int kc = (int)(q % KC);
    if (kc < VU / UPS) vstore(kc);  // this tile's V and nu (read at its last chunk, after a barrier)
    if (kc == 0) {
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) g[jb][ib] = d4v{0.0, 0.0, 0.0, 0.0};
    }
    if (q + 1 < nsteps) gload(q + 1);
#pragma unroll
    for (int sk = 0; sk < 8; ++sk) {
      double a[4], b[2];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) a[jb] = (double)sC[buf][(16 * jb + li) * F64B_LK + 4 * sk + lg];
#pragma unroll
      for (int ib = 0; ib < 2; ++ib)
        b[ib] = (double)sR[buf][(32 * w + 16 * ib + li) * F64B_LK + 4 * sk + lg];
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int ib = 0; ib < 2; ++ib)
          g[jb][ib] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[jb], b[ib], g[jb][ib], 0, 0, 0);
    }
    if (kc == KC - 1) {
      const int tq = (int)(q / KC);
      const int64_t I = item_rb(tq), J = item_j(tq);
      const bool col = SYM && J >= 2 * (I + 1);  // right of I's diagonal block (uniform)
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        // column side: D[c][j] = sum over the wave's 32 rows i of V[i][c] P[i][j]; lane holds
        // D[c = lg + 4 r][j = 16 jb + li]
        d4v dc = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) {
          // transposed P of the 16 x 16 block (jb, ib): (i = 16 ib + lg + 4 r, j = li)
          d4v tp = d4v{0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int jj = 16 * jb + lg + 4 * r;
            double p;
            if (epi == KV_POLY) {
              p = pk.value(g[jb][ib][r]);
            } else {
              const double D = nui[ib] + sN[jj] - 2.0 * g[jb][ib][r];  // >= 0 up to rounding
              p = exp_neg_tab(D * c, sE);
              if (epi == KV_DSIGMA) p *= D * dscale;
            }
#pragma unroll
            for (int ct = 0; ct < NCT; ++ct)
              acc[ib][ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(p, sV[jj * LV + 16 * ct + li],
                                                                 acc[ib][ct], 0, 0, 0);
            // selection E_r[k][c'] = (c' == k + 4 r): lane (li, lg) holds (li == lg + 4 r)
            if (col)
              tp = __builtin_amdgcn_mfma_f64_16x16x4f64(p, li == lg + 4 * r ? 1.0 : 0.0, tp, 0, 0, 0);
          }
          if (col) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
              dc = __builtin_amdgcn_mfma_f64_16x16x4f64(sVI[(32 * w + 16 * ib + lg + 4 * r) * 16 + li],
                                                        tp[r], dc, 0, 0, 0);
          }
        }
        if (col) {
          const int64_t row = J * F64B_TJ + 16 * jb + li;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int cc = lg + 4 * r;
            if (c0 + cc < m) {
              const double v = dc[r];
              if (__builtin_isfinite(v)) {
                int F1, F2;
                f64sym_scales(so, cc, F1, F2);
                const double hd = rint(ldexp(v, F1));
                const double lo = rint(ldexp(v - ldexp(hd, -F1), F2));
                atomicAdd(so.fh + row * 16 + cc, (unsigned long long)(long long)hd);
                atomicAdd(so.fl + row * 16 + cc, (unsigned long long)(long long)lo);
              } else {
                atomicOr(so.flag + row, 1u << cc);
              }
            }
          }
        }
      }
      if (SYM && tq == nA - 1 && nA < count) {
        // the first row block of the pair is done: write it and start on the second
        write_rows(rbA, false);
#pragma unroll
        for (int ib = 0; ib < 2; ++ib) acc[ib][0] = d4v{0.0, 0.0, 0.0, 0.0};
        load_rows(rbB);
      }
    }
    if (q + 1 < nsteps) lstore(q + 1);
    __syncthreads();
  }
  if (SYM) {
    const bool hasA = nA > 0, hasB = nA < count;
    write_rows(hasB ? rbB : rbA, false);
    if (!hasA && hasB) write_rows(rbA, true);
    if (!hasB && rbB != rbA) write_rows(rbB, true);
  } else {
    write_rows(rbA, false);
  }
}

// Adds the column side of a symmetric FP64 product to split 0 of the partial sums:
// part[i][c] += fh 2^-F1 + fl 2^-F2 (NaN where a contribution was not finite).
__global__ __launch_bounds__(256) void f64sym_fold_kernel(F64SymOut so, int64_t n, int64_t mc,
                                                          double* __restrict__ part,
                                                          int64_t ldp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * mc) return;
  const int64_t i = e / mc, cc = e % mc;
  int F1, F2;
  f64sym_scales(so, (int)cc, F1, F2);
  double v = ldexp((double)(long long)so.fh[i * 16 + cc], -F1) +
             ldexp((double)(long long)so.fl[i * 16 + cc], -F2);
  if ((so.flag[i] >> cc) & 1u) v = __builtin_nan("");
  part[i * ldp + cc] += v;
}

// FP64 kernel product with the inner products on int8 MFMA (16x16x64, exact int32 sums).
// With the slices of prep_points_i8, <x_i, x_j> = s_i s_j sum_{a,b} 256^(10 - a - b)
// <D_ia, D_jb>. The digit products of one diagonal s = a + b share a weight, so they
// accumulate in one int32 sum E_s (exact: |E_s| < 2^24 per 64-wide chunk); diagonals
// s <= 6 are kept (26 of the 36 products; the dropped ones weigh below 2^-50 of the
// largest), then combined in FP64:
//   G_int = 2^72 (256 E_0 + E_1) + 2^56 (256 E_2 + E_3) + 2^40 (256 E_4 + E_5) + 2^32 E_6,
// the two first brackets formed exactly in int32. D = nu_i + nu_j - 2 s_i s_j G_int,
// k = exp(-c D) in FP64 (table exp), OUT[i][:] += sum_j k V[j][:] on FP64 MFMA.
// Block: 4 waves x 16 rows; the row slices stay in registers as the B operand, the column
// points stream through LDS in 32-point tiles (register prefetch) as the A operand, so lane
// l holds S^T[j = 4 (l/16) + r][i = l % 16], r < 4, the A-operand layout of the FP64
// product's contraction over four j per MFMA. With VPV (at most 8 right-hand sides) the
// P V step runs on the VALU instead: lane l accumulates its row's 8 columns over its four
// j (V rows read as LDS broadcasts) and the four lane groups are summed at the end in a
// fixed order (4 m FMAs per lane and block instead of four FP64 MFMAs padded to 16 columns).
constexpr int F64I_TJ = 32;
typedef int i32x4 __attribute__((ext_vector_type(4)));
template <int KC, int NCT, bool VPV, int EPI>
__global__ __launch_bounds__(256, KC == 1 ? (VPV ? 2 : 3) : 1) void matmat_f64i8_kernel(
    const int8_t* __restrict__ Sa, const double* __restrict__ sca, const double* __restrict__ nua,
    const int8_t* __restrict__ Sb, const double* __restrict__ scb, const double* __restrict__ nub,
    const double* __restrict__ V, int64_t ldv, int64_t n1, int64_t n2, int64_t m, int c0, double c,
    double dscale, PolyF64 pk, double* __restrict__ part, int64_t ldp, int64_t part_stride,
    int tiles_per_split) {
  constexpr int KP = 64 * KC;              // bytes per slice row
  constexpr int RB = OZ_SLICES * KP;       // bytes per point
  constexpr int RS = RB + 16;              // LDS row stride: fragment reads conflict-free
  static_assert(!VPV || NCT == 1, "VALU P V covers one pass of at most 8 columns");
  constexpr int VC = VPV ? 8 : 16 * NCT;
  constexpr int LV = VPV ? 10 : VC + 1;    // VPV: 80-byte rows, 16-byte aligned, and rows
                                           // four apart fall on distinct banks
  constexpr int SCH = F64I_TJ * RB / 16;   // 16-byte pieces per column tile
  constexpr int SPT = (SCH + 255) / 256;
  constexpr int VPT = (F64I_TJ * VC + 255) / 256;
  __shared__ __attribute__((aligned(16))) int8_t sS[2][F64I_TJ * RS];
  __shared__ double sV[2][F64I_TJ * LV];
  __shared__ double sN[2][F64I_TJ];
  __shared__ double sC[2][F64I_TJ];
  __shared__ double sE[EXP_TAB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int li = lane & 15, lg = lane >> 4;
  const int64_t i0 = (int64_t)blockIdx.x * 64 + 16 * w;
  for (int e = tid; e < EXP_TAB; e += 256) sE[e] = exp2(-(double)e / EXP_TAB);  // read after the first barrier
  const int64_t ntiles = ceil_div(n2, F64I_TJ);
  const int64_t t_begin = (int64_t)blockIdx.y * tiles_per_split;
  const int64_t t_end = t_begin + tiles_per_split < ntiles ? t_begin + tiles_per_split : ntiles;

  i32x4 xr[OZ_SLICES][KC];
#pragma unroll
  for (int a = 0; a < OZ_SLICES; ++a)
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
      xr[a][kc] = *reinterpret_cast<const i32x4*>(Sa + ((i0 + li) * OZ_SLICES + a) * KP +
                                                  kc * 64 + 16 * lg);
  const double nui = nua[i0 + li];
  const double ai = -2.0 * 4294967296.0 * sca[i0 + li];  // -2 * 2^32 * s_i
  d4v acc[NCT];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) acc[ct] = d4v{0.0, 0.0, 0.0, 0.0};
  double accv[VPV ? 8 : 1];
#pragma unroll
  for (int cc = 0; cc < (VPV ? 8 : 1); ++cc) accv[cc] = 0.0;

  i32x4 rs[SPT];
  double rv[VPT], rn = 0.0;
  auto gload = [&](int64_t t) __attribute__((always_inline)) {
    const int64_t j0 = t * F64I_TJ;
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int e = tid + 256 * u;
      if (e < SCH) rs[u] = *reinterpret_cast<const i32x4*>(Sb + j0 * RB + 16 * (int64_t)e);
    }
    // right-hand sides: out-of-range entries load a valid element and are zeroed at the
    // store (a select right after the load would wait for it)
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int e = tid + 256 * u;
      const int r = e / VC, cc = e % VC;
      const int64_t j = j0 + r;
      const bool ok = e < F64I_TJ * VC && j < n2 && c0 + cc < m;
      rv[u] = V[ok ? j * ldv + c0 + cc : 0];
    }
    if (tid < F64I_TJ) rn = nub[j0 + tid];
    else if (tid < 2 * F64I_TJ) rn = scb[j0 + tid - F64I_TJ];
  };
  auto lstore = [&](int64_t t, int buf) __attribute__((always_inline)) {
    const int64_t j0 = t * F64I_TJ;
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int e = tid + 256 * u;
      if (e < SCH) {
        const int row = (16 * e) / RB, off = (16 * e) % RB;
        *reinterpret_cast<i32x4*>(&sS[buf][row * RS + off]) = rs[u];
      }
    }
#pragma unroll
    for (int u = 0; u < VPT; ++u) {
      const int e = tid + 256 * u;
      const int r = e / VC, cc = e % VC;
      if (e < F64I_TJ * VC) sV[buf][r * LV + cc] = (j0 + r < n2 && c0 + cc < m) ? rv[u] : 0.0;
    }
    if (tid < F64I_TJ) sN[buf][tid] = rn;
    else if (tid < 2 * F64I_TJ) sC[buf][tid - F64I_TJ] = rn;
  };

  // digit-diagonal sums E_s of the 16 x 16 pair block jb of the tile in buffer buf
  auto i8_block = [&](int buf, int jb, i32x4 (&E)[7]) __attribute__((always_inline)) {
#pragma unroll
    for (int q = 0; q < 7; ++q) E[q] = i32x4{0, 0, 0, 0};
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      i32x4 cf[OZ_SLICES];
#pragma unroll
      for (int b = 0; b < OZ_SLICES; ++b)
        cf[b] = *reinterpret_cast<const i32x4*>(&sS[buf][(16 * jb + li) * RS + b * KP +
                                                         kc * 64 + 16 * lg]);
#pragma unroll
      for (int b = 0; b < OZ_SLICES; ++b)
#pragma unroll
        for (int a = 0; a < OZ_SLICES; ++a)
          if (a + b <= 6)
            E[a + b] = __builtin_amdgcn_mfma_i32_16x16x64_i8(cf[b], xr[a][kc], E[a + b], 0, 0, 0);
    }
  };
  // kernel values of block jb from its diagonal sums, accumulated against V
  auto i8_epi = [&](int buf, int jb, const i32x4 (&E)[7]) __attribute__((always_inline)) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int jj = 16 * jb + 4 * lg + r;
      const int H = E[0][r] * 256 + E[1][r];  // |H| < 2^28, |L| < 2^31 (int32, exact)
      const int L = E[2][r] * 256 + E[3][r];
      double g = fma((double)H, 65536.0, (double)L);
      if (KC == 1)  // |256 E_4 + E_5| < 2^31 for one 64-wide chunk
        g = fma(g, 65536.0, (double)(E[4][r] * 256 + E[5][r]));
      else
        g = fma(g, 65536.0, fma((double)E[4][r], 256.0, (double)E[5][r]));
      g = fma(g, 256.0, (double)E[6][r]);  // = G_int / 2^32
      // D >= 0 up to rounding (|D| ~ 1e-15 nu for duplicate points): no clamp needed, the
      // exp below is exact in form for small negative arguments, and a NaN stays NaN
      double p;
      if (EPI == KV_POLY) {
        p = pk.value((-0.5 * ai) * sC[buf][jj] * g);  // <x_i, x_j> (power-of-two scales)
      } else {
        const double D = fma(ai * sC[buf][jj], g, nui + sN[buf][jj]);
        p = exp_neg_tab(D * c, sE);
        if (EPI == KV_DSIGMA) p *= D * dscale;
      }
      if (VPV) {
        const double* vr = &sV[buf][jj * LV];
#pragma unroll
        for (int cc = 0; cc < 8; ++cc) accv[cc] = fma(p, vr[cc], accv[cc]);
      } else {
#pragma unroll
        for (int ct = 0; ct < NCT; ++ct)
          acc[ct] = __builtin_amdgcn_mfma_f64_16x16x4f64(p, sV[buf][jj * LV + 16 * ct + li],
                                                         acc[ct], 0, 0, 0);
      }
    }
  };

  if (t_begin < t_end) {
    gload(t_begin);
    lstore(t_begin, 0);
  }
  wait_vmem_all();  // the row slices above included, on every path
  __syncthreads();
  for (int64_t t = t_begin; t < t_end; ++t) {
    const int buf = (int)((t - t_begin) & 1);
    const bool more = t + 1 < t_end;
    if (more) gload(t + 1);
#pragma unroll 1
    for (int jb = 0; jb < F64I_TJ / 16; ++jb) {
      i32x4 E[7];
      i8_block(buf, jb, E);
      i8_epi(buf, jb, E);
    }
    if (more) lstore(t + 1, buf ^ 1);
    __syncthreads();
  }
  double* pout = part + (int64_t)blockIdx.y * part_stride;
  if (VPV) {
    // lane (li, lg) holds row i0 + li summed over its lane group's j: add the four groups
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) {
      accv[cc] += __shfl_xor(accv[cc], 16, 64);
      accv[cc] += __shfl_xor(accv[cc], 32, 64);
    }
    const int64_t i = i0 + li;
    if (lg == 0 && i < n1) {
#pragma unroll
      for (int cc = 0; cc < 8; ++cc)
        if (c0 + cc < m) pout[i * ldp + c0 + cc] = accv[cc];
    }
    return;
  }
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct) {
    const int64_t cc = c0 + 16 * ct + li;
    if (cc < m) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + lg + 4 * r;
        if (i < n1) pout[i * ldp + cc] = acc[ct][r];
      }
    }
  }
}

hipError_t matmat_f64(const F64Points& A, const F64Points& B, const double* V, int64_t ldv,
                      int64_t m, int epi, double c, double dscale, const PolyF64& pk,
                      double* part, int64_t ldp, int64_t part_stride, int nsplit,
                      hipStream_t st, const F64SymBuf* sym) {
  if (A.dp != B.dp) return hipErrorInvalidValue;
  if (epi != KV_GAUSS && epi != KV_DSIGMA && epi != KV_POLY) return hipErrorInvalidValue;
  dim3 grid(ceil_div(A.n, 64), nsplit);
  if (A.S && B.S) {
    // int8-slice kernel (d <= 128): 32-point column tiles, up to 32 right-hand sides per pass
    if (A.d != B.d || A.d > 128 || A.d < 1) return hipErrorInvalidValue;
    const int kc = (int)(oz_kp(A.d) / 64);
    const int tps = (int)ceil_div(ceil_div(B.n, F64I_TJ), nsplit);
    for (int64_t c0 = 0; c0 < m; c0 += 32) {
      const int nct = m - c0 > 16 ? 2 : 1;
#define KRR_I8(KC_, NCT_, VPV_, DV_)                                                           \
  matmat_f64i8_kernel<KC_, NCT_, VPV_, DV_><<<grid, 256, 0, st>>>(                             \
      A.S, A.scale, A.nu, B.S, B.scale, B.nu, V, ldv, A.n, B.n, m, (int)c0, c, dscale, pk,     \
      part, ldp, part_stride, tps)
#define KRR_I8D(KC_, NCT_, VPV_)                                                               \
  do {                                                                                         \
    if (epi == KV_DSIGMA) KRR_I8(KC_, NCT_, VPV_, KV_DSIGMA);                                  \
    else if (epi == KV_POLY) KRR_I8(KC_, NCT_, VPV_, KV_POLY);                                 \
    else KRR_I8(KC_, NCT_, VPV_, KV_GAUSS);                                                    \
  } while (0)
      const bool vpv = m - c0 <= 8;  // P V on the VALU
      if (kc == 1 && vpv) KRR_I8D(1, 1, true);
      else if (kc == 1 && nct == 1) KRR_I8D(1, 1, false);
      else if (kc == 1) KRR_I8D(1, 2, false);
      else if (vpv) KRR_I8D(2, 1, true);
      else if (nct == 1) KRR_I8D(2, 1, false);
      else KRR_I8D(2, 2, false);
#undef KRR_I8D
#undef KRR_I8
      KRR_LAUNCH_CHECK();
    }
    return hipSuccess;
  }
  if (!A.Xf || !B.Xf || A.dp % 32) return hipErrorInvalidValue;
  const int tpsb = (int)ceil_div(ceil_div(B.n, F64B_TJ), nsplit);
  dim3 gridb(ceil_div(A.n, 128), nsplit);
  F64SymOut so;
  if (sym && A.n == B.n && m <= 16 && epi != KV_POLY) {
    // symmetric product (one 16-column pass): column side in two-word fixed point
    const int64_t rows_pad = round_up(A.n, 128);
    so.fh = sym->fh;
    so.fl = sym->fl;
    so.flag = sym->flag;
    so.vmax = sym->vmax;
    so.pmax = epi == KV_DSIGMA ? 1.01 * std::fabs(dscale) / (c * 2.718281828459045) + 1e-300 : 2.0;
    so.nsplit = nsplit;
    so.nrb = ceil_div(A.n, 128);
    hipError_t e = fill_f64(reinterpret_cast<double*>(so.fh), rows_pad * 16, 0.0, st);
    if (e == hipSuccess) e = fill_f64(reinterpret_cast<double*>(so.fl), rows_pad * 16, 0.0, st);
    if (e == hipSuccess) e = fill_i32(reinterpret_cast<int*>(so.flag), rows_pad, 0, st);
    if (e == hipSuccess) e = fill_f64(reinterpret_cast<double*>(sym->vmax), 16, 0.0, st);
    if (e != hipSuccess) return e;
    f64_colmax_kernel<<<(unsigned)std::min<int64_t>(1024, ceil_div(A.n, 16)), 256, 0, st>>>(
        V, A.n, m, ldv, sym->vmax);
    KRR_LAUNCH_CHECK();
    const dim3 gs((unsigned)((so.nrb + 1) / 2), nsplit);
    matmat_f64big_kernel<1, true><<<gs, 256, 0, st>>>(A.Xf, A.nu, B.Xf, B.nu, V, ldv, A.n, B.n, m,
                                                      0, (int)A.dp, c, epi, dscale, pk, part, ldp,
                                                      part_stride, tpsb, so);
    KRR_LAUNCH_CHECK();
    f64sym_fold_kernel<<<(unsigned)ceil_div(A.n * m, 256), 256, 0, st>>>(so, A.n, m, part, ldp);
    KRR_LAUNCH_CHECK();
    return hipSuccess;
  }
  // passes of up to 160 right-hand sides: the inner products dominate a pass's work
  for (int64_t c0 = 0; c0 < m; c0 += 160) {
#define KRR_F64B(NCT_)                                                                        \
  matmat_f64big_kernel<NCT_><<<gridb, 256, 0, st>>>(A.Xf, A.nu, B.Xf, B.nu, V, ldv, A.n, B.n, m, \
                                                    (int)c0, (int)A.dp, c, epi, dscale, pk,    \
                                                    part, ldp, part_stride, tpsb, so)
    if (m - c0 > 64) KRR_F64B(10);
    else if (m - c0 > 32) KRR_F64B(4);
    else if (m - c0 > 16) KRR_F64B(2);
    else KRR_F64B(1);
#undef KRR_F64B
    KRR_LAUNCH_CHECK();
  }
  return hipSuccess;
}

// OUT[i, c] = sum_s part[s][i][c] (fixed order) + shift * Vs[i, c]
template <typename VS>
__global__ void matmat_finalize_kernel(const double* __restrict__ part, int64_t part_stride,
                                       int nsplit, int64_t n, int64_t m, int64_t ldp,
                                       double shift, const VS* __restrict__ Vs, int64_t ldvs,
                                       double* __restrict__ out, int64_t ldo) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * m) return;
  const int64_t i = e / m, c = e % m;
  double s = 0.0;
  for (int k = 0; k < nsplit; ++k) s += part[k * part_stride + i * ldp + c];
  if (shift != 0.0) s += shift * (double)Vs[i * ldvs + c];
  out[i * ldo + c] = s;
}

template <typename VS>
hipError_t matmat_finalize(const double* part, int64_t part_stride, int nsplit, int64_t n,
                           int64_t m, int64_t ldp, double shift, const VS* Vs, int64_t ldvs,
                           double* out, int64_t ldo, hipStream_t st) {
  matmat_finalize_kernel<VS><<<ceil_div(n * m, 256), 256, 0, st>>>(
      part, part_stride, nsplit, n, m, ldp, shift, Vs, ldvs, out, ldo);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
template hipError_t matmat_finalize<double>(const double*, int64_t, int, int64_t, int64_t,
                                            int64_t, double, const double*, int64_t, double*,
                                            int64_t, hipStream_t);
template hipError_t matmat_finalize<float>(const double*, int64_t, int, int64_t, int64_t, int64_t,
                                           double, const float*, int64_t, double*, int64_t,
                                           hipStream_t);

}  // namespace krr
