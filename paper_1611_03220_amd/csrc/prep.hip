// Point preparation and operand splitting for the MFMA products.
//
// The Gaussian kernel (Sec. 6) is evaluated through the norm expansion
//   -||x_i - x_j||^2 c = 2c <x_i, x_j> - c nu_i - c nu_j,   nu = ||x||^2, c = log2(e)/(2 sigma^2),
// which becomes ONE inner product of augmented rows
//   a_i = q [sqrt(2c) x_i, -c nu_i, 1],   b_j = q [sqrt(2c) x_j, 1, -c nu_j],
// so that <a_i, b_j> = q^2 log2 k(x_i, x_j). q is a power of two that keeps every entry
// below 2^14, so the FP16 hi/lo split loses no range (exact scaling, undone in the
// epilogue); q = 1 whenever the entries already lie in [2^-3, 2^14].
#include "kernels.hpp"

namespace krr {

__global__ void fill_f32_kernel(float* p, int64_t count, float v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}
__global__ void fill_f64_kernel(double* p, int64_t count, double v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}
__global__ void fill_i32_kernel(int* p, int64_t count, int v) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) p[i] = v;
}

hipError_t fill_f32(float* p, int64_t count, float v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  fill_f32_kernel<<<ceil_div(count, 256), 256, 0, st>>>(p, count, v);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
hipError_t fill_f64(double* p, int64_t count, double v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  fill_f64_kernel<<<ceil_div(count, 256), 256, 0, st>>>(p, count, v);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
__global__ void fill2d_f64_kernel(double* p, int64_t ld, int64_t rows, int64_t cols, double v) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < rows * cols) p[(e / cols) * ld + e % cols] = v;
}
hipError_t fill2d_f64(double* p, int64_t ld, int64_t rows, int64_t cols, double v, hipStream_t st) {
  if (rows * cols <= 0) return hipSuccess;
  fill2d_f64_kernel<<<ceil_div(rows * cols, 256), 256, 0, st>>>(p, ld, rows, cols, v);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
hipError_t fill_i32(int* p, int64_t count, int v, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  fill_i32_kernel<<<ceil_div(count, 256), 256, 0, st>>>(p, count, v);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// stats[0] = max |x_ik|, stats[1] = max ||x_i||^2 over all rows: each wave walks rows with a
// grid stride, the block reduces its four waves, one atomic max per block and statistic
// (atomic max on the float bit pattern, valid for non-negative values; stats start at 0).
__global__ __launch_bounds__(256) void point_stats_kernel(const float* __restrict__ X, int64_t n,
                                                          int64_t d, int64_t ldx, float* stats) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float amax = 0.0f, numax = 0.0f;
  for (int64_t row = (int64_t)blockIdx.x * 4 + w; row < n; row += (int64_t)gridDim.x * 4) {
    const float* x = X + row * ldx;
    double nu = 0.0;
    for (int64_t k = lane; k < d; k += 64) {
      const float v = x[k];
      nu += (double)v * (double)v;
      amax = fmaxf(amax, fabsf(v));
    }
    nu = wave_sum(nu);
    numax = fmaxf(numax, (float)nu);
  }
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  __shared__ float red[2][4];
  if (lane == 0) { red[0][w] = amax; red[1][w] = numax; }
  __syncthreads();
  if (threadIdx.x == 0) {
    atomic_max_pos(&stats[0], fmaxf(fmaxf(red[0][0], red[0][1]), fmaxf(red[0][2], red[0][3])));
    atomic_max_pos(&stats[1], fmaxf(fmaxf(red[1][0], red[1][1]), fmaxf(red[1][2], red[1][3])));
  }
}

hipError_t point_stats(const float* X, int64_t n, int64_t d, int64_t ldx, float* stats,
                       hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>(1024, ceil_div(n, 4));
  point_stats_kernel<<<blocks, 256, 0, st>>>(X, n, d, ldx, stats);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// Augmented, scaled, split rows (one wave per row). side 0 writes a_i, side 1 writes b_j.
// Gaussian rows (see the top of the file): <a_i, b_j> = q^2 log2 k. With pshift > 0 a third
// augmented column (a: q, b: q * pshift) adds pshift to every log2 k, i.e. the products
// return k * 2^pshift.
// Polynomial rows (kernel (gamma x^T z + c)^deg, Sec. 6): a_i = q [sqrt(gamma / T) x_i,
// sqrt(c / T)] on both sides, so <a_i, b_j> = q^2 (gamma <x_i, x_j> + c) / T, where T is the
// even power of two at or above t_max = gamma max ||x||^2 + c (the Cauchy-Schwarz bound of
// |gamma x^T z + c|): the scaled value lies in [-1, 1] and its deg-th power cannot overflow;
// the products are multiplied back by T^deg.
// With nrm (Gaussian rows only), the two norm columns are left out (Kp >= d) and
// nrm[row] = -q^2 c nu_row is written instead, the same for both sides; the product then
// adds nrm_i + nrm_j to the accumulated q^2 2c <x_i, x_j> in FP32 (rows n..rows_pad-1: 0).
// Rows n..rows_pad-1 and the remaining columns up to Kp are zero. Thread 0 of block 0 of
// side 0 also stores the kernel parameters kpar[0] = 1/q^2, kpar[1] = log2 T^deg and
// kpar[2] = deg (identical for both sides: they depend only on the shared stats).
template <typename T>
__global__ __launch_bounds__(256) void prep_points_kernel(
    const float* __restrict__ X, int64_t n, int64_t d, int64_t ldx, int64_t rows_pad, int64_t Kp,
    RowSpec rs, const float* __restrict__ stats, int side, int pshift, T* __restrict__ hi,
    T* __restrict__ lo, float* __restrict__ kpar, float* __restrict__ nrm) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  double t, cterm = 0.0;
  float amax;
  int tlog = 0;
  if (rs.poly) {
    int e;
    frexp(rs.gamma * (double)stats[1] + rs.coef0, &e);  // t_max < 2^e
    tlog = e + (e & 1);                                  // even, so sqrt(1/T) is exact
    const double tinv = ldexp(1.0, -tlog);
    t = sqrt(rs.gamma * tinv);
    cterm = sqrt(rs.coef0 * tinv);
    amax = fmaxf(fmaxf((float)(t * stats[0]), (float)cterm), 1.0f);
  } else {
    t = sqrt(2.0 * rs.c2);
    amax = fmaxf(fmaxf((float)(t * stats[0]), (float)(rs.c2 * stats[1])),
                 fmaxf(1.0f, (float)pshift));
  }
  const float q = point_scale(amax);
  if (blockIdx.x == 0 && threadIdx.x == 0 && kpar) {
    kpar[0] = 1.0f / (q * q);
    kpar[1] = (float)(tlog * rs.deg);
    kpar[2] = (float)rs.deg;
  }
  if (row >= rows_pad) return;
  T* h = hi + row * Kp;
  T* l = lo + row * Kp;
  if (row >= n) {
    for (int64_t k = lane; k < Kp; k += 64) { h[k] = (T)0.0f; l[k] = (T)0.0f; }
    if (nrm && lane == 0) nrm[row] = 0.0f;
    return;
  }
  const float* x = X + row * ldx;
  double nu = 0.0;
  if (!rs.poly) {
    for (int64_t k = lane; k < d; k += 64) nu += (double)x[k] * (double)x[k];
    nu = wave_sum(nu);
  }
  const double qt = (double)q * t;
  const double qnu = -(double)q * rs.c2 * nu;
  if (nrm && lane == 0) nrm[row] = (float)((double)q * qnu);
  for (int64_t k = lane; k < Kp; k += 64) {
    double v;
    if (k < d) v = qt * (double)x[k];
    else if (nrm) v = 0.0;
    else if (rs.poly) v = k == d ? (double)q * cterm : 0.0;
    else if (k == d) v = side == 0 ? qnu : (double)q;
    else if (k == d + 1) v = side == 0 ? (double)q : qnu;
    else if (k == d + 2 && pshift > 0) v = side == 0 ? (double)q : (double)q * pshift;
    else v = 0.0;
    T a, b;
    Elem<T>::split((float)v, a, b);
    h[k] = a;
    l[k] = b;
  }
}

template <typename T>
hipError_t prep_points(const float* X, int64_t n, int64_t d, int64_t ldx, int64_t rows_pad,
                       int64_t Kp, const RowSpec& rs, const float* stats, int side, int pshift,
                       T* hi, T* lo, float* kpar, hipStream_t st, float* nrm) {
  if (nrm && (rs.poly || pshift != 0 || Kp < d)) return hipErrorInvalidValue;
  prep_points_kernel<T><<<ceil_div(rows_pad, 4), 256, 0, st>>>(X, n, d, ldx, rows_pad, Kp, rs,
                                                               stats, side, pshift, hi, lo, kpar,
                                                               nrm);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
template hipError_t prep_points<_Float16>(const float*, int64_t, int64_t, int64_t, int64_t,
                                          int64_t, const RowSpec&, const float*, int, int,
                                          _Float16*, _Float16*, float*, hipStream_t, float*);
template hipError_t prep_points<__bf16>(const float*, int64_t, int64_t, int64_t, int64_t, int64_t,
                                        const RowSpec&, const float*, int, int, __bf16*, __bf16*,
                                        float*, hipStream_t, float*);

// ------------------------------------------- right-hand sides for the MFMA accumulation
// colmax[c] = max_i |V[i, c]| (atomic max on the float bit pattern; colmax starts at 0).
__global__ __launch_bounds__(256) void vec_colmax_kernel(const float* __restrict__ V, int64_t n,
                                                         int64_t m, int64_t ldv,
                                                         float* __restrict__ colmax) {
  __shared__ float sh[256];
  const int tid = threadIdx.x;
  for (int64_t cbase = 0; cbase < m; cbase += 256) {
    const int64_t mc = m - cbase < 256 ? m - cbase : 256;
    const int rif = (int)(256 / mc);
    const int ro = tid / (int)mc;
    const int64_t c = cbase + tid % mc;
    float mx = 0.0f;
    if (ro < rif)
      for (int64_t i = (int64_t)blockIdx.x * rif + ro; i < n; i += (int64_t)gridDim.x * rif)
        mx = fmaxf(mx, fabsf(V[i * ldv + c]));
    sh[tid] = ro < rif ? mx : 0.0f;
    __syncthreads();
    if (tid < mc) {
      float r = 0.0f;
      for (int k = 0; k < rif; ++k) r = fmaxf(r, sh[k * mc + tid]);
      atomic_max_pos(&colmax[cbase + tid], r);
    }
    __syncthreads();
  }
}

// Vt_hi/Vt_lo[c][j] = split(qv_c V[j, c]) (FP16, c < mpad, j < rows_pad, zero padded) with
// qv_c = split_scale(colmax[c]); V[j, c] is overwritten by the value the split represents
// exactly, (hi + lo) / qv_c, so later updates use the vector the products saw.
// vscale[c] = 1 / (qv_c 2^pshift) undoes both the V scale and the 2^pshift of the kernel.
// Packed (m <= 8, mpad = 16): row c < 8 of hi holds the high part of column c and row c + 8
// its low part; lo is not written. One 16-row operand then carries both halves.
__global__ __launch_bounds__(256) void vec_split_t_kernel(float* __restrict__ V, int64_t n,
                                                          int64_t m, int64_t ldv, int64_t rows_pad,
                                                          int64_t mpad,
                                                          const float* __restrict__ colmax,
                                                          int pshift, int packed,
                                                          _Float16* __restrict__ hi,
                                                          _Float16* __restrict__ lo,
                                                          float* __restrict__ vscale) {
  __shared__ float tile[32][33];
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  const int64_t j0 = (int64_t)blockIdx.x * 32, c0 = (int64_t)blockIdx.y * 32;
  // load V[j0 + yy][c0 + tx]
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t j = j0 + yy, c = c0 + tx;
    tile[yy][tx] = (j < n && c < m) ? V[j * ldv + c] : 0.0f;
  }
  __syncthreads();
  // write Vt[c0 + yy][j0 + tx] (coalesced along j)
  for (int yy = ty; yy < 32; yy += 8) {
    const int64_t c = c0 + yy, j = j0 + tx;
    if (c < mpad && j < rows_pad) {
      const int64_t cv = packed ? (c & 7) : c;  // source column
      const bool low_row = packed && c >= 8;
      const float qv = cv < m ? split_scale(colmax[cv]) : 1.0f;
      const float v = tile[tx][cv - c0] * qv;
      _Float16 h, l;
      Elem<_Float16>::split(v, h, l);
      if (packed) {
        hi[c * rows_pad + j] = low_row ? l : h;
      } else {
        hi[c * rows_pad + j] = h;
        lo[c * rows_pad + j] = l;
      }
      if (!low_row) {
        if (j < n && c < m) V[j * ldv + c] = ((float)h + (float)l) / qv;
        if (j == 0) vscale[c] = c < m ? 1.0f / (qv * ldexpf(1.0f, pshift)) : 0.0f;
      } else if (j == 0) {
        vscale[c] = 0.0f;
      }
    }
  }
}

hipError_t vec_split_t(float* V, int64_t n, int64_t m, int64_t ldv, int64_t rows_pad, int64_t mpad,
                       float* colmax, int pshift, bool packed, _Float16* hi, _Float16* lo,
                       float* vscale, hipStream_t st) {
  if (packed && (m > 8 || mpad != 16)) return hipErrorInvalidValue;
  hipError_t e = fill_f32(colmax, m, 0.0f, st);
  if (e != hipSuccess) return e;
  const int64_t blocks = std::min<int64_t>(512, std::max<int64_t>(1, ceil_div(n, 256)));
  vec_colmax_kernel<<<blocks, 256, 0, st>>>(V, n, m, ldv, colmax);
  KRR_LAUNCH_CHECK();
  dim3 grid(ceil_div(rows_pad, 32), ceil_div(mpad, 32));
  vec_split_t_kernel<<<grid, 256, 0, st>>>(V, n, m, ldv, rows_pad, mpad, colmax, pshift,
                                           packed ? 1 : 0, hi, lo, vscale);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// Integer slices of the points for the FP64 product on int8 MFMA. This is the error-free
// splitting of a matrix product into products of short-integer matrices (Ozaki, Ogita,
// Oishi and Rump, 2012) in its fixed-point form: row i is scaled by 2^(46 - e_i), e_i the
// exponent with max_k |x_ik| < 2^e_i, and rounded to integers X_ik (exact for every element
// within 22 binades of the row maximum, since an FP32 value carries 24 bits); then
// X_ik = sum_a D_iak 256^(5 - a) with balanced digits D_iak in [-128, 127] (|D_i0k| <= 65).
// S[(row * 6 + a) * kp + k] = D_iak (int8, zero padded to kp and rows_pad),
// scale[row] = 2^(e_i - 46), nu[row] = sum_k x_ik^2 in FP64 (NaN if the row holds a
// non-finite value, so that it propagates as in the plain FP64 product).
__global__ __launch_bounds__(256) void prep_points_i8_kernel(const float* __restrict__ X,
                                                             int64_t n, int64_t d, int64_t ldx,
                                                             int64_t rows_pad, int64_t kp,
                                                             int8_t* __restrict__ S,
                                                             double* __restrict__ scale,
                                                             double* __restrict__ nu) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows_pad) return;
  float mx = 0.0f;
  double ss = 0.0;
  int bad = 0;
  for (int64_t k = lane; k < d; k += 64) {
    const float v = row < n ? X[row * ldx + k] : 0.0f;
    if (!isfinite(v)) bad = 1;
    mx = fmaxf(mx, fabsf(v));
    ss += (double)v * (double)v;
  }
  mx = wave_max(mx);
  ss = wave_sum(ss);
  bad = wave_max(bad);
  int e = 0;
  if (!bad && mx > 0.0f) frexpf(mx, &e);  // mx = f 2^e, f in [0.5, 1): every |x| < 2^e
  const double up = ldexp(1.0, OZ_BITS - e);
  for (int64_t k = lane; k < kp; k += 64) {
    const double v = (row < n && k < d && !bad) ? (double)X[row * ldx + k] : 0.0;
    long long q = (long long)rint(v * up);  // |q| < 2^46
    for (int a = OZ_SLICES - 1; a > 0; --a) {
      const long long dg = ((q + 128) & 255) - 128;  // q = dg (mod 256), dg in [-128, 127]
      S[(row * OZ_SLICES + a) * kp + k] = (int8_t)dg;
      q = (q - dg) >> 8;  // exact: q - dg is a multiple of 256
    }
    S[(row * OZ_SLICES) * kp + k] = (int8_t)q;
  }
  if (lane == 0) {
    scale[row] = ldexp(1.0, e - OZ_BITS);
    nu[row] = bad ? __builtin_nan("") : ss;
  }
}

hipError_t prep_points_i8(const float* X, int64_t n, int64_t d, int64_t ldx, int64_t rows_pad,
                          int8_t* S, double* scale, double* nu, hipStream_t st) {
  prep_points_i8_kernel<<<ceil_div(rows_pad, 4), 256, 0, st>>>(X, n, d, ldx, rows_pad, oz_kp(d),
                                                              S, scale, nu);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// Point copies for the large-d FP64 product: X64 (rows_pad x dp, zero padded; an FP32 copy
// holds the FP32 values exactly) and nu (rows_pad) formed in FP64.
template <typename T>
__global__ __launch_bounds__(256) void prep_points_f64_kernel(const float* __restrict__ X,
                                                              int64_t n, int64_t d, int64_t ldx,
                                                              int64_t rows_pad, int64_t dp,
                                                              T* __restrict__ X64,
                                                              double* __restrict__ nu) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows_pad) return;
  double s = 0.0;
  for (int64_t k = lane; k < dp; k += 64) {
    double v = (row < n && k < d) ? (double)X[row * ldx + k] : 0.0;
    X64[row * dp + k] = (T)v;  // exact for both types: v is an FP32 value
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) nu[row] = s;
}

// Same with the coordinates kept in FP32 (an exact copy, zero padded) for the large-d FP64
// product, which converts them on the fly; nu is still formed in FP64.
hipError_t prep_points_f64x(const float* X, int64_t n, int64_t d, int64_t ldx, int64_t rows_pad,
                            int64_t dp, float* X32, double* nu, hipStream_t st) {
  prep_points_f64_kernel<float><<<ceil_div(rows_pad, 4), 256, 0, st>>>(X, n, d, ldx, rows_pad,
                                                                       dp, X32, nu);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// V (FP64, n x m, ldv) -> FP32 (rows_pad x ldo), zero padded rows and columns.
__global__ void vec_to_f32_kernel(const double* __restrict__ V, int64_t n, int64_t m, int64_t ldv,
                                  int64_t rows_pad, int64_t ldo, float* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows_pad * ldo) return;
  int64_t i = e / ldo, c = e % ldo;
  out[e] = (i < n && c < m) ? (float)V[i * ldv + c] : 0.0f;
}

hipError_t vec_to_f32(const double* V, int64_t n, int64_t m, int64_t ldv, int64_t rows_pad,
                      int64_t ldo, float* out, hipStream_t st) {
  vec_to_f32_kernel<<<ceil_div(rows_pad * ldo, 256), 256, 0, st>>>(V, n, m, ldv, rows_pad, ldo,
                                                                   out);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// V (FP64) -> FP64 copy (rows_pad x ldo), zero padded.
__global__ void vec_pad_f64_kernel(const double* __restrict__ V, int64_t n, int64_t m, int64_t ldv,
                                   int64_t rows_pad, int64_t ldo, double* __restrict__ out) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows_pad * ldo) return;
  int64_t i = e / ldo, c = e % ldo;
  out[e] = (i < n && c < m) ? V[i * ldv + c] : 0.0;
}

hipError_t vec_pad_f64(const double* V, int64_t n, int64_t m, int64_t ldv, int64_t rows_pad,
                       int64_t ldo, double* out, hipStream_t st) {
  vec_pad_f64_kernel<<<ceil_div(rows_pad * ldo, 256), 256, 0, st>>>(V, n, m, ldv, rows_pad, ldo,
                                                                    out);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// ------------------------------------------------- generic operand splitting (GEMMs)
// max |src| over a rows x cols FP32 or FP64 matrix -> atomic max into *amax (starts at 0).
// Each wave takes whole rows (lanes along the row, so reads coalesce and no index division
// is needed; four loads per lane in flight); the waves' maxima meet in LDS and one atomic
// per block.
template <typename S>
__global__ __launch_bounds__(256) void absmax_kernel(const S* __restrict__ src, int64_t rows,
                                                     int64_t cols, int64_t ld, float* amax) {
  float m = 0.0f;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int64_t r = (int64_t)blockIdx.x * 4 + w; r < rows; r += (int64_t)gridDim.x * 4) {
    const S* row = src + r * ld;
    int64_t c = lane;
    for (; c + 192 < cols; c += 256) {  // four independent loads in flight per lane
      const S a = row[c], b = row[c + 64], d = row[c + 128], e = row[c + 192];
      m = fmaxf(fmaxf(m, (float)fabs((double)a)), (float)fabs((double)b));
      m = fmaxf(fmaxf(m, (float)fabs((double)d)), (float)fabs((double)e));
    }
    for (; c < cols; c += 64) m = fmaxf(m, (float)fabs((double)row[c]));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
  __shared__ float red[4];
  if (lane == 0) red[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) atomic_max_pos(amax, fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3])));
}

template <typename S>
hipError_t absmax(const S* src, int64_t rows, int64_t cols, int64_t ld, float* amax,
                  hipStream_t st) {
  int64_t blocks = std::min<int64_t>(2048, std::max<int64_t>(1, ceil_div(rows, 4)));
  absmax_kernel<S><<<blocks, 256, 0, st>>>(src, rows, cols, ld, amax);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
template hipError_t absmax<float>(const float*, int64_t, int64_t, int64_t, float*, hipStream_t);
template hipError_t absmax<double>(const double*, int64_t, int64_t, int64_t, float*, hipStream_t);

// dst (rows_pad x cols_pad, k contiguous) = split(q * src), q = split_scale(*amax).
// transpose = 0: dst[r][c] = src[r][c]; transpose = 1: dst[c][r] = src[r][c] (dst is
// cols_pad x rows_pad). Padding is zero. Block: 32 output rows x 64 output columns; each
// thread writes two adjacent columns (4-byte stores of the hi and lo pairs), so a wave's
// stores cover 128-byte row segments; the transposed case goes through a 64 x 32 LDS tile
// (rows of 33 floats: the column-pair reads hit distinct banks). cols_pad must be even.
template <typename S, typename T>
__global__ __launch_bounds__(256) void split_kernel(const S* __restrict__ src, int64_t rows,
                                                    int64_t cols, int64_t ld,
                                                    const float* __restrict__ amax, int transpose,
                                                    int64_t out_rows, int64_t out_cols,
                                                    T* __restrict__ hi, T* __restrict__ lo) {
  __shared__ float tile[64][33];
  const float q = split_scale(*amax);
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  const int64_t orow0 = (int64_t)blockIdx.y * 32, ocol0 = (int64_t)blockIdx.x * 64;
  auto put = [&](int64_t r, int64_t c, float v0, float v1) __attribute__((always_inline)) {
    T h0, l0, h1, l1;
    Elem<T>::split(v0, h0, l0);
    Elem<T>::split(v1, h1, l1);
    typedef T pair_t __attribute__((ext_vector_type(2)));
    *reinterpret_cast<pair_t*>(&hi[r * out_cols + c]) = pair_t{h0, h1};
    *reinterpret_cast<pair_t*>(&lo[r * out_cols + c]) = pair_t{l0, l1};
  };
  auto val = [&](int64_t sr, int64_t sc) __attribute__((always_inline)) {
    return (sr < rows && sc < cols) ? (float)((double)q * (double)src[sr * ld + sc]) : 0.0f;
  };
  if (!transpose) {
    for (int yy = ty; yy < 32; yy += 8) {
      const int64_t r = orow0 + yy, c = ocol0 + 2 * tx;
      if (r < out_rows && c < out_cols) put(r, c, val(r, c), val(r, c + 1));
    }
  } else {
    // source rows ocol0 .. ocol0 + 63 (output columns), source columns orow0 .. + 31
    for (int yy = ty; yy < 64; yy += 8) tile[yy][tx] = val(ocol0 + yy, orow0 + tx);
    __syncthreads();
    for (int yy = ty; yy < 32; yy += 8) {
      const int64_t r = orow0 + yy, c = ocol0 + 2 * tx;
      if (r < out_rows && c < out_cols) put(r, c, tile[2 * tx][yy], tile[2 * tx + 1][yy]);
    }
  }
}

template <typename S, typename T>
hipError_t split_operand(const S* src, int64_t rows, int64_t cols, int64_t ld, const float* amax,
                         int transpose, int64_t out_rows, int64_t out_cols, T* hi, T* lo,
                         hipStream_t st) {
  if (out_cols % 2) return hipErrorInvalidValue;
  dim3 grid(ceil_div(out_cols, 64), ceil_div(out_rows, 32));
  split_kernel<S, T><<<grid, 256, 0, st>>>(src, rows, cols, ld, amax, transpose, out_rows,
                                           out_cols, hi, lo);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
template hipError_t split_operand<float, _Float16>(const float*, int64_t, int64_t, int64_t,
                                                   const float*, int, int64_t, int64_t, _Float16*,
                                                   _Float16*, hipStream_t);
template hipError_t split_operand<double, _Float16>(const double*, int64_t, int64_t, int64_t,
                                                    const float*, int, int64_t, int64_t,
                                                    _Float16*, _Float16*, hipStream_t);

}  // namespace krr
