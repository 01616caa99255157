// TensorSketch features for the polynomial kernel (Sec. 2.2; the feature map of Thm. 1).
//
// For the kernel (gamma x^T z + c)^q each point is augmented to x' = [sqrt(gamma) x, sqrt(c)]
// (one constant feature, as the remark after Thm. 1 suggests) and sketched to
//     phi(x') = IFFT( prod_k FFT( CountSketch_k(x') ) ),
// the circular convolution of q CountSketches with hashes h_k and signs g_k, which equals
// S v_q(x') for the TensorSketch matrix S (H = sum_k h_k(i_k) mod s, G = prod_k g_k(i_k)).
//
// One block of 256 threads per point. The FFT runs in LDS (complex FP32, radix 2,
// decimation in time, the CountSketch scattered straight into bit-reversed bins so no
// reordering pass is needed); the product of the q spectra is kept in registers, each
// thread owning the frequencies tid + 256 u; the inverse transform reuses the forward one
// with conjugated twiddles after a bit-reversed store of the product. s is a power of two,
// 2 <= s <= 8192.
#include "kernels.hpp"

namespace krr {

constexpr int TS_THREADS = 256;
constexpr int TS_MAX_LOG = 13;
constexpr int TS_SPT = (1 << TS_MAX_LOG) / TS_THREADS;  // frequencies per thread at s = 8192

__device__ inline int bitrev(int i, int logs) { return (int)(__brev((unsigned)i) >> (32 - logs)); }

// In-place radix-2 DIT FFT of bit-reversed input in (re, im); dir = -1 forward, +1 inverse
// (unnormalised). Twiddles exp(dir 2 pi i k / len) from sincospi (accurate FP32).
__device__ inline void lds_fft(float* re, float* im, int logs, float dir) {
  const int s = 1 << logs;
  for (int st = 1; st <= logs; ++st) {
    const int half = 1 << (st - 1);
    const float step = dir * 2.0f / (float)(2 * half);  // angle / pi per unit k
    for (int b = threadIdx.x; b < s / 2; b += TS_THREADS) {
      const int k = b & (half - 1);
      const int i0 = ((b >> (st - 1)) << st) + k;
      const int i1 = i0 + half;
      float sn, cs;
      sincospif(step * (float)k, &sn, &cs);
      const float xr = re[i1], xi = im[i1];
      const float tr = cs * xr - sn * xi, ti = cs * xi + sn * xr;
      const float ur = re[i0], ui = im[i0];
      re[i0] = ur + tr;
      im[i0] = ui + ti;
      re[i1] = ur - tr;
      im[i1] = ui - ti;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(TS_THREADS) void tensor_sketch_kernel(
    const float* __restrict__ X, int64_t n, int64_t d, int64_t ldx, float sg, float sc, int q,
    const int* __restrict__ hash, const float* __restrict__ sign, int logs, float* __restrict__ Z,
    int64_t ldz) {
  __shared__ float re[1 << TS_MAX_LOG];
  __shared__ float im[1 << TS_MAX_LOG];
  const int s = 1 << logs;
  const int tid = threadIdx.x;
  const int64_t row = blockIdx.x;
  const float* x = X + row * ldx;
  const int64_t da = d + 1;  // augmented length
  float ar[TS_SPT], ai[TS_SPT];
#pragma unroll
  for (int u = 0; u < TS_SPT; ++u) { ar[u] = 1.0f; ai[u] = 0.0f; }

  for (int k = 0; k < q; ++k) {
    for (int i = tid; i < s; i += TS_THREADS) { re[i] = 0.0f; im[i] = 0.0f; }
    __syncthreads();
    const int* hk = hash + (int64_t)k * da;
    const float* gk = sign + (int64_t)k * da;
    for (int64_t j = tid; j < da; j += TS_THREADS) {
      const float v = j < d ? sg * x[j] : sc;
      if (v != 0.0f) atomicAdd(&re[bitrev(hk[j] & (s - 1), logs)], gk[j] * v);
    }
    __syncthreads();
    lds_fft(re, im, logs, -1.0f);
#pragma unroll
    for (int u = 0; u < TS_SPT; ++u) {
      const int i = tid + TS_THREADS * u;
      if (i < s) {
        const float br = re[i], bi = im[i];
        const float nr = ar[u] * br - ai[u] * bi;
        ai[u] = ar[u] * bi + ai[u] * br;
        ar[u] = nr;
      }
    }
    __syncthreads();
  }
  // inverse transform of the product: bit-reversed store, conjugate twiddles, scale 1/s
#pragma unroll
  for (int u = 0; u < TS_SPT; ++u) {
    const int i = tid + TS_THREADS * u;
    if (i < s) {
      const int r = bitrev(i, logs);
      re[r] = ar[u];
      im[r] = ai[u];
    }
  }
  __syncthreads();
  lds_fft(re, im, logs, 1.0f);
  const float inv = 1.0f / (float)s;
  float* z = Z + row * ldz;
  for (int i = tid; i < s; i += TS_THREADS) z[i] = re[i] * inv;
}

hipError_t tensor_sketch(const float* X, int64_t n, int64_t d, int64_t ldx, double gamma,
                         double coef0, int q, const int* hash, const float* sign, int logs,
                         float* Z, int64_t ldz, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  if (logs < 1 || logs > TS_MAX_LOG) return hipErrorInvalidValue;
  tensor_sketch_kernel<<<n, TS_THREADS, 0, st>>>(X, n, d, ldx, (float)sqrt(gamma),
                                                 (float)sqrt(coef0), q, hash, sign, logs, Z, ldz);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace krr
