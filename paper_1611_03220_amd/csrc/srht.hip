// Second level of the multiple-level sketch of Alg. 2 (Sec. 4): a subsampled randomized
// Walsh-Hadamard transform applied to the rows of a first-level sketch Z_1,
//     Z_2 = Z_1 S_2^T,  S_2 = s_2^{-1/2} P H D  (Def. 2),
// with D the random signs, H the +-1 Walsh-Hadamard matrix of the recursion
// H_m = [[H, H], [H, -H]], P the sampled coordinates. A width s_1 that is not a power of two
// is zero-padded to the next one (zero columns leave Z_1 Z_1^T unchanged).
//
// One 256-thread block per row: the signed row is staged in LDS and transformed in place by
// the iterative fast transform (log2 s_1 stages of sum/difference butterflies, the
// Kronecker factors of H taken one bit at a time), then the sampled coordinates are
// gathered and scaled. FP32 throughout; s_1 (padded) <= 16384.
#include "kernels.hpp"

namespace krr {

constexpr int SRHT_THREADS = 256;
constexpr int SRHT_MAX = 16384;

__global__ __launch_bounds__(SRHT_THREADS) void srht_kernel(
    const float* __restrict__ Z1, int64_t s1, int64_t ldz1, const float* __restrict__ signs,
    int logp, const int* __restrict__ sample, int64_t s2, float scale, float* __restrict__ Z2,
    int64_t ldz2) {
  __shared__ float buf[SRHT_MAX];
  const int p = 1 << logp;
  const int tid = threadIdx.x;
  const int64_t row = blockIdx.x;
  const float* z = Z1 + row * ldz1;
  for (int j = tid; j < p; j += SRHT_THREADS) buf[j] = j < s1 ? z[j] * signs[j] : 0.0f;
  __syncthreads();
  for (int h = 1; h < p; h <<= 1) {
    for (int b = tid; b < p / 2; b += SRHT_THREADS) {
      const int i0 = ((b / h) * 2 * h) + (b % h);
      const int i1 = i0 + h;
      const float a = buf[i0], c = buf[i1];
      buf[i0] = a + c;
      buf[i1] = a - c;
    }
    __syncthreads();
  }
  float* out = Z2 + row * ldz2;
  for (int64_t t = tid; t < s2; t += SRHT_THREADS) out[t] = buf[sample[t] & (p - 1)] * scale;
}

hipError_t srht_rows(const float* Z1, int64_t n, int64_t s1, int64_t ldz1, const float* signs,
                     const int* sample, int64_t s2, float* Z2, int64_t ldz2, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int logp = 0;
  while ((int64_t(1) << logp) < s1) ++logp;
  if ((1 << logp) > SRHT_MAX || s2 < 1) return hipErrorInvalidValue;
  srht_kernel<<<n, SRHT_THREADS, 0, st>>>(Z1, s1, ldz1, signs, logp, sample, s2,
                                          (float)(1.0 / std::sqrt((double)s2)), Z2, ldz2);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace krr
