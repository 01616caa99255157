// Symmetric eigen-decomposition of a small Gram matrix G = C C^T (s x s, FP64) by one-sided
// Jacobi rotations on the rows of its Cholesky factor C (Hestenes' method): rotating pairs
// of rows until all rows are mutually orthogonal gives Vt C = W^T with orthogonal rows, so
// Vt G Vt^T = diag(||row_i||^2): the eigenvalues are the squared row norms and the
// eigenvectors the rows of Vt (the accumulated rotations). Working on C instead of G keeps
// small eigenvalues at the relative accuracy of C (the condition number is the square root
// of G's).
//
// One launch per round of the round-robin (circle) ordering: s/2 disjoint row pairs, one
// 256-thread block per pair, so rounds need no other synchronisation; s - 1 rounds form a
// sweep in which every pair meets once. Each block records the largest |cos| of the angle
// between its two rows for the sweep's convergence test.
#include <cstring>

#include "kernels.hpp"

namespace krr {

constexpr int JAC_THREADS = 256;

__device__ inline double block_sum3(double& a, double& b, double& c, double* red) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) { red[w] = a; red[4 + w] = b; red[8 + w] = c; }
  __syncthreads();
  a = red[0] + red[1] + red[2] + red[3];
  b = red[4] + red[5] + red[6] + red[7];
  c = red[8] + red[9] + red[10] + red[11];
  return a;
}

// Pair i of round r among sp (even) indices: index 0 stays, the others rotate on a circle.
__device__ inline void rr_pair(int r, int i, int sp, int& p, int& q) {
  const int m = sp - 1;
  if (i == 0) {
    p = 0;
    q = 1 + (r % m);
  } else {
    p = 1 + ((r + i) % m);
    q = 1 + ((r + m - i) % m);
  }
}

__global__ __launch_bounds__(JAC_THREADS) void jacobi_round_kernel(
    double* __restrict__ A, double* __restrict__ Vt, int s, int sp, int r,
    unsigned long long* __restrict__ off) {
  __shared__ double red[12];
  int p, q;
  rr_pair(r, blockIdx.x, sp, p, q);
  if (p >= s || q >= s) return;  // the padding index of an odd s
  double* ap = A + (int64_t)p * s;
  double* aq = A + (int64_t)q * s;
  double al = 0.0, be = 0.0, ga = 0.0;
  for (int k = threadIdx.x; k < s; k += JAC_THREADS) {
    const double x = ap[k], y = aq[k];
    al = fma(x, x, al);
    be = fma(y, y, be);
    ga = fma(x, y, ga);
  }
  block_sum3(al, be, ga, red);
  if (!(fabs(ga) > 0.0) || !(al > 0.0) || !(be > 0.0)) return;
  const double cosang = fabs(ga) / sqrt(al * be);
  if (threadIdx.x == 0) atomicMax(off, (unsigned long long)__double_as_longlong(cosang));
  if (cosang < 1e-300) return;
  const double z = (be - al) / (2.0 * ga);
  const double t = (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z));
  const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
  double* vp = Vt + (int64_t)p * s;
  double* vq = Vt + (int64_t)q * s;
  for (int k = threadIdx.x; k < s; k += JAC_THREADS) {
    const double x = ap[k], y = aq[k];
    ap[k] = c * x - sn * y;
    aq[k] = sn * x + c * y;
    const double u = vp[k], v = vq[k];
    vp[k] = c * u - sn * v;
    vq[k] = sn * u + c * v;
  }
}

// A (s x s, in: C, out: the rotated rows), Vt (s x s, out), ev (s, out: squared row norms).
// Returns the sweeps taken in *sweeps; stops when every pair's |cos| fell below tol in a
// sweep or after max_sweeps. off: one device word of scratch.
__global__ void jacobi_init_kernel(double* Vt, int s) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < (int64_t)s * s) Vt[e] = (e / s == e % s) ? 1.0 : 0.0;
}
__global__ void jacobi_rownorm_kernel(const double* __restrict__ A, int s, double* __restrict__ ev) {
  __shared__ double red[12];
  double a = 0.0, b = 0.0, c = 0.0;
  const double* row = A + (int64_t)blockIdx.x * s;
  for (int k = threadIdx.x; k < s; k += JAC_THREADS) a = fma(row[k], row[k], a);
  block_sum3(a, b, c, red);
  if (threadIdx.x == 0) ev[blockIdx.x] = a;
}
__global__ void zero_u64_kernel(unsigned long long* p) { *p = 0ull; }

hipError_t jacobi_eig(double* A, int s, double* Vt, double* ev, unsigned long long* off,
                      double tol, int max_sweeps, int* sweeps, hipStream_t st) {
  if (s < 1) return hipErrorInvalidValue;
  jacobi_init_kernel<<<ceil_div((int64_t)s * s, 256), 256, 0, st>>>(Vt, s);
  KRR_LAUNCH_CHECK();
  const int sp = s + (s & 1);
  int sw = 0;
  for (; sw < max_sweeps && s > 1; ++sw) {
    zero_u64_kernel<<<1, 1, 0, st>>>(off);
    KRR_LAUNCH_CHECK();
    for (int r = 0; r < sp - 1; ++r) {
      jacobi_round_kernel<<<sp / 2, JAC_THREADS, 0, st>>>(A, Vt, s, sp, r, off);
      KRR_LAUNCH_CHECK();
    }
    unsigned long long h = 0;
    hipError_t e = hipMemcpyAsync(&h, off, sizeof(h), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return e;
    double worst;
    memcpy(&worst, &h, sizeof(worst));
    if (!(worst > tol)) { ++sw; break; }
  }
  jacobi_rownorm_kernel<<<s, JAC_THREADS, 0, st>>>(A, s, ev);
  KRR_LAUNCH_CHECK();
  *sweeps = sw;
  return hipSuccess;
}

}  // namespace krr

namespace krr {

// ------------------------------------------------ pieces of the preconditioner test (Thm. 4)
// Bk[j][:] = Vt[idx[j]][:] * scale[j] (FP32): the kept eigenvectors of Z^T Z, scaled so that
// Z Bk^T has orthonormal columns (the eigenvectors of Z Z^T above the threshold).
__global__ void gather_scaled_rows_kernel(const double* __restrict__ Vt, int s,
                                          const int* __restrict__ idx,
                                          const double* __restrict__ scale, int k,
                                          float* __restrict__ Bk) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)k * s) return;
  const int j = (int)(e / s), c = (int)(e % s);
  Bk[e] = (float)(Vt[(int64_t)idx[j] * s + c] * scale[j]);
}
hipError_t gather_scaled_rows(const double* Vt, int s, const int* idx, const double* scale, int k,
                              float* Bk, hipStream_t st) {
  if (k <= 0) return hipSuccess;
  gather_scaled_rows_kernel<<<ceil_div((int64_t)k * s, 256), 256, 0, st>>>(Vt, s, idx, scale, k, Bk);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// y[c] = sum_i U[i][c] r[i] (U n x k FP32, ld), partial sums per block over row chunks:
// part[b][c]; one thread per column c within a block, rows strided by the grid.
__global__ __launch_bounds__(256) void gemv_t_partial_kernel(const float* __restrict__ U,
                                                             int64_t ldu, int64_t n, int k,
                                                             const double* __restrict__ r,
                                                             double* __restrict__ part) {
  const int64_t rows_per = ceil_div(n, (int64_t)gridDim.y);
  const int64_t i0 = (int64_t)blockIdx.y * rows_per;
  const int64_t i1 = i0 + rows_per < n ? i0 + rows_per : n;
  for (int c = blockIdx.x * 256 + threadIdx.x; c < k; c += gridDim.x * 256) {
    double acc = 0.0;
    for (int64_t i = i0; i < i1; ++i) acc = fma((double)U[i * ldu + c], r[i], acc);
    part[(int64_t)blockIdx.y * k + c] = acc;
  }
}
__global__ void sum_parts_kernel(const double* __restrict__ part, int nparts, int k,
                                 const double* __restrict__ w, double* __restrict__ y) {
  const int c = blockIdx.x * 256 + threadIdx.x;
  if (c >= k) return;
  double acc = 0.0;
  for (int b = 0; b < nparts; ++b) acc += part[(int64_t)b * k + c];
  y[c] = w ? acc * w[c] : acc;
}
constexpr int GEMV_PARTS = 128;
// y = diag(w) U^T r (w may be null); part: GEMV_PARTS x k doubles of scratch
hipError_t gemv_t(const float* U, int64_t ldu, int64_t n, int k, const double* r, const double* w,
                  double* y, double* part, hipStream_t st) {
  dim3 grid((unsigned)ceil_div(k, 256), GEMV_PARTS);
  gemv_t_partial_kernel<<<grid, 256, 0, st>>>(U, ldu, n, k, r, part);
  KRR_LAUNCH_CHECK();
  sum_parts_kernel<<<ceil_div(k, 256), 256, 0, st>>>(part, GEMV_PARTS, k, w, y);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
// r[i] = sum_c U[i][c] (w[c] x[c]) (w may be null): one wave per row
__global__ __launch_bounds__(256) void gemv_n_kernel(const float* __restrict__ U, int64_t ldu,
                                                     int64_t n, int k, const double* __restrict__ x,
                                                     const double* __restrict__ w,
                                                     double* __restrict__ r) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= n) return;
  double acc = 0.0;
  for (int c = lane; c < k; c += 64) acc = fma((double)U[i * ldu + c], w ? w[c] * x[c] : x[c], acc);
  acc = wave_sum(acc);
  if (lane == 0) r[i] = acc;
}
hipError_t gemv_n(const float* U, int64_t ldu, int64_t n, int k, const double* x, const double* w,
                  double* r, hipStream_t st) {
  gemv_n_kernel<<<ceil_div(n, 4), 256, 0, st>>>(U, ldu, n, k, x, w, r);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

// A deterministic start vector for the power iterations: v[i] = a hash of i in [-1, 1).
__global__ void hash_fill_kernel(double* v, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = (uint64_t)i + seed + 0x9E3779B97F4A7C15ull;  // SplitMix64 finaliser
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  v[i] = (double)(z >> 11) * (1.0 / 4503599627370496.0) - 1.0;  // [0, 2) - 1
}
hipError_t hash_fill(double* v, int64_t n, uint64_t seed, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hash_fill_kernel<<<ceil_div(n, 256), 256, 0, st>>>(v, n, seed);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}

}  // namespace krr

namespace krr {
// out = a x + b y (y may be null: out = a x)
__global__ void axpby_kernel(int64_t n, double a, const double* __restrict__ x, double b,
                             const double* __restrict__ y, double* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = y ? fma(a, x[i], b * y[i]) : a * x[i];
}
hipError_t axpby(int64_t n, double a, const double* x, double b, const double* y, double* out,
                 hipStream_t st) {
  if (n <= 0) return hipSuccess;
  axpby_kernel<<<ceil_div(n, 256), 256, 0, st>>>(n, a, x, b, y, out);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
}  // namespace krr

namespace krr {
// out (n x cols, ld cols) = FP64 copy of a (n x cols, lda) in FP32
__global__ void f32_to_f64_2d_kernel(const float* __restrict__ a, int64_t n, int64_t cols,
                                     int64_t lda, double* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n * cols) out[e] = (double)a[(e / cols) * lda + e % cols];
}
hipError_t f32_to_f64_2d(const float* a, int64_t n, int64_t cols, int64_t lda, double* out,
                         hipStream_t st) {
  if (n * cols <= 0) return hipSuccess;
  f32_to_f64_2d_kernel<<<ceil_div(n * cols, 256), 256, 0, st>>>(a, n, cols, lda, out);
  KRR_LAUNCH_CHECK();
  return hipSuccess;
}
}  // namespace krr
