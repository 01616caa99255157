// Shared device/host definitions for libkrr (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace krr {

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

constexpr int WAVE = 64;

// Padding of the prepared point arrays: rows to a multiple of ROW_PAD, the contraction
// (feature) dimension to a multiple of K_STEP (one 16x16x32 MFMA step).
constexpr int ROW_PAD = 128;
constexpr int K_STEP = 32;
// Output tile of the split GEMMs; their operand rows are padded to a multiple of it.
constexpr int GEMM_TILE = 128;

__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Largest finite magnitude we let a scaled operand reach before the hi/lo split: the hi
// part must stay below the FP16 maximum (65504) with margin.
constexpr float SPLIT_TARGET = 16384.0f;

// ---------------------------------------------------------------- element traits
// Split a float into hi + lo of a 16-bit MFMA type: hi = rn(x), lo = rn(x - hi).
template <typename T> struct Elem;
template <> struct Elem<_Float16> {
  typedef half8 vec8;
  __device__ static inline void split(float x, _Float16& hi, _Float16& lo) {
    hi = (_Float16)x;
    lo = (_Float16)(x - (float)hi);
  }
  __device__ static inline f32x4 mfma(vec8 a, vec8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};
template <> struct Elem<__bf16> {
  typedef bf16x8 vec8;
  __device__ static inline void split(float x, __bf16& hi, __bf16& lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
  }
  __device__ static inline f32x4 mfma(vec8 a, vec8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// Scale of the point operands: 1 when the largest entry already lies in [2^-3, 2^14]
// (products then need no rescaling), else the power of two of split_scale.
__device__ inline float point_scale(float amax) {
  if (amax >= 0.125f && amax <= SPLIT_TARGET) return 1.0f;
  if (!(amax > 0.0f) || !(amax < 3.0e38f)) return 1.0f;
  int e;
  frexpf(SPLIT_TARGET / amax, &e);
  return ldexpf(1.0f, e - 1);
}

// Power of two q with q * amax <= SPLIT_TARGET (amax > 0 finite), else 1.
__device__ inline float split_scale(float amax) {
  if (!(amax > 0.0f) || !(amax < 3.0e38f)) return 1.0f;
  int e;
  frexpf(SPLIT_TARGET / amax, &e);  // SPLIT_TARGET/amax = f * 2^e, f in [0.5, 1)
  return ldexpf(1.0f, e - 1);
}

// Positive floats order like their bit patterns: atomic max through unsigned ints.
__device__ inline void atomic_max_pos(float* addr, float v) {
  if (v > 0.0f) atomicMax(reinterpret_cast<unsigned int*>(addr), __float_as_uint(v));
}

// s_waitcnt vmcnt(0): wait for all outstanding vector memory loads (gfx9 encoding, expcnt
// and lgkmcnt left at their maxima). Issued before a loop, it keeps loads of the prologue
// from reaching the loop as pending, which would make the compiler's wait counts inside
// the loop stall on the loop's own prefetch.
__device__ inline void wait_vmem_all() { __builtin_amdgcn_s_waitcnt(0x0F70); }

template <typename T> __device__ inline T wave_sum(T v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <typename T> __device__ inline T wave_max(T v) {
  for (int o = 32; o > 0; o >>= 1) {
    const T u = __shfl_xor(v, o, 64);
    v = u > v ? u : v;
  }
  return v;
}

// Exact int8 slices of the points for the FP64 product on int8 MFMA: OZ_SLICES balanced
// base-256 digits of a 46-bit fixed-point form of each row, OZ_KC(d) chunks of 64 bytes
// per slice.
constexpr int OZ_SLICES = 6;
constexpr int OZ_BITS = 46;
__host__ __device__ inline int64_t oz_kp(int64_t d) { return round_up(d, 64); }

}  // namespace krr

// ------------------------------------------------------------------ host helpers
#define KRR_LAUNCH_CHECK()                                    \
  do {                                                        \
    hipError_t e_ = hipGetLastError();                        \
    if (e_ != hipSuccess) return e_;                          \
  } while (0)
