// Shared device/host helpers for the CRL kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace crl {

typedef uint16_t bf16_t;  // BF16 bit pattern
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));  // 16-byte register vector

constexpr int kWave = 64;

// FP32 -> BF16 round to nearest even (NaN kept quiet).
__host__ __device__ inline bf16_t f2bf(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (bf16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (bf16_t)(u >> 16);
}
__host__ __device__ inline float bf2f(bf16_t h) {
  return __builtin_bit_cast(float, (uint32_t)h << 16);
}

// Storage-type traits: float or BF16 (stored as bf16_t).
template <typename T> struct Store;
template <> struct Store<float> {
  __device__ static inline float to_f(float x) { return x; }
  __device__ static inline float from_f(float x) { return x; }
};
template <> struct Store<bf16_t> {
  __device__ static inline float to_f(bf16_t x) { return bf2f(x); }
  __device__ static inline bf16_t from_f(float x) { return f2bf(x); }
};

// Butterfly sum / max over the 64 lanes of a wavefront.
__device__ inline float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

// Merge of two online log-sum-exp states (m, s) meaning log(s) + m, s >= 0.
__device__ inline void lse_merge(float& m, float& s, float m2, float s2) {
  if (s2 == 0.f) return;
  if (s == 0.f) { m = m2; s = s2; return; }
  if (m2 > m) { s = s * __expf(m - m2) + s2; m = m2; }
  else        { s = s + s2 * __expf(m2 - m); }
}

__device__ inline float sigmoidf_(float y) { return 1.f / (1.f + __expf(-y)); }

}  // namespace crl
