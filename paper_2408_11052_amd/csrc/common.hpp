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

// FP32 -> BF16, round to nearest even: the hardware conversion
// (v_cvt_pk_bf16_f32 on gfx950; NaN stays NaN).
__device__ inline bf16_t f2bf(float f) {
  return __builtin_bit_cast(bf16_t, (__bf16)f);
}
// Two values packed low/high into one 32-bit word: one v_cvt_pk_bf16_f32 (the
// two-element vector conversion; two scalar conversions would take four
// instructions with the shift and the merge).
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ inline uint32_t pack2bf(float lo, float hi) {
  const f32x2_t f = {lo, hi};
  return __builtin_bit_cast(uint32_t, __builtin_convertvector(f, bf16x2_t));
}
__device__ inline float bf2f(bf16_t h) {
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
// Sum over the wavefront for code where all 64 lanes are active: a butterfly
// inside each 16-lane row by DPP moves (pairs within quads, then the half-row
// and row mirrors), then the four row sums read out of lanes 0, 16, 32 and 48
// and added in a fixed order.  Every lane gets the same bits; no LDS traffic.
template <int CTRL> __device__ __forceinline__ float dpp_mov(float v) {
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), CTRL,
                                                               0xF, 0xF, false));
}
__device__ __forceinline__ float wave_sum_full(float v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror
  const int u = __builtin_bit_cast(int, v);
  const float a = __builtin_bit_cast(float, __builtin_amdgcn_readlane(u, 0));
  const float b = __builtin_bit_cast(float, __builtin_amdgcn_readlane(u, 16));
  const float c = __builtin_bit_cast(float, __builtin_amdgcn_readlane(u, 32));
  const float d = __builtin_bit_cast(float, __builtin_amdgcn_readlane(u, 48));
  return (a + b) + (c + d);
}
__device__ inline float wave_max(float v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
  return v;
}

// Merge of two online log-sum-exp states (m, s) meaning log(s) + m, s >= 0
// (s == 0: empty).  Branch-free: the larger max keeps its sum exactly
// (exp(0) = 1), the other is scaled down; an empty state contributes 0.
__device__ inline void lse_merge(float& m, float& s, float m2, float s2) {
  const float mn = s2 == 0.f ? m : (s == 0.f ? m2 : fmaxf(m, m2));
  const float a = s == 0.f ? 0.f : s * __expf(m - mn);
  const float b = s2 == 0.f ? 0.f : s2 * __expf(m2 - mn);
  s = a + b;
  m = mn;
}

// The L2 distance from the norm expansion d^2 = |x|^2 + |y|^2 - 2 <x, y>.
// Below 2^-14 (|x|^2 + |y|^2) the expansion's value is rounding noise of the
// product and the norms (an FP32 sum over up to 256 terms errs by about
// 2^-18 of them), so the distance is taken as 0 there: the energy is 0 and
// its subgradient, scaled by 1/d, is 0 too.  Both tests are written so that
// a NaN operand fails them and stays NaN (the loss then reports it).
constexpr float kL2Floor = 1.f / 16384.f;
__device__ __forceinline__ float l2_dist(float nx, float ny, float v) {
  const float d2 = nx + ny - 2.f * v;
  return d2 <= kL2Floor * (nx + ny) ? 0.f : sqrtf(d2);
}
// The squared distance from the same expansion, clamped at 0 (NaN kept).
__device__ __forceinline__ float l2sq_dist(float nx, float ny, float v) {
  const float d2 = nx + ny - 2.f * v;
  return d2 < 0.f ? 0.f : d2;
}

// logistic function with the hardware reciprocal (about 1 ulp)
__device__ inline float sigmoidf_(float y) { return __builtin_amdgcn_rcpf(1.f + __expf(-y)); }


// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): 10 rounds of two 64x64->128 products,
// key bumped by the Weyl constants between rounds.
// ---------------------------------------------------------------------------
__device__ inline void philox4x64_10(uint64_t (&x)[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += W0; k1 += W1; }
    uint64_t lo0 = M0 * x[0], hi0 = __umul64hi(M0, x[0]);
    uint64_t lo1 = M1 * x[2], hi1 = __umul64hi(M1, x[2]);
    uint64_t y0 = hi1 ^ x[1] ^ k0;
    uint64_t y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0; x[1] = lo1; x[2] = y2; x[3] = lo0;
  }
}

// Compensated (Kahan) summation step.
__device__ inline void kahan_add(float& s, float& comp, float x) {
  float y = x - comp;
  float t = s + y;
  comp = (t - s) - y;
  s = t;
}

}  // namespace crl
