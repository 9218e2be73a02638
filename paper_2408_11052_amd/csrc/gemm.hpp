// MFMA GEMM for the encoder layers and the logit products (gfx950).
//
// C[M][N] = epilogue(alpha * A[M][K] . B[K][N]) for up to two independent
// problems per launch (the phi and psi encoders run side by side).
//
// Operands are either "KC" (the contraction index is contiguous:
// A(m,k) = A[m*lda + k], B(k,n) = B[n*ldb + k]) or "MC" (the row/column index
// is contiguous: A(m,k) = A[k*lda + m], B(k,n) = B[k*ldb + n]).  Tiles are
// staged through LDS in one layout, [row][k] with a 16-byte pad, so that every
// MFMA operand fragment is one 16-byte LDS read; MC operands are transposed on
// the way in (4 k-rows per thread, repacked in registers).
//
// Tile: 128 x 128 per workgroup of 256 threads (4 waves, 2 x 2), 64 x 64 per
// wave as 4 x 4 MFMA 16x16 blocks.  K step: 128 bytes of each row per stage
// (64 BF16 or 32 FP32), double-buffered in LDS with one barrier per stage;
// global loads run two steps ahead through two register sets.
//   BF16: v_mfma_f32_16x16x32_bf16, FP32 accumulation.
//   FP32: v_mfma_f32_16x16x4_f32.
#pragma once

#include "common.hpp"

namespace crl {

enum : int { LAY_KC = 0, LAY_MC = 1 };
enum : int {
  EPI_NONE = 0,      // v
  EPI_BIAS = 1,      // v + bias[n]
  EPI_BIAS_RELU = 2, // max(v + bias[n], 0)
  EPI_MASK_POS = 3,  // aux(m,n) > 0 ? v : 0      (ReLU backward)
  EPI_L2 = 4,        // -l2_dist(rowv[m], colv[n], v)
  EPI_L2SQ = 5       // -l2sq_dist(rowv[m], colv[n], v)
};

struct GemmDesc {
  const void* A;
  const void* B;
  void* C;
  const float* bias;
  const void* aux;    // same storage type and leading dim as C
  const float* rowv;
  const float* colv;
  int M, N, K;
  int lda, ldb, ldc;
  int epi;
  float alpha;
  int accumulate;     // C += result (read-modify-write of C)
  int kb;             // rows k < kb of an MC-layout B exist (0: all K).  The
                      // direct-to-LDS kernel re-reads row kb-1 for k >= kb;
                      // the caller guarantees A is zero in those columns
};

constexpr int kGemmMaxGroup = 2;
constexpr int kBM = 128, kBN = 128, kGemmThreads = 256;

struct GemmParams {
  GemmDesc d[kGemmMaxGroup];
  int count;
  int tiles_n[kGemmMaxGroup];
  int tiles[kGemmMaxGroup];
  int splits;          // split-K factor (>= 1)
  int k_chunk;         // K range per split (multiple of the K step)
  float* partial;      // splits > 1: partial[g][s][M][N] (FP32, no epilogue)
  int64_t partial_len; // floats per problem in `partial`
  int defer_reduce;    // splits > 1: leave the partials for a later reduction
  int frag;            // with defer_reduce: the direct-to-LDS kernel stores the
                       // partials in fragment order (see frag_partial_floats)
};

// Work item (tile, split, problem) of a workgroup.  Workgroups are dealt to
// the 8 XCDs round-robin by linear id; the linear id is remapped so that each
// XCD gets one contiguous eighth of the (problem, split, tile) order -- a run
// of tiles sharing one K range of one problem, whose operand panels then stay
// in that XCD's L2.
struct WorkItem { int tile, split, prob; };
// lin = launch-order id within a grid of gx tiles x gy splits x problems
// (total ids), whose first id sits on XCD 0
__device__ __forceinline__ WorkItem work_item_of(int lin, int gx, int gy, int total) {
  if ((total & 7) == 0) lin = (lin & 7) * (total >> 3) + (lin >> 3);
  WorkItem w;
  w.tile = lin % gx;
  w.split = (lin / gx) % gy;
  w.prob = lin / (gx * gy);
  return w;
}
__device__ __forceinline__ WorkItem gemm_work_item() {
  const int gx = gridDim.x, gy = gridDim.y;
  return work_item_of(blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z), gx, gy,
                      gx * gy * gridDim.z);
}

template <typename T> struct GemmCfg;
template <> struct GemmCfg<bf16_t> { static constexpr int BK = 64, VEC = 8; };
template <> struct GemmCfg<float> { static constexpr int BK = 32, VEC = 4; };

// ---------------------------------------------------------------------------
// global -> register staging
// ---------------------------------------------------------------------------
template <typename T> struct Vec16 { T e[16 / sizeof(T)]; };
struct Words4 { uint32_t w[4]; };
struct Floats4 { float f[4]; };

template <typename T>
__device__ __forceinline__ u32x4 load_vec_guarded(const T* base, int64_t off, int valid) {
  // `valid` = number of in-range elements of the VEC-wide vector at base+off
  constexpr int VEC = GemmCfg<T>::VEC;
  if (valid >= VEC) return *reinterpret_cast<const u32x4*>(base + off);
  Vec16<T> t;
#pragma unroll
  for (int i = 0; i < VEC; ++i) t.e[i] = (i < valid) ? base[off + i] : T(0);
  return __builtin_bit_cast(u32x4, t);
}

// KC operand tile: rows [r0, r0+128), k [k0, k0+BK).  4 vectors per thread.
// FAST: the whole tile is in range (no guards, straight-line vector loads).
template <typename T, bool FAST>
__device__ __forceinline__ void load_kc(u32x4 (&reg)[4], const T* __restrict__ X, int ld,
                               int r0, int R, int k0, int kend, int tid) {
  constexpr int VEC = GemmCfg<T>::VEC;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int v = tid + i * kGemmThreads;
    int row = v >> 3, c = v & 7;
    int gr = r0 + row, gk = k0 + c * VEC;
    if (FAST) {
      reg[i] = *reinterpret_cast<const u32x4*>(X + (int64_t)gr * ld + gk);
    } else {
      int valid = (gr < R) ? min(VEC, kend - gk) : 0;
      reg[i] = load_vec_guarded<T>(X, (int64_t)gr * ld + gk, valid);
    }
  }
}

// MC operand tile: k-rows [k0, k0+BK), row/col index [r0, r0+128).
// Thread (q, mv) loads k-rows 4q..4q+3 at columns mv*VEC..+VEC.
template <typename T, bool FAST>
__device__ __forceinline__ void load_mc(u32x4 (&reg)[4], const T* __restrict__ X, int ld,
                               int r0, int R, int k0, int kend, int tid) {
  constexpr int BK = GemmCfg<T>::BK, VEC = GemmCfg<T>::VEC;
  constexpr int QN = BK / 4;
  int q = tid % QN, mv = tid / QN;
  int gm = r0 + mv * VEC;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    int gk = k0 + 4 * q + j;
    if (FAST) {
      reg[j] = *reinterpret_cast<const u32x4*>(X + (int64_t)gk * ld + gm);
    } else {
      int valid = (gk < kend) ? min(VEC, R - gm) : 0;
      reg[j] = load_vec_guarded<T>(X, (int64_t)gk * ld + gm, valid);
    }
  }
}

// LDS row stride in elements: 128 data bytes + 16 pad bytes.
template <typename T> constexpr int lds_ld() { return (128 + 16) / (int)sizeof(T); }

template <typename T>
__device__ __forceinline__ void store_kc(T* __restrict__ S, const u32x4 (&reg)[4], int tid) {
  constexpr int VEC = GemmCfg<T>::VEC, LD = lds_ld<T>();
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int v = tid + i * kGemmThreads;
    int row = v >> 3, c = v & 7;
    *reinterpret_cast<u32x4*>(S + row * LD + c * VEC) = reg[i];
  }
}

__device__ __forceinline__ void store_mc(bf16_t* __restrict__ S, const u32x4 (&reg)[4], int tid) {
  constexpr int LD = lds_ld<bf16_t>();
  constexpr int QN = GemmCfg<bf16_t>::BK / 4;  // 16
  int q = tid % QN, mv = tid / QN;
  const Words4 w0 = __builtin_bit_cast(Words4, reg[0]);
  const Words4 w1 = __builtin_bit_cast(Words4, reg[1]);
  const Words4 w2 = __builtin_bit_cast(Words4, reg[2]);
  const Words4 w3 = __builtin_bit_cast(Words4, reg[3]);
#pragma unroll
  for (int d = 0; d < 4; ++d) {
    // elements 2d (low halves) and 2d+1 (high halves) of each k-row
    uint2 lo, hi;
    lo.x = (w0.w[d] & 0xffffu) | (w1.w[d] << 16);
    lo.y = (w2.w[d] & 0xffffu) | (w3.w[d] << 16);
    hi.x = (w0.w[d] >> 16) | (w1.w[d] & 0xffff0000u);
    hi.y = (w2.w[d] >> 16) | (w3.w[d] & 0xffff0000u);
    int m = mv * 8 + 2 * d;
    *reinterpret_cast<uint2*>(S + m * LD + 4 * q) = lo;
    *reinterpret_cast<uint2*>(S + (m + 1) * LD + 4 * q) = hi;
  }
}

__device__ __forceinline__ void store_mc(float* __restrict__ S, const u32x4 (&reg)[4], int tid) {
  constexpr int LD = lds_ld<float>();
  constexpr int QN = GemmCfg<float>::BK / 4;  // 8
  int q = tid % QN, mv = tid / QN;
  const Floats4 r0 = __builtin_bit_cast(Floats4, reg[0]);
  const Floats4 r1 = __builtin_bit_cast(Floats4, reg[1]);
  const Floats4 r2 = __builtin_bit_cast(Floats4, reg[2]);
  const Floats4 r3 = __builtin_bit_cast(Floats4, reg[3]);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    float4 v = make_float4(r0.f[i], r1.f[i], r2.f[i], r3.f[i]);
    *reinterpret_cast<float4*>(S + (mv * 4 + i) * LD + 4 * q) = v;
  }
}

// ---------------------------------------------------------------------------
// MFMA inner product over one LDS stage
// ---------------------------------------------------------------------------
__device__ __forceinline__ void mma_stage(floatx4 (&acc)[4][4], const bf16_t* __restrict__ As,
                                 const bf16_t* __restrict__ Bs, int wm, int wn, int lane) {
  constexpr int LD = lds_ld<bf16_t>();
  int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    bf16x8 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = *reinterpret_cast<const bf16x8*>(As + (wm * 64 + i * 16 + r16) * LD + g * 16 + h * 8);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(Bs + (wn * 64 + j * 16 + r16) * LD + g * 16 + h * 8);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
  }
}

__device__ __forceinline__ void mma_stage(floatx4 (&acc)[4][4], const float* __restrict__ As,
                                 const float* __restrict__ Bs, int wm, int wn, int lane) {
  constexpr int LD = lds_ld<float>();
  int r16 = lane & 15, g = lane >> 4;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float4 a[4], b[4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = *reinterpret_cast<const float4*>(As + (wm * 64 + i * 16 + r16) * LD + g * 8 + h * 4);
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *reinterpret_cast<const float4*>(Bs + (wn * 64 + j * 16 + r16) * LD + g * 8 + h * 4);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].x, b[j].x, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].y, b[j].y, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].z, b[j].z, acc[i][j], 0, 0, 0);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i].w, b[j].w, acc[i][j], 0, 0, 0);
      }
  }
}

// 8 consecutive values as FP32, from/to FP32 or BF16 storage (16-byte aligned)
__device__ inline void load8_any(const float* p, float (&o)[8]) {
  *reinterpret_cast<float4*>(o) = *reinterpret_cast<const float4*>(p);
  *reinterpret_cast<float4*>(o + 4) = *reinterpret_cast<const float4*>(p + 4);
}
__device__ inline void load8_any(const bf16_t* p, float (&o)[8]) {
  u32x4 u = *reinterpret_cast<const u32x4*>(p);
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    o[2 * i] = __builtin_bit_cast(float, w[i] << 16);
    o[2 * i + 1] = __builtin_bit_cast(float, w[i] & 0xffff0000u);
  }
}
__device__ inline void store8_any(float* p, const float (&o)[8]) {
  *reinterpret_cast<float4*>(p) = *reinterpret_cast<const float4*>(o);
  *reinterpret_cast<float4*>(p + 4) = *reinterpret_cast<const float4*>(o + 4);
}
__device__ inline void store8_any(bf16_t* p, const float (&o)[8]) {
  u32x4 u;
  u.x = pack2bf(o[0], o[1]);
  u.y = pack2bf(o[2], o[3]);
  u.z = pack2bf(o[4], o[5]);
  u.w = pack2bf(o[6], o[7]);
  *reinterpret_cast<u32x4*>(p) = u;
}

template <bool B> struct BoolTag { static constexpr bool value = B; };

// K loop.  Two register sets: tile t is fetched into set t&1 two steps
// before it is consumed (one full step of MFMA work between the load and the
// LDS store that waits for it).  LDS is double-buffered with one barrier per step.  All
// register arrays are indexed with constants so they stay in VGPRs.
template <typename T, int LA, int LB, bool FAST>
__device__ __forceinline__ void gemm_mainloop(floatx4 (&acc)[4][4], T* __restrict__ smem,
                                              const GemmDesc& D, int m0, int n0, int kbeg,
                                              int kend, int tid, int wm, int wn, int lane) {
  constexpr int BK = GemmCfg<T>::BK;
  constexpr int LD = lds_ld<T>();
  constexpr int STAGE = (kBM + kBN) * LD;
  const T* __restrict__ A = reinterpret_cast<const T*>(D.A);
  const T* __restrict__ B = reinterpret_cast<const T*>(D.B);
  const int nk = (kend > kbeg) ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk == 0) return;
#define CRL_GLOAD(ra, rb, k0)                                                    \
  do {                                                                           \
    if (LA == LAY_KC) load_kc<T, FAST>(ra, A, D.lda, m0, D.M, (k0), kend, tid);  \
    else              load_mc<T, FAST>(ra, A, D.lda, m0, D.M, (k0), kend, tid);  \
    if (LB == LAY_KC) load_kc<T, FAST>(rb, B, D.ldb, n0, D.N, (k0), kend, tid);  \
    else              load_mc<T, FAST>(rb, B, D.ldb, n0, D.N, (k0), kend, tid);  \
  } while (0)
#define CRL_SSTORE(ra, rb, buf)                                                  \
  do {                                                                           \
    T* As_ = smem + (buf) * STAGE;                                               \
    T* Bs_ = As_ + kBM * LD;                                                     \
    if (LA == LAY_KC) store_kc<T>(As_, ra, tid); else store_mc(As_, ra, tid);    \
    if (LB == LAY_KC) store_kc<T>(Bs_, rb, tid); else store_mc(Bs_, rb, tid);    \
  } while (0)
  // rac/rbc held tile kt (already in LDS) and now receive tile kt+2;
  // ran/rbn hold tile kt+1, which goes to the other LDS buffer.
#define CRL_STEP(kt, rac, rbc, ran, rbn)                                         \
  do {                                                                           \
    CRL_GLOAD(rac, rbc, kbeg + ((kt) + 2) * BK);                                 \
    const T* As_ = smem + ((kt) & 1) * STAGE;                                    \
    mma_stage(acc, As_, As_ + kBM * LD, wm, wn, lane);                           \
    CRL_SSTORE(ran, rbn, ((kt) + 1) & 1);                                        \
    __syncthreads();                                                             \
  } while (0)
  // the last two steps fetch nothing; the last one stores nothing
#define CRL_STEP_NOLOAD(kt, ran, rbn)                                            \
  do {                                                                           \
    const T* As_ = smem + ((kt) & 1) * STAGE;                                    \
    mma_stage(acc, As_, As_ + kBM * LD, wm, wn, lane);                           \
    CRL_SSTORE(ran, rbn, ((kt) + 1) & 1);                                        \
    __syncthreads();                                                             \
  } while (0)
  // the closing barrier lets the epilogue reuse the stage buffers
#define CRL_STEP_LAST(kt)                                                        \
  do {                                                                           \
    const T* As_ = smem + ((kt) & 1) * STAGE;                                    \
    mma_stage(acc, As_, As_ + kBM * LD, wm, wn, lane);                           \
    __syncthreads();                                                             \
  } while (0)
  u32x4 ra0[4], rb0[4], ra1[4], rb1[4];
  CRL_GLOAD(ra0, rb0, kbeg);
  if (nk == 1) {
    CRL_SSTORE(ra0, rb0, 0);
    __syncthreads();
    CRL_STEP_LAST(0);
    return;
  }
  CRL_GLOAD(ra1, rb1, kbeg + BK);
  CRL_SSTORE(ra0, rb0, 0);
  __syncthreads();
  // Steady state in pairs, with every step fetching and storing.  The loop
  // has a single back edge with the same loads in flight as on entry (tile
  // kt+1 in set 1), so the compiler's wait before each LDS store covers
  // only the older register set and never the loads just issued.
  int kt = 0;
  for (; kt + 3 < nk; kt += 2) {
    CRL_STEP(kt, ra0, rb0, ra1, rb1);
    CRL_STEP(kt + 1, ra1, rb1, ra0, rb0);
  }
  // 2 or 3 steps remain; set 1 holds tile kt+1
  if (kt + 2 < nk) {
    CRL_STEP(kt, ra0, rb0, ra1, rb1);        // fetches the last tile kt+2
    CRL_STEP_NOLOAD(kt + 1, ra0, rb0);
    CRL_STEP_LAST(kt + 2);
  } else {
    CRL_STEP_NOLOAD(kt, ra1, rb1);
    CRL_STEP_LAST(kt + 1);
  }
#undef CRL_STEP_LAST
#undef CRL_STEP_NOLOAD
#undef CRL_STEP
#undef CRL_SSTORE
#undef CRL_GLOAD
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
template <typename T, int LA, int LB, typename OutT>
__global__ __launch_bounds__(kGemmThreads) __attribute__((amdgpu_waves_per_eu(2, 2)))
void gemm_kernel(GemmParams P) {
  constexpr int BK = GemmCfg<T>::BK;
  constexpr int LD = lds_ld<T>();
  constexpr int STAGE = (kBM + kBN) * LD;
  __shared__ __attribute__((aligned(16))) T smem[2 * STAGE];
  static_assert(sizeof(T) * 2 * STAGE >= sizeof(float) * kBM * (kBN + 4),
                "the epilogue tile must fit in the stage buffers");

  const WorkItem wi = gemm_work_item();
  const int g = wi.prob;
  const GemmDesc& D = P.d[g];
  const int ntile = P.tiles[g];
  const int pid = wi.tile;
  if (pid >= ntile) return;
  const int tm = pid / P.tiles_n[g], tn = pid % P.tiles_n[g];
  const int m0 = tm * kBM, n0 = tn * kBN;
  const int kbeg = wi.split * P.k_chunk;
  const int kend = min(D.K, kbeg + P.k_chunk);

  const T* __restrict__ A = reinterpret_cast<const T*>(D.A);
  const T* __restrict__ B = reinterpret_cast<const T*>(D.B);
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int wm = wid >> 1, wn = wid & 1;

  floatx4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  // Workgroups whose tile lies entirely inside M x N, with a K range made of
  // whole K steps, run the unguarded loop; the others run the guarded one.
  // The choice is made once per workgroup, so each loop is straight-line code
  // and the compiler can wait for exactly the loads each LDS store needs.
  const bool fast = (m0 + kBM <= D.M) && (n0 + kBN <= D.N) && ((kend - kbeg) % BK == 0);
  if (fast) gemm_mainloop<T, LA, LB, true>(acc, smem, D, m0, n0, kbeg, kend, tid, wm, wn, lane);
  else      gemm_mainloop<T, LA, LB, false>(acc, smem, D, m0, n0, kbeg, kend, tid, wm, wn, lane);

  // Epilogue.  Row/column-only operations (scale, bias, ReLU, L2) are applied
  // in registers; the 128 x 128 FP32 tile is then staged through LDS so that
  // global memory sees 16-byte row-contiguous stores (and 16-byte reads of
  // aux / C where the epilogue needs them).
  // Lane holds rows 4*(lane/16)+r, column lane%16 of each 16x16 MFMA block.
  const int r16 = lane & 15, gq = lane >> 4;
  float* Cs = reinterpret_cast<float*>(smem);  // [128][kLdc], fits in the stage buffers
  constexpr int kLdc = kBN + 4;
  const bool split = P.splits > 1;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int cl = wn * 64 + j * 16 + r16;
      const int col = n0 + cl;
      float bcol = 0.f, ccol = 0.f;
      if (!split && col < D.N) {
        if (D.epi == EPI_BIAS || D.epi == EPI_BIAS_RELU) bcol = D.bias[col];
        if (D.epi == EPI_L2 || D.epi == EPI_L2SQ) ccol = D.colv[col];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = wm * 64 + i * 16 + gq * 4 + r;
        float v = acc[i][j][r];
        if (!split) {
          v *= D.alpha;
          if (D.epi == EPI_BIAS) v += bcol;
          else if (D.epi == EPI_BIAS_RELU) v = fmaxf(v + bcol, 0.f);
          else if (D.epi == EPI_L2 || D.epi == EPI_L2SQ) {
            const int row = m0 + rl;
            const float rv = row < D.M ? D.rowv[row] : 0.f;
            v = D.epi == EPI_L2 ? -l2_dist(rv, ccol, v) : -l2sq_dist(rv, ccol, v);
          }
        }
        Cs[rl * kLdc + cl] = v;
      }
    }
  __syncthreads();
  // 128 rows x 16 chunks of 8 values; thread t handles chunk (t & 15) of rows
  // t/16, t/16 + 16, ...
  const int ch = tid & 15;
  const int col0 = n0 + ch * 8;
  if (split) {
    float* out = P.partial + (int64_t)g * P.partial_len + (int64_t)wi.split * D.M * D.N;
    const bool vec = (D.N % 4 == 0) && (col0 + 8 <= D.N);
    for (int rl = tid >> 4; rl < kBM; rl += 16) {
      const int row = m0 + rl;
      if (row >= D.M) break;
      const float* src = Cs + rl * kLdc + ch * 8;
      float* dst = out + (int64_t)row * D.N + col0;
      if (vec) {
        *reinterpret_cast<float4*>(dst) = *reinterpret_cast<const float4*>(src);
        *reinterpret_cast<float4*>(dst + 4) = *reinterpret_cast<const float4*>(src + 4);
      } else {
        for (int k = 0; k < 8; ++k)
          if (col0 + k < D.N) dst[k] = src[k];
      }
    }
    return;
  }
  OutT* __restrict__ C = reinterpret_cast<OutT*>(D.C);
  const OutT* __restrict__ aux = reinterpret_cast<const OutT*>(D.aux);
  const bool vec = (D.N % 8 == 0) && (D.ldc % 8 == 0) && (col0 + 8 <= D.N);
  for (int rl = tid >> 4; rl < kBM; rl += 16) {
    const int row = m0 + rl;
    if (row >= D.M) break;
    const float* src = Cs + rl * kLdc + ch * 8;
    const int64_t o = (int64_t)row * D.ldc + col0;
    if (vec) {
      float v[8];
      *reinterpret_cast<float4*>(v) = *reinterpret_cast<const float4*>(src);
      *reinterpret_cast<float4*>(v + 4) = *reinterpret_cast<const float4*>(src + 4);
      if (D.epi == EPI_MASK_POS) {
        float a8[8];
        load8_any(aux + o, a8);
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] = a8[k] > 0.f ? v[k] : 0.f;
      }
      if (D.accumulate) {
        float c8[8];
        load8_any(C + o, c8);
#pragma unroll
        for (int k = 0; k < 8; ++k) v[k] += c8[k];
      }
      store8_any(C + o, v);
    } else {
      for (int k = 0; k < 8; ++k) {
        if (col0 + k >= D.N) break;
        float v = src[k];
        if (D.epi == EPI_MASK_POS) v = Store<OutT>::to_f(aux[o + k]) > 0.f ? v : 0.f;
        if (D.accumulate) v += Store<OutT>::to_f(C[o + k]);
        C[o + k] = Store<OutT>::from_f(v);
      }
    }
  }
}

}  // namespace crl
