// BF16 GEMM whose operand tiles go from global memory straight into LDS
// (global_load_lds_dwordx4: no staging registers, so only an explicit wait
// orders a tile's arrival before its use), double-buffered.  Tiles that are
// contiguous along K (KC) are read with ds_read_b128 through an XOR swizzle of
// their 16-byte chunks; tiles contiguous along M or N (MC) are read with the
// 16-bit transpose read ds_read_b64_tr_b16, which turns four rows of 4 x 16-bit
// chunks into the per-lane K runs the MFMA wants.  Tiles are 128 x BN with BN
// 128 or 64, computed by BN/16 waves of 64 x 32 each (eight or four waves: more
// resident waves hide more of the load and barrier latency than larger
// per-wave blocks save in LDS reads).  M and N may be ragged (loads past the edge are clamped into the
// operand and the results they feed are not stored; an N that is not a multiple of 8 is stored
// element by element); every K range must be a
// whole number of 64-deep steps, otherwise gemm_kernel takes the launch.
#pragma once
#include "gemm.hpp"

namespace crl {
namespace lds {

constexpr int BM = 128, BK = 64;
// waves and threads of a 128 x BN tile: a 2 x (BN/32) grid of 64 x 32 blocks
template <int BN> constexpr int waves() { return BN / 16; }
template <int BN> constexpr int threads() { return 64 * waves<BN>(); }
typedef short v4s __attribute__((ext_vector_type(4)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) v4s lds_v4s;

// bytes of a ROWS x 64 BF16 operand tile
template <int ROWS> constexpr int tile_bytes() { return ROWS * BK * 2; }

// KC tile: row r holds 64 k values (8 chunks of 16 B); logical chunk c sits
// in slot c ^ kc_swz(r).  A ds_read_b128 pass of 16 rows then touches 16
// distinct (bank window, slot) pairs.
__device__ __forceinline__ int kc_swz(int r) { return (r >> 1) & 7; }

// MC tile of W columns: k-row kr holds W values (W/8 chunks); chunk c sits in
// slot c ^ mc_swz<W>(kr).  A half-wave of transpose reads covers 8 k-rows x 2
// adjacent chunks; the swizzle gives those 16 chunks distinct banks.
template <int W> __device__ __forceinline__ int mc_swz(int kr);
template <> __device__ __forceinline__ int mc_swz<128>(int kr) {
  return 2 * ((kr & 3) + 4 * ((kr >> 3) & 1));
}
template <> __device__ __forceinline__ int mc_swz<64>(int kr) {
  return 2 * (((kr >> 1) & 1) + 2 * ((kr >> 3) & 1));
}

// One wave instruction fills one 1 KB block of the tile; the NW waves take
// blocks wave, wave+NW, ...  W = extent of the tile along M or N; R = extent of
// the operand along it; KR = k-rows of an MC operand that exist.  A KC row
// past R re-reads row R-1, an MC chunk past the row stride re-reads the last
// chunk (in bounds, and only ever feeding outputs that are not stored); an MC
// k-row past KR re-reads row KR-1, which meets zero columns of the other
// operand.
template <int LAY, int W, int NW>
__device__ __forceinline__ void issue_tile(const bf16_t* __restrict__ X, int ld, int r0, int R,
                                           int KR, int k0, char* tile, int wave, int lane) {
  constexpr int NBLK = tile_bytes<W>() / 1024;
  static_assert(NBLK % NW == 0, "whole blocks per wave");
#pragma unroll
  for (int i = 0; i < NBLK / NW; ++i) {
    const int blk = wave + NW * i;
    const bf16_t* src;
    if (LAY == LAY_KC) {  // 8 rows of 128 B per block
      const int r = blk * 8 + (lane >> 3);
      const int c = (lane & 7) ^ kc_swz(r);
      src = X + (int64_t)min(r0 + r, R - 1) * ld + k0 + 8 * c;
    } else {              // 1024 / (2W) k-rows per block
      constexpr int LPR = W / 8;  // lanes (chunks) per k-row
      const int kr = blk * (64 / LPR) + lane / LPR;
      const int c = (lane % LPR) ^ mc_swz<W>(kr);
      src = X + (int64_t)min(k0 + kr, KR - 1) * ld + min(r0 + 8 * c, ld - 8);
    }
    __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(tile + blk * 1024),
                                     16, 0, 0);
  }
}

// KC fragment: 8 consecutive k (32-k half hh, lane group g) of row `row`
__device__ __forceinline__ bf16x8 frag_kc(const char* tile, int row, int hh, int g) {
  const int c = 4 * hh + g;
  return *reinterpret_cast<const bf16x8*>(tile + row * 128 + ((c ^ kc_swz(row)) << 4));
}
// MC fragment: lane (g, j) gets k = 32hh + 8g + 0..7 of column mb + j.  In a
// 16-lane group, lane j addresses k-row 4t + j/4 at columns 4(j%4)..+3; the
// transpose read hands lane j the column-j values of those four rows.
template <int W>
__device__ __forceinline__ bf16x8 frag_mc(const char* tile, int mb, int hh, int g, int j) {
  v4s h[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int kr = 32 * hh + 8 * g + 4 * t + (j >> 2);
    const int m = mb + 4 * (j & 3);
    const int off = kr * (2 * W) + (((m >> 3) ^ mc_swz<W>(kr)) << 4) + (m & 7) * 2;
    h[t] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(tile + off));
  }
  v8s r = {h[0][0], h[0][1], h[0][2], h[0][3], h[1][0], h[1][1], h[1][2], h[1][3]};
  return __builtin_bit_cast(bf16x8, r);
}

// one 64-deep stage: wave (wm, wn) owns rows wm*64 + 0..63, columns
// wn*32 + 0..31 of the tile
template <int LA, int LB, int BN>
__device__ __forceinline__ void compute_tile(floatx4 (&acc)[4][2], const char* At,
                                             const char* Bt, int wm, int wn, int lane) {
  constexpr int NJ = 2;
  const int g = lane >> 4, j = lane & 15;
#pragma unroll
  for (int hh = 0; hh < 2; ++hh) {
    bf16x8 a[4], b[NJ];
#pragma unroll
    for (int i = 0; i < 4; ++i)
      a[i] = LA == LAY_KC ? frag_kc(At, wm * 64 + i * 16 + j, hh, g)
                          : frag_mc<BM>(At, wm * 64 + i * 16, hh, g, j);
#pragma unroll
    for (int i = 0; i < NJ; ++i)
      b[i] = LB == LAY_KC ? frag_kc(Bt, wn * 32 + i * 16 + j, hh, g)
                          : frag_mc<BN>(Bt, wn * 32 + i * 16, hh, g, j);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj)
        acc[i][jj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[jj], acc[i][jj], 0, 0, 0);
  }
}

// s_waitcnt on the vector-memory counter only
template <int N> __device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 16, "vmcnt range");
  __builtin_amdgcn_s_waitcnt(N | 0x70 | 0xF00);
}

// LDS bytes of a 128 x BN tile: two stages, or the FP32 epilogue tile
template <int BN> constexpr int smem_bytes() {
  constexpr int stage2 = 2 * (tile_bytes<BM>() + tile_bytes<BN>());
  constexpr int epi = (int)sizeof(float) * BM * (BN + 4);
  return stage2 > epi ? stage2 : epi;
}
}  // namespace lds

// One workgroup's work item wi of launch P; smem holds smem_bytes<BN>().
template <int LA, int LB, typename OutT, int BN>
__device__ __forceinline__ void gemm_lds_tile(const GemmParams& P, const WorkItem wi, char* smem) {
  using namespace lds;
  constexpr int NW = waves<BN>(), NT = threads<BN>();
  constexpr int TA = tile_bytes<BM>(), TB = tile_bytes<BN>();
  constexpr int STAGE = TA + TB;
  constexpr int kLdc = BN + 4;
  constexpr int NJ = 2;
  const int gi = wi.prob;
  const GemmDesc& D = P.d[gi];
  const int ntile = P.tiles[gi];
  const int pid = wi.tile;
  if (pid >= ntile) return;
  const int tm = pid / P.tiles_n[gi], tn = pid % P.tiles_n[gi];
  const int m0 = tm * BM, n0 = tn * BN;
  const int kbeg = wi.split * P.k_chunk;
  const int nk = (min(D.K, kbeg + P.k_chunk) - kbeg) / BK;  // <= 0: empty split
  const bf16_t* A = reinterpret_cast<const bf16_t*>(D.A);
  const bf16_t* B = reinterpret_cast<const bf16_t*>(D.B);
  const int kb = D.kb > 0 ? D.kb : D.K;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / (NW / 2), wn = wave % (NW / 2);
  floatx4 acc[4][NJ];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};

  auto issue = [&](int t) {
    char* st = smem + (t & 1) * STAGE;
    issue_tile<LA, BM, NW>(A, D.lda, m0, D.M, D.K, kbeg + t * BK, st, wave, lane);
    issue_tile<LB, BN, NW>(B, D.ldb, n0, D.N, kb, kbeg + t * BK, st + TA, wave, lane);
  };
  if (nk > 0) issue(0);
  for (int kt = 0; kt < nk; ++kt) {
    // this thread's loads of tile kt are the only ones in flight; the barrier
    // then makes every thread's part of it visible and guarantees that the
    // other buffer (tile kt-1) is no longer being read
    wait_vm<0>();
    __syncthreads();
    if (kt + 1 < nk) issue(kt + 1);
    const char* st = smem + (kt & 1) * STAGE;
    compute_tile<LA, LB, BN>(acc, st, st + TA, wm, wn, lane);
  }
  const bool split = P.splits > 1;
  if (split && P.defer_reduce && P.frag) {
    // deferred split-K partial in fragment order: wave w's accumulators
    // acc[i][j] go to floats ((tile * NW + w) * 8 + i * 2 + j) * 256 + 4 lane
    // of this split's block, one 1 KB store per wave and fragment
    float* out = P.partial + (int64_t)gi * P.partial_len +
                 (int64_t)wi.split * ntile * BM * BN + ((int64_t)pid * NW + wave) * (4 * NJ * 256);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < NJ; ++j)
        *reinterpret_cast<floatx4*>(out + (i * NJ + j) * 256 + lane * 4) = acc[i][j];
    return;
  }
  __syncthreads();

  // epilogue: stage the FP32 tile in LDS, then 16-byte row stores
  const int r16 = lane & 15, gq = lane >> 4;
  float* Cs = reinterpret_cast<float*>(smem);
  const bool has_bias = !split && (D.epi == EPI_BIAS || D.epi == EPI_BIAS_RELU);
  float bcol[NJ];
#pragma unroll
  for (int j = 0; j < NJ; ++j)  // clamped column: past-the-edge values are not stored
    bcol[j] = has_bias ? D.bias[min(n0 + wn * 32 + j * 16 + r16, D.N - 1)] : 0.f;
  const float alpha = split ? 1.f : D.alpha;
  const bool relu = !split && D.epi == EPI_BIAS_RELU;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
      const int cl = wn * 32 + j * 16 + r16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int rl = wm * 64 + i * 16 + gq * 4 + r;
        float v = acc[i][j][r] * alpha + bcol[j];
        if (relu) v = fmaxf(v, 0.f);
        Cs[rl * kLdc + cl] = v;
      }
    }
  __syncthreads();
  // BN/8 threads per row, 8 values each; N is a multiple of 8, so a chunk is
  // either wholly inside or wholly past the edge
  constexpr int TPR = BN / 8, RSTEP = NT / TPR;
  const int ch = tid % TPR;
  const int col0 = n0 + ch * 8;
  const int rows = min(BM, D.M - m0);
  if (col0 >= D.N) return;
  // N not a multiple of 8 (a few output columns, no mask epilogue): element stores
  const int nc = min(8, D.N - col0);
  const bool ragged = (D.N & 7) != 0;
  if (split) {
    float* out = P.partial + (int64_t)gi * P.partial_len + (int64_t)wi.split * D.M * D.N;
    for (int rl = tid / TPR; rl < rows; rl += RSTEP) {
      const float* src = Cs + rl * kLdc + ch * 8;
      float* dst = out + (int64_t)(m0 + rl) * D.N + col0;
      if (ragged) {  // unrolled with constant indices: no private-memory array
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k < nc) dst[k] = src[k];
        continue;
      }
      *reinterpret_cast<float4*>(dst) = *reinterpret_cast<const float4*>(src);
      *reinterpret_cast<float4*>(dst + 4) = *reinterpret_cast<const float4*>(src + 4);
    }
    return;
  }
  OutT* __restrict__ C = reinterpret_cast<OutT*>(D.C);
  const OutT* __restrict__ aux = reinterpret_cast<const OutT*>(D.aux);
  for (int rl = tid / TPR; rl < rows; rl += RSTEP) {
    const float* src = Cs + rl * kLdc + ch * 8;
    const int64_t o = (int64_t)(m0 + rl) * D.ldc + col0;
    float v[8];
    *reinterpret_cast<float4*>(v) = *reinterpret_cast<const float4*>(src);
    *reinterpret_cast<float4*>(v + 4) = *reinterpret_cast<const float4*>(src + 4);
    if (D.epi == EPI_MASK_POS) {
      float a8[8];
      load8_any(aux + o, a8);
#pragma unroll
      for (int k = 0; k < 8; ++k) v[k] = a8[k] > 0.f ? v[k] : 0.f;
    }
    if (ragged) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (k < nc) C[o + k] = Store<OutT>::from_f(v[k]);
      continue;
    }
    store8_any(C + o, v);
  }
}

// two workgroups per CU: 2 * waves<BN>() waves over the 4 SIMDs
template <int LA, int LB, typename OutT, int BN>
__global__ __launch_bounds__(lds::threads<BN>())
__attribute__((amdgpu_waves_per_eu(lds::waves<BN>() / 2, lds::waves<BN>() / 2)))
void gemm_lds_kernel(GemmParams P) {
  __shared__ __attribute__((aligned(1024))) char smem[lds::smem_bytes<BN>()];
  gemm_lds_tile<LA, LB, OutT, BN>(P, gemm_work_item(), smem);
}

// Two independent launches of 128 x 128 tiles in one grid: ids [0, n1) take
// launch P1 (grid g1 = tiles x splits x problems), the rest launch P2.  One
// launch instead of two saves a launch's fixed cost (first stage, epilogue,
// ramp) and lets the second launch's tiles fill the first one's tail.
struct PairGrid { int n1, gx1, gy1, gx2, gy2, n2; };
template <int LA1, int LB1, typename Out1, int LA2, int LB2, typename Out2>
__global__ __launch_bounds__(lds::threads<128>())
__attribute__((amdgpu_waves_per_eu(lds::waves<128>() / 2, lds::waves<128>() / 2)))
void gemm_lds_pair_kernel(GemmParams P1, GemmParams P2, PairGrid G) {
  __shared__ __attribute__((aligned(1024))) char smem[lds::smem_bytes<128>()];
  const int id = blockIdx.x;
  if (id < G.n1)
    gemm_lds_tile<LA1, LB1, Out1, 128>(P1, work_item_of(id, G.gx1, G.gy1, G.n1), smem);
  else
    gemm_lds_tile<LA2, LB2, Out2, 128>(P2, work_item_of(id - G.n1, G.gx2, G.gy2, G.n2), smem);
}

}  // namespace crl
