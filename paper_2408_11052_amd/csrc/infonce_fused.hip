// Fused InfoNCE over the B x B critic matrix without storing it.
//
// Forward: each workgroup owns 64 rows of phi (4 wavefronts x 16 rows, held
// in registers as MFMA A fragments) and one split of the columns.  For every
// 64-column tile of psi (staged in LDS) it forms the tile F = phi . psi^T with
// v_mfma_f32_16x16x32_bf16, applies the energy, and keeps
//   - per row: an online (max, sum exp) pair over its columns,
//   - per column: the (max, sum exp) over the workgroup's 64 rows,
//   - the diagonal F_ii.
// Row pairs of all splits and column pairs of all row blocks are merged by
// lse_merge_kernel; the loss is then a reduction over r, c and the diagonal.
//
// Backward: G_ij = dL/dF_ij = (1/B)[Pr_ij (wf + 2 beta r_i) - wf d_ij
// + wb (Pc_ij - d_ij)] (wf, wb in {0, 1}: the row and column directions of
// InfoNCE / FlatNCE) is recomputed tile by tile from r and c (never stored)
// and multiplied into the streamed operand with a second MFMA:
// dphi = G psi (row pass) and dpsi = G^T phi (column pass, the same kernel
// with the roles of phi and psi exchanged).  For the L2 energy H = G / d
// replaces G (H = 2 G without the root) and the row sums of H give the
// -(sum_j H_ij) phi_i term.  The cosine energy runs as the dot product of
// unit rows; the reduction then projects out the row's own direction and
// divides by its norm.  Each split writes its own partial, summed in a fixed
// order afterwards (no atomics).
#include <cmath>

#include "internal.hpp"

namespace crl {

constexpr int kFRows = 64;   // rows per workgroup
constexpr int kFCols = 64;   // columns per tile

// Energy applied to a tile value v = <x_i, y_j> (x, y the BF16 rows, or the
// BF16 unit rows for the cosine energy) with squared norms nx, ny.
enum : int { kEnDot = 0, kEnL2 = 1, kEnL2sq = 2 };
static int fused_energy(int energy) {
  return energy == CRL_ENERGY_L2 ? kEnL2 : energy == CRL_ENERGY_L2SQ ? kEnL2sq : kEnDot;
}

// Column splits: enough workgroups for four waves per SIMD (1024 x 4 waves
// over 1024 SIMDs), at most 16 partials per row to merge.
int fused_splits(int B) {
  int nrb = (B + kFRows - 1) / kFRows;
  int S = 1024 / nrb;
  if (S < 1) S = 1;
  if (S > 16) S = 16;
  int cps = (B + S - 1) / S;
  cps = (cps + kFCols - 1) / kFCols * kFCols;
  return (B + cps - 1) / cps;
}
static inline int cols_per_split(int B, int S) {
  int cps = (B + S - 1) / S;
  return (cps + kFCols - 1) / kFCols * kFCols;
}

// BF16 copies of phi, psi and the squared norms of the rounded rows; for the
// cosine energy (unit != 0) the BF16 copies are of the unit rows x / |x| and
// the norm slot holds |x| (FP32).
__device__ __forceinline__ void prep_row(float* X, bf16_t* Xb, float* nrm, int row, int D,
                                         int lane, int unit) {
  float s = 0.f;
  if (unit) {
    for (int d = lane; d < D; d += 64) s += X[d] * X[d];
    s = wave_sum(s);
    const float n = sqrtf(s);
    const float inv = n > 0.f ? 1.f / n : 0.f;
    for (int d = lane; d < D; d += 64) Xb[d] = f2bf(X[d] * inv);
    if (lane == 0) nrm[row] = n;
    return;
  }
  for (int d = lane; d < D; d += 64) {
    const bf16_t h = f2bf(X[d]);
    Xb[d] = h;
    const float v = bf2f(h);
    s += v * v;
  }
  s = wave_sum(s);
  if (lane == 0) nrm[row] = s;
}

__global__ void fused_prep_kernel(FusedArgs a, int B, int D, int unit) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int which = blockIdx.y;
  if (row >= B) return;
  const float* X = (which ? a.psi : a.phi) + (int64_t)row * D;
  bf16_t* Xb = (which ? a.psi_b : a.phi_b) + (int64_t)row * D;
  prep_row(const_cast<float*>(X), Xb, which ? a.npsi : a.nphi, row, D, lane, unit);
}

// The same from the output layer's split-K partials: phi / psi = sum of the
// splits in order + bias (FP32, as the split-K reduction writes them), then
// the BF16 copies and norms.
__global__ void fused_prep_reduce_kernel(FusedArgs a, GemmParams P, int B, int D, int unit) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int which = blockIdx.y;
  if (row >= B) return;
  const GemmDesc& G = P.d[which];
  const int64_t MN = (int64_t)G.M * G.N;
  const float* __restrict__ src = P.partial + (int64_t)which * P.partial_len + (int64_t)row * D;
  float* X = reinterpret_cast<float*>(G.C) + (int64_t)row * G.ldc;
  for (int d = lane; d < D; d += 64) {
    float v = 0.f;
    for (int k = 0; k < P.splits; ++k) v += src[k * MN + d];
    X[d] = v + G.bias[d];
  }
  prep_row(X, (which ? a.psi_b : a.phi_b) + (int64_t)row * D, which ? a.npsi : a.nphi, row, D,
           lane, unit);
}

// A 64-row tile of Y [B][D] (BF16) moves global -> registers -> LDS.  Each
// of the 256 threads holds D/32 16-byte vectors; rows past B are zero.  The
// next tile is fetched into registers while the current one is computed on.
template <int D>
struct TileRegs { u32x4 v[D / 32]; };

// A tile inside the batch (the common case) loads without bounds checks from
// one tile base and per-lane 32-bit offsets; only the last tile of the batch
// checks its rows.
template <int D>
__device__ __forceinline__ void tile_load(TileRegs<D>& t, const bf16_t* __restrict__ Y, int j0,
                                          int B, int tid) {
  constexpr int VPR = D / 8;  // 16-byte vectors per row
  const bf16_t* __restrict__ base = Y + (int64_t)j0 * D;
  if (j0 + kFCols <= B) {
#pragma unroll
    for (int i = 0; i < D / 32; ++i)
      t.v[i] = *reinterpret_cast<const u32x4*>(base + (tid + i * 256) * 8);
    return;
  }
#pragma unroll
  for (int i = 0; i < D / 32; ++i) {
    const int v = tid + i * 256;
    const int r = v / VPR;
    u32x4 val = {0u, 0u, 0u, 0u};
    if (j0 + r < B) val = *reinterpret_cast<const u32x4*>(base + v * 8);
    t.v[i] = val;
  }
}

// LDS rows of D BF16 values are padded to D + 16 (a stride of 2 mod 16 in
// 16-byte bank groups; 64 banks of 4 bytes) and, inside each group of 16
// rows, row r is stored at r with its bits 2 and 3 exchanged.  The three
// accesses to the tile are then free of bank conflicts, given the lane groups
// the LDS serves together (measured on gfx950 with the bank-conflict
// counter): ds_write_b128 serves 8 consecutive lanes, each storing 16
// contiguous bytes of one row here; ds_read_b128 serves the 16 lanes that
// share lane bit 5 and the parity of bits 2..4, which for the MFMA row
// operand (lane (g, j): row j, chunk g) meet 16 distinct bank groups; the
// 8-byte transpose read serves a half-wave, rows c..c+3 and c+8..c+11 with
// 32 bytes each, again 16 distinct groups.  The earlier order (padding 8,
// rows 8a + 4b + t at 8a + 2t + b) left the row operand two-way conflicted.
// Both reads keep one per-lane base plus compile-time offsets: row 16 m + j
// (j < 16) is at 16 m + lds_row(j), and row 32 k + 8 g + 4 q + i (g, i < 4)
// at 32 k + 8 q + lds_row(8 g + i).
__device__ __forceinline__ int lds_row(int r) {
  return (r & ~12) | ((r & 4) << 1) | ((r >> 1) & 4);
}
// element offset of position p (a permuted row), column d
template <int D>
__device__ __forceinline__ int lds_pos(int p, int d) {
  return p * (D + 16) + d;
}
// element offset of row r, column d
template <int D>
__device__ __forceinline__ int lds_at(int r, int d) {
  return lds_pos<D>(lds_row(r), d);
}

// rows layout Ys[r][d] (row order and stride as above)
template <int D, int LDY>
__device__ __forceinline__ void tile_store_rows(bf16_t* __restrict__ Ys, const TileRegs<D>& t,
                                                int tid) {
  constexpr int VPR = D / 8;
#pragma unroll
  for (int i = 0; i < D / 32; ++i) {
    const int v = tid + i * 256;
    const int r = v / VPR, c = v % VPR;
    *reinterpret_cast<u32x4*>(Ys + lds_at<D>(r, c * 8)) = t.v[i];
  }
}

// Exponentials are one v_exp_f32 (2^x) of a scaled argument: exp(x - m) is
// exp2((x - m) * log2(e)) in the forward, where x = m must give exactly 1
// (B = 1 gives r_i = F_ii exactly), and exp2(x * log2(e) - s) with the
// shift s = lse * log2(e) + log2(B) formed once per row or column in the
// backward.
constexpr float kL2E = 1.4426950408889634f;  // log2(e)

// Tile entry of the energy from v = <x_i, y_j> (norms nx, ny for the
// distances), and for L2 the distance d (0 below the norm-expansion noise,
// as l2_dist; the hardware square root, whose 1-ulp error is far below the
// BF16 rounding of the operands).  A NaN operand stays NaN in f and d.
template <int EN>
__device__ __forceinline__ float energy_f(float v, float nx, float ny, float& d) {
  if (EN == kEnL2) {
    const float t = nx + ny;
    const float d2 = __builtin_fmaf(-2.f, v, t);
    d = d2 <= kL2Floor * t ? 0.f : __builtin_amdgcn_sqrtf(d2);
    return -d;
  }
  if (EN == kEnL2sq) {
    const float d2 = __builtin_fmaf(-2.f, v, nx + ny);
    d = d2 < 0.f ? 0.f : d2;
    return -d;
  }
  d = 0.f;
  return v;
}
// The same for the backward, with the factor w that turns the gradient of the
// energy's argument into the tile entry: for L2, 1 / d (0 where d is 0) from
// one reciprocal square root, d = d2 / sqrt(d2) (a NaN operand stays NaN in
// both); 2 for the squared distance; 1 for the product.
template <int EN>
__device__ __forceinline__ float energy_fw(float v, float nx, float ny, float& w) {
  if (EN == kEnL2) {
    const float t = nx + ny;
    const float d2 = __builtin_fmaf(-2.f, v, t);
    // the masked entries take r = 0, so that f = -(d2 r) is a signed zero:
    // only exponentials of f are taken, and those do not see the sign (a
    // squared norm that overflows to inf gives NaN here, as it should)
    const float r = d2 <= kL2Floor * t ? 0.f : __builtin_amdgcn_rsqf(d2);
    w = r;
    return -(d2 * r);
  }
  if (EN == kEnL2sq) {
    const float d2 = __builtin_fmaf(-2.f, v, nx + ny);
    w = 2.f;
    return d2 < 0.f ? -0.f : -d2;
  }
  w = 1.f;
  return v;
}
// The maxima of the online log-sum-exp: IEEE maximum, which returns NaN if
// either operand is NaN and needs no canonicalising of its operands (two
// three-operand instructions for a row's four entries and its running max,
// where fmaxf took seven).  A NaN entry makes its row's and column's LSE NaN
// either way: with fmaxf it was skipped by the max but reached the sum.
__device__ __forceinline__ float max_nan(float a, float b) {
  return __builtin_elementwise_maximum(a, b);
}
__device__ __forceinline__ float exp_diff(float x, float m) {
  return __builtin_amdgcn_exp2f((x - m) * kL2E);
}

// Per workgroup: 64 rows (wave w: rows 16w + 4g + r of lane (r16, g), r < 4)
// against the 64-column tiles of one column split.  Tiles inside the batch
// on every side skip the masking, and only the tile that holds a wave's
// diagonal entries looks for them (both are wave-uniform branches).
// The 16 x 64 tile F = X[16 rows] . Y[64 columns]^T of one wave: four
// 16-column accumulators, the K loop outside, so that the four products of
// a K step are independent and their B fragments can be read together.
template <int KS>
__device__ __forceinline__ void tile_product(floatx4 (&acc)[4], const bf16x8 (&xa)[KS],
                                             const bf16_t* __restrict__ Ys, int r16, int g) {
#pragma unroll
  for (int jb = 0; jb < 4; ++jb) acc[jb] = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    bf16x8 b[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
      b[jb] = *reinterpret_cast<const bf16x8*>(Ys + lds_pos<KS * 32>(jb * 16 + lds_row(r16), ks * 32 + g * 8));
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
      acc[jb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(xa[ks], b[jb], acc[jb], 0, 0, 0);
  }
}

// Occupancy targets (wavefronts per SIMD) that the register allocation must
// meet: the forward's LDS holds three workgroups per CU at D = 256, the
// backward passes need about 256 registers per lane there.
template <int KS> constexpr int fwd_waves() { return KS >= 8 ? 3 : 4; }
template <int KS> constexpr int bwd_waves() { return KS >= 4 ? 2 : 4; }

template <int KS, int EN>
__global__ __launch_bounds__(256, fwd_waves<KS>()) void infonce_fwd_kernel(FusedArgs a, int B, int cps) {
  constexpr bool L2 = EN != kEnDot;
  constexpr int D = KS * 32;
  constexpr int LDY = D + 16;
  constexpr int LDC = kFCols + 16;  // column-partial rows
  __shared__ __attribute__((aligned(16))) bf16_t Ys[kFCols * LDY];
  // column (max, sum) of each (wave, 4-row group) for the current tile
  __shared__ float cm_s[16][LDC], cs_s[16][LDC];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15, g = lane >> 4;
  const int rb = blockIdx.x;
  const int row_base = rb * kFRows + wave * 16;
  const int c0 = blockIdx.y * cps, c1 = min(B, c0 + cps);
  const bool rows_full = row_base + 16 <= B;

  bf16x8 xa[KS];
  {
    const int row = row_base + r16;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (row < B) xa[ks] = *reinterpret_cast<const bf16x8*>(a.phi_b + (int64_t)row * D + ks * 32 + g * 8);
      else xa[ks] = bf16x8{};
    }
  }
  float nx[4], rm[4], rsum[4];
  bool rvalid[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int row = row_base + 4 * g + r;
    rvalid[r] = row < B;
    nx[r] = (L2 && rvalid[r]) ? a.nphi[row] : 0.f;
    rm[r] = -INFINITY;
    rsum[r] = 0.f;
  }

  // column (max, sum) partials of a finished tile, merged over the 16
  // (wave, row group) entries: their max first, then the rescaled sums.  Each
  // wave takes 16 of the tile's columns, four lanes per column, each lane four
  // of the entries; the lanes' maxima and sums then meet by butterflies over
  // the lane groups (a fixed order).  Every wave does its share every tile, so
  // no wave arrives at the next barrier with the whole merge.
  auto flush_cols = [&](int jp) {
    const int cl = wave * 16 + r16;
    float mv[4], sv[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) { mv[i] = cm_s[4 * g + i][cl]; sv[i] = cs_s[4 * g + i][cl]; }
    float cm = max_nan(max_nan(mv[0], mv[1]), max_nan(mv[2], mv[3]));
    cm = max_nan(cm, __shfl_xor(cm, 16, 64));
    cm = max_nan(cm, __shfl_xor(cm, 32, 64));
    float cs = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) cs += sv[i] == 0.f ? 0.f : sv[i] * exp_diff(mv[i], cm);
    cs += __shfl_xor(cs, 16, 64);
    cs += __shfl_xor(cs, 32, 64);
    const int col = jp + cl;
    if (g == 0 && col < c1) {
      a.col_m[(int64_t)rb * B + col] = cm;
      a.col_s[(int64_t)rb * B + col] = cs;
    }
  };
  // the prefetch is unconditional (clamped to the last tile) so the wait
  // before each LDS store covers exactly the previous fetch
  const int jlast = c0 + ((c1 - c0 - 1) / kFCols) * kFCols;
  TileRegs<D> pf;
  float nypf[4] = {0.f, 0.f, 0.f, 0.f};
  auto ny_load = [&](int j0) {
    if (!L2) return;
    const float* __restrict__ base = a.npsi + j0;
    if (j0 + kFCols <= c1) {
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) nypf[jb] = base[jb * 16 + r16];
      return;
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) nypf[jb] = j0 + jb * 16 + r16 < c1 ? base[jb * 16 + r16] : 0.f;
  };
  if (c0 < c1) { tile_load<D>(pf, a.psi_b, c0, B, tid); ny_load(c0); }
  for (int j0 = c0; j0 < c1; j0 += kFCols) {
    __syncthreads();
    if (j0 > c0) flush_cols(j0 - kFCols);
    tile_store_rows<D, LDY>(Ys, pf, tid);
    float nyv[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) nyv[jb] = nypf[jb];
    tile_load<D>(pf, a.psi_b, min(j0 + kFCols, jlast), B, tid);
    ny_load(min(j0 + kFCols, jlast));
    __syncthreads();
    floatx4 acc[4];
    tile_product<KS>(acc, xa, Ys, r16, g);
    float f[4][4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        float d;
        f[jb][r] = energy_f<EN>(acc[jb][r], nx[r], nyv[jb], d);
      }
    if (j0 <= row_base && row_base < j0 + kFCols) {  // this wave's diagonal entries
#pragma unroll
      for (int jb = 0; jb < 4; ++jb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row_base + 4 * g + r;
          if (row == j0 + jb * 16 + r16 && row < c1 && rvalid[r]) a.diag[row] = f[jb][r];
        }
    }
    const bool edge = !rows_full || j0 + kFCols > c1;
    if (edge) {  // entries outside the batch or the split become -inf
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        const bool cv = j0 + jb * 16 + r16 < c1;
#pragma unroll
        for (int r = 0; r < 4; ++r) f[jb][r] = (cv && rvalid[r]) ? f[jb][r] : -INFINITY;
      }
    }
    // rows: online (max, sum)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float nm = max_nan(rm[r], max_nan(max_nan(f[0][r], f[1][r]), max_nan(f[2][r], f[3][r])));
      float sr = rsum[r] * exp_diff(rm[r], nm);
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) sr += exp_diff(f[jb][r], nm);
      if (edge) sr = nm == -INFINITY ? 0.f : sr;  // nothing of this row seen yet
      rsum[r] = sr;
      rm[r] = nm;
    }
    // columns: (max, sum) over this lane's 4 rows, one entry per (wave, row
    // group); the merge runs after the next barrier
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      const float cm = max_nan(max_nan(f[jb][0], f[jb][1]), max_nan(f[jb][2], f[jb][3]));
      float cs = 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) cs += exp_diff(f[jb][r], cm);
      if (edge) cs = cm == -INFINITY ? 0.f : cs;
      cm_s[wave * 4 + g][jb * 16 + r16] = cm;
      cs_s[wave * 4 + g][jb * 16 + r16] = cs;
    }
  }
  if (c0 < c1) {
    __syncthreads();
    flush_cols(jlast);
  }
  // merge the row states across the 16 lanes that share each row: the max
  // by a butterfly, then the sums rescaled to it by a butterfly (every lane
  // ends with the same value: each level adds the same two operands)
  float mrow[4], srow[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) mrow[r] = rm[r];
#pragma unroll
  for (int o = 1; o <= 8; o <<= 1)
#pragma unroll
    for (int r = 0; r < 4; ++r) mrow[r] = max_nan(mrow[r], __shfl_xor(mrow[r], o, 64));
#pragma unroll
  for (int r = 0; r < 4; ++r)
    srow[r] = rsum[r] == 0.f ? 0.f : rsum[r] * exp_diff(rm[r], mrow[r]);
#pragma unroll
  for (int o = 1; o <= 8; o <<= 1)
#pragma unroll
    for (int r = 0; r < 4; ++r) srow[r] += __shfl_xor(srow[r], o, 64);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const float m = mrow[r], s = srow[r];
    const int row = row_base + 4 * g + r;
    if (r16 == 0 && row < B) {
      a.row_m[(int64_t)blockIdx.y * B + row] = m;
      a.row_s[(int64_t)blockIdx.y * B + row] = s;
    }
  }
}

// Element offset of (column c, row e) in a wave's transposed G strip: 64
// columns of 16 BF16 rows (32 bytes each).  Inside each group of 16 columns,
// column c8 + 8t (c8 < 8, t = 0 or 1) sits in 32-byte slot (c8 + 4t) mod 8 of
// the group's t-th 256-byte half, its two 16-byte halves swapped when t = 1.
// A half-wave's transpose read (columns c..c+3 and c+8..c+11, 32 bytes each)
// then falls on 64 distinct banks, and a strip store (16 lanes at a time over
// 32 banks, measured) is two-way conflicted; with plain 32-byte rows they
// were two-way and four-way.  Permuting each column's four 8-byte chunks by
// bits 2 and 3 of c as well makes the store conflict-free too, but measured
// about 1% slower at D = 256, so the simpler form stays.
__device__ __forceinline__ int gt_at(int c, int e) {
  const int t = (c >> 3) & 1;
  return (c & ~15) * 16 + t * 128 + (((c & 7) + 4 * t) & 7) * 16 + (e ^ (8 * t));
}

// TRANS = 0: rows are phi, streamed operand psi -> partials of dphi.
// TRANS = 1: rows are psi, streamed operand phi -> partials of dpsi.
// Per 64-column tile: F (MFMA), G (or H) into the wave's own LDS strip, then
// dX += G . Y with the Y operand read from the row-major tile by the 16-bit
// transpose read (no transposed copy of the tile is kept).  For D >= 128 the
// product is split over D instead of rows: after a workgroup barrier each
// wave multiplies all four strips (64 rows) by its quarter of the tile's
// columns, so the tile is read once per workgroup in that product rather
// than once per wave; for D <= 64 a wave reads its own strip back.  The tile's
// column values (the other side's LSE, |y|^2) are fetched together with the
// tile, one tile ahead.
//
// Entry (i, j) of G (rows pass; the columns pass exchanges the roles) is
//   P^r_ij (wf + 2 beta r_i) / B + wb P^c_ij / B - (wf + wb) delta_ij / B,
// and each P / B is one exp2 of f log2(e) - (lse log2(e) + log2 B), the shifts
// formed once per row and per column: the weight wb (0 or 1) of the other
// direction is folded into its shift (+inf when it is 0).  The strip is kept
// transposed, [column][row], so that each lane stores its four rows of a
// column as one 8-byte write; the transpose read gives back the row-major A
// operand of the product.
template <int KS, int EN, int TRANS>
__global__ __launch_bounds__(256, bwd_waves<KS>()) void infonce_bwd_kernel(FusedArgs a, int B, int cps,
                                                          float beta, float wf, float wb,
                                                          float log2b) {
  constexpr bool L2 = EN != kEnDot;
  constexpr int D = KS * 32;
  constexpr int LDY = D + 16;
  constexpr int LDG = 16;     // transposed G strip: [64 columns][16 rows]
  constexpr int NB = D / 16;  // 16-wide output blocks of dX
  // D >= 128: wave w owns columns [w D/4, (w+1) D/4) of dX for all 64 rows
  constexpr bool DSPLIT = NB >= 8;
  constexpr int NW = NB / 4;  // 16-wide output blocks per wave when split
  typedef short v4s __attribute__((ext_vector_type(4)));
  typedef short v8s __attribute__((ext_vector_type(8)));
  typedef __attribute__((address_space(3))) v4s lds_v4s;
  // two tile buffers: the next tile is stored while this one is in use
  __shared__ __attribute__((aligned(16))) bf16_t Ys[2][kFCols * LDY];
  __shared__ __attribute__((aligned(16))) bf16_t Gt[4][kFCols * LDG];

  const bf16_t* Xb = TRANS ? a.psi_b : a.phi_b;
  const bf16_t* Yb = TRANS ? a.phi_b : a.psi_b;
  const float* nX = TRANS ? a.npsi : a.nphi;
  const float* nY = TRANS ? a.nphi : a.npsi;
  // TRANS=0: rows own r_i (and the penalty), columns own c_j; TRANS=1: swapped
  const float* lseX = TRANS ? a.c : a.r;
  const float* lseY = TRANS ? a.r : a.c;

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15, g = lane >> 4;
  const int rb = blockIdx.x;
  const int row_base = rb * kFRows + wave * 16;
  const int c0 = blockIdx.y * cps, c1 = min(B, c0 + cps);
  const bool rows_full = row_base + 16 <= B;
  const float beta2 = 2.f * beta;
  const float dgv = (wf + wb) / (float)B;  // the diagonal's -delta_ij terms
  // shift and weight of the row direction (the penalty rides on the rows'
  // own LSE r_i) and the shift of the column direction, folded with wb
  auto main_shift = [&](float lse) { return __builtin_fmaf(lse, kL2E, log2b); };
  auto other_shift = [&](float lse) {
    return wb != 0.f ? __builtin_fmaf(lse, kL2E, log2b) : INFINITY;
  };

  bf16x8 xa[KS];
  {
    const int row = row_base + r16;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (row < B) xa[ks] = *reinterpret_cast<const bf16x8*>(Xb + (int64_t)row * D + ks * 32 + g * 8);
      else xa[ks] = bf16x8{};
    }
  }
  float nx[4], sh_a[4], k_a[4], hsum[4];
  bool rvalid[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = row_base + 4 * g + r;
    rvalid[r] = row < B;
    nx[r] = (L2 && rvalid[r]) ? nX[row] : 0.f;
    const float l = rvalid[r] ? lseX[row] : 0.f;
    sh_a[r] = TRANS ? other_shift(l) : main_shift(l);
    k_a[r] = wf + beta2 * l;  // used by the rows pass only
    hsum[r] = 0.f;
  }
  floatx4 acc_dx[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc_dx[nb] = floatx4{0.f, 0.f, 0.f, 0.f};

  // per-lane column values of a tile (columns j0 + jb*16 + r16)
  struct ColVals { float lse[4], ny[4]; };
  auto col_load = [&](ColVals& cvv, int j0) {
    if (j0 + kFCols <= c1) {
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        cvv.lse[jb] = lseY[j0 + jb * 16 + r16];
        cvv.ny[jb] = L2 ? nY[j0 + jb * 16 + r16] : 0.f;
      }
      return;
    }
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      const int col = j0 + jb * 16 + r16;
      const bool cv = col < c1;
      cvv.lse[jb] = cv ? lseY[col] : 0.f;
      cvv.ny[jb] = (L2 && cv) ? nY[col] : 0.f;
    }
  };

  // tile j0 sits in Ys[buf]; pf holds tile j0 + 64 (stored into the other
  // buffer at the top of the iteration) and cpf its column values
  const int jlast = c0 + ((c1 - c0 - 1) / kFCols) * kFCols;
  TileRegs<D> pf;
  ColVals cvals, cpf;
  if (c0 < c1) {
    tile_load<D>(pf, Yb, c0, B, tid);
    col_load(cvals, c0);
    tile_store_rows<D, LDY>(Ys[0], pf, tid);
    tile_load<D>(pf, Yb, min(c0 + kFCols, jlast), B, tid);
    col_load(cpf, min(c0 + kFCols, jlast));
  }
  int buf = 0;
  for (int j0 = c0; j0 < c1; j0 += kFCols, buf ^= 1) {
    // Ys[buf] is complete, and every wave is past the previous tile's reads
    // of Ys[buf ^ 1] and of the G strips
    __syncthreads();
    if (j0 + kFCols < c1) {
      tile_store_rows<D, LDY>(Ys[buf ^ 1], pf, tid);
      tile_load<D>(pf, Yb, min(j0 + 2 * kFCols, jlast), B, tid);
    }
    const bf16_t* __restrict__ Yt = Ys[buf];
    floatx4 acc[4];
    tile_product<KS>(acc, xa, Yt, r16, g);
    float sh_b[4], k_b[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      sh_b[jb] = TRANS ? main_shift(cvals.lse[jb]) : other_shift(cvals.lse[jb]);
      k_b[jb] = wf + beta2 * cvals.lse[jb];  // used by the columns pass only
    }
    const bool edge = !rows_full || j0 + kFCols > c1;
    const bool diag = j0 <= row_base && row_base < j0 + kFCols;
    // one 16-column block at a time: its four rows' G, the diagonal and edge
    // terms, H, the rows' sums and the strip store
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      float h[4], wv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float fv = energy_fw<EN>(acc[jb][r], nx[r], cvals.ny[jb], wv[r]);
        const float pa = __builtin_amdgcn_exp2f(__builtin_fmaf(fv, kL2E, -sh_a[r]));
        const float pb = __builtin_amdgcn_exp2f(__builtin_fmaf(fv, kL2E, -sh_b[jb]));
        h[r] = TRANS ? __builtin_fmaf(pb, k_b[jb], pa) : __builtin_fmaf(pa, k_a[r], pb);
      }
      if (diag) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row_base + 4 * g + r == j0 + jb * 16 + r16) h[r] -= dgv;
      }
      if (edge) {
        const bool cv = j0 + jb * 16 + r16 < c1;
#pragma unroll
        for (int r = 0; r < 4; ++r) h[r] = (cv && rvalid[r]) ? h[r] : 0.f;
      }
      // H = G / d (L2; 0 where d = 0) or 2 G (L2 without the root)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (EN != kEnDot) h[r] *= wv[r];
        hsum[r] += h[r];
      }
      uint2 w;
      w.x = pack2bf(h[0], h[1]);
      w.y = pack2bf(h[2], h[3]);
      *reinterpret_cast<uint2*>(&Gt[wave][gt_at(jb * 16 + r16, 4 * g)]) = w;
    }
    if constexpr (DSPLIT) {
      // every wave reads all four strips: a workgroup barrier
      __syncthreads();
      // dX[64 rows][this wave's D/4 columns] += G[64][64] . Y[64][D/4 columns];
      // the A fragments of the four strips are read once and each used NW times
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        bf16x8 ga[4];
#pragma unroll
        for (int st = 0; st < 4; ++st) {
          v4s gq[2];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int krow = kk * 32 + 8 * g + 4 * q + (r16 >> 2);
            gq[q] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
                (lds_v4s*)(&Gt[st][gt_at(krow, 4 * (r16 & 3))]));
          }
          v8s gv8 = {gq[0][0], gq[0][1], gq[0][2], gq[0][3], gq[1][0], gq[1][1], gq[1][2], gq[1][3]};
          ga[st] = __builtin_bit_cast(bf16x8, gv8);
        }
#pragma unroll
        for (int u = 0; u < NW; ++u) {
          v4s hq[2];
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int jpos = kk * 32 + 8 * q + lds_row(8 * g + (r16 >> 2));
            const int dcol = (wave * NW + u) * 16 + 4 * (r16 & 3);
            hq[q] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(Yt + lds_pos<D>(jpos, dcol)));
          }
          v8s yv = {hq[0][0], hq[0][1], hq[0][2], hq[0][3], hq[1][0], hq[1][1], hq[1][2], hq[1][3]};
#pragma unroll
          for (int st = 0; st < 4; ++st)
            acc_dx[st * NW + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                ga[st], __builtin_bit_cast(bf16x8, yv), acc_dx[st * NW + u], 0, 0, 0);
        }
      }
    } else {
      // only this wave reads its strip back: a wave-local LDS wait suffices
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
      __builtin_amdgcn_wave_barrier();
      // dX[16 rows][D] += G[16][64] . Y[64][D]; lane (g, j) needs G[j][8g + 0..7]
      // and Y[8g + 0..7][d] of column d = nb*16 + j: transpose reads of 4 rows
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        v4s gq[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int krow = kk * 32 + 8 * g + 4 * q + (r16 >> 2);
          gq[q] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
              (lds_v4s*)(&Gt[wave][gt_at(krow, 4 * (r16 & 3))]));
        }
        v8s gv8 = {gq[0][0], gq[0][1], gq[0][2], gq[0][3], gq[1][0], gq[1][1], gq[1][2], gq[1][3]};
        const bf16x8 ga = __builtin_bit_cast(bf16x8, gv8);
        // up to four output blocks at a time: their B fragments read together
        constexpr int NU = NB < 4 ? NB : 4;
#pragma unroll
        for (int nb0 = 0; nb0 < NB; nb0 += NU) {
          v4s hq[NU][2];
#pragma unroll
          for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int q = 0; q < 2; ++q) {
              const int jpos = kk * 32 + 8 * q + lds_row(8 * g + (r16 >> 2));
              const int dcol = (nb0 + u) * 16 + 4 * (r16 & 3);
              hq[u][q] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(Yt + lds_pos<D>(jpos, dcol)));
            }
#pragma unroll
          for (int u = 0; u < NU; ++u) {
            v8s yv = {hq[u][0][0], hq[u][0][1], hq[u][0][2], hq[u][0][3],
                      hq[u][1][0], hq[u][1][1], hq[u][1][2], hq[u][1][3]};
            acc_dx[nb0 + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                ga, __builtin_bit_cast(bf16x8, yv), acc_dx[nb0 + u], 0, 0, 0);
          }
        }
      }
    }
    cvals = cpf;
    col_load(cpf, min(j0 + 2 * kFCols, jlast));
  }
  // write this split's partials (the two passes use separate halves)
  float* dst = a.dX_part + ((int64_t)TRANS * gridDim.y + blockIdx.y) * B * D;
  if constexpr (DSPLIT) {
#pragma unroll
    for (int st = 0; st < 4; ++st)
#pragma unroll
      for (int u = 0; u < NW; ++u)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = rb * kFRows + st * 16 + 4 * g + r;
          if (row < B) dst[(int64_t)row * D + (wave * NW + u) * 16 + r16] = acc_dx[st * NW + u][r];
        }
  } else {
#pragma unroll
    for (int nb = 0; nb < NB; ++nb)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = row_base + 4 * g + r;
        if (row < B) dst[(int64_t)row * D + nb * 16 + r16] = acc_dx[nb][r];
      }
  }
  if (L2) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float s = hsum[r];
#pragma unroll
      for (int o = 1; o <= 8; o <<= 1) s += __shfl_xor(s, o, 64);
      const int row = row_base + 4 * g + r;
      if (r16 == 0 && row < B) a.rs_part[((int64_t)TRANS * gridDim.y + blockIdx.y) * B + row] = s;
    }
  }
}

// Both gradients in one pass (D = 64): a workgroup of 16 wavefronts owns 256
// rows and 256 columns of the critic matrix, computes each 64-column tile of
// G once, and uses it twice:
//   dphi[rows] += G . psi[tile]        (wave w: its 16 rows, as in the row pass)
//   dpsi[tile]  = G^T . phi[rows]      (wave w: 16 columns x 16 features, K = 256)
// phi's 256 rows and the G tile stay in LDS, the tile transposed
// ([column][row]: each lane stores its four rows of a column as one 8-byte
// write); G^T rows are then plain 16-byte reads and the G strip of the first
// product a transpose read, as is phi in the second.  dphi partials go to
// split blockIdx.y (the column block), dpsi partials to split blockIdx.x (the
// row block); for L2 the row and column sums of H go with them.  The entries
// of G are formed as in infonce_bwd_kernel.
constexpr int kBRows = 256;  // rows (and columns) per workgroup of the one-pass backward
int fused_bwd_splits(int B) { return (B + kBRows - 1) / kBRows; }

template <int EN>
__global__ __launch_bounds__(1024) void infonce_bwd_both_kernel(FusedArgs a, int B, float beta,
                                                               float wf, float wb, float log2b) {
  constexpr bool L2 = EN != kEnDot;
  constexpr int D = 64, KS = 2, NB = 4;
  constexpr int LDX = D + 16;          // phi / psi rows in LDS (160 B, lds_at order)
  constexpr int LDGT = kBRows + 16;    // transposed G rows (one per column of the tile, lds_row order)
  // for the product energy, columns with bit 3 set swap adjacent 16-byte
  // chunks: the 8-byte G stores (16 lanes over 32 banks) are then two-way
  // instead of four-way conflicted, with both reads of the tile still
  // conflict-free (the distance energies have no registers to spare for it)
  const int hsw = EN == kEnDot ? 8 * ((threadIdx.x >> 3) & 1) : 0;  // column r16 + 16 m
  typedef short v4s __attribute__((ext_vector_type(4)));
  typedef short v8s __attribute__((ext_vector_type(8)));
  typedef __attribute__((address_space(3))) v4s lds_v4s;
  __shared__ __attribute__((aligned(16))) bf16_t Xs[kBRows * LDX];
  __shared__ __attribute__((aligned(16))) bf16_t Ys[2][kFCols * LDX];  // this tile and the next
  __shared__ __attribute__((aligned(16))) bf16_t Gt[kFCols * LDGT];
  __shared__ float csum[16][kFCols];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int r16 = lane & 15, g = lane >> 4;
  const int r0 = blockIdx.x * kBRows, cb0 = blockIdx.y * kBRows;
  const int row_base = r0 + wave * 16;
  const bool rows_full = row_base + 16 <= B;
  const float beta2 = 2.f * beta;
  const float dgv = (wf + wb) / (float)B;

  // phi rows of the block -> LDS (rows past B are zero)
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    const int v = tid + i * 1024;     // 16-byte vector: row v / 8, chunk v % 8
    const int r = v >> 3, c = v & 7;
    u32x4 val = {0u, 0u, 0u, 0u};
    if (r0 + r < B) val = *reinterpret_cast<const u32x4*>(a.phi_b + (int64_t)(r0 + r) * D + c * 8);
    *reinterpret_cast<u32x4*>(Xs + lds_at<D>(r, c * 8)) = val;
  }
  bf16x8 xa[KS];
  {
    const int row = row_base + r16;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      if (row < B) xa[ks] = *reinterpret_cast<const bf16x8*>(a.phi_b + (int64_t)row * D + ks * 32 + g * 8);
      else xa[ks] = bf16x8{};
    }
  }
  float nx[4], sh_r[4], k_r[4], hrow[4];
  bool rvalid[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = row_base + 4 * g + r;
    rvalid[r] = row < B;
    nx[r] = (L2 && rvalid[r]) ? a.nphi[row] : 0.f;
    const float lr = rvalid[r] ? a.r[row] : 0.f;
    sh_r[r] = __builtin_fmaf(lr, kL2E, log2b);
    k_r[r] = wf + beta2 * lr;
    hrow[r] = 0.f;
  }
  floatx4 acc_dx[NB];
#pragma unroll
  for (int nb = 0; nb < NB; ++nb) acc_dx[nb] = floatx4{0.f, 0.f, 0.f, 0.f};

  // psi tile loader: threads 0..511 move one 16-byte vector each
  auto y_load = [&](int j0) {
    u32x4 val = {0u, 0u, 0u, 0u};
    const int r = (tid & 511) >> 3, c = tid & 7;
    if (tid < 512 && j0 + r < B) val = *reinterpret_cast<const u32x4*>(a.psi_b + (int64_t)(j0 + r) * D + c * 8);
    return val;
  };
  const int ntiles = min(kBRows, B - cb0 + kFCols - 1) / kFCols;
  // tile t sits in Ys[t & 1]; ypf holds tile t + 1, stored into the other
  // buffer at the top of iteration t
  u32x4 ypf = y_load(cb0);
  if (tid < 512) *reinterpret_cast<u32x4*>(Ys[0] + lds_at<D>(tid >> 3, (tid & 7) * 8)) = ypf;
  if (ntiles > 1) ypf = y_load(cb0 + kFCols);
  for (int t = 0; t < ntiles; ++t) {
    const int j0 = cb0 + t * kFCols;
    // Ys[t & 1] and Xs are written; the previous tile's reads of Ys[(t + 1) & 1]
    // and of the G tile are done
    __syncthreads();
    if (t + 1 < ntiles) {
      if (tid < 512) *reinterpret_cast<u32x4*>(Ys[(t + 1) & 1] + lds_at<D>(tid >> 3, (tid & 7) * 8)) = ypf;
      if (t + 2 < ntiles) ypf = y_load(j0 + 2 * kFCols);
    }
    const bf16_t* __restrict__ Yt = Ys[t & 1];
    float sh_c[4], ny[4];
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      const int col = j0 + jb * 16 + r16;
      const bool cv = col < B;
      sh_c[jb] = (wb != 0.f && cv) ? __builtin_fmaf(a.c[col], kL2E, log2b) : INFINITY;
      ny[jb] = (L2 && cv) ? a.npsi[col] : 0.f;
    }
    floatx4 acc[4];
    tile_product<KS>(acc, xa, Yt, r16, g);
    // G (or H = G / d) of the wave's 16 rows, one 16-column block at a time;
    // row and column sums of H for L2
    const bool edge = !rows_full || j0 + kFCols > B;
    const bool diag = j0 <= row_base && row_base < j0 + kFCols;
    float hcol[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int jb = 0; jb < 4; ++jb) {
      float h[4], wv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float fv = energy_fw<EN>(acc[jb][r], nx[r], ny[jb], wv[r]);
        const float pa = __builtin_amdgcn_exp2f(__builtin_fmaf(fv, kL2E, -sh_r[r]));
        const float pb = __builtin_amdgcn_exp2f(__builtin_fmaf(fv, kL2E, -sh_c[jb]));
        h[r] = __builtin_fmaf(pa, k_r[r], pb);
      }
      if (diag) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          if (row_base + 4 * g + r == j0 + jb * 16 + r16) h[r] -= dgv;
      }
      if (edge) {
        const bool cv = j0 + jb * 16 + r16 < B;
#pragma unroll
        for (int r = 0; r < 4; ++r) h[r] = (cv && rvalid[r]) ? h[r] : 0.f;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (EN != kEnDot) h[r] *= wv[r];
        hrow[r] += h[r];
        hcol[jb] += h[r];
      }
      uint2 w;
      w.x = pack2bf(h[0], h[1]);
      w.y = pack2bf(h[2], h[3]);
      *reinterpret_cast<uint2*>(&Gt[(jb * 16 + lds_row(r16)) * LDGT + ((wave * 16 + 4 * g) ^ hsw)]) = w;
    }
    if (L2) {
#pragma unroll
      for (int jb = 0; jb < 4; ++jb) {
        float hc = hcol[jb];
        hc += __shfl_xor(hc, 16, 64);
        hc += __shfl_xor(hc, 32, 64);
        if (g == 0) csum[wave][jb * 16 + r16] = hc;
      }
    }
    // dphi[16 rows][D] += G[16][64] . Y[64][D] from the wave's own rows of
    // the tile (only this wave wrote them: a wave-local LDS wait suffices)
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      v4s gq[2];
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int kpos = kk * 32 + 8 * q + lds_row(8 * g + (r16 >> 2));
        gq[q] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
            (lds_v4s*)(&Gt[kpos * LDGT + ((wave * 16 + 4 * (r16 & 3)) ^ (EN == kEnDot ? 8 * (g & 1) : 0))]));
      }
      v8s gv8 = {gq[0][0], gq[0][1], gq[0][2], gq[0][3], gq[1][0], gq[1][1], gq[1][2], gq[1][3]};
      const bf16x8 ga = __builtin_bit_cast(bf16x8, gv8);
      // up to four output blocks at a time: their B fragments read together
      constexpr int NU = NB < 4 ? NB : 4;
#pragma unroll
      for (int nb0 = 0; nb0 < NB; nb0 += NU) {
        v4s hq[NU][2];
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const int jpos = kk * 32 + 8 * q + lds_row(8 * g + (r16 >> 2));
            const int dcol = (nb0 + u) * 16 + 4 * (r16 & 3);
            hq[u][q] = __builtin_amdgcn_ds_read_tr16_b64_v4i16((lds_v4s*)(Yt + lds_pos<D>(jpos, dcol)));
          }
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          v8s yv = {hq[u][0][0], hq[u][0][1], hq[u][0][2], hq[u][0][3],
                    hq[u][1][0], hq[u][1][1], hq[u][1][2], hq[u][1][3]};
          acc_dx[nb0 + u] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
              ga, __builtin_bit_cast(bf16x8, yv), acc_dx[nb0 + u], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // the whole G tile (and csum) is in LDS
    {
      // dpsi[16 columns cb16][16 features nb] = G^T . phi over the 256 rows:
      // A = G^T (lane (g, j): rows 32kk + 8g..+7 of column j, one 16-byte
      // read of the transposed tile), B = phi (rows 32kk + 8g..+7 of feature
      // j, transpose reads)
      const int cb16 = wave >> 2, nb = wave & 3;
      floatx4 acc_dy = floatx4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < kBRows / 32; ++kk) {
        const bf16x8 av =
            *reinterpret_cast<const bf16x8*>(&Gt[(cb16 * 16 + lds_row(r16)) * LDGT + ((kk * 32 + 8 * g) ^ hsw)]);
        v4s hb[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const int kpos = kk * 32 + 8 * q + lds_row(8 * g + (r16 >> 2));
          hb[q] = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
              (lds_v4s*)(Xs + lds_pos<D>(kpos, nb * 16 + 4 * (r16 & 3))));
        }
        v8s bv = {hb[0][0], hb[0][1], hb[0][2], hb[0][3], hb[1][0], hb[1][1], hb[1][2], hb[1][3]};
        acc_dy = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, __builtin_bit_cast(bf16x8, bv),
                                                         acc_dy, 0, 0, 0);
      }
      float* dst = a.dX_part + ((int64_t)gridDim.y + blockIdx.x) * B * D;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int col = j0 + cb16 * 16 + 4 * g + r;
        if (col < B) dst[(int64_t)col * D + nb * 16 + r16] = acc_dy[r];
      }
      if (L2 && tid < kFCols && j0 + tid < B) {
        float hs = 0.f;
#pragma unroll
        for (int w = 0; w < 16; ++w) hs += csum[w][tid];
        a.rs_part[((int64_t)gridDim.y + blockIdx.x) * B + j0 + tid] = hs;
      }
    }
  }
  // dphi partial of column block blockIdx.y
  float* dst = a.dX_part + (int64_t)blockIdx.y * B * D;
#pragma unroll
  for (int nb = 0; nb < NB; ++nb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row_base + 4 * g + r;
      if (row < B) dst[(int64_t)row * D + nb * 16 + r16] = acc_dx[nb][r];
    }
  if (L2) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      float hr = hrow[r];
#pragma unroll
      for (int o = 1; o <= 8; o <<= 1) hr += __shfl_xor(hr, o, 64);
      const int row = row_base + 4 * g + r;
      if (r16 == 0 && row < B) a.rs_part[(int64_t)blockIdx.y * B + row] = hr;
    }
  }
}

// dphi and dpsi (blockIdx.y) from the S split partials:
//   dX = sum_s part[s]  (- (sum_s rs[s]) * X_bf16 for the distance energies;
//   for the cosine energy, with U the BF16 unit rows: (dX - (dX . U) U) / |X|),
// FP32 and storage copies, four consecutive columns per thread (16-byte
// loads and stores); with bias_part set, also the column sums of each
// block's rows (the output layer's bias-gradient partials).  en: 0 dot,
// 1 distance, 2 cosine.  NT threads per block: red_threads(D).
constexpr int kRedVec = 4;  // columns per thread
template <typename OutT, int D, int NT>
__global__ __launch_bounds__(NT) void bwd_reduce_kernel(FusedArgs a, int S, int B, int en, int rounds) {
  constexpr int TPR = D / kRedVec;  // threads per row
  constexpr int TR = NT / TPR;      // rows per round; a block takes `rounds` rounds
  __shared__ float red[NT];
  __shared__ float4 redv[NT];
  const int side = blockIdx.y;
  const int c = threadIdx.x % TPR;
  const int64_t n = (int64_t)B * D;
  const bf16_t* __restrict__ Xb = side ? a.psi_b : a.phi_b;
  float4 bsum = make_float4(0.f, 0.f, 0.f, 0.f);  // this thread's columns over the block's rows
#pragma unroll 2
  for (int rd = 0; rd < rounds; ++rd) {
    const int row = (blockIdx.x * rounds + rd) * TR + threadIdx.x / TPR;
    const int64_t idx = (int64_t)row * D + c * kRedVec;
    float v[kRedVec] = {0.f, 0.f, 0.f, 0.f}, u[kRedVec] = {0.f, 0.f, 0.f, 0.f};
    if (row < B) {
      const float* __restrict__ part = a.dX_part + (int64_t)side * S * n + idx;
#pragma unroll 2
      for (int i = 0; i < S; ++i) {
        const float4 p = *reinterpret_cast<const float4*>(part + i * n);
        v[0] += p.x; v[1] += p.y; v[2] += p.z; v[3] += p.w;
      }
      if (en != 0) {
        const uint2 xw = *reinterpret_cast<const uint2*>(Xb + idx);
        u[0] = __builtin_bit_cast(float, xw.x << 16);
        u[1] = __builtin_bit_cast(float, xw.x & 0xffff0000u);
        u[2] = __builtin_bit_cast(float, xw.y << 16);
        u[3] = __builtin_bit_cast(float, xw.y & 0xffff0000u);
      }
      if (en == 1) {
        const float* __restrict__ rs = a.rs_part + (int64_t)side * S * B + row;
        float h = 0.f;
        for (int i = 0; i < S; ++i) h += rs[(int64_t)i * B];
#pragma unroll
        for (int k = 0; k < kRedVec; ++k) v[k] -= h * u[k];
      }
    }
    if (en == 2) {  // the row's dot product with its unit vector, a tree over its TPR threads
      red[threadIdx.x] = (v[0] * u[0] + v[1] * u[1]) + (v[2] * u[2] + v[3] * u[3]);
      __syncthreads();
      for (int o = TPR / 2; o > 0; o >>= 1) {
        if (c < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
      }
      const float dot = red[threadIdx.x - c];
      __syncthreads();
      if (row < B) {
        const float nr = (side ? a.npsi : a.nphi)[row];
#pragma unroll
        for (int k = 0; k < kRedVec; ++k) v[k] = nr > 0.f ? (v[k] - dot * u[k]) / nr : 0.f;
      }
    }
    if (row < B) {
      *reinterpret_cast<float4*>((side ? a.dpsi : a.dphi) + idx) = make_float4(v[0], v[1], v[2], v[3]);
      OutT* t = reinterpret_cast<OutT*>(side ? a.dpsi_t : a.dphi_t) + idx;
      if constexpr (sizeof(OutT) == 2)
        *reinterpret_cast<uint2*>(t) = make_uint2(pack2bf(v[0], v[1]), pack2bf(v[2], v[3]));
      else
        *reinterpret_cast<float4*>(t) = make_float4(v[0], v[1], v[2], v[3]);
      bsum.x += v[0]; bsum.y += v[1]; bsum.z += v[2]; bsum.w += v[3];  // rows past B add nothing
    }
  }
  float* bias = a.bias_part[side];
  if (bias == nullptr) return;
  redv[threadIdx.x] = bsum;
  __syncthreads();
  if (threadIdx.x < TPR) {
    float4 t = redv[threadIdx.x];
#pragma unroll
    for (int q = 1; q < TR; ++q) {
      const float4 w = redv[q * TPR + threadIdx.x];
      t.x += w.x; t.y += w.y; t.z += w.z; t.w += w.w;
    }
    *reinterpret_cast<float4*>(bias + (int64_t)blockIdx.x * D + threadIdx.x * kRedVec) = t;
  }
}

// Threads per block of the backward reduction: 1024 at D >= 128, so that a
// block's rounds (below) stay few and each SIMD holds eight wavefronts of
// them; 256 below.
static constexpr int red_threads(int D) { return D >= 128 ? 1024 : 256; }

// Rounds of red_threads(D) * kRedVec / D rows per block of the backward reduction:
// enough that the output layer's bias keeps at most 512 partial rows.  With
// one round it had 16384 at B = 16384, D = 256, which the gradient reduction
// sums serially per column (103 us for the reduction, 43.7 us with 512);
// capped at 256 the rounds left this kernel too few blocks (91 us against 56).
static int fused_bias_rounds(int B, int D) {
  const int tr = red_threads(D) * kRedVec / D;
  const int blocks = (B + tr - 1) / tr;
  return std::max(1, (blocks + 511) / 512);
}
int fused_bias_chunks(int B, int D) {
  const int rows = (red_threads(D) * kRedVec / D) * fused_bias_rounds(B, D);
  return (B + rows - 1) / rows;
}

#define CRL_FUSED_DISPATCH(KS_, BODY)                      \
  switch (D) {                                              \
    case 32:  { constexpr int KS_ = 1; BODY; } break;      \
    case 64:  { constexpr int KS_ = 2; BODY; } break;      \
    case 128: { constexpr int KS_ = 4; BODY; } break;      \
    case 256: { constexpr int KS_ = 8; BODY; } break;      \
    default: return hipErrorInvalidValue;                   \
  }

// Workgroups of the forward kernel for (D, energy) that the device holds at
// once (its register and LDS use decide how many fit on a CU), or 0 if unknown.
static int fwd_resident_wgs(int D, int en) {
  const void* k = nullptr;
#define CRL_FWD_PTR(KS_)                                                           \
  k = en == kEnL2 ? reinterpret_cast<const void*>(&infonce_fwd_kernel<KS_, kEnL2>)   \
    : en == kEnL2sq ? reinterpret_cast<const void*>(&infonce_fwd_kernel<KS_, kEnL2sq>) \
                    : reinterpret_cast<const void*>(&infonce_fwd_kernel<KS_, kEnDot>)
  switch (D) {
    case 32: CRL_FWD_PTR(1); break;
    case 64: CRL_FWD_PTR(2); break;
    case 128: CRL_FWD_PTR(4); break;
    case 256: CRL_FWD_PTR(8); break;
    default: return 0;
  }
#undef CRL_FWD_PTR
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// Column splits of the forward: fused_splits(B), or fewer where the kernel's
// resident capacity takes the launch in one round that way (D = 256 holds
// three workgroups per CU: 3 splits at B=16384 run in one round, 4 in two).
// The count returned is that of the non-empty splits once each split's
// columns are rounded up to whole 64-column tiles.
static int fused_fwd_splits(int B, int D, int en) {
  const int S = fused_splits(B);
  const int nrb = (B + kFRows - 1) / kFRows;
  const int cap = fwd_resident_wgs(D, en);
  if (cap <= 0 || (int64_t)nrb * S <= cap) return S;
  const int S1 = std::max(1, cap / nrb);
  // one round of S1 splits against ceil(nrb S / cap) rounds of S splits
  const int64_t rounds = ((int64_t)nrb * S + cap - 1) / cap;
  if ((int64_t)S1 * rounds <= S) return S;
  const int cps = cols_per_split(B, S1);
  return (B + cps - 1) / cps;
}

// Resident workgroups of the rows pass of the two-pass backward (the columns
// pass has the same resources).
static int bwd_resident_wgs(int D, int en) {
  const void* k = nullptr;
#define CRL_BWD_PTR(KS_)                                                              \
  k = en == kEnL2 ? reinterpret_cast<const void*>(&infonce_bwd_kernel<KS_, kEnL2, 0>)     \
    : en == kEnL2sq ? reinterpret_cast<const void*>(&infonce_bwd_kernel<KS_, kEnL2sq, 0>) \
                    : reinterpret_cast<const void*>(&infonce_bwd_kernel<KS_, kEnDot, 0>)
  switch (D) {
    case 32: CRL_BWD_PTR(1); break;
    case 64: CRL_BWD_PTR(2); break;
    case 128: CRL_BWD_PTR(4); break;
    case 256: CRL_BWD_PTR(8); break;
    default: return 0;
  }
#undef CRL_BWD_PTR
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, 256, 0) != hipSuccess)
    return 0;
  return per_cu * cus;
}

// Column splits of the two backward passes: each split writes a B x D
// partial of dX that bwd_reduce_kernel reads back, so take the fewest splits
// (at most fused_splits(B)) whose busiest workgroup slot carries no more
// 64-column tiles than with fused_splits(B): rounds of resident workgroups
// times tiles per workgroup (B=16384, D=256: 2 splits in one round of 512
// workgroups against 4 in two rounds, half the partials).
static int fused_bwd2_splits(int B, int D, int en) {
  const int S = fused_splits(B);
  const int nrb = (B + kFRows - 1) / kFRows;
  const int cap = bwd_resident_wgs(D, en);
  if (cap <= 0) return S;
  auto load = [&](int s) {
    const int64_t rounds = ((int64_t)nrb * s + cap - 1) / cap;
    return rounds * (cols_per_split(B, s) / kFCols);
  };
  const int64_t target = load(S);
  int best = S;
  for (int s = S - 1; s >= 1; --s)
    if (load(s) <= target) best = s;
  const int cps = cols_per_split(B, best);
  return (B + cps - 1) / cps;
}

#define CRL_EN_DISPATCH(EN_, BODY)                                  \
  switch (en) {                                                      \
    case kEnL2:   { constexpr int EN_ = kEnL2; BODY; } break;        \
    case kEnL2sq: { constexpr int EN_ = kEnL2sq; BODY; } break;      \
    default:      { constexpr int EN_ = kEnDot; BODY; } break;       \
  }

static const char* fused_name(const char* const names[3], int en) { return names[en]; }

hipError_t launch_fused_fwd(const FusedArgs& a, int B, int D, int energy, const GemmParams* top,
                            hipStream_t s) {
  const int en = fused_energy(energy);
  const int unit = energy == CRL_ENERGY_COS;
  if (top)
    CRL_TIMED("fused_prep_reduce_kernel", 0.0, 2.0 * B * D * (4.0 * top->splits + 10.0), s,
              fused_prep_reduce_kernel<<<dim3((B + 3) / 4, 2), 256, 0, s>>>(a, *top, B, D, unit));
  else
    CRL_TIMED("fused_prep_kernel", 0.0, 2.0 * B * D * 6.0, s,
              fused_prep_kernel<<<dim3((B + 3) / 4, 2), 256, 0, s>>>(a, B, D, unit));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int S = fused_fwd_splits(B, D, en), cps = cols_per_split(B, S);
  const int nrb = (B + kFRows - 1) / kFRows;
  dim3 grid(nrb, S);
  const double fw_flops = 2.0 * B * B * D;
  const double fw_bytes = 2.0 * 2.0 * B * D + 4.0 * 2.0 * ((double)S * B + (double)nrb * B);
  static const char* const names[3] = {"infonce_fwd_kernel<dot>", "infonce_fwd_kernel<l2>",
                                       "infonce_fwd_kernel<l2sq>"};
  KTimer t = timing_begin(fused_name(names, en), fw_flops, fw_bytes, s);
  CRL_EN_DISPATCH(EN, CRL_FUSED_DISPATCH(KS, (infonce_fwd_kernel<KS, EN><<<grid, 256, 0, s>>>(a, B, cps))))
  timing_end(t);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  LseMergeArgs m{};  // row LSEs over the column splits, column LSEs over the row blocks
  m.pm[0] = a.row_m; m.ps[0] = a.row_s; m.nparts[0] = S; m.out[0] = a.r;
  m.pm[1] = a.col_m; m.ps[1] = a.col_s; m.nparts[1] = nrb; m.out[1] = a.c;
  return launch_lse_merge(m, 2, B, s);
}

// The one-pass backward (D = 64) writes ceil(B / 256) partials per row of
// dphi and of dpsi, B x 64 floats each; above kBothMaxSplits partials the
// row and column passes run instead, whose partial count is bounded by
// fused_splits (at most 16).
constexpr int kBothMaxSplits = 16;
bool fused_bwd_one_pass(int B, int D) { return D == 64 && fused_bwd_splits(B) <= kBothMaxSplits; }

hipError_t launch_fused_bwd(const FusedArgs& a, int B, int D, int energy, int loss, float beta,
                            bool out_bf16, hipStream_t s) {
  const int en = fused_energy(energy);
  const float wf = (loss == CRL_LOSS_FWD || loss == CRL_LOSS_SYM || loss == CRL_LOSS_FLATNCE_FWD) ? 1.f : 0.f;
  const float wb = (loss == CRL_LOSS_SYM || loss == CRL_LOSS_BWD || loss == CRL_LOSS_FLATNCE_BWD) ? 1.f : 0.f;
  const int64_t n = (int64_t)B * D;
  const float l2b = (float)std::log2((double)B);
  const bool one = fused_bwd_one_pass(B, D);
  int S = one ? 0 : fused_bwd2_splits(B, D, en);
  if (one) {  // one pass for both gradients
    S = fused_bwd_splits(B);
    const dim3 grid(S, S);
    const double flops = 4.0 * B * B * D;  // G . psi and G^T . phi; the tile recompute is not counted
    const double bytes = 2.0 * 2.0 * B * D + 4.0 * 2.0 * B + 2.0 * 4.0 * (double)S * B * (D + 1.0);
    static const char* const names[3] = {"infonce_bwd_both_kernel<dot>",
                                         "infonce_bwd_both_kernel<l2>",
                                         "infonce_bwd_both_kernel<l2sq>"};
    KTimer t = timing_begin(fused_name(names, en), flops, bytes, s);
    CRL_EN_DISPATCH(EN, (infonce_bwd_both_kernel<EN><<<grid, 1024, 0, s>>>(a, B, beta, wf, wb, l2b)))
    timing_end(t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int cps = cols_per_split(B, S);
  const int nrb = (B + kFRows - 1) / kFRows;
  dim3 grid(nrb, S);
  const double bw_flops = 2.0 * B * B * D;  // G . Y per pass; the tile recompute is not counted
  const double bw_bytes = 2.0 * 2.0 * B * D + 4.0 * 2.0 * B + 4.0 * (double)S * B * (D + 1.0);
  for (int pass = 0; pass < (one ? 0 : 2); ++pass) {
    KTimer t = timing_begin(pass ? "infonce_bwd_kernel<cols>" : "infonce_bwd_kernel<rows>",
                            bw_flops, bw_bytes, s);
    if (pass == 0) {
      CRL_EN_DISPATCH(EN, CRL_FUSED_DISPATCH(KS, (infonce_bwd_kernel<KS, EN, 0><<<grid, 256, 0, s>>>(a, B, cps, beta, wf, wb, l2b))))
    } else {
      CRL_EN_DISPATCH(EN, CRL_FUSED_DISPATCH(KS, (infonce_bwd_kernel<KS, EN, 1><<<grid, 256, 0, s>>>(a, B, cps, beta, wf, wb, l2b))))
    }
    timing_end(t);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const int ren = energy == CRL_ENERGY_COS ? 2 : (en != kEnDot ? 1 : 0);
  const dim3 rgrid(fused_bias_chunks(B, D), 2);
  const int rounds = fused_bias_rounds(B, D);
  const double rb = 2.0 * (4.0 * (double)n * (S + 1.0) + (double)n * (out_bf16 ? 2 : 4));
  if (out_bf16) {
    CRL_TIMED("bwd_reduce_kernel", 0.0, rb, s,
              CRL_FUSED_DISPATCH(KS, (bwd_reduce_kernel<bf16_t, KS * 32, red_threads(KS * 32)>
                                      <<<rgrid, red_threads(KS * 32), 0, s>>>(a, S, B, ren, rounds))));
  } else {
    CRL_TIMED("bwd_reduce_kernel", 0.0, rb, s,
              CRL_FUSED_DISPATCH(KS, (bwd_reduce_kernel<float, KS * 32, red_threads(KS * 32)>
                                      <<<rgrid, red_threads(KS * 32), 0, s>>>(a, S, B, ren, rounds))));
  }
  return hipGetLastError();
}

}  // namespace crl
