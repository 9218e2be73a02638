// Relabel/gather, LayerNorm+Swish, column reductions, materialised InfoNCE,
// Adam and small utility kernels (gfx950, wave64).
#include "internal.hpp"
#include "relabel.hpp"

namespace crl {

// One wavefront per sample: draw (e, t, k), then copy the rows.
template <typename T>
__global__ __launch_bounds__(256) void relabel_kernel(
    const float* __restrict__ obs, const float* __restrict__ act, int E, int T_,
    int d_s, int d_a, int d_g, int goal_lo, uint64_t seed, const int64_t* __restrict__ step,
    const uint64_t* __restrict__ thr, int B, int32_t* __restrict__ idx,
    T* __restrict__ x_sa, int ld_sa, T* __restrict__ x_g, int ld_g,
    T* __restrict__ x_sg, int ld_sg) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;
  const GeomProbe probe = geom_prefetch(thr, T_ - 2, lane);
  uint64_t x[4] = {(uint64_t)b, (uint64_t)(*step), 0ull, 0ull};
  philox4x64_10(x, seed, 0ull);
  const int e = (int)__umul64hi(x[0], (uint64_t)E);
  const int t = (int)__umul64hi(x[1], (uint64_t)(T_ - 1));
  const int km1 = geom_count(thr, probe, x[2], lane);  // k - 1
  const int tg = min(t + 1 + km1, T_ - 1);
  if (lane == 0) {
    idx[3 * b + 0] = e;
    idx[3 * b + 1] = t;
    idx[3 * b + 2] = tg;
  }
  const float* s_row = obs + ((int64_t)e * T_ + t) * d_s;
  const float* a_row = act + ((int64_t)e * T_ + t) * d_a;
  const float* g_row = obs + ((int64_t)e * T_ + tg) * d_s + goal_lo;
  write_inputs<T>(s_row, a_row, g_row, d_s, d_a, d_g, b, lane, x_sa, ld_sa, x_g, ld_g, x_sg,
                  ld_sg);
}

hipError_t launch_relabel(const float* obs, const float* act, int E, int T, int d_s,
                          int d_a, int d_g, int goal_lo, uint64_t seed,
                          const int64_t* step, const uint64_t* thr, int B,
                          int32_t* idx, void* x_sa, int ld_sa, void* x_g, int ld_g,
                          void* x_sg, int ld_sg, bool bf16, hipStream_t s) {
  dim3 grid((B + 3) / 4), block(256);
  const double es = bf16 ? 2.0 : 4.0;
  const double bytes = (double)B * (4.0 * (d_s + d_a + d_g + (x_sg ? d_s + d_g : 0)) +
                                    es * (ld_sa + ld_g + (x_sg ? ld_sg : 0)) + 12.0);
  if (bf16)
    CRL_TIMED("relabel_kernel", 0.0, bytes, s,
      relabel_kernel<bf16_t><<<grid, block, 0, s>>>(obs, act, E, T, d_s, d_a, d_g, goal_lo,
        seed, step, thr, B, idx, (bf16_t*)x_sa, ld_sa, (bf16_t*)x_g, ld_g,
        (bf16_t*)x_sg, ld_sg));
  else
    CRL_TIMED("relabel_kernel", 0.0, bytes, s,
      relabel_kernel<float><<<grid, block, 0, s>>>(obs, act, E, T, d_s, d_a, d_g, goal_lo,
        seed, step, thr, B, idx, (float*)x_sa, ld_sa, (float*)x_g, ld_g,
        (float*)x_sg, ld_sg));
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// 8-element row chunks
// ---------------------------------------------------------------------------
__device__ inline void load8(const float* p, float (&o)[8]) {
  float4 a = *reinterpret_cast<const float4*>(p);
  float4 b = *reinterpret_cast<const float4*>(p + 4);
  o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
  o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
}
__device__ inline void load8(const bf16_t* p, float (&o)[8]) {
  uint4 u = *reinterpret_cast<const uint4*>(p);
  const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    o[2 * i] = __builtin_bit_cast(float, w[i] << 16);
    o[2 * i + 1] = __builtin_bit_cast(float, w[i] & 0xffff0000u);
  }
}
__device__ inline void store8(float* p, const float (&o)[8]) {
  *reinterpret_cast<float4*>(p) = make_float4(o[0], o[1], o[2], o[3]);
  *reinterpret_cast<float4*>(p + 4) = make_float4(o[4], o[5], o[6], o[7]);
}
__device__ inline void store8(bf16_t* p, const float (&o)[8]) {
  uint4 u;
  u.x = pack2bf(o[0], o[1]);
  u.y = pack2bf(o[2], o[3]);
  u.z = pack2bf(o[4], o[5]);
  u.w = pack2bf(o[6], o[7]);
  *reinterpret_cast<uint4*>(p) = u;
}

// ---------------------------------------------------------------------------
// LayerNorm (biased variance over the N features) -> affine -> Swish.
// One wavefront per row; lane owns chunks lane, lane+64, ... of 8 features.
// ---------------------------------------------------------------------------
// 16-byte raw chunk of a row (8 BF16 or 4 FP32 values; FP32 rows use two)
template <typename T> struct RawChunk;
template <> struct RawChunk<bf16_t> {
  u32x4 w;
  __device__ inline void load(const bf16_t* p) { w = *reinterpret_cast<const u32x4*>(p); }
  __device__ inline void get(float (&o)[8]) const {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      o[2 * i] = __builtin_bit_cast(float, w[i] << 16);
      o[2 * i + 1] = __builtin_bit_cast(float, w[i] & 0xffff0000u);
    }
  }
};
template <> struct RawChunk<float> {
  float4 a, b;
  __device__ inline void load(const float* p) {
    a = *reinterpret_cast<const float4*>(p);
    b = *reinterpret_cast<const float4*>(p + 4);
  }
  __device__ inline void get(float (&o)[8]) const {
    o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
    o[4] = b.x; o[5] = b.y; o[6] = b.z; o[7] = b.w;
  }
};

template <typename T, int CH>
__global__ __launch_bounds__(256) void ln_swish_fwd_kernel(LnArgs a, int B, int N, float eps) {
  const int e = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= B) return;  // whole wavefronts: the row sums below see all 64 lanes
  const int nch = N >> 3;
  const T* z = reinterpret_cast<const T*>(a.Z[e]) + (int64_t)row * N;
  T* h = reinterpret_cast<T*>(a.H[e]) + (int64_t)row * N;
  // every load of the wave is issued before the first value is used
  RawChunk<T> zr[CH];
  float v[CH][8], gv[CH][8], bv[CH][8];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int ch = lane + 64 * c;
    if (ch < nch) {
      zr[c].load(z + ch * 8);
      load8(a.g[e] + ch * 8, gv[c]);
      load8(a.b[e] + ch * 8, bv[c]);
    }
  }
#pragma unroll
  for (int c = 0; c < CH; ++c)
    if (lane + 64 * c < nch) zr[c].get(v[c]);
  float s = 0.f;
#pragma unroll
  for (int c = 0; c < CH; ++c)
    if (lane + 64 * c < nch)
#pragma unroll
      for (int i = 0; i < 8; ++i) s += v[c][i];
  const float inv_n = 1.f / (float)N;  // exact for the power-of-two widths
  const float mean = wave_sum_full(s) * inv_n;
  float q = 0.f;
#pragma unroll
  for (int c = 0; c < CH; ++c)
    if (lane + 64 * c < nch)
#pragma unroll
      for (int i = 0; i < 8; ++i) { float d = v[c][i] - mean; q += d * d; }
  const float var = wave_sum_full(q) * inv_n;
  const float rstd = __builtin_amdgcn_rsqf(var + eps);  // hardware 1/sqrt (1 ulp)
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int ch = lane + 64 * c;
    if (ch < nch) {
      float o[8];
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        float y = gv[c][i] * ((v[c][i] - mean) * rstd) + bv[c][i];
        o[i] = y * sigmoidf_(y);
      }
      store8(h + ch * 8, o);
    }
  }
  if (lane == 0) { a.mu[e][row] = mean; a.rstd[e][row] = rstd; }
}

hipError_t launch_ln_swish_fwd(const LnArgs& a, int count, int B, int N, float eps,
                               bool bf16, hipStream_t s) {
  dim3 grid((B + 3) / 4, count), block(256);
  int ch = (N / 8 + 63) / 64;
  const double lnf_bytes = (double)count * B * N * 2.0 * (bf16 ? 2 : 4);
#define LNF(T, C) CRL_TIMED("ln_swish_fwd_kernel", 0.0, lnf_bytes, s, \
                            ln_swish_fwd_kernel<T, C><<<grid, block, 0, s>>>(a, B, N, eps))
  // hidden widths are at most 1024 (checked at context creation): CH <= 2
  if (bf16) { if (ch <= 1) LNF(bf16_t, 1); else LNF(bf16_t, 2); }
  else      { if (ch <= 1) LNF(float, 1);  else LNF(float, 2); }
#undef LNF
  return hipGetLastError();
}

// Backward of h = Swish(g * zhat + b), zhat = (z - mu) * rstd.  Each
// workgroup owns `rows` rows (a multiple of kLnRows, taken kLnRows at a time,
// kLnRows / 4 per wavefront, one row at a time):
//   dy = dh * Swish'(y), dzhat = g * dy,
//   dz = rstd * (dzhat - mean(dzhat) - zhat * mean(dzhat * zhat)),
// and it accumulates the column sums dg = sum dy*zhat, db_ln = sum dy,
// db_linear = sum dz of its rows; the four wavefronts' sums are added in LDS
// in a fixed order and written as one partial row per workgroup.
constexpr int kLnRows = 16;

template <typename T, int CH>
__global__ __launch_bounds__(256) void ln_swish_bwd_kernel(LnArgs a, int B, int N, int rows) {
  extern __shared__ float red[];  // [4 waves][3][N]
  constexpr int R = kLnRows / 4;  // rows per wavefront
  const int e = blockIdx.y;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nch = N >> 3;
  const T* Zb = reinterpret_cast<const T*>(a.Z[e]);
  const T* dHb = reinterpret_cast<const T*>(a.dH[e]);
  T* dZb = reinterpret_cast<T*>(a.dZ[e]);
  float gv[CH][8], bv[CH][8], cg[CH][8], cb[CH][8], cz[CH][8];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int ch = lane + 64 * c;
#pragma unroll
    for (int i = 0; i < 8; ++i) { cg[c][i] = cb[c][i] = cz[c][i] = gv[c][i] = bv[c][i] = 0.f; }
    if (ch < nch) { load8(a.g[e] + ch * 8, gv[c]); load8(a.b[e] + ch * 8, bv[c]); }
  }
  const float inv_n = 1.f / (float)N;
  // rounds of kLnRows rows (R per wavefront) over the workgroup's rows; the
  // column sums run on across the rounds
  const int wg_end = min(B, (blockIdx.x + 1) * rows);
  for (int base = blockIdx.x * rows; base < wg_end; base += kLnRows) {
    const int r0 = base + wave * R;
    const int nr = max(0, min(R, B - r0));
    // all rows of this wavefront are requested before any is used
    RawChunk<T> zr[R][CH], hr[R][CH];
    float mu[R], rs[R];
#pragma unroll
    for (int j = 0; j < R; ++j) {
      mu[j] = rs[j] = 0.f;
      if (j < nr) {
        mu[j] = a.mu[e][r0 + j];
        rs[j] = a.rstd[e][r0 + j];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
          const int ch = lane + 64 * c;
          if (ch < nch) {
            zr[j][c].load(Zb + (int64_t)(r0 + j) * N + ch * 8);
            hr[j][c].load(dHb + (int64_t)(r0 + j) * N + ch * 8);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < R; ++j) {
      if (j >= nr) break;  // uniform over the wavefront, as the row sums need
      const int row = r0 + j;
      float zh[CH][8], dzh[CH][8];
      float s1 = 0.f, s2 = 0.f;
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int ch = lane + 64 * c;
        if (ch < nch) {
          float z[8], dh[8];
          zr[j][c].get(z);
          hr[j][c].get(dh);
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const float xh = (z[i] - mu[j]) * rs[j];
            const float y = __builtin_fmaf(gv[c][i], xh, bv[c][i]);
            const float sg = sigmoidf_(y);
            // Swish'(y) = sg (1 + y (1 - sg)) = sg + y sg (1 - sg)
            const float q = __builtin_fmaf(-sg, sg, sg);
            const float dy = dh[i] * __builtin_fmaf(y, q, sg);
            cg[c][i] += dy * xh;
            cb[c][i] += dy;
            const float d = dy * gv[c][i];
            zh[c][i] = xh;
            dzh[c][i] = d;
            s1 += d;
            s2 += d * xh;
          }
        }
      }
      // dz = rstd (dzhat - m1 - zhat m2) = rstd dzhat + (e zhat + k),
      // e = -rstd m2, k = -rstd m1
      const float k = -rs[j] * (wave_sum_full(s1) * inv_n);
      const float e = -rs[j] * (wave_sum_full(s2) * inv_n);
#pragma unroll
      for (int c = 0; c < CH; ++c) {
        const int ch = lane + 64 * c;
        if (ch < nch) {
          float o[8];
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            o[i] = __builtin_fmaf(rs[j], dzh[c][i], __builtin_fmaf(e, zh[c][i], k));
            cz[c][i] += o[i];
          }
          store8(dZb + (int64_t)row * N + ch * 8, o);
        }
      }
    }
  }
  float* mine = red + (int64_t)wave * 3 * N;
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int ch = lane + 64 * c;
    if (ch < nch) {
      store8(mine + ch * 8, cg[c]);
      store8(mine + N + ch * 8, cb[c]);
      store8(mine + 2 * N + ch * 8, cz[c]);
    }
  }
  __syncthreads();
  // N is a multiple of 8: the four wave rows and the partial row in float4s
  const float4* r4 = reinterpret_cast<const float4*>(red);
  float4* p4 = reinterpret_cast<float4*>(a.part[e] + (int64_t)blockIdx.x * 3 * N);
  const int n4 = 3 * N / 4;
  for (int k = threadIdx.x; k < n4; k += 256) {
    const float4 w0 = r4[k], w1 = r4[n4 + k], w2 = r4[2 * n4 + k], w3 = r4[3 * n4 + k];
    float4 o;
    o.x = (w0.x + w1.x) + (w2.x + w3.x);
    o.y = (w0.y + w1.y) + (w2.y + w3.y);
    o.z = (w0.z + w1.z) + (w2.z + w3.z);
    o.w = (w0.w + w1.w) + (w2.w + w3.w);
    p4[k] = o;
  }
}

// Rows per workgroup: kLnRows up to B = 4096 (one round of at most 512
// workgroups for two encoders), then more rounds per workgroup instead of
// more workgroups, so the column partials (3 N floats per workgroup, summed
// again in the gradient reduction) stop growing with B.
int ln_bwd_rows(int B) { return kLnRows * std::max(1, (B + 4095) / 4096); }
int ln_bwd_partials(int B, int) {
  const int rows = ln_bwd_rows(B);
  return (B + rows - 1) / rows;
}

hipError_t launch_ln_swish_bwd(const LnArgs& a, int count, int B, int N, bool bf16, int,
                               hipStream_t s) {
  const int ch = (N / 8 + 63) / 64;
  const int rows = ln_bwd_rows(B);
  const int nparts = ln_bwd_partials(B, 0);
  dim3 grid(nparts, count), block(256);
  const size_t lds = (size_t)4 * 3 * N * sizeof(float);
  const double bytes = (double)count * ((double)B * N * 3.0 * (bf16 ? 2 : 4) + 12.0 * nparts * N);
#define LNB(T, C) CRL_TIMED("ln_swish_bwd_kernel", 0.0, bytes, s, \
                            ln_swish_bwd_kernel<T, C><<<grid, block, lds, s>>>(a, B, N, rows))
  if (bf16) { if (ch <= 1) LNB(bf16_t, 1); else LNB(bf16_t, 2); }
  else      { if (ch <= 1) LNB(float, 1);  else LNB(float, 2); }
#undef LNB
  return hipGetLastError();
}

// 4-element chunks for the column kernels
__device__ inline void load4(const float* p, float (&o)[4]) {
  float4 a = *reinterpret_cast<const float4*>(p);
  o[0] = a.x; o[1] = a.y; o[2] = a.z; o[3] = a.w;
}
__device__ inline void load4(const bf16_t* p, float (&o)[4]) {
  uint2 u = *reinterpret_cast<const uint2*>(p);
  o[0] = __builtin_bit_cast(float, u.x << 16);
  o[1] = __builtin_bit_cast(float, u.x & 0xffff0000u);
  o[2] = __builtin_bit_cast(float, u.y << 16);
  o[3] = __builtin_bit_cast(float, u.y & 0xffff0000u);
}

constexpr int kColRows = 128;  // rows per chunk of the column-sum kernel

// out[k][n] = sum over w of part[w][k][n]: 16 outputs per workgroup, the
// parts split over 16 groups (w = grp, grp + 16, ...; four independent running
// sums per thread), then a fixed-order tree over the groups in LDS.
__global__ __launch_bounds__(256) void partial_reduce_kernel(ColReduceArgs a, int nparts,
                                                             int nk, int N) {
  __shared__ float red[16][17];
  const int e = blockIdx.y;
  const int col = threadIdx.x & 15, grp = threadIdx.x >> 4;
  const int i = blockIdx.x * 16 + col;
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  if (i < nk * N) {
    const float* p = a.part[e] + i;
    const int64_t st = (int64_t)nk * N;
    int w = grp;
    for (; w + 48 < nparts; w += 64) {
      s0 += p[w * st];
      s1 += p[(w + 16) * st];
      s2 += p[(w + 32) * st];
      s3 += p[(w + 48) * st];
    }
    for (; w < nparts; w += 16) s0 += p[w * st];
  }
  red[grp][col] = (s0 + s1) + (s2 + s3);
  __syncthreads();
  for (int h = 8; h >= 1; h >>= 1) {
    if (grp < h) red[grp][col] += red[grp + h][col];
    __syncthreads();
  }
  if (grp == 0 && i < nk * N) a.out[e][i / N][i % N] = red[0][col];
}

hipError_t launch_partial_reduce(const ColReduceArgs& a, int count, int nparts, int nk,
                                 int N, hipStream_t s) {
  dim3 grid((nk * N + 15) / 16, count), block(256);
  CRL_TIMED("partial_reduce_kernel", 0.0, 4.0 * count * (nparts + 1.0) * nk * N, s,
            partial_reduce_kernel<<<grid, block, 0, s>>>(a, nparts, nk, N));
  return hipGetLastError();
}

// Column sums of X [B][ld] over one chunk of rows (same block shape as above).
template <typename T>
__global__ __launch_bounds__(256) void colsum_partial_kernel(ColSumArgs a, int B, int N, int ld) {
  __shared__ float red[4][256];
  const int e = blockIdx.z;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int n0 = blockIdx.x * 256 + lane * 4;
  const int r0 = blockIdx.y * kColRows, r1 = min(B, r0 + kColRows);
  float acc[4] = {0, 0, 0, 0};
  if (n0 < N) {
    const T* X = reinterpret_cast<const T*>(a.X[e]);
    // the wavefront's rows r0 + wave, + 4, + 8, ... in that order, eight
    // rows' loads in flight before they are added
    int row = r0 + wave;
    for (; row + 28 < r1; row += 32) {
      float v[8][4];
#pragma unroll
      for (int k = 0; k < 8; ++k) load4(X + (int64_t)(row + 4 * k) * ld + n0, v[k]);
#pragma unroll
      for (int k = 0; k < 8; ++k)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[i] += v[k][i];
    }
    for (; row < r1; row += 4) {
      float v[4];
      load4(X + (int64_t)row * ld + n0, v);
#pragma unroll
      for (int i = 0; i < 4; ++i) acc[i] += v[i];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) red[wave][lane * 4 + i] = acc[i];
  __syncthreads();
  const int t = threadIdx.x;
  const int n = blockIdx.x * 256 + t;
  if (n < N)
    a.part[e][(int64_t)blockIdx.y * N + n] = (red[0][t] + red[1][t]) + (red[2][t] + red[3][t]);
}

int colsum_chunks(int B) { return (B + kColRows - 1) / kColRows; }

hipError_t launch_colsum_partials(const ColSumArgs& a, int count, int B, int N, int ld,
                                  bool bf16, hipStream_t s) {
  // N and ld must be multiples of 4 (vector loads of 4 elements)
  const int nrb = colsum_chunks(B);
  dim3 grid((N + 255) / 256, nrb, count), block(256);
  const double cs_bytes = (double)count * B * N * (bf16 ? 2 : 4);
  if (bf16) CRL_TIMED("colsum_partial_kernel", 0.0, cs_bytes, s,
                      colsum_partial_kernel<bf16_t><<<grid, block, 0, s>>>(a, B, N, ld));
  else      CRL_TIMED("colsum_partial_kernel", 0.0, cs_bytes, s,
                      colsum_partial_kernel<float><<<grid, block, 0, s>>>(a, B, N, ld));
  return hipGetLastError();
}

hipError_t launch_colsum(const ColSumArgs& a, int count, int B, int N, int ld, bool bf16,
                         hipStream_t s) {
  const int nrb = colsum_chunks(B);
  hipError_t err = launch_colsum_partials(a, count, B, N, ld, bf16, s);
  if (err != hipSuccess) return err;
  ColReduceArgs r{};
  for (int e = 0; e < count; ++e) { r.part[e] = a.part[e]; r.out[e][0] = a.out[e]; }
  return launch_partial_reduce(r, count, nrb, 1, N, s);
}

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
// One Adam update, written with explicit fused multiply-adds so that every
// kernel that applies it rounds the same way:
//   m = b1 m + (1-b1) g,  v = b2 v + (1-b2) g^2,
//   p -= lr (m c1) / (sqrt(v c2) + eps),  c1 = 1/(1 - b1^t), c2 = 1/(1 - b2^t).
__device__ __forceinline__ float adam_update(float& p, float g, float& m, float& v, float c1,
                                             float c2, const AdamCoef& c) {
  m = __builtin_fmaf(c.b1, m, c.omb1 * g);
  v = __builtin_fmaf(c.b2, v, (c.omb2 * g) * g);
  p = p - (c.lr * (m * c1)) / (sqrtf(v * c2) + c.eps);
  return p;
}
// bias-correction factors 1 / (1 - b^t) = -1 / expm1(t log b): full FP32
// relative accuracy (no cancellation in 1 - b^t)
__device__ __forceinline__ void adam_factors(const AdamCoef& c, const int64_t* step, float& c1,
                                             float& c2) {
  const float t = (float)(*step);
  c1 = 1.f / (-expm1f(t * c.log_b1));
  c2 = 1.f / (-expm1f(t * c.log_b2));
}
// Adam on parameter k with gradient gk
__device__ __forceinline__ void adam_at(const AdamArgs& A, float c1, float c2, int64_t k,
                                        float gk) {
  float pk = A.p[k], mk = A.m[k], vk = A.v[k];
  adam_update(pk, gk, mk, vk, c1, c2, A.c);
  A.p[k] = pk;
  A.m[k] = mk;
  A.v[k] = vk;
  if (A.pb) A.pb[k] = f2bf(pk);
}
// ... on the four parameters k4 * 4 + 0..3 (16-byte aligned)
__device__ __forceinline__ void adam_at4(const AdamArgs& A, float c1, float c2, int64_t k4,
                                         float4 gg) {
  float4 pp = reinterpret_cast<float4*>(A.p)[k4];
  float4 mm = reinterpret_cast<float4*>(A.m)[k4];
  float4 vv = reinterpret_cast<float4*>(A.v)[k4];
  adam_update(pp.x, gg.x, mm.x, vv.x, c1, c2, A.c);
  adam_update(pp.y, gg.y, mm.y, vv.y, c1, c2, A.c);
  adam_update(pp.z, gg.z, mm.z, vv.z, c1, c2, A.c);
  adam_update(pp.w, gg.w, mm.w, vv.w, c1, c2, A.c);
  reinterpret_cast<float4*>(A.p)[k4] = pp;
  reinterpret_cast<float4*>(A.m)[k4] = mm;
  reinterpret_cast<float4*>(A.v)[k4] = vv;
  if (A.pb) {
    uint2 u;
    u.x = pack2bf(pp.x, pp.y);
    u.y = pack2bf(pp.z, pp.w);
    reinterpret_cast<uint2*>(A.pb)[k4] = u;
  }
}

// last job whose `first` is <= v (jobs sorted by `first`)
__device__ inline int find_job(const RedJob* __restrict__ jobs, int njobs, int64_t v) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].first <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// sum of a float4 over the job's parts, in part order (four running sums)
__device__ __forceinline__ float4 sum_parts(const float4* __restrict__ p, int64_t st,
                                            int nparts) {
  float4 s[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) s[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  int k = 0;
  for (; k + 3 < nparts; k += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = p[(k + q) * st];
      s[q].x += t.x; s[q].y += t.y; s[q].z += t.z; s[q].w += t.w;
    }
  }
  for (; k < nparts; ++k) {
    const float4 t = p[k * st];
    s[0].x += t.x; s[0].y += t.y; s[0].z += t.z; s[0].w += t.w;
  }
  float4 r;
  r.x = (s[0].x + s[1].x) + (s[2].x + s[3].x);
  r.y = (s[0].y + s[1].y) + (s[2].y + s[3].y);
  r.z = (s[0].z + s[1].z) + (s[2].z + s[3].z);
  r.w = (s[0].w + s[1].w) + (s[2].w + s[3].w);
  return r;
}

// last job whose first_chunk is <= v
__device__ inline int find_job_chunk(const RedJob* __restrict__ jobs, int njobs, int64_t v) {
  int lo = 0, hi = njobs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (jobs[mid].first_chunk <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Few parts with the Adam epilogue: block blk takes chunk c of one job
// (kRedChunk4 float4 outputs, 4 per thread).  Dense jobs step their float4s
// in place.  Fragment-order jobs hold each tile wave by wave (64 x 32 per
// wave, bn / 32 waves per 64-row half); a chunk is two consecutive waves, a
// 64 x 64 block of the tile, whose partials are summed into an LDS copy of
// the block and then stepped row by row, so that p, m, v move in 256-byte
// row runs.  (Half-tile chunks took half the blocks, too few to fill the
// chip when the vector is small.)
constexpr int kRedWaves = kRedChunk4 * 4 / 2048;  // waves of a tile per chunk
constexpr int kRedCols = 32 * kRedWaves;          // block columns
constexpr int kRedLdsFloats = 64 * (kRedCols + 4);
static_assert(kRedWaves == 2, "a chunk is two waves: a 64 x 64 block of a 64- or 128-wide tile");
__device__ __forceinline__ void reduce_few_adam(const char* __restrict__ ws,
                                                float* __restrict__ g,
                                                const RedJob* __restrict__ jobs, int njobs,
                                                int64_t blk, const AdamArgs& A, float c1,
                                                float c2, float* __restrict__ T) {
  const RedJob J = jobs[find_job_chunk(jobs, njobs, blk)];
  const int64_t c = blk - J.first_chunk;
  const float4* src = reinterpret_cast<const float4*>(ws + J.src);
  const int64_t st = J.stride / 4, n4 = J.n / 4;
  const int tid = threadIdx.x;
  if (J.bn == 0) {
#pragma unroll
    for (int k = 0; k < kRedChunk4 / 256; ++k) {
      const int64_t i4 = c * kRedChunk4 + k * 256 + tid;
      if (i4 < n4) {
        const float4 r = sum_parts(src + i4, st, J.nparts);
        if (g) reinterpret_cast<float4*>(g + J.dst)[i4] = r;
        adam_at4(A, c1, c2, J.dst / 4 + i4, r);
      }
    }
    return;
  }
  // the chunk: tile t, waves [w0, w0 + 2): rows [R0, R0 + 64), columns
  // [C0, C0 + 64) of the tile
  const int bn = J.bn, wpr = bn / 32, ld = kRedCols + 4;
  const int64_t tsz4 = 32 * (int64_t)bn;  // float4s per tile
  const int t = (int)((c * kRedChunk4) / tsz4);
  const int w0 = (int)(((c * kRedChunk4) % tsz4) / kRedChunk4) * kRedWaves;
  const int R0 = (w0 / wpr) * 64, C0 = (w0 % wpr) * 32;
#pragma unroll
  for (int k = 0; k < kRedChunk4 / 256; ++k) {
    const int64_t i4 = c * kRedChunk4 + k * 256 + tid;
    const float4 r = sum_parts(src + i4, st, J.nparts);
    // float4 i4 = lane's 4 accumulator rows of fragment f of wave w of tile t
    const int rem = (int)(i4 * 4 - (int64_t)t * tsz4 * 4);
    const int w = rem >> 11, f = (rem >> 8) & 7, lane = (rem >> 2) & 63;
    const int rl = (w / wpr) * 64 + (f >> 1) * 16 + (lane >> 4) * 4 - R0;
    const int cl = (w % wpr) * 32 + (f & 1) * 16 + (lane & 15) - C0;
    T[rl * ld + cl] = r.x;
    T[(rl + 1) * ld + cl] = r.y;
    T[(rl + 2) * ld + cl] = r.z;
    T[(rl + 3) * ld + cl] = r.w;
  }
  __syncthreads();
  constexpr int q4 = kRedCols / 4;  // float4s per block row
  const int row0 = (t / J.tiles_n) * 128 + R0, col0 = (t % J.tiles_n) * bn + C0;
#pragma unroll
  for (int k = 0; k < kRedChunk4 / 256; ++k) {
    const int v = k * 256 + tid;
    const int rl = v / q4, cq = v % q4;
    const int row = row0 + rl, col = col0 + 4 * cq;
    if (row < J.M && col < J.N) {  // N is a multiple of 8: whole float4s
      const float4 r = *reinterpret_cast<const float4*>(T + rl * ld + 4 * cq);
      const int64_t k0 = J.dst + (int64_t)row * J.N + col;
      if (g) *reinterpret_cast<float4*>(g + k0) = r;
      adam_at4(A, c1, c2, k0 / 4, r);
    }
  }
}

// few parts (split-K partials): one float4 of one job per thread
template <bool ADAM>
__device__ __forceinline__ void reduce_few(const char* __restrict__ ws, float* __restrict__ g,
                                           const RedJob* __restrict__ jobs, int njobs,
                                           int64_t total4, int64_t blk, const AdamArgs& A,
                                           float c1, float c2) {
  const int64_t v = blk * 256ll + threadIdx.x;
  if (v >= total4) return;
  const RedJob J = jobs[find_job(jobs, njobs, v)];
  const int64_t i4 = v - J.first;
  int64_t o0 = -1;  // fragment order: row-major offset of this float4's first row
  if (J.bn > 0) {
    // float4 i4 = lane's 4 accumulator rows of fragment (i, j) of wave w of
    // tile t (the direct-to-LDS kernel's 64 x 32 wave blocks)
    const int64_t e = i4 * 4;
    const int64_t tsz = (int64_t)128 * J.bn;
    const int t = (int)(e / tsz);
    const int rem = (int)(e - (int64_t)t * tsz);
    const int w = rem >> 11, f = (rem >> 8) & 7, lane = (rem >> 2) & 63;
    const int wpr = J.bn / 32;  // waves per row of wave blocks
    const int row = (t / J.tiles_n) * 128 + (w / wpr) * 64 + (f >> 1) * 16 + (lane >> 4) * 4;
    const int col = (t % J.tiles_n) * J.bn + (w % wpr) * 32 + (f & 1) * 16 + (lane & 15);
    if (row >= J.M || col >= J.N) return;
    o0 = (int64_t)row * J.N + col;
  }
  const float4* p = reinterpret_cast<const float4*>(ws + J.src) + i4;
  const int64_t st = J.stride / 4;
  float4 s[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) s[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  int k = 0;
  for (; k + 3 < J.nparts; k += 4) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = p[(k + q) * st];
      s[q].x += t.x; s[q].y += t.y; s[q].z += t.z; s[q].w += t.w;
    }
  }
  for (; k < J.nparts; ++k) {
    const float4 t = p[k * st];
    s[0].x += t.x; s[0].y += t.y; s[0].z += t.z; s[0].w += t.w;
  }
  float4 r;
  r.x = (s[0].x + s[1].x) + (s[2].x + s[3].x);
  r.y = (s[0].y + s[1].y) + (s[2].y + s[3].y);
  r.z = (s[0].z + s[1].z) + (s[2].z + s[3].z);
  r.w = (s[0].w + s[1].w) + (s[2].w + s[3].w);
  if (o0 < 0) {
    if (!ADAM || g) reinterpret_cast<float4*>(g + J.dst)[i4] = r;
    if (ADAM) adam_at4(A, c1, c2, J.dst / 4 + i4, r);
  } else {  // rows past M inside the last tile are not stored
    const int64_t k = J.dst + o0;
    const int nrow = min(4, J.M - (int)(o0 / J.N));
    if (!ADAM || g) {
      float* q = g + k;
      q[0] = r.x;
      if (nrow > 1) q[J.N] = r.y;
      if (nrow > 2) q[2 * (int64_t)J.N] = r.z;
      if (nrow > 3) q[3 * (int64_t)J.N] = r.w;
    }
    if (ADAM) {
      adam_at(A, c1, c2, k, r.x);
      if (nrow > 1) adam_at(A, c1, c2, k + J.N, r.y);
      if (nrow > 2) adam_at(A, c1, c2, k + 2 * (int64_t)J.N, r.z);
      if (nrow > 3) adam_at(A, c1, c2, k + 3 * (int64_t)J.N, r.w);
    }
  }
}

// many parts (per-chunk column partials): kManyCols = 32 outputs per
// workgroup (a wavefront reads two whole 128-byte lines per load), the parts
// over 8 groups, then a fixed-order tree in LDS.  A job with no parts writes
// zeros (the padding between parameter tensors).
template <bool ADAM>
__device__ __forceinline__ void reduce_many(const char* __restrict__ ws, float* __restrict__ g,
                                            const RedJob* __restrict__ jobs, int njobs,
                                            int64_t blk, const AdamArgs& A, float c1, float c2) {
  constexpr int NG = 256 / kManyCols;  // groups
  __shared__ float red[NG][kManyCols + 1];
  const RedJob J = jobs[find_job(jobs, njobs, blk)];
  const int col = threadIdx.x % kManyCols, grp = threadIdx.x / kManyCols;
  const int64_t i = (blk - J.first) * kManyCols + col;
  // eight running sums: eight loads in flight per thread
  float sk[8];
#pragma unroll
  for (int q = 0; q < 8; ++q) sk[q] = 0.f;
  if (i < J.n) {
    const float* p = reinterpret_cast<const float*>(ws + J.src) + i;
    int k = grp;
    for (; k + 7 * NG < J.nparts; k += 8 * NG) {
#pragma unroll
      for (int q = 0; q < 8; ++q) sk[q] += p[(k + NG * q) * J.stride];
    }
    for (; k < J.nparts; k += NG) sk[0] += p[k * J.stride];
  }
  red[grp][col] = ((sk[0] + sk[1]) + (sk[2] + sk[3])) + ((sk[4] + sk[5]) + (sk[6] + sk[7]));
  __syncthreads();
  for (int h = NG / 2; h >= 1; h >>= 1) {
    if (grp < h) red[grp][col] += red[grp + h][col];
    __syncthreads();
  }
  if (grp == 0 && i < J.n) {
    const float r = red[0][col];
    if (!ADAM || g) g[J.dst + i] = r;
    if (ADAM) adam_at(A, c1, c2, J.dst + i, r);
  }
}

// Both reductions in one launch: blocks [0, nbf) take the few-part jobs,
// the rest the many-part jobs.  ADAM: each reduced element goes into the
// Adam step of its parameter (the jobs then cover the whole vector).
template <bool ADAM>
__global__ __launch_bounds__(256) void grad_reduce_kernel(const char* __restrict__ ws,
                                                          float* __restrict__ g,
                                                          const RedJob* __restrict__ few,
                                                          int nfew, int64_t total4,
                                                          const RedJob* __restrict__ many,
                                                          int nmany, int64_t nbf, AdamArgs A) {
  if constexpr (ADAM) {
    __shared__ __attribute__((aligned(16))) float T[kRedLdsFloats];
    float c1, c2;
    adam_factors(A.c, A.step, c1, c2);
    if (blockIdx.x < nbf) reduce_few_adam(ws, g, few, nfew, blockIdx.x, A, c1, c2, T);
    else reduce_many<true>(ws, g, many, nmany, blockIdx.x - nbf, A, c1, c2);
  } else {
    if (blockIdx.x < nbf) reduce_few<false>(ws, g, few, nfew, total4, blockIdx.x, A, 0.f, 0.f);
    else reduce_many<false>(ws, g, many, nmany, blockIdx.x - nbf, A, 0.f, 0.f);
  }
}

hipError_t launch_grad_reduce(const char* ws, float* g, const RedJob* few, int nfew,
                              int64_t total4, const RedJob* many, int nmany, int64_t nblocks,
                              double bytes, hipStream_t s, const AdamArgs* A) {
  // with Adam, total4 counts chunks of kRedChunk4 float4s
  const int64_t nbf = nfew > 0 ? (A ? total4 : (total4 + 255) / 256) : 0;
  const int64_t nbm = nmany > 0 ? nblocks : 0;
  if (nbf + nbm == 0) return hipSuccess;
  const dim3 grid((unsigned)(nbf + nbm));
  if (A)
    CRL_TIMED("grad_reduce_adam_kernel", 0.0, bytes, s,
              grad_reduce_kernel<true><<<grid, 256, 0, s>>>(ws, g, few, nfew, total4, many,
                                                            nmany, nbf, *A));
  else
    CRL_TIMED("grad_reduce_kernel", 0.0, bytes, s,
              grad_reduce_kernel<false><<<grid, 256, 0, s>>>(ws, g, few, nfew, total4, many,
                                                             nmany, nbf, AdamArgs{}));
  return hipGetLastError();
}

__global__ void sqnorm_kernel(const float* __restrict__ X, float* __restrict__ out, int B, int D) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= B) return;
  float s = 0.f;
  for (int d = lane; d < D; d += 64) { float v = X[(int64_t)row * D + d]; s += v * v; }
  s = wave_sum(s);
  if (lane == 0) out[row] = s;
}
hipError_t launch_sqnorm(const float* X, float* out, int B, int D, hipStream_t s) {
  CRL_TIMED("sqnorm_kernel", 2.0 * B * D, 4.0 * B * (D + 1.0), s,
            sqnorm_kernel<<<(B + 3) / 4, 256, 0, s>>>(X, out, B, D));
  return hipGetLastError();
}

__global__ void cast_bf16_kernel(const float* __restrict__ src, bf16_t* __restrict__ dst, int64_t n) {
  int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) * 4;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x * 4) {
    if (i + 4 <= n) {
      float4 v = *reinterpret_cast<const float4*>(src + i);
      uint2 u;
      u.x = pack2bf(v.x, v.y);
      u.y = pack2bf(v.z, v.w);
      *reinterpret_cast<uint2*>(dst + i) = u;
    } else {
      for (int64_t j = i; j < n; ++j) dst[j] = f2bf(src[j]);
    }
  }
}
hipError_t launch_cast_bf16(const float* src, bf16_t* dst, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 1023) / 1024;
  if (blocks > 8192) blocks = 8192;
  CRL_TIMED("cast_bf16_kernel", 0.0, 6.0 * n, s,
            cast_bf16_kernel<<<(int)blocks, 256, 0, s>>>(src, dst, n));
  return hipGetLastError();
}

// Adam on a flat vector (adam_update on every element).
__global__ __launch_bounds__(256) void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                                                   float* __restrict__ m, float* __restrict__ v,
                                                   bf16_t* __restrict__ pb, int64_t n,
                                                   const int64_t* __restrict__ step, AdamCoef c) {
  float c1, c2;
  adam_factors(c, step, c1, c2);
  const AdamArgs A{p, m, v, pb, step, c};
  const int64_t n4 = n >> 2;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n4;
       i += (int64_t)gridDim.x * blockDim.x)
    adam_at4(A, c1, c2, i, reinterpret_cast<const float4*>(g)[i]);
  if (blockIdx.x == 0 && threadIdx.x < (n & 3)) {
    const int64_t k = n4 * 4 + threadIdx.x;
    adam_at(A, c1, c2, k, g[k]);
  }
}
hipError_t launch_adam(float* p, const float* g, float* m, float* v, bf16_t* pb, int64_t n,
                       const int64_t* step, const AdamCoef& c, hipStream_t s) {
  int64_t blocks = (n / 4 + 255) / 256;
  if (blocks < 1) blocks = 1;
  if (blocks > 16384) blocks = 16384;
  CRL_TIMED("adam_kernel", 0.0, (28.0 + (pb ? 2.0 : 0.0)) * n, s,
            adam_kernel<<<(int)blocks, 256, 0, s>>>(p, g, m, v, pb, n, step, c));
  return hipGetLastError();
}

__global__ void counter_add_kernel(int64_t* c, int64_t inc) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c += inc;
}
hipError_t launch_counter_add(int64_t* c, int64_t inc, hipStream_t s) {
  counter_add_kernel<<<1, 64, 0, s>>>(c, inc);
  return hipGetLastError();
}

// ranges: [nranges][2] = (offset, length) in floats

// ---------------------------------------------------------------------------
// materialised InfoNCE: F [B][B] FP32 in memory
// ---------------------------------------------------------------------------
// per (row chunk, column) online (max, sum) over the chunk's rows
__global__ void col_lse_partial_kernel(const float* __restrict__ F, int B, int ld, int rows_per,
                                       float* __restrict__ pm, float* __restrict__ ps) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= B) return;
  const int i0 = blockIdx.y * rows_per, i1 = min(B, i0 + rows_per);
  float m = -INFINITY, s = 0.f;
  for (int i = i0; i < i1; ++i) {
    float f = F[(int64_t)i * ld + j];
    if (f > m) { s = s * __expf(m - f) + 1.f; m = f; }
    else s += __expf(f - m);
  }
  pm[(int64_t)blockIdx.y * B + j] = m;
  ps[(int64_t)blockIdx.y * B + j] = s;
}
hipError_t launch_col_lse_partial(const float* F, int B, int ld, int rchunks, float* pm, float* ps,
                                  hipStream_t s) {
  int rows_per = (B + rchunks - 1) / rchunks;
  dim3 grid((B + 255) / 256, rchunks);
  CRL_TIMED("col_lse_partial_kernel", 0.0, 4.0 * B * B, s,
            col_lse_partial_kernel<<<grid, 256, 0, s>>>(F, B, ld, rows_per, pm, ps));
  return hipGetLastError();
}

__global__ __launch_bounds__(1024) void lse_merge_kernel(LseMergeArgs a, int B) {
  // problem blockIdx.y; 64 columns per workgroup (a wavefront reads 256
  // contiguous bytes of one part), the parts split over the 16 wavefronts
  // (p = grp, grp + 16, ...), then a fixed-order tree over them in LDS
  __shared__ float sm[16][65], ss[16][65];
  const int e = blockIdx.y;
  const float* __restrict__ pm = a.pm[e];
  const float* __restrict__ ps = a.ps[e];
  const int nparts = a.nparts[e];
  const int col = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + col;
  float m = -INFINITY, s = 0.f;
  if (j < B)
    for (int p = grp; p < nparts; p += 16)
      lse_merge(m, s, pm[(int64_t)p * B + j], ps[(int64_t)p * B + j]);
  sm[grp][col] = m;
  ss[grp][col] = s;
  __syncthreads();
  for (int h = 8; h >= 1; h >>= 1) {
    if (grp < h) {
      float mm = sm[grp][col], s2 = ss[grp][col];
      lse_merge(mm, s2, sm[grp + h][col], ss[grp + h][col]);
      sm[grp][col] = mm;
      ss[grp][col] = s2;
    }
    __syncthreads();
  }
  if (grp == 0 && j < B) a.out[e][j] = sm[0][col] + __logf(ss[0][col]);
}
hipError_t launch_lse_merge(const LseMergeArgs& a, int count, int B, hipStream_t s) {
  double parts = 0.0;
  for (int e = 0; e < count; ++e) parts += a.nparts[e];
  CRL_TIMED("lse_merge_kernel", 0.0, 4.0 * B * (2.0 * parts + count), s,
            lse_merge_kernel<<<dim3((B + 63) / 64, count), 1024, 0, s>>>(a, B));
  return hipGetLastError();
}
hipError_t launch_lse_merge(const float* pm, const float* ps, int nparts, int B, float* out,
                            hipStream_t s) {
  LseMergeArgs a{};
  a.pm[0] = pm; a.ps[0] = ps; a.nparts[0] = nparts; a.out[0] = out;
  return launch_lse_merge(a, 1, B, s);
}

// Loss from r, c, diag (and the per-row objective terms of the pairwise
// objectives) in one workgroup: per-thread Kahan sums, then an ordered
// pairwise tree over the threads (deterministic).
//   loss_out = {L_obj + L_pen, mean(r - diag), mean(c - diag), L_pen,
//               mean r, mean c, #non-finite rows, L_obj}
// with L_obj the objective `loss` (CRL_LOSS_*): the two InfoNCE directions,
// their sum, FlatNCE (exp(x - x) per row, x = r - diag or c - diag), or the
// mean of term[] (Forward-Backward, DPO, IPO, SPPO).
__global__ __launch_bounds__(1024) void loss_kernel(const float* __restrict__ r,
                                                    const float* __restrict__ c,
                                                    const float* __restrict__ diag,
                                                    const float* __restrict__ term, int B,
                                                    int loss, float beta,
                                                    float* __restrict__ loss_out,
                                                    int64_t* __restrict__ advance) {
  __shared__ float sh[7][1024];
  float acc[6] = {0, 0, 0, 0, 0, 0}, cmp[6] = {0, 0, 0, 0, 0, 0};
  float bad = 0.f;
  const bool pairwise = loss >= CRL_LOSS_FB;
  for (int i = threadIdx.x; i < B; i += 1024) {
    float ri = r[i], ci = c[i], di = diag[i];
    float o = 0.f;
    if (loss == CRL_LOSS_FLATNCE_FWD) { const float x = ri - di; o = __expf(x - x); }
    else if (loss == CRL_LOSS_FLATNCE_BWD) { const float x = ci - di; o = __expf(x - x); }
    else if (pairwise) o = term[i];
    float t[6] = {ri - di, ci - di, ri * ri, ri, ci, o};
#pragma unroll
    for (int k = 0; k < 6; ++k) kahan_add(acc[k], cmp[k], t[k]);
    if (!isfinite(ri) || !isfinite(ci) || !isfinite(di) || !isfinite(o)) bad += 1.f;
  }
#pragma unroll
  for (int k = 0; k < 6; ++k) sh[k][threadIdx.x] = acc[k] - cmp[k];
  sh[6][threadIdx.x] = bad;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w)
#pragma unroll
      for (int k = 0; k < 7; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float inv = 1.f / (float)B;
    const float lf = sh[0][0] * inv, lb = sh[1][0] * inv, lp = beta * sh[2][0] * inv;
    float obj;
    if (loss == CRL_LOSS_FWD) obj = lf;
    else if (loss == CRL_LOSS_SYM) obj = lf + lb;
    else if (loss == CRL_LOSS_BWD) obj = lb;
    else obj = sh[5][0] * inv;
    loss_out[0] = obj + lp;
    loss_out[1] = lf;
    loss_out[2] = lb;
    loss_out[3] = lp;
    loss_out[4] = sh[3][0] * inv;
    loss_out[5] = sh[4][0] * inv;
    loss_out[6] = sh[6][0];
    loss_out[7] = obj;
    if (advance) *advance += 1;
  }
}
hipError_t launch_loss(const float* r, const float* c, const float* diag, const float* term,
                       int B, int loss, float beta, float* loss_out, int64_t* advance,
                       hipStream_t s) {
  CRL_TIMED("loss_kernel", 0.0, 16.0 * B, s,
            loss_kernel<<<1, 1024, 0, s>>>(r, c, diag, term, B, loss, beta, loss_out, advance));
  return hipGetLastError();
}

// dX[i][d] -= rs[i] * X[i][d]
__global__ void l2_fix_kernel(float* __restrict__ dX, const float* __restrict__ X,
                              const float* __restrict__ rs, int B, int D) {
  int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= (int64_t)B * D) return;
  dX[k] -= rs[k / D] * X[k];
}
hipError_t launch_l2_fix(float* dX, const float* X, const float* rs, int B, int D,
                         hipStream_t s) {
  int64_t n = (int64_t)B * D;
  CRL_TIMED("l2_fix_kernel", 2.0 * n, 12.0 * n, s,
            l2_fix_kernel<<<(int)((n + 255) / 256), 256, 0, s>>>(dX, X, rs, B, D));
  return hipGetLastError();
}

}  // namespace crl
