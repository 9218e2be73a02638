// Instantiations and host dispatch of the MFMA GEMM.
#include "internal.hpp"
#include "gemm_lds.hpp"

namespace crl {

// Sum of split-K partials: C[m][n] (+)= sum_s partial[s][m][n] (+ bias[n]),
// FP32 out; the only epilogues used with split-K are none and bias.
__global__ void splitk_reduce_kernel(GemmParams P) {
  const int g = blockIdx.y;
  const GemmDesc& D = P.d[g];
  const int64_t MN = (int64_t)D.M * D.N;
  const float* src = P.partial + (int64_t)g * P.partial_len;
  float* C = reinterpret_cast<float*>(D.C);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < MN;
       i += (int64_t)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int k = 0; k < P.splits; ++k) s += src[k * MN + i];
    int64_t row = i / D.N, col = i % D.N;
    int64_t o = row * D.ldc + col;
    if (D.epi == EPI_BIAS) s += D.bias[col];
    if (D.accumulate) s += C[o];
    C[o] = s;
  }
}


template <typename T, int LA, int LB, typename OutT>
static const char* kernel_name() {
  static const char* names[2][2][2][2] = {
      {{{"gemm_kernel<f32,KC,KC,f32>", "gemm_kernel<f32,KC,KC,bf16>"},
        {"gemm_kernel<f32,KC,MC,f32>", "gemm_kernel<f32,KC,MC,bf16>"}},
       {{"gemm_kernel<f32,MC,KC,f32>", "gemm_kernel<f32,MC,KC,bf16>"},
        {"gemm_kernel<f32,MC,MC,f32>", "gemm_kernel<f32,MC,MC,bf16>"}}},
      {{{"gemm_kernel<bf16,KC,KC,f32>", "gemm_kernel<bf16,KC,KC,bf16>"},
        {"gemm_kernel<bf16,KC,MC,f32>", "gemm_kernel<bf16,KC,MC,bf16>"}},
       {{"gemm_kernel<bf16,MC,KC,f32>", "gemm_kernel<bf16,MC,KC,bf16>"},
        {"gemm_kernel<bf16,MC,MC,f32>", "gemm_kernel<bf16,MC,MC,bf16>"}}}};
  return names[sizeof(T) == 2][LA][LB][sizeof(OutT) == 2];
}

template <int LA, int LB, typename OutT, int BN>
static const char* lds_kernel_name() {
  static const char* names[2][2][2][2] = {
      {{{"gemm_lds_kernel<KC,KC,f32,64>", "gemm_lds_kernel<KC,KC,bf16,64>"},
        {"gemm_lds_kernel<KC,MC,f32,64>", "gemm_lds_kernel<KC,MC,bf16,64>"}},
       {{"gemm_lds_kernel<MC,KC,f32,64>", "gemm_lds_kernel<MC,KC,bf16,64>"},
        {"gemm_lds_kernel<MC,MC,f32,64>", "gemm_lds_kernel<MC,MC,bf16,64>"}}},
      {{{"gemm_lds_kernel<KC,KC,f32>", "gemm_lds_kernel<KC,KC,bf16>"},
        {"gemm_lds_kernel<KC,MC,f32>", "gemm_lds_kernel<KC,MC,bf16>"}},
       {{"gemm_lds_kernel<MC,KC,f32>", "gemm_lds_kernel<MC,KC,bf16>"},
        {"gemm_lds_kernel<MC,MC,f32>", "gemm_lds_kernel<MC,MC,bf16>"}}}};
  return names[BN == 128][LA][LB][sizeof(OutT) == 2];
}

// The direct-to-LDS kernel takes a launch whose K ranges are all whole 64-deep
// steps, with 16-byte rows (ragged M and N are handled by clamped loads and
// guarded stores).  N not a multiple of 8 is taken only where the results are
// stored plainly (no mask epilogue, no fragment-order partials): those column
// tails are stored element by element.  Its column tile is 128 wide, as the
// planned grid; or 64 wide when no problem is wider than 64 (one column tile
// either way).
static int lds_path_bn(const GemmParams& P) {
  int nmax = 0;
  for (int g = 0; g < P.count; ++g) {
    const GemmDesc& d = P.d[g];
    if (d.K % lds::BK || P.k_chunk % lds::BK) return 0;
    if (d.N % 8 && (P.defer_reduce || (d.epi != EPI_NONE && d.epi != EPI_BIAS))) return 0;
    if (d.lda % 8 || d.ldb % 8 || d.ldc % 8) return 0;
    if (d.epi == EPI_L2 || d.epi == EPI_L2SQ || d.accumulate) return 0;
    if ((reinterpret_cast<uintptr_t>(d.A) | reinterpret_cast<uintptr_t>(d.B) |
         reinterpret_cast<uintptr_t>(d.C)) & 15u)
      return 0;
    nmax = d.N > nmax ? d.N : nmax;
  }
  return nmax > 64 ? 128 : 64;
}

int gemm_lds_bn(const GemmParams& P, bool bf16) { return bf16 ? lds_path_bn(P) : 0; }

int64_t frag_partial_floats(const GemmParams& P, int g, int bn) {
  const GemmDesc& d = P.d[g];
  if (bn == 0) return (int64_t)d.M * d.N;
  return (int64_t)((d.M + lds::BM - 1) / lds::BM) * ((d.N + bn - 1) / bn) * lds::BM * bn;
}

// algorithmic FLOPs and bytes of one launch (the unpadded K)
static void algo_counts(const GemmParams& P, double esize, double osize, double& flops,
                        double& bytes) {
  for (int g = 0; g < P.count; ++g) {
    const GemmDesc& d = P.d[g];
    const double k = d.kb > 0 ? d.kb : d.K;
    flops += 2.0 * d.M * d.N * k;
    bytes += esize * ((double)d.M * k + k * d.N) + (P.splits > 1 ? 4.0 : osize) * d.M * d.N;
  }
}

static int max_tiles(const GemmParams& P) {
  int maxt = 0;
  for (int g = 0; g < P.count; ++g) maxt = P.tiles[g] > maxt ? P.tiles[g] : maxt;
  return maxt;
}

template <typename T, int LA, int LB, typename OutT>
static hipError_t run(GemmParams& P, hipStream_t s) {
  const int maxt = max_tiles(P);
  if (maxt == 0) return hipSuccess;
  dim3 grid(maxt, P.splits, P.count), block(kGemmThreads);
  int bn = 0;
  if constexpr (sizeof(T) == 2) bn = lds_path_bn(P);
  if (bn == 0)  // the register-staged kernel handles any K: drop zero-padded K
    for (int g = 0; g < P.count; ++g)
      if (P.d[g].kb > 0) {
        P.d[g].K = P.d[g].kb;
        P.d[g].kb = 0;
      }
  double flops = 0.0, bytes = 0.0;
  algo_counts(P, sizeof(T), sizeof(OutT), flops, bytes);
  if (bn == 128) {
    KTimer t = timing_begin(lds_kernel_name<LA, LB, OutT, 128>(), flops, bytes, s);
    gemm_lds_kernel<LA, LB, OutT, 128><<<grid, lds::threads<128>(), 0, s>>>(P);
    timing_end(t);
  } else if (bn == 64) {
    KTimer t = timing_begin(lds_kernel_name<LA, LB, OutT, 64>(), flops, bytes, s);
    gemm_lds_kernel<LA, LB, OutT, 64><<<grid, lds::threads<64>(), 0, s>>>(P);
    timing_end(t);
  } else {
    KTimer t = timing_begin(kernel_name<T, LA, LB, OutT>(), flops, bytes, s);
    gemm_kernel<T, LA, LB, OutT><<<grid, block, 0, s>>>(P);
    timing_end(t);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || P.splits <= 1 || P.defer_reduce) return e;
  int64_t mn = 0;
  for (int g = 0; g < P.count; ++g) {
    int64_t v = (int64_t)P.d[g].M * P.d[g].N;
    mn = v > mn ? v : mn;
  }
  int64_t blocks = (mn + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  KTimer tr = timing_begin("splitk_reduce_kernel", 0.0, (double)(P.splits + 1) * 4.0 * mn * P.count, s);
  splitk_reduce_kernel<<<dim3((unsigned)blocks, P.count), 256, 0, s>>>(P);
  timing_end(tr);
  return hipGetLastError();
}

template <typename T, typename OutT>
static hipError_t run_layout(GemmParams& P, int la, int lb, hipStream_t s) {
  if (la == LAY_KC && lb == LAY_KC) return run<T, LAY_KC, LAY_KC, OutT>(P, s);
  if (la == LAY_KC && lb == LAY_MC) return run<T, LAY_KC, LAY_MC, OutT>(P, s);
  if (la == LAY_MC && lb == LAY_KC) return run<T, LAY_MC, LAY_KC, OutT>(P, s);
  return run<T, LAY_MC, LAY_MC, OutT>(P, s);
}

bool gemm_pair_ok(const GemmParams& Pw, const GemmParams& Px, bool bf16) {
  return bf16 && lds_path_bn(Pw) != 0 && lds_path_bn(Px) == 128 &&
         (Pw.splits == 1 || Pw.defer_reduce) && Px.splits == 1 && max_tiles(Pw) > 0 &&
         max_tiles(Px) > 0;
}

hipError_t launch_gemm_dw_dx(GemmParams& Pw, GemmParams& Px, hipStream_t s) {
  if (!gemm_pair_ok(Pw, Px, true)) return hipErrorInvalidValue;
  PairGrid G;
  G.gx1 = max_tiles(Pw);
  G.gy1 = Pw.splits;
  G.n1 = G.gx1 * G.gy1 * Pw.count;
  G.gx2 = max_tiles(Px);
  G.gy2 = 1;
  G.n2 = G.gx2 * Px.count;
  double flops = 0.0, bytes = 0.0;
  algo_counts(Pw, 2.0, 4.0, flops, bytes);
  algo_counts(Px, 2.0, 2.0, flops, bytes);
  KTimer t = timing_begin("gemm_lds_pair_kernel<dW,dX>", flops, bytes, s);
  gemm_lds_pair_kernel<LAY_MC, LAY_MC, float, LAY_KC, LAY_KC, bf16_t>
      <<<G.n1 + G.n2, lds::threads<128>(), 0, s>>>(Pw, Px, G);
  timing_end(t);
  return hipGetLastError();
}

void plan_split_k(GemmParams& P, bool bf16, int target_wgs, int min_steps) {
  const int BK = bf16 ? GemmCfg<bf16_t>::BK : GemmCfg<float>::BK;
  int tiles = 0, kmax = 0;
  for (int g = 0; g < P.count; ++g) {
    P.tiles_n[g] = (P.d[g].N + kBN - 1) / kBN;
    P.tiles[g] = ((P.d[g].M + kBM - 1) / kBM) * P.tiles_n[g];
    tiles += P.tiles[g];
    kmax = P.d[g].K > kmax ? P.d[g].K : kmax;
  }
  int splits = 1;
  if (tiles > 0 && P.partial != nullptr) {
    int max_splits = kmax / (min_steps * BK);
    while (splits * 2 <= max_splits && tiles * splits * 2 <= target_wgs) splits *= 2;
  }
  int kc = (kmax + splits - 1) / splits;
  kc = (kc + BK - 1) / BK * BK;
  if (kc == 0) kc = BK;
  P.splits = splits;
  P.k_chunk = kc;
}

hipError_t launch_gemm(GemmParams& P, bool bf16, int la, int lb, bool out_bf16, hipStream_t s) {
  if (bf16) {
    if (out_bf16) return run_layout<bf16_t, bf16_t>(P, la, lb, s);
    return run_layout<bf16_t, float>(P, la, lb, s);
  }
  if (out_bf16) return run_layout<float, bf16_t>(P, la, lb, s);
  return run_layout<float, float>(P, la, lb, s);
}

}  // namespace crl
