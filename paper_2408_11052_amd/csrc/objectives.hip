// Energies and contrastive objectives on the materialised critic matrix
// F [B][ld] (FP32): the per-row reductions, the in-place gradient dL/dF, and
// the energy backward passes that are not plain products.
//
// Objectives (Appendix A.2 list of tested objectives, with the logsumexp
// penalty of Section 5.3 on every one): InfoNCE forward / backward /
// symmetric, FlatNCE forward / backward (value 1 per row, the gradient of
// the log of its sum), Forward-Backward, DPO, IPO and SPPO, each averaged
// over the positives i with the sum over j taken over the whole batch.
//
// Energies (Appendix A.2): dot and L2 / L2-without-root come from the logit
// GEMM's epilogue; cosine is the dot product of unit rows (unit_rows_kernel);
// L1 is not a product and has its own vector-ALU kernels here.
#include "internal.hpp"

namespace crl {

__device__ __forceinline__ float softplusf(float x) {
  return fmaxf(x, 0.f) + log1pf(__expf(-fabsf(x)));
}


// U[i] = X[i] / |X[i]| (0 for a zero row) and nrm[i] = |X[i]|, one wave per row.
__global__ __launch_bounds__(256) void unit_rows_kernel(const float* __restrict__ X,
                                                        float* __restrict__ U,
                                                        float* __restrict__ nrm, int B, int D) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= B) return;
  const float* x = X + (int64_t)row * D;
  float s = 0.f;
  for (int d = lane; d < D; d += 64) s += x[d] * x[d];
  s = wave_sum(s);
  const float n = sqrtf(s);
  const float inv = n > 0.f ? 1.f / n : 0.f;
  for (int d = lane; d < D; d += 64) U[(int64_t)row * D + d] = x[d] * inv;
  if (lane == 0) nrm[row] = n;
}
hipError_t launch_unit_rows(const float* X, float* U, float* nrm, int B, int D, hipStream_t s) {
  CRL_TIMED("unit_rows_kernel", 3.0 * B * D, 4.0 * B * (2.0 * D + 1.0), s,
            unit_rows_kernel<<<(B + 3) / 4, 256, 0, s>>>(X, U, nrm, B, D));
  return hipGetLastError();
}

// F_ij = -sum_k |phi_ik - psi_jk| for a 64 x 64 tile per workgroup; each of
// the 256 threads owns a 4 x 4 block.  32-feature slices of both operands go
// through LDS (transposed, so a thread's four rows are one 16-byte read).
constexpr int kL1T = 64, kL1K = 32;
__global__ __launch_bounds__(256) void l1_energy_kernel(const float* __restrict__ phi,
                                                        const float* __restrict__ psi,
                                                        float* __restrict__ F, int B, int D,
                                                        int ld) {
  __shared__ __attribute__((aligned(16))) float As[kL1K][kL1T + 4];
  __shared__ __attribute__((aligned(16))) float Bs[kL1K][kL1T + 4];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int i0 = blockIdx.y * kL1T, j0 = blockIdx.x * kL1T;
  float acc[4][4] = {};
  for (int k0 = 0; k0 < D; k0 += kL1K) {
    __syncthreads();
    // 64 rows x 32 features of each operand: 8 values per thread
    for (int v = tid; v < kL1T * kL1K; v += 256) {
      const int r = v / kL1K, k = v % kL1K;
      const bool kin = k0 + k < D;
      As[k][r] = (i0 + r < B && kin) ? phi[(int64_t)(i0 + r) * D + k0 + k] : 0.f;
      Bs[k][r] = (j0 + r < B && kin) ? psi[(int64_t)(j0 + r) * D + k0 + k] : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < kL1K; ++k) {
      const float4 a = *reinterpret_cast<const float4*>(&As[k][ty * 4]);
      const float4 b = *reinterpret_cast<const float4*>(&Bs[k][tx * 4]);
      const float av[4] = {a.x, a.y, a.z, a.w}, bv[4] = {b.x, b.y, b.z, b.w};
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += fabsf(av[p] - bv[q]);
    }
  }
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int i = i0 + ty * 4 + p;
    if (i >= B) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + tx * 4 + q;
      if (j < B) F[(int64_t)i * ld + j] = -acc[p][q];
    }
  }
}
hipError_t launch_l1_energy(const float* phi, const float* psi, float* F, int B, int D, int ld,
                            hipStream_t s) {
  const dim3 grid((B + kL1T - 1) / kL1T, (B + kL1T - 1) / kL1T);
  CRL_TIMED("l1_energy_kernel", 3.0 * B * B * D, 4.0 * (2.0 * B * D + (double)B * B), s,
            l1_energy_kernel<<<grid, 256, 0, s>>>(phi, psi, F, B, D, ld));
  return hipGetLastError();
}

// dX_xk = -sum_y C(x, y) sign(X_xk - Y_yk), C(x, y) = G[x][y] (trans = 0:
// X = phi, Y = psi, giving dphi) or G[y][x] (trans = 1: X = psi, Y = phi,
// giving dpsi, since dF_ij/dpsi_jk = +sign(phi_ik - psi_jk) =
// -sign(psi_jk - phi_ik)).  A workgroup owns 32 rows x all D features (a
// thread: one row, features t%8 + 8m); 32-row slices of Y and the matching
// 32 x 32 block of C go through LDS.
constexpr int kL1R = 32;
template <int TRANS>
__global__ __launch_bounds__(256) void l1_backward_kernel(const float* __restrict__ X,
                                                          const float* __restrict__ Y,
                                                          const float* __restrict__ G, int ldg,
                                                          float* __restrict__ dX, int B, int D) {
  extern __shared__ float sm[];
  float* Ys = sm;                       // [kL1R][D + 1]
  float* Cs = sm + kL1R * (D + 1);      // [kL1R x rows][kL1R y] (+1 pad)
  const int tid = threadIdx.x;
  const int rl = tid >> 3, kq = tid & 7;
  const int x = blockIdx.x * kL1R + rl;
  const int nk = (D + 7) / 8;           // features per thread (<= 32)
  float acc[32] = {};
  float xv[32];
#pragma unroll
  for (int m = 0; m < 32; ++m) {
    const int k = kq + 8 * m;
    xv[m] = (m < nk && k < D && x < B) ? X[(int64_t)x * D + k] : 0.f;
  }
  for (int y0 = 0; y0 < B; y0 += kL1R) {
    __syncthreads();
    for (int v = tid; v < kL1R * D; v += 256) {
      const int r = v / D, k = v % D;
      Ys[r * (D + 1) + k] = (y0 + r < B) ? Y[(int64_t)(y0 + r) * D + k] : 0.f;
    }
    for (int v = tid; v < kL1R * kL1R; v += 256) {
      const int a = v / kL1R, b = v % kL1R;     // a: x row in the block, b: y
      const int xa = blockIdx.x * kL1R + a, yb = y0 + b;
      float c = 0.f;
      if (xa < B && yb < B) c = TRANS ? G[(int64_t)yb * ldg + xa] : G[(int64_t)xa * ldg + yb];
      Cs[a * (kL1R + 1) + b] = c;
    }
    __syncthreads();
    const int ny = min(kL1R, B - y0);
    for (int b = 0; b < ny; ++b) {
      const float c = Cs[rl * (kL1R + 1) + b];
      const float* yr = Ys + b * (D + 1);
#pragma unroll
      for (int m = 0; m < 32; ++m) {
        if (m >= nk) break;
        const int k = kq + 8 * m;
        const float dlt = xv[m] - (k < D ? yr[k] : 0.f);
        const float sg = dlt > 0.f ? 1.f : (dlt < 0.f ? -1.f : 0.f);
        acc[m] -= c * sg;
      }
    }
  }
  if (x >= B) return;
#pragma unroll
  for (int m = 0; m < 32; ++m) {
    const int k = kq + 8 * m;
    if (m < nk && k < D) dX[(int64_t)x * D + k] = acc[m];
  }
}
hipError_t launch_l1_backward(const float* X, const float* Y, const float* G, int ldg, int trans,
                              float* dX, int B, int D, hipStream_t s) {
  if (D > 256) return hipErrorInvalidValue;
  const size_t lds = sizeof(float) * (kL1R * (D + 1) + kL1R * (kL1R + 1));
  const dim3 grid((B + kL1R - 1) / kL1R);
  if (trans)
    CRL_TIMED("l1_backward_kernel<cols>", 3.0 * B * B * D, 4.0 * (3.0 * B * D + (double)B * B), s,
              l1_backward_kernel<1><<<grid, 256, lds, s>>>(X, Y, G, ldg, dX, B, D));
  else
    CRL_TIMED("l1_backward_kernel<rows>", 3.0 * B * B * D, 4.0 * (3.0 * B * D + (double)B * B), s,
              l1_backward_kernel<0><<<grid, 256, lds, s>>>(X, Y, G, ldg, dX, B, D));
  return hipGetLastError();
}

// Per row i of F: r_i = LSE_j F_ij (max-subtracted), F_ii, and for the
// pairwise objectives the row's term of the objective and the sum that
// forms dL/dF_ii:
//   FB:   term = -exp(F_ii) + sum_{j != i} exp(2 F_ij) / (2 (B - 1))
//   DPO:  term = sum_j softplus(F_ij - F_ii),      aux = sum_{j != i} sigmoid(F_ij - F_ii)
//   IPO:  term = sum_j (F_ii - F_ij - 1)^2,        aux = sum_{j != i} (F_ii - F_ij - 1)
//   SPPO: term = B (F_ii - 1)^2 + sum_j (F_ij + 1)^2
template <int LOSS>
__global__ __launch_bounds__(256) void row_obj_kernel(const float* __restrict__ F, int B, int ld,
                                                      float* __restrict__ r,
                                                      float* __restrict__ diag,
                                                      float* __restrict__ term,
                                                      float* __restrict__ aux) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= B) return;
  const float* row = F + (int64_t)i * ld;
  const float fii = row[i];
  float m = -INFINITY;
  for (int j = lane; j < B; j += 64) m = fmaxf(m, row[j]);
  m = wave_max(m);
  float s = 0.f, t = 0.f, a = 0.f;
  for (int j = lane; j < B; j += 64) {
    const float f = row[j];
    s += __expf(f - m);
    if (LOSS == CRL_LOSS_FB) {
      if (j != i) t += __expf(2.f * f);
    } else if (LOSS == CRL_LOSS_DPO) {
      t += softplusf(f - fii);
      if (j != i) a += sigmoidf_(f - fii);
    } else if (LOSS == CRL_LOSS_IPO) {
      const float e = (fii - f) - 1.f;
      t += e * e;
      if (j != i) a += e;
    } else if (LOSS == CRL_LOSS_SPPO) {
      t += (f + 1.f) * (f + 1.f);
    }
  }
  s = wave_sum(s);
  if (LOSS >= CRL_LOSS_FB) t = wave_sum(t);
  if (LOSS == CRL_LOSS_DPO || LOSS == CRL_LOSS_IPO) a = wave_sum(a);
  if (lane == 0) {
    r[i] = m + __logf(s);
    diag[i] = fii;
    if (LOSS == CRL_LOSS_FB) {
      const float scale = B > 1 ? 0.5f / (float)(B - 1) : 0.f;
      term[i] = -__expf(fii) + scale * t;
    } else if (LOSS == CRL_LOSS_SPPO) {
      term[i] = (float)B * (fii - 1.f) * (fii - 1.f) + t;
    } else if (LOSS >= CRL_LOSS_FB) {
      term[i] = t;
    }
    if (LOSS == CRL_LOSS_DPO || LOSS == CRL_LOSS_IPO) aux[i] = a;
  }
}
hipError_t launch_row_obj(const float* F, int B, int ld, int loss, float* r, float* diag,
                          float* term, float* aux, hipStream_t s) {
  const dim3 grid((B + 3) / 4);
  const double bytes = 4.0 * ((double)B * B + 4.0 * B);
  switch (loss) {
#define CRL_ROW_OBJ(L_, NAME)                                                       \
  case L_:                                                                          \
    CRL_TIMED(NAME, 0.0, bytes, s,                                                  \
              row_obj_kernel<L_><<<grid, 256, 0, s>>>(F, B, ld, r, diag, term, aux)); \
    break;
    CRL_ROW_OBJ(CRL_LOSS_FB, "row_obj_kernel<fb>")
    CRL_ROW_OBJ(CRL_LOSS_DPO, "row_obj_kernel<dpo>")
    CRL_ROW_OBJ(CRL_LOSS_IPO, "row_obj_kernel<ipo>")
    CRL_ROW_OBJ(CRL_LOSS_SPPO, "row_obj_kernel<sppo>")
#undef CRL_ROW_OBJ
    default:  // the InfoNCE family needs only r and the diagonal
      CRL_TIMED("row_obj_kernel<lse>", 0.0, bytes, s,
                row_obj_kernel<CRL_LOSS_FWD><<<grid, 256, 0, s>>>(F, B, ld, r, diag, term, aux));
  }
  return hipGetLastError();
}

// In place: F_ij -> G_ij = dL/dF_ij, then through the energy's pointwise
// factor: H_ij = G_ij / d_ij for L2 (d_ij = -F_ij, 0 where d_ij = 0),
// H_ij = 2 G_ij for L2 without the root, G_ij otherwise; rowsum_i = sum_j H_ij
// for the two distance energies.  B G_ij =
//   2 beta r_i Pr_ij                                  (penalty, every objective)
// + wf (Pr_ij - d_ij) + wb (Pc_ij - d_ij)             (InfoNCE, FlatNCE)
// + FB:   -exp(F_ii) d_ij + (1 - d_ij) exp(2 F_ij) / (B - 1)
// + DPO:  (1 - d_ij) sigmoid(F_ij - F_ii) - d_ij aux_i
// + IPO:  -2 (1 - d_ij) (F_ii - F_ij - 1) + 2 d_ij aux_i
// + SPPO: 2 (F_ij + 1) + 2 B d_ij (F_ii - 1)
template <int LOSS, int EN>
__global__ __launch_bounds__(256) void grad_obj_kernel(float* __restrict__ F, int B, int ld,
                                                       const float* __restrict__ r,
                                                       const float* __restrict__ c,
                                                       const float* __restrict__ diag,
                                                       const float* __restrict__ aux,
                                                       float beta, float* __restrict__ rowsum) {
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= B) return;
  const float inv = 1.f / (float)B;
  const float ri = r[i];
  const float pen = 2.f * beta * ri;
  const float fii = diag[i];
  const float ai = (LOSS == CRL_LOSS_DPO || LOSS == CRL_LOSS_IPO) ? aux[i] : 0.f;
  constexpr bool wf = LOSS == CRL_LOSS_FWD || LOSS == CRL_LOSS_SYM || LOSS == CRL_LOSS_FLATNCE_FWD;
  constexpr bool wb = LOSS == CRL_LOSS_SYM || LOSS == CRL_LOSS_BWD || LOSS == CRL_LOSS_FLATNCE_BWD;
  float* row = F + (int64_t)i * ld;
  float rs = 0.f;
  for (int j = lane; j < B; j += 64) {
    const float f = row[j];
    const bool dg = j == i;
    const float pr = __expf(f - ri);
    float g = pr * pen;
    if (wf) g += pr - (dg ? 1.f : 0.f);
    if (wb) g += __expf(f - c[j]) - (dg ? 1.f : 0.f);
    if (LOSS == CRL_LOSS_FB)
      g += dg ? -__expf(fii) : __expf(2.f * f) / (float)(B - 1);
    if (LOSS == CRL_LOSS_DPO) g += dg ? -ai : sigmoidf_(f - fii);
    if (LOSS == CRL_LOSS_IPO) g += dg ? 2.f * ai : -2.f * ((fii - f) - 1.f);
    if (LOSS == CRL_LOSS_SPPO) g += 2.f * (f + 1.f) + (dg ? 2.f * (float)B * (fii - 1.f) : 0.f);
    g *= inv;
    if (EN == CRL_ENERGY_L2) {
      const float d = -f;
      g = d > 0.f ? g / d : 0.f;
    } else if (EN == CRL_ENERGY_L2SQ) {
      g *= 2.f;
    }
    if (EN == CRL_ENERGY_L2 || EN == CRL_ENERGY_L2SQ) rs += g;
    row[j] = g;
  }
  if (EN == CRL_ENERGY_L2 || EN == CRL_ENERGY_L2SQ) {
    rs = wave_sum(rs);
    if (lane == 0) rowsum[i] = rs;
  }
}

template <int LOSS>
static void grad_obj_launch(float* F, int B, int ld, const float* r, const float* c,
                            const float* diag, const float* aux, int energy, float beta,
                            float* rowsum, hipStream_t s) {
  const dim3 grid((B + 3) / 4);
  switch (energy) {
    case CRL_ENERGY_L2:
      grad_obj_kernel<LOSS, CRL_ENERGY_L2><<<grid, 256, 0, s>>>(F, B, ld, r, c, diag, aux, beta, rowsum);
      break;
    case CRL_ENERGY_L2SQ:
      grad_obj_kernel<LOSS, CRL_ENERGY_L2SQ><<<grid, 256, 0, s>>>(F, B, ld, r, c, diag, aux, beta, rowsum);
      break;
    default:  // dot, cosine and L1 use G itself
      grad_obj_kernel<LOSS, CRL_ENERGY_DOT><<<grid, 256, 0, s>>>(F, B, ld, r, c, diag, aux, beta, rowsum);
  }
}

hipError_t launch_grad_obj(float* F, int B, int ld, const float* r, const float* c,
                           const float* diag, const float* aux, int loss, int energy, float beta,
                           float* rowsum, hipStream_t s) {
  KTimer t = timing_begin("grad_obj_kernel", 0.0, 8.0 * B * B, s);
  switch (loss) {
    case CRL_LOSS_FWD: grad_obj_launch<CRL_LOSS_FWD>(F, B, ld, r, c, diag, aux, energy, beta, rowsum, s); break;
    case CRL_LOSS_SYM: grad_obj_launch<CRL_LOSS_SYM>(F, B, ld, r, c, diag, aux, energy, beta, rowsum, s); break;
    case CRL_LOSS_BWD: grad_obj_launch<CRL_LOSS_BWD>(F, B, ld, r, c, diag, aux, energy, beta, rowsum, s); break;
    case CRL_LOSS_FLATNCE_FWD: grad_obj_launch<CRL_LOSS_FLATNCE_FWD>(F, B, ld, r, c, diag, aux, energy, beta, rowsum, s); break;
    case CRL_LOSS_FLATNCE_BWD: grad_obj_launch<CRL_LOSS_FLATNCE_BWD>(F, B, ld, r, c, diag, aux, energy, beta, rowsum, s); break;
    case CRL_LOSS_FB: grad_obj_launch<CRL_LOSS_FB>(F, B, ld, r, c, diag, aux, energy, beta, rowsum, s); break;
    case CRL_LOSS_DPO: grad_obj_launch<CRL_LOSS_DPO>(F, B, ld, r, c, diag, aux, energy, beta, rowsum, s); break;
    case CRL_LOSS_IPO: grad_obj_launch<CRL_LOSS_IPO>(F, B, ld, r, c, diag, aux, energy, beta, rowsum, s); break;
    case CRL_LOSS_SPPO: grad_obj_launch<CRL_LOSS_SPPO>(F, B, ld, r, c, diag, aux, energy, beta, rowsum, s); break;
    default: return hipErrorInvalidValue;
  }
  timing_end(t);
  return hipGetLastError();
}

// Cosine energy backward: with dU = G V (rows of unit vectors U, V),
// dX_i = (dU_i - (dU_i . U_i) U_i) / |X_i| (0 for a zero row), in place on dX.
__global__ __launch_bounds__(256) void cos_fix_kernel(float* __restrict__ dX,
                                                      const float* __restrict__ U,
                                                      const float* __restrict__ nrm, int B,
                                                      int D) {
  const int lane = threadIdx.x & 63;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= B) return;
  float* dx = dX + (int64_t)row * D;
  const float* u = U + (int64_t)row * D;
  float s = 0.f;
  for (int d = lane; d < D; d += 64) s += dx[d] * u[d];
  s = wave_sum(s);
  const float n = nrm[row];
  const float inv = n > 0.f ? 1.f / n : 0.f;
  for (int d = lane; d < D; d += 64) dx[d] = (dx[d] - s * u[d]) * inv;
}
hipError_t launch_cos_fix(float* dX, const float* U, const float* nrm, int B, int D, hipStream_t s) {
  CRL_TIMED("cos_fix_kernel", 4.0 * B * D, 4.0 * B * (3.0 * D + 1.0), s,
            cos_fix_kernel<<<(B + 3) / 4, 256, 0, s>>>(dX, U, nrm, B, D));
  return hipGetLastError();
}

}  // namespace crl
