// Policy (actor) step kernels: the tanh-Gaussian head with its reparameterised
// sample, the energy of the policy's action under the frozen critic, the head
// backward and the loss reduction (Section 3.2, policy learning; Section 5.1
// setup, tunable entropy coefficient).  The MLPs around them are the encoder
// GEMM / LayerNorm kernels.
#include "internal.hpp"

namespace crl {

namespace {

constexpr float kSigmaMin = 1e-3f;
constexpr float kHalfLog2Pi = 0.91893853320467274f;  // log(2 pi) / 2
constexpr float kLog2 = 0.69314718055994531f;

// log(1 + e^x) without overflow
__device__ inline float softplusf_(float x) { return fmaxf(x, 0.f) + log1pf(expf(-fabsf(x))); }

// 23-bit uniform in (0, 1) from the top bits of a 64-bit word: (2k + 1) / 2^24,
// exact in FP32.
__device__ inline float uniform23(uint64_t w) {
  return (float)(2u * (uint32_t)(w >> 41) + 1u) * 5.9604644775390625e-08f;
}

// Standard normal for action coordinate k of sample b: Box-Muller pair k/2
// takes words (2p, 2p+1), p = (k/2) % 2, of the Philox block with counter
// (b, n, 1, k/4); even k take the cosine branch, odd k the sine branch.
__device__ inline float box_muller(uint64_t seed, uint64_t b, uint64_t n, int k) {
  const int pair = k >> 1;
  uint64_t x[4] = {b, n, 1ull, (uint64_t)(pair >> 1)};
  philox4x64_10(x, seed, 0ull);
  const int w = (pair & 1) * 2;
  const float u1 = uniform23(x[w]), u2 = uniform23(x[w + 1]);
  const float r = sqrtf(-2.f * logf(u1));
  float sn, cs;
  sincospif(2.f * u2, &sn, &cs);
  return r * ((k & 1) ? sn : cs);
}

}  // namespace

// One wavefront per sample.  From the policy output o = [mu | rho | pad]:
// sigma = softplus(rho) + sigma_min, u = mu + sigma eps, a = tanh(u),
// log pi = sum_k [-eps_k^2/2 - log sigma_k - log(2 pi)/2 - 2(log 2 - u_k - softplus(-2 u_k))].
// Writes the critic input [s, a] (state columns copied from x_sa), eps and log pi.
template <typename T>
__global__ __launch_bounds__(256) void actor_head_fwd_kernel(
    const float* __restrict__ out, int ldo, int A, uint64_t seed,
    const int64_t* __restrict__ step, const T* __restrict__ x_sa, T* __restrict__ x_sa2,
    int ld, int d_s, float* __restrict__ eps, float* __restrict__ logpi, int B) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;
  const uint64_t n = (uint64_t)(*step);
  const float* o = out + (int64_t)b * ldo;
  T* row2 = x_sa2 + (int64_t)b * ld;
  float lp = 0.f;
  for (int k = lane; k < A; k += 64) {
    const float z = box_muller(seed, (uint64_t)b, n, k);
    const float mu = o[k], rho = o[A + k];
    const float sigma = softplusf_(rho) + kSigmaMin;
    const float u = fmaf(sigma, z, mu);
    const float a = tanhf(u);
    const float log_det = 2.f * (kLog2 - u - softplusf_(-2.f * u));
    lp += -0.5f * z * z - logf(sigma) - kHalfLog2Pi - log_det;
    eps[(int64_t)b * A + k] = z;
    row2[d_s + k] = Store<T>::from_f(a);
  }
  const T* row = x_sa + (int64_t)b * ld;
  for (int c = lane; c < ld; c += 64) {
    if (c < d_s) row2[c] = row[c];
    else if (c >= d_s + A) row2[c] = Store<T>::from_f(0.f);
  }
  lp = wave_sum(lp);
  if (lane == 0) logpi[b] = lp;
}

// One wavefront per sample: the critic's diagonal energy f_b of the policy's
// action and d(-mean_b f_b)/dphi_b (the critic is frozen), for each energy:
//   dot   f = p.q                       -> -q / B
//   L2    f = -|p - q|                  -> (p - q) / (|p - q| B)  (0 at p = q)
//   cos   f = p.q / (|p| |q|)           -> -(q/|q| - f p/|p|) / (|p| B)
//   L2sq  f = -|p - q|^2                -> 2 (p - q) / B
//   L1    f = -sum |p - q|              -> sign(p - q) / B
template <typename T>
__global__ __launch_bounds__(256) void actor_energy_kernel(
    const float* __restrict__ phi, const float* __restrict__ psi, int D, int energy,
    float* __restrict__ f, T* __restrict__ dphi, int B) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;
  const float* p = phi + (int64_t)b * D;
  const float* q = psi + (int64_t)b * D;
  T* d = dphi + (int64_t)b * D;
  const float invB = 1.f / (float)B;
  float pq = 0.f, pp = 0.f, qq = 0.f, dd = 0.f, l1 = 0.f;
  for (int k = lane; k < D; k += 64) {
    const float x = p[k], y = q[k];
    pq += x * y;
    pp += x * x;
    qq += y * y;
    dd += (x - y) * (x - y);
    l1 += fabsf(x - y);
  }
  pq = wave_sum(pq);
  pp = wave_sum(pp);
  qq = wave_sum(qq);
  dd = wave_sum(dd);
  l1 = wave_sum(l1);
  float fb;
  if (energy == CRL_ENERGY_L2) {
    const float dist = sqrtf(dd);
    const float s = dist > 0.f ? invB / dist : 0.f;
    for (int k = lane; k < D; k += 64) d[k] = Store<T>::from_f((p[k] - q[k]) * s);
    fb = -dist;
  } else if (energy == CRL_ENERGY_COS) {
    const float np = sqrtf(pp), nq = sqrtf(qq);
    const float ip = np > 0.f ? 1.f / np : 0.f, iq = nq > 0.f ? 1.f / nq : 0.f;
    fb = pq * ip * iq;
    for (int k = lane; k < D; k += 64)
      d[k] = Store<T>::from_f(-(q[k] * iq - fb * p[k] * ip) * ip * invB);
  } else if (energy == CRL_ENERGY_L2SQ) {
    for (int k = lane; k < D; k += 64) d[k] = Store<T>::from_f(2.f * (p[k] - q[k]) * invB);
    fb = -dd;
  } else if (energy == CRL_ENERGY_L1) {
    for (int k = lane; k < D; k += 64) {
      const float dl = p[k] - q[k];
      d[k] = Store<T>::from_f((dl > 0.f ? invB : (dl < 0.f ? -invB : 0.f)));
    }
    fb = -l1;
  } else {
    for (int k = lane; k < D; k += 64) d[k] = Store<T>::from_f(-q[k] * invB);
    fb = pq;
  }
  if (lane == 0) f[b] = fb;
}

// One wavefront per sample: the policy-output gradient
//   g_u   = (alpha/B) 2 tanh(u) + da (1 - tanh^2 u)
//   g_mu  = g_u,  g_rho = [(alpha/B)(-1/sigma) + g_u eps] sigmoid(rho)
// with da = d(-mean f)/da' from the frozen critic; columns past 2A are 0.
template <typename T>
__global__ __launch_bounds__(256) void actor_head_bwd_kernel(
    const float* __restrict__ out, int ldo, int A, const float* __restrict__ eps,
    const float* __restrict__ da, int ldd, const float* __restrict__ log_alpha,
    float* dout, T* dout_t, int B) {  // dout_t may alias dout (FP32)
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;
  const float c = expf(*log_alpha) / (float)B;
  const float* o = out + (int64_t)b * ldo;
  float* g = dout + (int64_t)b * ldo;
  T* gt = dout_t + (int64_t)b * ldo;
  for (int k = lane; k < A; k += 64) {
    const float z = eps[(int64_t)b * A + k];
    const float mu = o[k], rho = o[A + k];
    const float sigma = softplusf_(rho) + kSigmaMin;
    const float t = tanhf(fmaf(sigma, z, mu));
    const float gu = 2.f * c * t + da[(int64_t)b * ldd + k] * (1.f - t * t);
    const float gr = (gu * z - c / sigma) / (1.f + expf(-rho));
    g[k] = gu;
    g[A + k] = gr;
    gt[k] = Store<T>::from_f(gu);
    gt[A + k] = Store<T>::from_f(gr);
  }
  for (int k = 2 * A + lane; k < ldo; k += 64) {
    g[k] = 0.f;
    gt[k] = Store<T>::from_f(0.f);
  }
}

// loss_out = {L_pi, mean log pi, L_alpha, mean f}; *alpha_grad = dL_alpha/dlog alpha.
//   L_pi = alpha mean(log pi) - mean(f),  L_alpha = -log alpha (mean(log pi) + H)
// Per-thread Kahan sums, then an ordered tree over the workgroup.
__global__ __launch_bounds__(1024) void actor_loss_kernel(
    const float* __restrict__ logpi, const float* __restrict__ f, int B,
    const float* __restrict__ log_alpha, float target_entropy, float* __restrict__ loss_out,
    float* __restrict__ alpha_grad) {
  __shared__ float sh[2][1024];
  float s0 = 0.f, c0 = 0.f, s1 = 0.f, c1 = 0.f;
  for (int i = threadIdx.x; i < B; i += 1024) {
    kahan_add(s0, c0, logpi[i]);
    kahan_add(s1, c1, f[i]);
  }
  sh[0][threadIdx.x] = s0 - c0;
  sh[1][threadIdx.x] = s1 - c1;
  __syncthreads();
  for (int w = 512; w >= 1; w >>= 1) {
    if ((int)threadIdx.x < w) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + w];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const float la = *log_alpha;
    const float mlp = sh[0][0] / (float)B, mf = sh[1][0] / (float)B;
    loss_out[0] = expf(la) * mlp - mf;
    loss_out[1] = mlp;
    loss_out[2] = -la * (mlp + target_entropy);
    loss_out[3] = mf;
    *alpha_grad = -(mlp + target_entropy);
  }
}

hipError_t launch_actor_head_fwd(const float* out, int ldo, int A, uint64_t seed,
                                 const int64_t* step, const void* x_sa, void* x_sa2, int ld,
                                 int d_s, float* eps, float* logpi, int B, bool bf16,
                                 hipStream_t s) {
  dim3 grid((B + 3) / 4), block(256);
  const double es = bf16 ? 2.0 : 4.0;
  const double bytes = (double)B * (8.0 * A + es * (d_s + ld) + 4.0 * A + 4.0);
  if (bf16)
    CRL_TIMED("actor_head_fwd_kernel", 0.0, bytes, s,
      actor_head_fwd_kernel<bf16_t><<<grid, block, 0, s>>>(out, ldo, A, seed, step,
        (const bf16_t*)x_sa, (bf16_t*)x_sa2, ld, d_s, eps, logpi, B));
  else
    CRL_TIMED("actor_head_fwd_kernel", 0.0, bytes, s,
      actor_head_fwd_kernel<float><<<grid, block, 0, s>>>(out, ldo, A, seed, step,
        (const float*)x_sa, (float*)x_sa2, ld, d_s, eps, logpi, B));
  return hipGetLastError();
}

hipError_t launch_actor_energy(const float* phi, const float* psi, int D, int energy, float* f,
                               void* dphi, int B, bool bf16, hipStream_t s) {
  dim3 grid((B + 3) / 4), block(256);
  const double bytes = (double)B * (8.0 * D + (bf16 ? 2.0 : 4.0) * D + 4.0);
  if (bf16)
    CRL_TIMED("actor_energy_kernel", 2.0 * B * D, bytes, s,
      actor_energy_kernel<bf16_t><<<grid, block, 0, s>>>(phi, psi, D, energy, f, (bf16_t*)dphi, B));
  else
    CRL_TIMED("actor_energy_kernel", 2.0 * B * D, bytes, s,
      actor_energy_kernel<float><<<grid, block, 0, s>>>(phi, psi, D, energy, f, (float*)dphi, B));
  return hipGetLastError();
}

hipError_t launch_actor_head_bwd(const float* out, int ldo, int A, const float* eps,
                                 const float* da, int ldd, const float* log_alpha, float* dout,
                                 void* dout_t, int B, bool bf16, hipStream_t s) {
  dim3 grid((B + 3) / 4), block(256);
  const double bytes = (double)B * (8.0 * A + 8.0 * A + (4.0 + (bf16 ? 2.0 : 4.0)) * ldo);
  if (bf16)
    CRL_TIMED("actor_head_bwd_kernel", 0.0, bytes, s,
      actor_head_bwd_kernel<bf16_t><<<grid, block, 0, s>>>(out, ldo, A, eps, da, ldd, log_alpha,
                                                           dout, (bf16_t*)dout_t, B));
  else
    CRL_TIMED("actor_head_bwd_kernel", 0.0, bytes, s,
      actor_head_bwd_kernel<float><<<grid, block, 0, s>>>(out, ldo, A, eps, da, ldd, log_alpha,
                                                          dout, (float*)dout_t, B));
  return hipGetLastError();
}

// One wavefront per sample: the Philox block (b, n, 2, 0) decides whether
// sample b takes another sample's goal and whose.  Storage values are copied
// as they are, so a mixed row equals the row the sampler would have written
// for that goal.
template <typename T>
__global__ __launch_bounds__(256) void goal_mix_kernel(
    const T* __restrict__ x_g, int ld_g, const T* __restrict__ x_sg, int ld_sg, int d_s,
    int d_g, uint64_t seed, const int64_t* __restrict__ step, uint64_t thr53, int B,
    T* __restrict__ xg_out, T* __restrict__ xsg_out) {
  const int lane = threadIdx.x & 63;
  const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (b >= B) return;
  uint64_t x[4] = {(uint64_t)b, (uint64_t)(*step), 2ull, 0ull};
  philox4x64_10(x, seed, 0ull);
  int j = b;
  if (B >= 2 && (x[0] >> 11) < thr53) {
    j = b + 1 + (int)__umul64hi(x[1], (uint64_t)(B - 1));
    if (j >= B) j -= B;
  }
  const T* __restrict__ g = x_g + (int64_t)j * ld_g;
  for (int c = lane; c < ld_g; c += 64) xg_out[(int64_t)b * ld_g + c] = g[c];
  const T* __restrict__ sg = x_sg + (int64_t)b * ld_sg;
  for (int c = lane; c < ld_sg; c += 64) {
    T v = sg[c];
    if (c >= d_s && c < d_s + d_g) v = g[c - d_s];
    xsg_out[(int64_t)b * ld_sg + c] = v;
  }
}

hipError_t launch_goal_mix(const void* x_g, int ld_g, const void* x_sg, int ld_sg, int d_s,
                           int d_g, uint64_t seed, const int64_t* step, uint64_t thr53, int B,
                           void* xg_out, void* xsg_out, bool bf16, hipStream_t s) {
  dim3 grid((B + 3) / 4), block(256);
  const double bytes = 2.0 * B * (ld_g + ld_sg) * (bf16 ? 2.0 : 4.0);
  if (bf16)
    CRL_TIMED("goal_mix_kernel", 0.0, bytes, s,
      goal_mix_kernel<bf16_t><<<grid, block, 0, s>>>((const bf16_t*)x_g, ld_g,
        (const bf16_t*)x_sg, ld_sg, d_s, d_g, seed, step, thr53, B, (bf16_t*)xg_out,
        (bf16_t*)xsg_out));
  else
    CRL_TIMED("goal_mix_kernel", 0.0, bytes, s,
      goal_mix_kernel<float><<<grid, block, 0, s>>>((const float*)x_g, ld_g,
        (const float*)x_sg, ld_sg, d_s, d_g, seed, step, thr53, B, (float*)xg_out,
        (float*)xsg_out));
  return hipGetLastError();
}

hipError_t launch_actor_loss(const float* logpi, const float* f, int B, const float* log_alpha,
                             float target_entropy, float* loss_out, float* alpha_grad,
                             hipStream_t s) {
  CRL_TIMED("actor_loss_kernel", 0.0, 8.0 * B, s,
            actor_loss_kernel<<<1, 1024, 0, s>>>(logpi, f, B, log_alpha, target_entropy,
                                                 loss_out, alpha_grad));
  return hipGetLastError();
}

}  // namespace crl
