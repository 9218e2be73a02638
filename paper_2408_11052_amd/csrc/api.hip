// C ABI of the CRL update hot path: context, layouts, argument checks and the
// orchestration of the kernels for each entry point.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <vector>

#include "../../include/crl.h"
#include "internal.hpp"

using namespace crl;

namespace {

thread_local char g_err[512] = "";

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}
int hip_fail(hipError_t e, const char* what) {
  return fail(CRL_EHIP, "%s: %s", what, hipGetErrorString(e));
}
#define CRL_HIP(expr, what)                       \
  do {                                            \
    hipError_t _e = (expr);                       \
    if (_e != hipSuccess) return hip_fail(_e, what); \
  } while (0)

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct LayerOff {
  int64_t w, b, g, be;
  int fan_in, fan_out;
};

}  // namespace

struct crl_ctx {
  crl_config cfg;
  int device;
  bool bf16, ln, l2, sym, fused;
  int B, H, D, L;            // batch, hidden width, repr dim, hidden layers
  int fan_in0[2];            // d_s + d_a, d_g
  int ld_in[2];              // ld_sa, ld_g
  int ld_sg;
  int esz;                   // bytes per activation element
  std::vector<LayerOff> lay[2];
  int64_t nparam;
  std::vector<int64_t> gaps; // (offset, len) pairs of padding
  // device tables
  uint64_t* d_thr;
  int64_t* d_gaps;
  int n_gaps;
  // workspace plan (byte offsets)
  int64_t ws_bytes;
  std::vector<int64_t> Z[2], Hh[2], mu[2], rstd[2];
  int64_t out[2], dout[2], dout_t[2], dH[2], dZ[2][2], lnpart[2], cpart[2];
  int64_t splitk, splitk_len;  // floats per problem
  int64_t r, c, diag, nphi, npsi, logits, cpm, cps, rowsumH, colsumH, cpartB;
  int64_t phi_b, psi_b, row_m, row_s, col_m, col_s, dx_part, rs_part;
  int ln_rows_per_wave, ln_nparts, rchunks;
  int ldF;                     // row stride of the materialised logits
};

namespace {

int validate(const crl_config* c) {
  if (!c) return fail(CRL_EINVAL, "config is NULL");
  for (int i = 0; i < 7; ++i)
    if (c->reserved[i] != 0) return fail(CRL_EINVAL, "reserved config fields must be zero");
  if (c->batch < 1 || c->batch > 65536) return fail(CRL_EINVAL, "batch must be in [1, 65536]");
  if (c->obs_dim < 1 || c->act_dim < 0 || c->goal_dim < 1)
    return fail(CRL_EINVAL, "obs_dim >= 1, act_dim >= 0, goal_dim >= 1 required");
  if (c->goal_lo < 0 || c->goal_lo + c->goal_dim > c->obs_dim)
    return fail(CRL_EINVAL, "goal slice [goal_lo, goal_lo + goal_dim) outside the observation");
  if (c->n_hidden < 1 || c->n_hidden > 16) return fail(CRL_EINVAL, "n_hidden must be in [1, 16]");
  if (c->hidden < 8 || c->hidden % 8 || c->hidden > 1024)
    return fail(CRL_EINVAL, "hidden must be a multiple of 8 in [8, 1024]");
  if (c->repr_dim < 8 || c->repr_dim % 8 || c->repr_dim > 1024)
    return fail(CRL_EINVAL, "repr_dim must be a multiple of 8 in [8, 1024]");
  if (c->activation != CRL_ACT_RELU && c->activation != CRL_ACT_LN_SWISH)
    return fail(CRL_EINVAL, "unknown activation %d", c->activation);
  if (c->energy != CRL_ENERGY_DOT && c->energy != CRL_ENERGY_L2)
    return fail(CRL_EINVAL, "unknown energy %d", c->energy);
  if (c->loss != CRL_LOSS_FWD && c->loss != CRL_LOSS_SYM)
    return fail(CRL_EINVAL, "unknown loss %d", c->loss);
  if (c->precision != CRL_PREC_FP32 && c->precision != CRL_PREC_BF16)
    return fail(CRL_EINVAL, "unknown precision %d", c->precision);
  if (c->logits != CRL_LOGITS_MATERIALISED && c->logits != CRL_LOGITS_FUSED)
    return fail(CRL_EINVAL, "unknown logits mode %d", c->logits);
  if (c->logits == CRL_LOGITS_FUSED) {
    if (c->precision != CRL_PREC_BF16)
      return fail(CRL_EUNSUPPORTED, "fused logits are implemented for BF16 tiles only");
    if (c->repr_dim != 32 && c->repr_dim != 64 && c->repr_dim != 128 && c->repr_dim != 256)
      return fail(CRL_EUNSUPPORTED, "fused logits need repr_dim in {32, 64, 128, 256}");
  } else if (c->batch > 32768) {
    return fail(CRL_EUNSUPPORTED, "materialised logits are limited to batch <= 32768");
  }
  if (!(c->logsumexp_penalty >= 0.f) || !std::isfinite(c->logsumexp_penalty))
    return fail(CRL_EINVAL, "logsumexp_penalty must be finite and >= 0");
  if (!(c->ln_eps > 0.f) || !std::isfinite(c->ln_eps)) return fail(CRL_EINVAL, "ln_eps must be > 0");
  if (!(c->discount > 0.0 && c->discount < 1.0)) return fail(CRL_EINVAL, "discount must lie in (0, 1)");
  if (c->max_episode_len < 2) return fail(CRL_EINVAL, "max_episode_len must be >= 2");
  return CRL_OK;
}

void plan_params(crl_ctx* x) {
  int64_t off = 0;
  auto take = [&](int64_t n) {
    int64_t o = align_up(off, 64);
    if (o > off) { x->gaps.push_back(off); x->gaps.push_back(o - off); }
    off = o + n;
    return o;
  };
  for (int e = 0; e < 2; ++e) {
    x->lay[e].clear();
    int in = x->fan_in0[e];
    for (int l = 0; l <= x->L; ++l) {
      const bool last = l == x->L;
      const int out = last ? x->D : x->H;
      LayerOff lo;
      lo.fan_in = in;
      lo.fan_out = out;
      lo.w = take((int64_t)in * out);
      lo.b = take(out);
      lo.g = lo.be = -1;
      if (!last && x->ln) { lo.g = take(out); lo.be = take(out); }
      x->lay[e].push_back(lo);
      in = out;
    }
  }
  int64_t end = align_up(off, 64);
  if (end > off) { x->gaps.push_back(off); x->gaps.push_back(end - off); }
  x->nparam = end;
  x->n_gaps = (int)(x->gaps.size() / 2);
}

// split-K planning for the dW products (and the materialised dphi/dpsi)
int64_t splitk_need(crl_ctx* x) {
  int64_t need = 0;
  auto consider = [&](int M0, int N0, int M1, int N1, int K) {
    GemmParams P{};
    P.count = 2;
    P.d[0].M = M0; P.d[0].N = N0; P.d[0].K = K;
    P.d[1].M = M1; P.d[1].N = N1; P.d[1].K = K;
    P.partial = reinterpret_cast<float*>(1);
    plan_split_k(P, x->bf16, 512);
    int64_t len = (int64_t)P.splits * (std::max((int64_t)M0 * N0, (int64_t)M1 * N1));
    if (P.splits > 1 && len > need) need = len;
  };
  for (int l = 0; l <= x->L; ++l)
    consider(x->lay[0][l].fan_in, x->lay[0][l].fan_out, x->lay[1][l].fan_in,
             x->lay[1][l].fan_out, x->B);
  // forward output layer: [B x H] . [H x D]
  consider(x->B, x->D, x->B, x->D, x->H);
  if (!x->fused) {
    // dphi = G psi and dpsi = G^T phi run as single problems with FP32 tiles
    GemmParams P{};
    P.count = 1;
    P.d[0].M = x->B; P.d[0].N = x->D; P.d[0].K = x->B;
    P.partial = reinterpret_cast<float*>(1);
    plan_split_k(P, false, 512);
    int64_t len = (int64_t)P.splits * x->B * x->D;
    if (P.splits > 1 && len > need) need = len;
  }
  return need;
}

void plan_workspace(crl_ctx* x) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) {
    int64_t o = align_up(off, 256);
    off = o + (bytes > 0 ? bytes : 1);
    return o;
  };
  const int64_t B = x->B, H = x->H, D = x->D;
  const int64_t es = x->esz;
  x->ln_rows_per_wave = 16;
  x->ln_nparts = ln_bwd_partials(x->B, x->ln_rows_per_wave);
  for (int e = 0; e < 2; ++e) {
    x->Z[e].assign(x->L, -1);
    x->Hh[e].assign(x->L, -1);
    x->mu[e].assign(x->L, -1);
    x->rstd[e].assign(x->L, -1);
    for (int l = 0; l < x->L; ++l) {
      if (x->ln) {
        x->Z[e][l] = take(B * H * es);
        x->mu[e][l] = take(B * 4);
        x->rstd[e][l] = take(B * 4);
      }
      x->Hh[e][l] = take(B * H * es);
    }
    x->out[e] = take(B * D * 4);
    x->dout[e] = take(B * D * 4);
    x->dout_t[e] = x->bf16 ? take(B * D * es) : x->dout[e];  // FP32: the same buffer
    x->dH[e] = take(B * H * es);
    x->dZ[e][0] = take(B * H * es);
    x->dZ[e][1] = take(B * H * es);
    x->lnpart[e] = x->ln ? take((int64_t)x->ln_nparts * 3 * H * 4) : -1;
    x->cpart[e] = take(((B + 127) / 128) * std::max(H, D) * 4);
  }
  x->splitk_len = splitk_need(x);
  x->splitk = take(2 * x->splitk_len * 4);
  x->r = take(B * 4);
  x->c = take(B * 4);
  x->diag = take(B * 4);
  x->nphi = take(B * 4);
  x->npsi = take(B * 4);
  x->logits = x->cpm = x->cps = x->rowsumH = x->colsumH = x->cpartB = -1;
  x->phi_b = x->psi_b = x->row_m = x->row_s = x->col_m = x->col_s = x->dx_part = x->rs_part = -1;
  if (!x->fused) {
    x->rchunks = 64;
    x->ldF = (int)align_up(B, 8);
    x->logits = take(B * x->ldF * 4);
    x->cpm = take((int64_t)x->rchunks * B * 4);
    x->cps = take((int64_t)x->rchunks * B * 4);
    x->rowsumH = take(B * 4);
    x->colsumH = take(B * 4);
    x->cpartB = take(((B + 127) / 128) * x->ldF * 4);
  } else {
    const int S = fused_splits(x->B);
    const int nrb = (x->B + 63) / 64;
    x->phi_b = take(B * D * 2);
    x->psi_b = take(B * D * 2);
    x->row_m = take((int64_t)S * B * 4);
    x->row_s = take((int64_t)S * B * 4);
    x->col_m = take((int64_t)nrb * B * 4);
    x->col_s = take((int64_t)nrb * B * 4);
    x->dx_part = take((int64_t)S * B * D * 4);
    x->rs_part = take((int64_t)S * B * 4);
  }
  x->ws_bytes = align_up(off, 256);
}

inline char* W(void* ws, int64_t off) { return static_cast<char*>(ws) + off; }
inline float* WF(void* ws, int64_t off) { return reinterpret_cast<float*>(W(ws, off)); }

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

int check_device(const crl_ctx* x) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev != x->device)
    return fail(CRL_EINVAL, "context was created on device %d, current device is %d", x->device, dev);
  return CRL_OK;
}

}  // namespace

extern "C" {

CRL_API const char* crl_last_error(void) { return g_err; }

CRL_API int crl_create(const crl_config* cfg, crl_ctx** out) {
  if (!out) return fail(CRL_EINVAL, "out is NULL");
  *out = nullptr;
  int rc = validate(cfg);
  if (rc) return rc;
  crl_ctx* x = new crl_ctx();
  x->cfg = *cfg;
  CRL_HIP(hipGetDevice(&x->device), "hipGetDevice");
  x->bf16 = cfg->precision == CRL_PREC_BF16;
  x->ln = cfg->activation == CRL_ACT_LN_SWISH;
  x->l2 = cfg->energy == CRL_ENERGY_L2;
  x->sym = cfg->loss == CRL_LOSS_SYM;
  x->fused = cfg->logits == CRL_LOGITS_FUSED;
  x->B = cfg->batch;
  x->H = cfg->hidden;
  x->D = cfg->repr_dim;
  x->L = cfg->n_hidden;
  x->fan_in0[0] = cfg->obs_dim + cfg->act_dim;
  x->fan_in0[1] = cfg->goal_dim;
  x->ld_in[0] = (int)align_up(x->fan_in0[0], 8);
  x->ld_in[1] = (int)align_up(x->fan_in0[1], 8);
  x->ld_sg = (int)align_up(cfg->obs_dim + cfg->goal_dim, 8);
  x->esz = x->bf16 ? 2 : 4;
  plan_params(x);
  plan_workspace(x);
  // geometric-offset thresholds thr[1..T-2] (stored from index 0)
  const int nthr = std::max(1, cfg->max_episode_len - 2);
  std::vector<uint64_t> thr(nthr, 0);
  const uint64_t G = (uint64_t)(cfg->discount * 18446744073709551616.0);
  uint64_t t = G;
  for (int m = 0; m < nthr; ++m) {
    thr[m] = t;
    t = (uint64_t)(((unsigned __int128)t * G) >> 64);
  }
  x->d_thr = nullptr;
  x->d_gaps = nullptr;
  hipError_t e = hipMalloc(&x->d_thr, nthr * sizeof(uint64_t));
  if (e == hipSuccess) e = hipMemcpy(x->d_thr, thr.data(), nthr * sizeof(uint64_t), hipMemcpyHostToDevice);
  if (e == hipSuccess && x->n_gaps > 0) {
    e = hipMalloc(&x->d_gaps, x->gaps.size() * sizeof(int64_t));
    if (e == hipSuccess)
      e = hipMemcpy(x->d_gaps, x->gaps.data(), x->gaps.size() * sizeof(int64_t), hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    if (x->d_thr) (void)hipFree(x->d_thr);
    if (x->d_gaps) (void)hipFree(x->d_gaps);
    delete x;
    return hip_fail(e, "crl_create device tables");
  }
  *out = x;
  return CRL_OK;
}

CRL_API int crl_destroy(crl_ctx* x) {
  if (!x) return CRL_OK;
  if (x->d_thr) (void)hipFree(x->d_thr);
  if (x->d_gaps) (void)hipFree(x->d_gaps);
  delete x;
  return CRL_OK;
}

CRL_API int crl_param_count(const crl_ctx* x, int64_t* n) {
  if (!x || !n) return fail(CRL_EINVAL, "NULL argument");
  *n = x->nparam;
  return CRL_OK;
}

CRL_API int crl_layer_layout(const crl_ctx* x, int32_t enc, int32_t layer, crl_layer_info* out) {
  if (!x || !out) return fail(CRL_EINVAL, "NULL argument");
  if (enc < 0 || enc > 1) return fail(CRL_EINVAL, "encoder must be 0 (phi) or 1 (psi)");
  if (layer < 0 || layer > x->L) return fail(CRL_EINVAL, "layer %d out of range [0, %d]", layer, x->L);
  const LayerOff& l = x->lay[enc][layer];
  out->w = l.w;
  out->b = l.b;
  out->ln_g = l.g;
  out->ln_b = l.be;
  out->fan_in = l.fan_in;
  out->fan_out = l.fan_out;
  return CRL_OK;
}

CRL_API int crl_workspace_size(const crl_ctx* x, int64_t* bytes) {
  if (!x || !bytes) return fail(CRL_EINVAL, "NULL argument");
  *bytes = x->ws_bytes;
  return CRL_OK;
}

CRL_API int crl_input_layout(const crl_ctx* x, int32_t* ld_sa, int32_t* ld_g, int32_t* ld_sg,
                             int32_t* elem_bytes) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (ld_sa) *ld_sa = x->ld_in[0];
  if (ld_g) *ld_g = x->ld_in[1];
  if (ld_sg) *ld_sg = x->ld_sg;
  if (elem_bytes) *elem_bytes = x->esz;
  return CRL_OK;
}

CRL_API int crl_workspace_view(const crl_ctx* x, int32_t which, int64_t* offset, int64_t* bytes) {
  if (!x || !offset || !bytes) return fail(CRL_EINVAL, "NULL argument");
  const int64_t B = x->B, D = x->D;
  switch (which) {
    case CRL_WS_PHI: *offset = x->out[0]; *bytes = B * D * 4; break;
    case CRL_WS_PSI: *offset = x->out[1]; *bytes = B * D * 4; break;
    case CRL_WS_ROW_LSE: *offset = x->r; *bytes = B * 4; break;
    case CRL_WS_COL_LSE: *offset = x->c; *bytes = B * 4; break;
    case CRL_WS_DIAG: *offset = x->diag; *bytes = B * 4; break;
    case CRL_WS_DPHI: *offset = x->dout[0]; *bytes = B * D * 4; break;
    case CRL_WS_DPSI: *offset = x->dout[1]; *bytes = B * D * 4; break;
    case CRL_WS_LOGITS:
      if (x->fused) return fail(CRL_EUNSUPPORTED, "fused logits are never materialised");
      *offset = x->logits; *bytes = B * x->ldF * 4; break;
    default: return fail(CRL_EINVAL, "unknown workspace view %d", which);
  }
  return CRL_OK;
}

CRL_API int crl_sample_relabel(crl_ctx* x, const float* obs, const float* act, int32_t E,
                               int32_t T, uint64_t seed, const int64_t* step, int32_t* idx,
                               void* x_sa, void* x_g, void* x_sg, void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!obs || !step || !idx || !x_sa || !x_g) return fail(CRL_EINVAL, "NULL buffer argument");
  if (!act && x->cfg.act_dim > 0) return fail(CRL_EINVAL, "act is NULL");
  if (E < 1) return fail(CRL_EINVAL, "num_envs must be >= 1");
  if (T < 2 || T > x->cfg.max_episode_len)
    return fail(CRL_EINVAL, "episode_len %d outside [2, %d]", T, x->cfg.max_episode_len);
  int rc = check_device(x);
  if (rc) return rc;
  CRL_HIP(launch_relabel(obs, act, E, T, x->cfg.obs_dim, x->cfg.act_dim, x->cfg.goal_dim,
                         x->cfg.goal_lo, seed, step, x->d_thr, x->B, idx, x_sa, x->ld_in[0],
                         x_g, x->ld_in[1], x_sg, x->ld_sg, x->bf16, (hipStream_t)stream),
          "relabel launch");
  return CRL_OK;
}

CRL_API int crl_critic_fwd(crl_ctx* x, const float* params, const uint16_t* params_bf16,
                           const void* x_sa, const void* x_g, void* ws, float* loss_out,
                           void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!params || !x_sa || !x_g || !ws || !loss_out) return fail(CRL_EINVAL, "NULL buffer argument");
  if (x->bf16 && !params_bf16) return fail(CRL_EINVAL, "BF16 precision needs params_bf16");
  if (!aligned16(params) || !aligned16(x_sa) || !aligned16(x_g) || !aligned16(ws) ||
      (params_bf16 && !aligned16(params_bf16)))
    return fail(CRL_EINVAL, "buffers must be 16-byte aligned");
  int rc = check_device(x);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int B = x->B, H = x->H, D = x->D, L = x->L;
  const void* xin[2] = {x_sa, x_g};

  // encoders, both in every launch
  for (int l = 0; l <= L; ++l) {
    const bool last = l == L;
    GemmParams P{};
    P.count = 2;
    for (int e = 0; e < 2; ++e) {
      const LayerOff& lo = x->lay[e][l];
      GemmDesc& d = P.d[e];
      d.A = l == 0 ? xin[e] : (const void*)W(ws, x->Hh[e][l - 1]);
      d.lda = l == 0 ? x->ld_in[e] : H;
      d.B = x->bf16 ? (const void*)(params_bf16 + lo.w) : (const void*)(params + lo.w);
      d.ldb = lo.fan_out;
      d.M = B; d.N = lo.fan_out; d.K = lo.fan_in;
      d.bias = params + lo.b;
      d.alpha = 1.f;
      if (last) { d.C = W(ws, x->out[e]); d.epi = EPI_BIAS; }
      else if (!x->ln) { d.C = W(ws, x->Hh[e][l]); d.epi = EPI_BIAS_RELU; }
      else { d.C = W(ws, x->Z[e][l]); d.epi = EPI_BIAS; }
      d.ldc = lo.fan_out;
    }
    if (last) P.partial = WF(ws, x->splitk);  // few output tiles: split K
    plan_split_k(P, x->bf16, 512);
    if (P.splits > 1)
      P.partial_len = (int64_t)P.splits * std::max((int64_t)P.d[0].M * P.d[0].N,
                                                   (int64_t)P.d[1].M * P.d[1].N);
    CRL_HIP(launch_gemm(P, x->bf16, LAY_KC, LAY_MC, x->bf16 && !last, s), "encoder GEMM");
    if (!last && x->ln) {
      LnArgs a{};
      for (int e = 0; e < 2; ++e) {
        const LayerOff& lo = x->lay[e][l];
        a.Z[e] = W(ws, x->Z[e][l]);
        a.H[e] = W(ws, x->Hh[e][l]);
        a.mu[e] = WF(ws, x->mu[e][l]);
        a.rstd[e] = WF(ws, x->rstd[e][l]);
        a.g[e] = params + lo.g;
        a.b[e] = params + lo.be;
      }
      CRL_HIP(launch_ln_swish_fwd(a, 2, B, H, x->cfg.ln_eps, x->bf16, s), "LayerNorm forward");
    }
  }

  float* phi = WF(ws, x->out[0]);
  float* psi = WF(ws, x->out[1]);
  float* r = WF(ws, x->r);
  float* c = WF(ws, x->c);
  float* dg = WF(ws, x->diag);
  if (!x->fused) {
    float* F = WF(ws, x->logits);
    GemmParams P{};
    P.count = 1;
    GemmDesc& d = P.d[0];
    d.A = phi; d.lda = D;
    d.B = psi; d.ldb = D;
    d.C = F; d.ldc = x->ldF;
    d.M = B; d.N = B; d.K = D;
    d.alpha = 1.f;
    d.epi = EPI_NONE;
    if (x->l2) {
      CRL_HIP(launch_sqnorm(phi, WF(ws, x->nphi), B, D, s), "norms");
      CRL_HIP(launch_sqnorm(psi, WF(ws, x->npsi), B, D, s), "norms");
      d.epi = EPI_L2;
      d.rowv = WF(ws, x->nphi);
      d.colv = WF(ws, x->npsi);
    }
    plan_split_k(P, false, 512);
    CRL_HIP(launch_gemm(P, false, LAY_KC, LAY_KC, false, s), "logits GEMM");
    CRL_HIP(launch_row_lse(F, B, x->ldF, r, dg, s), "row LSE");
    const int rc_ = std::min(x->rchunks, B);
    CRL_HIP(launch_col_lse_partial(F, B, x->ldF, rc_, WF(ws, x->cpm), WF(ws, x->cps), s), "column LSE");
    CRL_HIP(launch_lse_merge(WF(ws, x->cpm), WF(ws, x->cps), rc_, B, c, s), "column LSE merge");
  } else {
    FusedArgs a{};
    a.phi = phi; a.psi = psi;
    a.phi_b = reinterpret_cast<bf16_t*>(W(ws, x->phi_b));
    a.psi_b = reinterpret_cast<bf16_t*>(W(ws, x->psi_b));
    a.nphi = WF(ws, x->nphi); a.npsi = WF(ws, x->npsi);
    a.row_m = WF(ws, x->row_m); a.row_s = WF(ws, x->row_s);
    a.col_m = WF(ws, x->col_m); a.col_s = WF(ws, x->col_s);
    a.r = r; a.c = c; a.diag = dg;
    CRL_HIP(launch_fused_fwd(a, B, D, x->l2, s), "fused InfoNCE forward");
  }
  CRL_HIP(launch_loss(r, c, dg, B, x->sym, x->cfg.logsumexp_penalty, loss_out, s), "loss");
  return CRL_OK;
}

CRL_API int crl_critic_bwd(crl_ctx* x, const float* params, const uint16_t* params_bf16,
                           const void* x_sa, const void* x_g, void* ws, float* grads,
                           void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!params || !x_sa || !x_g || !ws || !grads) return fail(CRL_EINVAL, "NULL buffer argument");
  if (x->bf16 && !params_bf16) return fail(CRL_EINVAL, "BF16 precision needs params_bf16");
  if (!aligned16(params) || !aligned16(ws) || !aligned16(grads) || !aligned16(x_sa) ||
      !aligned16(x_g) || (params_bf16 && !aligned16(params_bf16)))
    return fail(CRL_EINVAL, "buffers must be 16-byte aligned");
  int rc = check_device(x);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int B = x->B, H = x->H, D = x->D, L = x->L;
  const float beta = x->cfg.logsumexp_penalty;
  const void* xin[2] = {x_sa, x_g};
  float* phi = WF(ws, x->out[0]);
  float* psi = WF(ws, x->out[1]);
  float* r = WF(ws, x->r);
  float* c = WF(ws, x->c);
  float* dphi = WF(ws, x->dout[0]);
  float* dpsi = WF(ws, x->dout[1]);
  float* splitk = WF(ws, x->splitk);

  CRL_HIP(launch_zero_ranges(grads, x->d_gaps, x->n_gaps, s), "zero padding");

  // dL/dphi, dL/dpsi
  if (!x->fused) {
    float* F = WF(ws, x->logits);
    float* rsH = WF(ws, x->rowsumH);
    CRL_HIP(launch_grad_matrix(F, B, x->ldF, r, c, x->sym, beta, x->l2, rsH, s), "grad matrix");
    for (int side = 0; side < 2; ++side) {
      // side 0: dphi = G psi (G as KC); side 1: dpsi = G^T phi (G as MC)
      GemmParams P{};
      P.count = 1;
      GemmDesc& d = P.d[0];
      d.A = F; d.lda = x->ldF;
      d.B = side == 0 ? psi : phi; d.ldb = D;
      d.C = side == 0 ? dphi : dpsi; d.ldc = D;
      d.M = B; d.N = D; d.K = B;
      d.alpha = 1.f;
      d.epi = EPI_NONE;
      P.partial = splitk;
      plan_split_k(P, false, 512);
      P.partial_len = (int64_t)P.splits * B * D;
      CRL_HIP(launch_gemm(P, false, side == 0 ? LAY_KC : LAY_MC, LAY_MC, false, s), "dphi/dpsi GEMM");
    }
    if (x->l2) {
      CRL_HIP(launch_l2_fix(dphi, phi, rsH, B, D, s), "L2 row term");
      ColSumArgs ca{};
      ca.X[0] = F; ca.out[0] = WF(ws, x->colsumH); ca.part[0] = WF(ws, x->cpartB);
      CRL_HIP(launch_colsum(ca, 1, B, B, x->ldF, false, s), "L2 column sums");
      CRL_HIP(launch_l2_fix(dpsi, psi, WF(ws, x->colsumH), B, D, s), "L2 column term");
    }
    if (x->bf16) {
      CRL_HIP(launch_cast_bf16(dphi, reinterpret_cast<bf16_t*>(W(ws, x->dout_t[0])), (int64_t)B * D, s), "cast");
      CRL_HIP(launch_cast_bf16(dpsi, reinterpret_cast<bf16_t*>(W(ws, x->dout_t[1])), (int64_t)B * D, s), "cast");
    }
  } else {
    FusedArgs a{};
    a.phi = phi; a.psi = psi;
    a.phi_b = reinterpret_cast<bf16_t*>(W(ws, x->phi_b));
    a.psi_b = reinterpret_cast<bf16_t*>(W(ws, x->psi_b));
    a.nphi = WF(ws, x->nphi); a.npsi = WF(ws, x->npsi);
    a.r = r; a.c = c;
    a.dX_part = WF(ws, x->dx_part);
    a.rs_part = WF(ws, x->rs_part);
    a.dphi = dphi; a.dpsi = dpsi;
    a.dphi_t = W(ws, x->dout_t[0]);
    a.dpsi_t = W(ws, x->dout_t[1]);
    CRL_HIP(launch_fused_bwd(a, B, D, x->l2, x->sym, beta, x->bf16, s), "fused InfoNCE backward");
  }

  // encoders, last layer first; dZ of hidden layers ping-pongs between two buffers
  int cur = 0;
  for (int l = L; l >= 0; --l) {
    const bool last = l == L;
    const void* dZ[2];
    for (int e = 0; e < 2; ++e)
      dZ[e] = last ? (const void*)W(ws, x->dout_t[e]) : (const void*)W(ws, x->dZ[e][cur]);
    {  // dW = in^T . dZ  (contraction over the batch)
      GemmParams P{};
      P.count = 2;
      for (int e = 0; e < 2; ++e) {
        const LayerOff& lo = x->lay[e][l];
        GemmDesc& d = P.d[e];
        d.A = l == 0 ? xin[e] : (const void*)W(ws, x->Hh[e][l - 1]);
        d.lda = l == 0 ? x->ld_in[e] : H;
        d.B = dZ[e]; d.ldb = lo.fan_out;
        d.C = grads + lo.w; d.ldc = lo.fan_out;
        d.M = lo.fan_in; d.N = lo.fan_out; d.K = B;
        d.alpha = 1.f;
        d.epi = EPI_NONE;
      }
      P.partial = splitk;
      plan_split_k(P, x->bf16, 512);
      int64_t mn = std::max((int64_t)P.d[0].M * P.d[0].N, (int64_t)P.d[1].M * P.d[1].N);
      P.partial_len = (int64_t)P.splits * mn;
      CRL_HIP(launch_gemm(P, x->bf16, LAY_MC, LAY_MC, false, s), "dW GEMM");
    }
    // bias gradients of this layer (LayerNorm layers got theirs with dZ)
    if (last || !x->ln) {
      ColSumArgs ca{};
      for (int e = 0; e < 2; ++e) {
        ca.X[e] = last ? (const void*)(e == 0 ? dphi : dpsi) : dZ[e];
        ca.out[e] = grads + x->lay[e][l].b;
        ca.part[e] = WF(ws, x->cpart[e]);
      }
      const int N = last ? D : H;
      CRL_HIP(launch_colsum(ca, 2, B, N, N, last ? false : x->bf16, s), "bias gradient");
    }
    if (l == 0) break;
    // dZ of layer l-1: dH = dZ . W^T, then through ReLU or Swish(LayerNorm)
    const int nxt = last ? 0 : (cur ^ 1);
    {
      GemmParams P{};
      P.count = 2;
      for (int e = 0; e < 2; ++e) {
        const LayerOff& lo = x->lay[e][l];
        GemmDesc& d = P.d[e];
        d.A = dZ[e]; d.lda = lo.fan_out;
        d.B = x->bf16 ? (const void*)(params_bf16 + lo.w) : (const void*)(params + lo.w);
        d.ldb = lo.fan_out;
        d.M = B; d.N = lo.fan_in; d.K = lo.fan_out;
        d.alpha = 1.f;
        d.ldc = lo.fan_in;
        if (x->ln) { d.C = W(ws, x->dH[e]); d.epi = EPI_NONE; }
        else { d.C = W(ws, x->dZ[e][nxt]); d.epi = EPI_MASK_POS; d.aux = W(ws, x->Hh[e][l - 1]); }
      }
      plan_split_k(P, x->bf16, 512);
      CRL_HIP(launch_gemm(P, x->bf16, LAY_KC, LAY_KC, x->bf16, s), "dX GEMM");
    }
    if (x->ln) {
      LnArgs a{};
      ColReduceArgs ra{};
      for (int e = 0; e < 2; ++e) {
        const LayerOff& lp = x->lay[e][l - 1];
        a.Z[e] = W(ws, x->Z[e][l - 1]);
        a.mu[e] = WF(ws, x->mu[e][l - 1]);
        a.rstd[e] = WF(ws, x->rstd[e][l - 1]);
        a.g[e] = params + lp.g;
        a.b[e] = params + lp.be;
        a.dH[e] = W(ws, x->dH[e]);
        a.dZ[e] = W(ws, x->dZ[e][nxt]);
        a.part[e] = WF(ws, x->lnpart[e]);
        ra.part[e] = a.part[e];
        ra.out[e][0] = grads + lp.g;
        ra.out[e][1] = grads + lp.be;
        ra.out[e][2] = grads + lp.b;
      }
      CRL_HIP(launch_ln_swish_bwd(a, 2, B, H, x->bf16, x->ln_rows_per_wave, s), "LayerNorm backward");
      CRL_HIP(launch_partial_reduce(ra, 2, x->ln_nparts, 3, H, s), "LayerNorm parameter gradients");
    }
    cur = nxt;
  }
  return CRL_OK;
}

CRL_API int crl_adam_step(float* p, const float* g, float* m, float* v, uint16_t* p_bf16,
                          int64_t n, const int64_t* step, double lr, double b1, double b2,
                          double eps, void* stream) {
  if (!p || !g || !m || !v || !step) return fail(CRL_EINVAL, "NULL buffer argument");
  if (n < 0) return fail(CRL_EINVAL, "n must be >= 0");
  if (!aligned16(p) || !aligned16(g) || !aligned16(m) || !aligned16(v) ||
      (p_bf16 && (reinterpret_cast<uintptr_t>(p_bf16) & 7u)))
    return fail(CRL_EINVAL, "Adam buffers must be 16-byte aligned (p_bf16 8-byte)");
  if (!(b1 > 0.0 && b1 < 1.0 && b2 > 0.0 && b2 < 1.0 && eps >= 0.0 && std::isfinite(lr)))
    return fail(CRL_EINVAL, "Adam hyperparameters out of range");
  if (n == 0) return CRL_OK;
  AdamCoef c;
  c.lr = (float)lr;
  c.b1 = (float)b1;
  c.b2 = (float)b2;
  c.omb1 = (float)(1.0 - b1);
  c.omb2 = (float)(1.0 - b2);
  c.log_b1 = (float)std::log(b1);
  c.log_b2 = (float)std::log(b2);
  c.eps = (float)eps;
  CRL_HIP(launch_adam(p, g, m, v, reinterpret_cast<bf16_t*>(p_bf16), n, step, c,
                      (hipStream_t)stream), "Adam launch");
  return CRL_OK;
}

CRL_API int crl_counter_add(int64_t* counter, int64_t inc, void* stream) {
  if (!counter) return fail(CRL_EINVAL, "NULL counter");
  CRL_HIP(launch_counter_add(counter, inc, (hipStream_t)stream), "counter launch");
  return CRL_OK;
}

CRL_API int crl_cast_bf16(const float* src, uint16_t* dst, int64_t n, void* stream) {
  if (!src || !dst) return fail(CRL_EINVAL, "NULL buffer argument");
  if (n < 0) return fail(CRL_EINVAL, "n must be >= 0");
  if (!aligned16(src) || (reinterpret_cast<uintptr_t>(dst) & 7u))
    return fail(CRL_EINVAL, "src must be 16-byte aligned, dst 8-byte aligned");
  CRL_HIP(launch_cast_bf16(src, reinterpret_cast<bf16_t*>(dst), n, (hipStream_t)stream), "cast launch");
  return CRL_OK;
}

}  // extern "C"
