// C ABI of the CRL update hot path: context, layouts, argument checks and the
// orchestration of the kernels for each entry point.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "crl.h"
#include "internal.hpp"

using namespace crl;

// Scratch memory of crl_infonce_fwd_noalloc: one copy per device, held from
// the library's first use on that device until the process ends.  In host
// code `scratch` names the symbol only; its device address comes from
// hipGetSymbolAddress (scratch_address below) and is what kernels receive.
static __device__ __align__(256) unsigned char scratch[CRL_NOALLOC_SCRATCH_BYTES];

namespace {

// This device's address of `scratch`, looked up once per device with that
// device current (crl_create calls it).
hipError_t scratch_address(int dev, void** out) {
  constexpr int kMaxDev = 64;
  static std::mutex mu;
  static void* addr[kMaxDev] = {};
  *out = nullptr;
  if (dev < 0 || dev >= kMaxDev) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *out = addr[dev];
  return hipSuccess;
}

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
#define CRL_TRY(expr)          \
  do {                         \
    int _rc = (expr);          \
    if (_rc != CRL_OK) return _rc; \
  } while (0)

int64_t align_up(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

struct LayerOff {
  int64_t w, b, g, be;
  int fan_in, fan_out;
};

// Static shape of one MLP: phi (0), psi (1) or the policy (2).
struct Net {
  std::vector<LayerOff> lay;  // offsets in the flat vector the net lives in
  int fan_in0;                // input features
  int ld_in;                  // row stride of its input
  int H, L;                   // hidden width and hidden layers
  int out_dim;                // output width (repr dim, or the padded policy head)
};

// Workspace byte offsets of one MLP's activations and gradients.
struct Slots {
  std::vector<int64_t> Z, Hh, mu, rstd;  // per hidden layer
  int64_t out, dout, dout_t;             // [B][out_dim] FP32, FP32, storage type
  int64_t dH, dZ[2];                     // [B][H] storage type
  std::vector<int64_t> lnp;              // per hidden layer: LayerNorm column partials
  std::vector<int64_t> bp;               // per layer: bias column partials, -1 if none
};

// The nets whose backward runs in the same launches, and the reductions of
// their gradient partials that follow it.
struct Group {
  int nets[2], count;
  std::vector<int64_t> dwp;              // per layer: dW split-K partials, -1 if unsplit
  std::vector<int> dwbn;                 // per layer: column tile of the LDS kernel (0: dense partials)
  std::vector<int64_t> dwu;              // per layer: with the Adam epilogue, where an
                                         // unsplit dW goes (-1 if split)
  std::vector<RedJob> few, many;         // reduction jobs (few / many parts); the few
                                         // list ends with the unsplit dW copies, which
                                         // only the Adam epilogue runs
  RedJob* d_few = nullptr;
  RedJob* d_many = nullptr;
  int nfew_plain = 0;                    // few jobs of the plain reduction
  int64_t total4_plain = 0;
  int64_t chunks = 0;                    // blocks of the few jobs with the Adam epilogue
  int64_t total4 = 0, nblocks = 0;
  double few_bytes = 0, many_bytes = 0;
};

// Byte offsets of the buffers the loss forward (critic matrix, log-sum-exps,
// objective terms) uses, inside whichever scratch memory it runs on.
struct LossWs {
  int64_t r, c, diag, nphi, npsi, rowterm, rowaux, uphi, upsi;
  int64_t logits, cpm, cps;                          // materialised logits
  int64_t phi_b, psi_b, row_m, row_s, col_m, col_s;  // fused logits
};

}  // namespace

struct crl_ctx {
  crl_config cfg;
  int device;
  bool bf16, ln, fused, actor;
  int energy, loss;          // CRL_ENERGY_*, CRL_LOSS_*
  int B, H, D, L;            // batch, critic hidden width, repr dim, hidden layers
  int A, P;                  // action dim, padded policy-output width (actor only)
  int ld_sg;
  int esz;                   // bytes per activation element
  Net net[3];
  Slots sl[3];
  Group grp[2];                  // 0: phi and psi, 1: the policy
  int64_t nparam, nparam_actor;
  std::vector<int64_t> gaps[2];  // (offset, len) pairs of padding: critic, actor vector
  // device tables
  uint64_t* d_thr;
  // workspace plan (byte offsets)
  int64_t ws_bytes;
  int64_t splitk, splitk_floats;
  int64_t r, c, diag, nphi, npsi, logits, cpm, cps, rowsumH, colsumH, cpartB;
  int64_t rowterm, rowaux, uphi, upsi;  // pairwise objectives; cosine unit rows
  int64_t phi_b, psi_b, row_m, row_s, col_m, col_s, dx_part, rs_part;
  int64_t xsa2, noise, logpi, fpol, dact;  // actor step
  int64_t xg_mix, xsg_mix;                 // random-goal inputs of the actor step, or -1
  uint64_t mix_thr;                        // floor(random_goal_ratio * 2^53)
  int ldd;                                 // row stride of dact
  int ln_rows_per_wave, ln_nparts, rchunks;
  int ldF;                     // row stride of the materialised logits
  LossWs na;                   // the loss forward packed from offset 0 (no-alloc entry point)
  int64_t na_bytes;            // bytes that layout needs
  void* scratch;               // this device's address of `scratch`, NULL if unavailable
  hipError_t scratch_err;      // why it is unavailable
};

namespace {

int validate(const crl_config* c) {
  if (!c) return fail(CRL_EINVAL, "config is NULL");
  for (int i = 0; i < 2; ++i)
    if (c->reserved[i] != 0) return fail(CRL_EINVAL, "reserved config fields must be zero");
  if (!(c->random_goal_ratio >= 0.0 && c->random_goal_ratio <= 1.0))
    return fail(CRL_EINVAL, "random_goal_ratio must lie in [0, 1]");
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
  if (c->energy < CRL_ENERGY_DOT || c->energy > CRL_ENERGY_L1)
    return fail(CRL_EINVAL, "unknown energy %d", c->energy);
  if (c->loss < CRL_LOSS_FWD || c->loss > CRL_LOSS_SPPO)
    return fail(CRL_EINVAL, "unknown loss %d", c->loss);
  if (c->energy == CRL_ENERGY_L1 && c->repr_dim > 256)
    return fail(CRL_EUNSUPPORTED, "the L1 energy supports repr_dim <= 256");
  if (c->precision != CRL_PREC_FP32 && c->precision != CRL_PREC_BF16)
    return fail(CRL_EINVAL, "unknown precision %d", c->precision);
  if (c->logits != CRL_LOGITS_MATERIALISED && c->logits != CRL_LOGITS_FUSED)
    return fail(CRL_EINVAL, "unknown logits mode %d", c->logits);
  if (c->logits == CRL_LOGITS_FUSED) {
    if (c->precision != CRL_PREC_BF16)
      return fail(CRL_EUNSUPPORTED, "fused logits are implemented for BF16 tiles only");
    if (c->repr_dim != 32 && c->repr_dim != 64 && c->repr_dim != 128 && c->repr_dim != 256)
      return fail(CRL_EUNSUPPORTED, "fused logits need repr_dim in {32, 64, 128, 256}");
    if (c->energy == CRL_ENERGY_L1)
      return fail(CRL_EUNSUPPORTED, "the L1 energy is not a product: materialised logits only");
    if (c->loss > CRL_LOSS_FLATNCE_BWD)
      return fail(CRL_EUNSUPPORTED,
                  "fused logits take the InfoNCE and FlatNCE objectives; the pairwise ones "
                  "(FB, DPO, IPO, SPPO) need materialised logits");
  } else if (c->batch > 32768) {
    return fail(CRL_EUNSUPPORTED, "materialised logits are limited to batch <= 32768");
  }
  if (!(c->logsumexp_penalty >= 0.f) || !std::isfinite(c->logsumexp_penalty))
    return fail(CRL_EINVAL, "logsumexp_penalty must be finite and >= 0");
  if (!(c->ln_eps > 0.f) || !std::isfinite(c->ln_eps)) return fail(CRL_EINVAL, "ln_eps must be > 0");
  if (!(c->discount > 0.0 && c->discount < 1.0)) return fail(CRL_EINVAL, "discount must lie in (0, 1)");
  if (c->max_episode_len < 2) return fail(CRL_EINVAL, "max_episode_len must be >= 2");
  if (c->actor_n_hidden < 0 || c->actor_n_hidden > 16)
    return fail(CRL_EINVAL, "actor_n_hidden must be in [0, 16]");
  if (c->actor_n_hidden == 0) {
    if (c->actor_hidden != 0) return fail(CRL_EINVAL, "actor_hidden must be 0 without an actor");
  } else {
    if (c->actor_hidden < 8 || c->actor_hidden % 8 || c->actor_hidden > 1024)
      return fail(CRL_EINVAL, "actor_hidden must be a multiple of 8 in [8, 1024]");
    if (c->act_dim < 1 || c->act_dim > 256)
      return fail(CRL_EINVAL, "the actor needs act_dim in [1, 256]");
    if (!std::isfinite(c->target_entropy)) return fail(CRL_EINVAL, "target_entropy must be finite");
  }
  return CRL_OK;
}

// Lays out the nets `first..last` one after another in one flat vector; each
// tensor starts on a 64-element boundary and the gaps are recorded.
int64_t plan_params(crl_ctx* x, int first, int last, std::vector<int64_t>& gaps) {
  int64_t off = 0;
  auto take = [&](int64_t n) {
    int64_t o = align_up(off, 64);
    if (o > off) { gaps.push_back(off); gaps.push_back(o - off); }
    off = o + n;
    return o;
  };
  gaps.clear();
  for (int e = first; e <= last; ++e) {
    Net& N = x->net[e];
    N.lay.clear();
    int in = N.fan_in0;
    for (int l = 0; l <= N.L; ++l) {
      const bool top = l == N.L;
      const int out = top ? N.out_dim : N.H;
      LayerOff lo;
      lo.fan_in = in;
      lo.fan_out = out;
      lo.w = take((int64_t)in * out);
      lo.b = take(out);
      lo.g = lo.be = -1;
      if (!top && x->ln) { lo.g = take(out); lo.be = take(out); }
      N.lay.push_back(lo);
      in = out;
    }
  }
  int64_t end = align_up(off, 64);
  if (end > off) { gaps.push_back(off); gaps.push_back(end - off); }
  return end;
}

// Floats of split-K partials that the largest split GEMM launch needs.
int64_t splitk_need(crl_ctx* x) {
  int64_t need = 0;
  auto consider = [&](int count, const int (*mnk)[3], bool bf16) {
    GemmParams P{};
    P.count = count;
    int64_t mn = 0;
    for (int g = 0; g < count; ++g) {
      P.d[g].M = mnk[g][0]; P.d[g].N = mnk[g][1]; P.d[g].K = mnk[g][2];
      mn = std::max(mn, (int64_t)mnk[g][0] * mnk[g][1]);
    }
    P.partial = reinterpret_cast<float*>(1);
    plan_split_k(P, bf16, 512);
    if (P.splits > 1) need = std::max(need, (int64_t)count * P.splits * mn);
  };
  const Net* n = x->net;
  // critic: dW of every layer, and the forward output layer
  for (int l = 0; l <= x->L; ++l) {
    const int d[2][3] = {{n[0].lay[l].fan_in, n[0].lay[l].fan_out, x->B},
                         {n[1].lay[l].fan_in, n[1].lay[l].fan_out, x->B}};
    consider(2, d, x->bf16);
  }
  {
    const int d[2][3] = {{x->B, x->D, x->H}, {x->B, x->D, x->H}};
    consider(2, d, x->bf16);
  }
  if (!x->fused) {  // dphi = G psi and dpsi = G^T phi, single FP32 problems
    const int d[1][3] = {{x->B, x->D, x->B}};
    consider(1, d, false);
  }
  if (x->actor) {
    for (int l = 0; l <= n[2].L; ++l) {
      const int d[1][3] = {{n[2].lay[l].fan_in, n[2].lay[l].fan_out, x->B}};
      consider(1, d, x->bf16);
    }
    const int fo[1][3] = {{x->B, x->P, n[2].H}};
    consider(1, fo, x->bf16);
    const int da[1][3] = {{x->B, x->A, x->H}};  // action columns of phi's input gradient
    consider(1, da, x->bf16);
  }
  return need;
}

int64_t take_bytes(crl_ctx*, int64_t& off, int64_t bytes) {
  int64_t o = align_up(off, 256);
  off = o + (bytes > 0 ? bytes : 1);
  return o;
}

void plan_slots(crl_ctx* x, int e, int64_t (*take)(crl_ctx*, int64_t&, int64_t), int64_t& off) {
  const Net& N = x->net[e];
  Slots& S = x->sl[e];
  const int64_t B = x->B, H = N.H, O = N.out_dim, es = x->esz;
  S.Z.assign(N.L, -1);
  S.Hh.assign(N.L, -1);
  S.mu.assign(N.L, -1);
  S.rstd.assign(N.L, -1);
  for (int l = 0; l < N.L; ++l) {
    if (x->ln) {
      S.Z[l] = take(x, off, B * H * es);
      S.mu[l] = take(x, off, B * 4);
      S.rstd[l] = take(x, off, B * 4);
    }
    S.Hh[l] = take(x, off, B * H * es);
  }
  S.out = take(x, off, B * O * 4);
  S.dout = take(x, off, B * O * 4);
  S.dout_t = x->bf16 ? take(x, off, B * O * es) : S.dout;  // FP32: the same buffer
  S.dH = take(x, off, B * H * es);
  S.dZ[0] = take(x, off, B * H * es);
  S.dZ[1] = take(x, off, B * H * es);
}

// dX = dZ . W^T of layer l > 0 for the nets of a group: shapes and split plan
// (no split: the launch has no partial buffer)
GemmParams dx_params(const crl_ctx* x, const Group& G, int l) {
  GemmParams P{};
  P.count = G.count;
  for (int e = 0; e < G.count; ++e) {
    const LayerOff& lo = x->net[G.nets[e]].lay[l];
    GemmDesc& d = P.d[e];
    d.M = x->B; d.N = lo.fan_in; d.K = lo.fan_out;
    d.lda = d.ldb = lo.fan_out;
    d.ldc = lo.fan_in;
    d.alpha = 1.f;
    d.epi = x->ln ? EPI_NONE : EPI_MASK_POS;
  }
  plan_split_k(P, x->bf16, 512);
  return P;
}

// dW = in^T . dZ of layer l for the nets of a group: shapes and split plan
// (the same function plans the workspace and the launch)
GemmParams dw_params(const crl_ctx* x, const Group& G, int l) {
  GemmParams P{};
  P.count = G.count;
  for (int e = 0; e < G.count; ++e) {
    const Net& N = x->net[G.nets[e]];
    const LayerOff& lo = N.lay[l];
    P.d[e].M = lo.fan_in;
    P.d[e].N = lo.fan_out;
    P.d[e].K = x->B;
    P.d[e].lda = l == 0 ? N.ld_in : N.H;
    P.d[e].ldb = P.d[e].ldc = lo.fan_out;
  }
  // Each split's partial (a full M x N block) is written out and read back by
  // the reduction, so splits stay at least 8 steps deep and there are no more
  // than the launch needs.  Alone, dW fills the 512 resident workgroups (two
  // per CU).  In one launch with its layer's dX (launch_gemm_dw_dx) the launch
  // takes about (total 64-deep steps) / 512 steps, and dW is split only until
  // one split is no deeper than that, and than 64 steps (deeper splits leave
  // the end of the launch to a few long work items).
  P.partial = reinterpret_cast<float*>(1);
  int target = 512;
  if (l > 0) {
    GemmParams P1 = P;
    plan_split_k(P1, x->bf16, 0, 8);  // unsplit: the tile counts
    const GemmParams Px = dx_params(x, G, l);
    if (gemm_pair_ok(P1, Px, x->bf16)) {
      int64_t tiles = 0, work = 0;
      for (int e = 0; e < G.count; ++e) {
        tiles += P1.tiles[e];
        work += (int64_t)Px.tiles[e] * (Px.d[e].K / 64);
      }
      const int64_t ksteps = x->B / 64;
      work += tiles * ksteps;
      const int64_t span = (work + 511) / 512;
      int64_t sp = 1;
      while ((ksteps / sp > span || ksteps / sp > 64) && ksteps / (2 * sp) >= 8) sp *= 2;
      target = (int)(tiles * sp);
    }
  }
  plan_split_k(P, x->bf16, target, 8);
  P.partial = nullptr;
  return P;
}

// Whether layer l's dW runs in one launch with its dX (launch_gemm_dw_dx).
// The dW split-K partials are then in the 128-wide fragment order, also where
// dW alone would take 64-wide tiles (N <= 64: the output layer).  Shapes
// decide it; the workspace and every operand are 16-byte aligned.
bool dw_dx_paired(const crl_ctx* x, const Group& G, int l) {
  if (l == 0) return false;
  GemmParams Pw = dw_params(x, G, l);
  Pw.defer_reduce = Pw.splits > 1;
  return gemm_pair_ok(Pw, dx_params(x, G, l), x->bf16);
}

// Partial buffers of a group's backward and the jobs that reduce them into
// the gradient vector: dW split-K partials, bias column partials (output
// layer, and ReLU hidden layers), LayerNorm column partials (dg, db_ln, db).
void plan_group(crl_ctx* x, int gi, int64_t& off) {
  Group& G = x->grp[gi];
  const int64_t B = x->B;
  const int L = x->net[G.nets[0]].L;
  const int nrb = colsum_chunks(x->B);
  G.dwp.assign(L + 1, -1);
  G.dwu.assign(L + 1, -1);
  G.dwbn.assign(L + 1, 0);
  std::vector<RedJob> unsplit;  // dW blocks that the GEMM writes whole
  G.few.clear();
  G.many.clear();
  auto add = [](std::vector<RedJob>& v, int64_t src, int64_t stride, int64_t dst, int nparts,
                int n) {
    RedJob j{};
    j.src = src; j.stride = stride; j.dst = dst; j.nparts = nparts; j.n = n;
    v.push_back(j);
  };
  for (int e = 0; e < G.count; ++e) {
    Slots& S = x->sl[G.nets[e]];
    S.lnp.assign(L, -1);
    S.bp.assign(L + 1, -1);
  }
  for (int l = 0; l <= L; ++l) {
    const GemmParams P = dw_params(x, G, l);
    if (P.splits > 1) {
      // partial layout of the kernel that will run: fragment order on the
      // direct-to-LDS kernel, dense otherwise
      const int bn = dw_dx_paired(x, G, l) ? 128 : gemm_lds_bn(P, x->bf16);
      int64_t ps = 0;
      for (int e = 0; e < G.count; ++e) ps = std::max(ps, frag_partial_floats(P, e, bn));
      G.dwbn[l] = bn;
      G.dwp[l] = take_bytes(x, off, (int64_t)G.count * P.splits * ps * 4);
      for (int e = 0; e < G.count; ++e) {
        RedJob j{};
        j.src = G.dwp[l] + (int64_t)e * P.splits * ps * 4;
        j.stride = frag_partial_floats(P, e, bn);
        j.dst = x->net[G.nets[e]].lay[l].w;
        j.nparts = P.splits;
        j.n = (int32_t)j.stride;
        j.M = P.d[e].M; j.N = P.d[e].N; j.tiles_n = P.tiles_n[e]; j.bn = bn;
        G.few.push_back(j);
      }
    } else {
      // the Adam epilogue needs every element in a job: the unsplit dW is
      // written to the workspace and taken as a one-part job
      int64_t mn = 0;
      for (int e = 0; e < G.count; ++e) mn = std::max(mn, (int64_t)P.d[e].M * P.d[e].N);
      G.dwu[l] = take_bytes(x, off, (int64_t)G.count * mn * 4);
      for (int e = 0; e < G.count; ++e) {
        RedJob j{};
        j.src = G.dwu[l] + (int64_t)e * mn * 4;
        j.stride = (int64_t)P.d[e].M * P.d[e].N;
        j.dst = x->net[G.nets[e]].lay[l].w;
        j.nparts = 1;
        j.n = (int32_t)j.stride;
        j.M = P.d[e].M; j.N = P.d[e].N; j.tiles_n = 0; j.bn = 0;
        unsplit.push_back(j);
      }
    }
    const bool top = l == L;
    for (int e = 0; e < G.count; ++e) {
      const Net& N = x->net[G.nets[e]];
      Slots& S = x->sl[G.nets[e]];
      const LayerOff& lo = N.lay[l];
      if (top || !x->ln) {
        // the critic's output-layer partials come from the fused InfoNCE
        // backward reduction (blocks of 256 / D rows), the others from the
        // column sums
        const int np = (top && gi == 0 && x->fused) ? fused_bias_chunks(x->B, lo.fan_out) : nrb;
        S.bp[l] = take_bytes(x, off, (int64_t)np * lo.fan_out * 4);
        add(G.many, S.bp[l], lo.fan_out, lo.b, np, lo.fan_out);
      }
      if (!top && x->ln) {
        const int H = N.H;
        S.lnp[l] = take_bytes(x, off, (int64_t)x->ln_nparts * 3 * H * 4);
        const int64_t dst[3] = {lo.g, lo.be, lo.b};
        for (int k = 0; k < 3; ++k)
          add(G.many, S.lnp[l] + (int64_t)k * H * 4, 3 * H, dst[k], x->ln_nparts, H);
      }
    }
  }
  // the padding between the vector's tensors: written as zeros
  const std::vector<int64_t>& gaps = x->gaps[gi];
  for (size_t k = 0; k + 1 < gaps.size(); k += 2) add(G.many, 0, 0, gaps[k], 0, (int)gaps[k + 1]);
  G.total4 = 0;
  G.few_bytes = 0;
  G.nfew_plain = (int)G.few.size();
  for (const RedJob& j : unsplit) G.few.push_back(j);
  G.chunks = 0;
  for (size_t k = 0; k < G.few.size(); ++k) {
    RedJob& j = G.few[k];
    if ((int)k == G.nfew_plain) G.total4_plain = G.total4;
    j.first = G.total4;
    G.total4 += j.n / 4;
    // fragment-order jobs are whole tiles: whole chunks
    j.first_chunk = G.chunks;
    G.chunks += (j.n / 4 + kRedChunk4 - 1) / kRedChunk4;
    if ((int)k < G.nfew_plain) G.few_bytes += 4.0 * j.M * j.N * (j.nparts + 1.0);
  }
  if (G.nfew_plain == (int)G.few.size()) G.total4_plain = G.total4;
  G.nblocks = 0;
  G.many_bytes = 0;
  for (RedJob& j : G.many) {
    j.first = G.nblocks;
    G.nblocks += (j.n + kManyCols - 1) / kManyCols;
    G.many_bytes += 4.0 * j.n * (j.nparts + 1.0);
  }
  (void)B;
}

void plan_workspace(crl_ctx* x) {
  int64_t off = 0;
  auto take = [&](int64_t bytes) { return take_bytes(x, off, bytes); };
  const int64_t B = x->B, D = x->D;
  x->ln_rows_per_wave = 16;
  x->ln_nparts = ln_bwd_partials(x->B, x->ln_rows_per_wave);
  for (int e = 0; e < (x->actor ? 3 : 2); ++e) plan_slots(x, e, take_bytes, off);
  x->grp[0].nets[0] = 0; x->grp[0].nets[1] = 1; x->grp[0].count = 2;
  x->grp[1].nets[0] = 2; x->grp[1].nets[1] = 2; x->grp[1].count = 1;
  for (int gi = 0; gi < (x->actor ? 2 : 1); ++gi) plan_group(x, gi, off);
  x->splitk_floats = splitk_need(x);
  x->splitk = take(x->splitk_floats * 4);
  x->r = take(B * 4);
  x->c = take(B * 4);
  x->diag = take(B * 4);
  x->nphi = take(B * 4);
  x->npsi = take(B * 4);
  x->rowterm = take(B * 4);
  x->rowaux = take(B * 4);
  x->uphi = x->upsi = -1;
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
    if (x->energy == CRL_ENERGY_COS) {
      x->uphi = take(B * D * 4);
      x->upsi = take(B * D * 4);
    }
  } else {
    // the one-pass backward (D = 64) indexes its partials by 256-row blocks
    const int S = fused_bwd_one_pass(x->B, x->D)
                      ? std::max(fused_splits(x->B), fused_bwd_splits(x->B))
                      : fused_splits(x->B);
    const int nrb = (x->B + 63) / 64;
    x->phi_b = take(B * D * 2);
    x->psi_b = take(B * D * 2);
    x->row_m = take((int64_t)S * B * 4);
    x->row_s = take((int64_t)S * B * 4);
    x->col_m = take((int64_t)nrb * B * 4);
    x->col_s = take((int64_t)nrb * B * 4);
    x->dx_part = take((int64_t)2 * S * B * D * 4);
    x->rs_part = take((int64_t)2 * S * B * 4);
  }
  x->xsa2 = x->noise = x->logpi = x->fpol = x->dact = -1;
  x->xg_mix = x->xsg_mix = -1;
  x->mix_thr = 0;
  x->ldd = 0;
  if (x->actor) {
    x->ldd = (int)align_up(x->A, 8);
    x->xsa2 = take(B * x->net[0].ld_in * x->esz);
    x->noise = take(B * x->A * 4);
    x->logpi = take(B * 4);
    x->fpol = take(B * 4);
    x->dact = take(B * x->ldd * 4);
    // r * 2^53 is exact in double (a power-of-two scaling of r <= 1)
    x->mix_thr = (uint64_t)std::floor(x->cfg.random_goal_ratio * 9007199254740992.0);
    if (x->mix_thr > 0) {
      x->xg_mix = take(B * x->net[1].ld_in * x->esz);
      x->xsg_mix = take(B * x->ld_sg * x->esz);
    }
  }
  x->ws_bytes = align_up(off, 256);

  // The loss forward alone, packed from offset 0: the layout
  // crl_infonce_fwd_noalloc uses inside the static scratch array.
  int64_t so = 0;
  auto st = [&](int64_t bytes) { return take_bytes(x, so, bytes); };
  LossWs& n = x->na;
  n.r = st(B * 4); n.c = st(B * 4); n.diag = st(B * 4);
  n.nphi = st(B * 4); n.npsi = st(B * 4);
  n.rowterm = st(B * 4); n.rowaux = st(B * 4);
  n.uphi = n.upsi = n.logits = n.cpm = n.cps = -1;
  n.phi_b = n.psi_b = n.row_m = n.row_s = n.col_m = n.col_s = -1;
  if (!x->fused) {
    n.logits = st(B * x->ldF * 4);
    n.cpm = st((int64_t)x->rchunks * B * 4);
    n.cps = st((int64_t)x->rchunks * B * 4);
    if (x->energy == CRL_ENERGY_COS) { n.uphi = st(B * D * 4); n.upsi = st(B * D * 4); }
  } else {
    const int S = fused_splits(x->B);  // bounds the forward's split count
    const int nrb = (x->B + 63) / 64;
    n.phi_b = st(B * D * 2); n.psi_b = st(B * D * 2);
    n.row_m = st((int64_t)S * B * 4); n.row_s = st((int64_t)S * B * 4);
    n.col_m = st((int64_t)nrb * B * 4); n.col_s = st((int64_t)nrb * B * 4);
  }
  x->na_bytes = align_up(so, 256);
}

// The same offsets inside the context's own workspace.
LossWs loss_ws(const crl_ctx* x) {
  LossWs o;
  o.r = x->r; o.c = x->c; o.diag = x->diag; o.nphi = x->nphi; o.npsi = x->npsi;
  o.rowterm = x->rowterm; o.rowaux = x->rowaux; o.uphi = x->uphi; o.upsi = x->upsi;
  o.logits = x->logits; o.cpm = x->cpm; o.cps = x->cps;
  o.phi_b = x->phi_b; o.psi_b = x->psi_b; o.row_m = x->row_m; o.row_s = x->row_s;
  o.col_m = x->col_m; o.col_s = x->col_s;
  return o;
}

// Adam hyperparameters for the device: 1 - b and log b formed in double
AdamCoef adam_coef(double lr, double b1, double b2, double eps) {
  AdamCoef c;
  c.lr = (float)lr;
  c.b1 = (float)b1;
  c.b2 = (float)b2;
  c.omb1 = (float)(1.0 - b1);
  c.omb2 = (float)(1.0 - b2);
  c.log_b1 = (float)std::log(b1);
  c.log_b2 = (float)std::log(b2);
  c.eps = (float)eps;
  return c;
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

// One MLP taking part in a forward or backward pass.
struct NetCall {
  int net;                 // 0 phi, 1 psi, 2 policy
  const void* x;           // layer-0 input [B][ld] (storage type)
  int ld;
  const float* p;          // FP32 flat vector the net lives in
  const bf16_t* pb;        // its BF16 shadow (BF16 precision)
  float* g;                // gradient vector, or nullptr: no parameter gradients
  float* dx;               // optional FP32 gradient of input columns [dx_c0, dx_c0 + dx_n)
  int dx_c0, dx_n, ldd;
};

const void* weights(const crl_ctx* x, const NetCall& c, int64_t off) {
  return x->bf16 ? (const void*)(c.pb + off) : (const void*)(c.p + off);
}

// Forward of `count` MLPs with the same depth and width, layer by layer in
// grouped launches: GEMM (bias, and ReLU, in the epilogue), then LayerNorm +
// Swish.  Outputs and the activations the backward needs stay in ws.
// top_deferred: the output layer's split-K partials are left unreduced and
// its launch parameters returned (splits == 1 there: nothing deferred).
int mlp_forward(crl_ctx* x, const NetCall* nc, int count, void* ws, hipStream_t s,
                GemmParams* top_deferred = nullptr) {
  const Net& N0 = x->net[nc[0].net];
  const int B = x->B;
  for (int l = 0; l <= N0.L; ++l) {
    const bool top = l == N0.L;
    GemmParams P{};
    P.count = count;
    for (int e = 0; e < count; ++e) {
      const Net& N = x->net[nc[e].net];
      const Slots& S = x->sl[nc[e].net];
      const LayerOff& lo = N.lay[l];
      GemmDesc& d = P.d[e];
      d.A = l == 0 ? nc[e].x : (const void*)W(ws, S.Hh[l - 1]);
      d.lda = l == 0 ? nc[e].ld : N.H;
      d.B = weights(x, nc[e], lo.w);
      d.ldb = lo.fan_out;
      d.M = B; d.N = lo.fan_out; d.K = lo.fan_in;
      if (l == 0 && x->bf16) {  // zero input columns up to the padded stride
        d.K = (int)align_up(lo.fan_in, 64);
        d.kb = lo.fan_in;
      }
      d.bias = nc[e].p + lo.b;
      d.alpha = 1.f;
      if (top) { d.C = W(ws, S.out); d.epi = EPI_BIAS; }
      else if (!x->ln) { d.C = W(ws, S.Hh[l]); d.epi = EPI_BIAS_RELU; }
      else { d.C = W(ws, S.Z[l]); d.epi = EPI_BIAS; }
      d.ldc = lo.fan_out;
    }
    if (top) P.partial = WF(ws, x->splitk);  // few output tiles: split K
    plan_split_k(P, x->bf16, 512);
    if (P.splits > 1)
      P.partial_len = (int64_t)P.splits * std::max((int64_t)P.d[0].M * P.d[0].N,
                                                   (int64_t)P.d[count - 1].M * P.d[count - 1].N);
    if (top && top_deferred) {
      P.defer_reduce = P.splits > 1;
      *top_deferred = P;
    }
    CRL_HIP(launch_gemm(P, x->bf16, LAY_KC, LAY_MC, x->bf16 && !top, s), "encoder GEMM");
    if (!top && x->ln) {
      LnArgs a{};
      for (int e = 0; e < count; ++e) {
        const Slots& S = x->sl[nc[e].net];
        const LayerOff& lo = x->net[nc[e].net].lay[l];
        a.Z[e] = W(ws, S.Z[l]);
        a.H[e] = W(ws, S.Hh[l]);
        a.mu[e] = WF(ws, S.mu[l]);
        a.rstd[e] = WF(ws, S.rstd[l]);
        a.g[e] = nc[e].p + lo.g;
        a.b[e] = nc[e].p + lo.be;
      }
      CRL_HIP(launch_ln_swish_fwd(a, count, B, N0.H, x->cfg.ln_eps, x->bf16, s), "LayerNorm forward");
    }
  }
  return CRL_OK;
}

// Backward of `count` MLPs from the output gradients in their dout / dout_t
// slots, last layer first.  With a gradient vector: dW, bias and LayerNorm
// parameter gradients of every layer.  A net with dx set (count must be 1)
// also gets the gradient of the chosen input columns.
int mlp_backward(crl_ctx* x, const NetCall* nc, int count, void* ws, hipStream_t s,
                 bool top_bias_ready = false, const AdamArgs* adam = nullptr) {
  const Net& N0 = x->net[nc[0].net];
  const int B = x->B, H = N0.H, L = N0.L;
  // adam: the parameter gradients go into the Adam step of the vector as
  // they are reduced (nc[0].g, if not NULL, receives them too)
  const bool grads = nc[0].g != nullptr || adam != nullptr;
  const Group& G = x->grp[nc[0].net == 2 ? 1 : 0];
  if (grads && G.count != count) return fail(CRL_EINVAL, "internal: backward group mismatch");
  float* splitk = WF(ws, x->splitk);
  int cur = 0;
  for (int l = L; l >= 0; --l) {
    const bool top = l == L;
    const void* dZ[2];
    for (int e = 0; e < count; ++e) {
      const Slots& S = x->sl[nc[e].net];
      dZ[e] = top ? (const void*)W(ws, S.dout_t) : (const void*)W(ws, S.dZ[cur]);
    }
    // dZ of layer l-1 (l > 0): dH = dZ . W^T, then through ReLU or Swish(LayerNorm)
    const int nxt = top ? 0 : (cur ^ 1);
    GemmParams Px{};
    if (l > 0) {
      Px.count = count;
      for (int e = 0; e < count; ++e) {
        const Slots& S = x->sl[nc[e].net];
        const LayerOff& lo = x->net[nc[e].net].lay[l];
        GemmDesc& d = Px.d[e];
        d.A = dZ[e]; d.lda = lo.fan_out;
        d.B = weights(x, nc[e], lo.w);
        d.ldb = lo.fan_out;
        d.M = B; d.N = lo.fan_in; d.K = lo.fan_out;
        d.alpha = 1.f;
        d.ldc = lo.fan_in;
        if (x->ln) { d.C = W(ws, S.dH); d.epi = EPI_NONE; }
        else { d.C = W(ws, S.dZ[nxt]); d.epi = EPI_MASK_POS; d.aux = W(ws, S.Hh[l - 1]); }
      }
      plan_split_k(Px, x->bf16, 512);
    }
    // dW = in^T . dZ (contraction over the batch); split-K partials are
    // reduced once, after the last layer
    GemmParams Pw{};
    bool paired = false;
    if (grads) {
      Pw = dw_params(x, G, l);
      for (int e = 0; e < count; ++e) {
        const Net& N = x->net[nc[e].net];
        const Slots& S = x->sl[nc[e].net];
        const LayerOff& lo = N.lay[l];
        GemmDesc& d = Pw.d[e];
        d.A = l == 0 ? nc[e].x : (const void*)W(ws, S.Hh[l - 1]);
        d.lda = l == 0 ? nc[e].ld : N.H;
        d.B = dZ[e]; d.ldb = lo.fan_out;
        d.ldc = lo.fan_out;
        d.alpha = 1.f;
        d.epi = EPI_NONE;
        if (G.dwu[l] >= 0 && (adam || !nc[e].g)) {  // unsplit: a one-part reduction job
          const GemmDesc& d0 = Pw.d[0];
          const GemmDesc& d1 = Pw.d[count - 1];
          const int64_t mn = std::max((int64_t)d0.M * d0.N, (int64_t)d1.M * d1.N);
          d.C = WF(ws, G.dwu[l]) + (int64_t)e * mn;
        } else {
          d.C = nc[e].g ? nc[e].g + lo.w : WF(ws, G.dwp[l]);  // split: C is not written
        }
      }
      Pw.defer_reduce = Pw.splits > 1;
      paired = dw_dx_paired(x, G, l);
      if (paired != (l > 0 && gemm_pair_ok(Pw, Px, x->bf16)))
        return fail(CRL_EINVAL, "internal: dW + dX launch plan mismatch");
      if (Pw.splits > 1) {
        const int bn = paired ? 128 : gemm_lds_bn(Pw, x->bf16);
        if (bn != G.dwbn[l]) return fail(CRL_EINVAL, "internal: dW partial layout mismatch");
        int64_t ps = 0;
        for (int e = 0; e < count; ++e) ps = std::max(ps, frag_partial_floats(Pw, e, bn));
        Pw.partial = WF(ws, G.dwp[l]);
        Pw.partial_len = (int64_t)Pw.splits * ps;
        Pw.frag = 1;
      }
      // bias column partials of this layer (LayerNorm layers get theirs with dZ;
      // top_bias_ready: the output layer's were written with dout)
      if ((top && !top_bias_ready) || (!top && !x->ln)) {
        ColSumArgs ca{};
        for (int e = 0; e < count; ++e) {
          const Slots& S = x->sl[nc[e].net];
          ca.X[e] = top ? (const void*)WF(ws, S.dout) : dZ[e];
          ca.part[e] = WF(ws, S.bp[l]);
        }
        const int Nc = top ? N0.out_dim : H;
        CRL_HIP(launch_colsum_partials(ca, count, B, Nc, Nc, top ? false : x->bf16, s),
                "bias gradient");
      }
    }
    if (paired) {
      // both products read dZ; one launch, the dW work items first
      CRL_HIP(launch_gemm_dw_dx(Pw, Px, s), "dW + dX GEMM");
    } else if (grads) {
      CRL_HIP(launch_gemm(Pw, x->bf16, LAY_MC, LAY_MC, false, s), "dW GEMM");
    }
    if (l == 0) {
      if (nc[0].dx) {  // dx[:, j] = dZ . W[c0 + j, :]^T for the requested input columns
        const LayerOff& lo = N0.lay[0];
        GemmParams P{};
        P.count = 1;
        GemmDesc& d = P.d[0];
        d.A = dZ[0]; d.lda = lo.fan_out;
        d.B = weights(x, nc[0], lo.w + (int64_t)nc[0].dx_c0 * lo.fan_out);
        d.ldb = lo.fan_out;
        d.M = B; d.N = nc[0].dx_n; d.K = lo.fan_out;
        d.C = nc[0].dx; d.ldc = nc[0].ldd;
        d.alpha = 1.f;
        d.epi = EPI_NONE;
        P.partial = splitk;
        plan_split_k(P, x->bf16, 512);
        P.partial_len = (int64_t)P.splits * d.M * d.N;
        CRL_HIP(launch_gemm(P, x->bf16, LAY_KC, LAY_KC, false, s), "input gradient GEMM");
      }
      break;
    }
    if (!paired) CRL_HIP(launch_gemm(Px, x->bf16, LAY_KC, LAY_KC, x->bf16, s), "dX GEMM");
    if (x->ln) {  // column partials of dg, db_ln, db go to the layer's own region
      LnArgs a{};
      for (int e = 0; e < count; ++e) {
        const Slots& S = x->sl[nc[e].net];
        const LayerOff& lp = x->net[nc[e].net].lay[l - 1];
        a.Z[e] = W(ws, S.Z[l - 1]);
        a.mu[e] = WF(ws, S.mu[l - 1]);
        a.rstd[e] = WF(ws, S.rstd[l - 1]);
        a.g[e] = nc[e].p + lp.g;
        a.b[e] = nc[e].p + lp.be;
        a.dH[e] = W(ws, S.dH);
        a.dZ[e] = W(ws, S.dZ[nxt]);
        a.part[e] = WF(ws, S.lnp[l - 1]);
      }
      CRL_HIP(launch_ln_swish_bwd(a, count, B, H, x->bf16, x->ln_rows_per_wave, s), "LayerNorm backward");
    }
    cur = nxt;
  }
  if (grads) {
    const char* wsc = static_cast<const char*>(ws);
    if (adam) {
      // every element of the vector (unsplit dW blocks included) is reduced
      // once, then stepped: the gradient read, the parameter, m, v read and written
      double bytes = G.few_bytes + G.many_bytes;
      for (size_t k = G.nfew_plain; k < G.few.size(); ++k) bytes += 8.0 * G.few[k].n;
      const int64_t n = nc[0].net == 2 ? x->nparam_actor : x->nparam;
      bytes += (24.0 + (adam->pb ? 2.0 : 0.0)) * n - (nc[0].g ? 0.0 : 4.0 * n);
      CRL_HIP(launch_grad_reduce(wsc, nc[0].g, G.d_few, (int)G.few.size(), G.chunks, G.d_many,
                                 (int)G.many.size(), G.nblocks, bytes, s, adam),
              "gradient reductions with the Adam step");
    } else {
      CRL_HIP(launch_grad_reduce(wsc, nc[0].g, G.d_few, G.nfew_plain, G.total4_plain, G.d_many,
                                 (int)G.many.size(), G.nblocks, G.few_bytes + G.many_bytes, s),
              "gradient reductions");
    }
  }
  return CRL_OK;
}

// The critic matrix of phi and psi (FP32 [B][D]), its row and column
// log-sum-exps and diagonal, and the loss parts, for the context's energy and
// objective, with its buffers at the offsets o inside ws.  top (fused logits): the output layer's deferred split-K launch,
// whose sum the prep kernel takes (phi and psi are then its outputs).
// advance (may be NULL): a step counter that the loss kernel advances by one.
int contrastive_fwd(crl_ctx* x, const float* phi, const float* psi, void* ws, const LossWs& o,
                    float* loss_out, const GemmParams* top, hipStream_t s,
                    int64_t* advance = nullptr) {
  const int B = x->B, D = x->D;
  float* r = WF(ws, o.r);
  float* c = WF(ws, o.c);
  float* dg = WF(ws, o.diag);
  float* term = WF(ws, o.rowterm);
  if (!x->fused) {
    float* F = WF(ws, o.logits);
    if (x->energy == CRL_ENERGY_L1) {
      CRL_HIP(launch_l1_energy(phi, psi, F, B, D, x->ldF, s), "L1 energy");
    } else {
      GemmParams P{};
      P.count = 1;
      GemmDesc& d = P.d[0];
      d.A = phi; d.lda = D;
      d.B = psi; d.ldb = D;
      d.C = F; d.ldc = x->ldF;
      d.M = B; d.N = B; d.K = D;
      d.alpha = 1.f;
      d.epi = EPI_NONE;
      if (x->energy == CRL_ENERGY_COS) {
        CRL_HIP(launch_unit_rows(phi, WF(ws, o.uphi), WF(ws, o.nphi), B, D, s), "unit rows");
        CRL_HIP(launch_unit_rows(psi, WF(ws, o.upsi), WF(ws, o.npsi), B, D, s), "unit rows");
        d.A = WF(ws, o.uphi);
        d.B = WF(ws, o.upsi);
      } else if (x->energy == CRL_ENERGY_L2 || x->energy == CRL_ENERGY_L2SQ) {
        CRL_HIP(launch_sqnorm(phi, WF(ws, o.nphi), B, D, s), "norms");
        CRL_HIP(launch_sqnorm(psi, WF(ws, o.npsi), B, D, s), "norms");
        d.epi = x->energy == CRL_ENERGY_L2 ? EPI_L2 : EPI_L2SQ;
        d.rowv = WF(ws, o.nphi);
        d.colv = WF(ws, o.npsi);
      }
      plan_split_k(P, false, 512);
      CRL_HIP(launch_gemm(P, false, LAY_KC, LAY_KC, false, s), "logits GEMM");
    }
    CRL_HIP(launch_row_obj(F, B, x->ldF, x->loss, r, dg, term, WF(ws, o.rowaux), s),
            "row log-sum-exp and objective terms");
    const int rc_ = std::min(x->rchunks, B);
    CRL_HIP(launch_col_lse_partial(F, B, x->ldF, rc_, WF(ws, o.cpm), WF(ws, o.cps), s), "column LSE");
    CRL_HIP(launch_lse_merge(WF(ws, o.cpm), WF(ws, o.cps), rc_, B, c, s), "column LSE merge");
  } else {
    FusedArgs a{};
    a.phi = phi; a.psi = psi;
    a.phi_b = reinterpret_cast<bf16_t*>(W(ws, o.phi_b));
    a.psi_b = reinterpret_cast<bf16_t*>(W(ws, o.psi_b));
    a.nphi = WF(ws, o.nphi); a.npsi = WF(ws, o.npsi);
    a.row_m = WF(ws, o.row_m); a.row_s = WF(ws, o.row_s);
    a.col_m = WF(ws, o.col_m); a.col_s = WF(ws, o.col_s);
    a.r = r; a.c = c; a.diag = dg;
    CRL_HIP(launch_fused_fwd(a, B, D, x->energy, (top && top->splits > 1) ? top : nullptr, s),
            "fused InfoNCE forward");
  }
  CRL_HIP(launch_loss(r, c, dg, term, B, x->loss, x->cfg.logsumexp_penalty, loss_out, advance, s),
          "loss");
  return CRL_OK;
}

// dL/dphi and dL/dpsi (FP32) after contrastive_fwd on the same phi, psi and
// ws; dphi_t / dpsi_t get storage-type copies (BF16 precision; FP32: they
// must be dphi / dpsi themselves); bias: the fused reduction also writes the
// critic output layer's bias partials.
int contrastive_bwd(crl_ctx* x, const float* phi, const float* psi, void* ws, float* dphi,
                    float* dpsi, void* dphi_t, void* dpsi_t, bool bias, hipStream_t s) {
  const int B = x->B, D = x->D;
  const float beta = x->cfg.logsumexp_penalty;
  const float* r = WF(ws, x->r);
  const float* c = WF(ws, x->c);
  if (!x->fused) {
    float* F = WF(ws, x->logits);
    float* rsH = WF(ws, x->rowsumH);
    const bool dist = x->energy == CRL_ENERGY_L2 || x->energy == CRL_ENERGY_L2SQ;
    const bool cosine = x->energy == CRL_ENERGY_COS;
    CRL_HIP(launch_grad_obj(F, B, x->ldF, r, c, WF(ws, x->diag), WF(ws, x->rowaux), x->loss,
                            x->energy, beta, rsH, s), "objective gradient");
    if (x->energy == CRL_ENERGY_L1) {
      CRL_HIP(launch_l1_backward(phi, psi, F, x->ldF, 0, dphi, B, D, s), "L1 backward");
      CRL_HIP(launch_l1_backward(psi, phi, F, x->ldF, 1, dpsi, B, D, s), "L1 backward");
    } else {
      float* splitk = WF(ws, x->splitk);
      for (int side = 0; side < 2; ++side) {
        // side 0: dphi = G psi (G as KC); side 1: dpsi = G^T phi (G as MC);
        // the unit rows stand in for phi and psi with the cosine energy
        const float* Y = side == 0 ? (cosine ? WF(ws, x->upsi) : psi)
                                   : (cosine ? WF(ws, x->uphi) : phi);
        GemmParams P{};
        P.count = 1;
        GemmDesc& d = P.d[0];
        d.A = F; d.lda = x->ldF;
        d.B = Y; d.ldb = D;
        d.C = side == 0 ? dphi : dpsi; d.ldc = D;
        d.M = B; d.N = D; d.K = B;
        d.alpha = 1.f;
        d.epi = EPI_NONE;
        P.partial = splitk;
        plan_split_k(P, false, 512);
        P.partial_len = (int64_t)P.splits * B * D;
        CRL_HIP(launch_gemm(P, false, side == 0 ? LAY_KC : LAY_MC, LAY_MC, false, s), "dphi/dpsi GEMM");
      }
      if (dist) {
        CRL_HIP(launch_l2_fix(dphi, phi, rsH, B, D, s), "distance row term");
        ColSumArgs ca{};
        ca.X[0] = F; ca.out[0] = WF(ws, x->colsumH); ca.part[0] = WF(ws, x->cpartB);
        CRL_HIP(launch_colsum(ca, 1, B, B, x->ldF, false, s), "distance column sums");
        CRL_HIP(launch_l2_fix(dpsi, psi, WF(ws, x->colsumH), B, D, s), "distance column term");
      }
      if (cosine) {
        CRL_HIP(launch_cos_fix(dphi, WF(ws, x->uphi), WF(ws, x->nphi), B, D, s), "cosine backward");
        CRL_HIP(launch_cos_fix(dpsi, WF(ws, x->upsi), WF(ws, x->npsi), B, D, s), "cosine backward");
      }
    }
    if (x->bf16) {
      CRL_HIP(launch_cast_bf16(dphi, reinterpret_cast<bf16_t*>(dphi_t), (int64_t)B * D, s), "cast");
      CRL_HIP(launch_cast_bf16(dpsi, reinterpret_cast<bf16_t*>(dpsi_t), (int64_t)B * D, s), "cast");
    }
  } else {
    FusedArgs a{};
    a.phi = phi; a.psi = psi;
    a.phi_b = reinterpret_cast<bf16_t*>(W(ws, x->phi_b));
    a.psi_b = reinterpret_cast<bf16_t*>(W(ws, x->psi_b));
    a.nphi = WF(ws, x->nphi); a.npsi = WF(ws, x->npsi);
    a.r = const_cast<float*>(r); a.c = const_cast<float*>(c);
    a.dX_part = WF(ws, x->dx_part);
    a.rs_part = WF(ws, x->rs_part);
    a.dphi = dphi; a.dpsi = dpsi;
    a.dphi_t = dphi_t;
    a.dpsi_t = dpsi_t;
    a.bias_part[0] = bias ? WF(ws, x->sl[0].bp[x->L]) : nullptr;
    a.bias_part[1] = bias ? WF(ws, x->sl[1].bp[x->L]) : nullptr;
    CRL_HIP(launch_fused_bwd(a, B, D, x->energy, x->loss, beta, x->bf16, s),
            "fused InfoNCE backward");
  }
  return CRL_OK;
}

int upload(void** dst, const void* src, size_t bytes) {
  *dst = nullptr;
  if (bytes == 0) return CRL_OK;
  hipError_t e = hipMalloc(dst, bytes);
  if (e == hipSuccess) e = hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (*dst) (void)hipFree(*dst);
    *dst = nullptr;
    return hip_fail(e, "crl_create device tables");
  }
  return CRL_OK;
}

void free_tables(crl_ctx* x) {
  if (x->d_thr) (void)hipFree(x->d_thr);
  for (int i = 0; i < 2; ++i) {
    if (x->grp[i].d_few) (void)hipFree(x->grp[i].d_few);
    if (x->grp[i].d_many) (void)hipFree(x->grp[i].d_many);
  }
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
  hipError_t he = hipGetDevice(&x->device);
  if (he != hipSuccess) { delete x; return hip_fail(he, "hipGetDevice"); }
  // the no-alloc entry point's scratch; without it only that entry point fails
  x->scratch_err = scratch_address(x->device, &x->scratch);
  if (x->scratch_err != hipSuccess) (void)hipGetLastError();
  x->bf16 = cfg->precision == CRL_PREC_BF16;
  x->ln = cfg->activation == CRL_ACT_LN_SWISH;
  x->energy = cfg->energy;
  x->loss = cfg->loss;
  x->fused = cfg->logits == CRL_LOGITS_FUSED;
  x->actor = cfg->actor_n_hidden > 0;
  x->B = cfg->batch;
  x->H = cfg->hidden;
  x->D = cfg->repr_dim;
  x->L = cfg->n_hidden;
  x->A = cfg->act_dim;
  // the policy head's width, padded to whole 64-deep K steps so that its
  // input gradient (K = P) runs on the direct-to-LDS GEMM, paired with its dW
  x->P = (int)align_up(2 * cfg->act_dim, 64);
  x->esz = x->bf16 ? 2 : 4;
  const int fan_in0[3] = {cfg->obs_dim + cfg->act_dim, cfg->goal_dim, cfg->obs_dim + cfg->goal_dim};
  for (int e = 0; e < 3; ++e) {
    Net& N = x->net[e];
    N.fan_in0 = fan_in0[e];
    // BF16 inputs are padded with zero columns to whole 64-deep K steps, so
    // the first layer runs on the direct-to-LDS GEMM too
    N.ld_in = (int)align_up(fan_in0[e], x->bf16 ? 64 : 8);
    N.H = e < 2 ? x->H : cfg->actor_hidden;
    N.L = e < 2 ? x->L : cfg->actor_n_hidden;
    N.out_dim = e < 2 ? x->D : x->P;
  }
  x->ld_sg = x->net[2].ld_in;
  x->nparam = plan_params(x, 0, 1, x->gaps[0]);
  x->nparam_actor = x->actor ? plan_params(x, 2, 2, x->gaps[1]) : 0;
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
  rc = upload(reinterpret_cast<void**>(&x->d_thr), thr.data(), nthr * sizeof(uint64_t));
  for (int i = 0; i < 2 && rc == CRL_OK; ++i) {
    Group& G = x->grp[i];
    rc = upload(reinterpret_cast<void**>(&G.d_few), G.few.data(), G.few.size() * sizeof(RedJob));
    if (rc == CRL_OK)
      rc = upload(reinterpret_cast<void**>(&G.d_many), G.many.data(), G.many.size() * sizeof(RedJob));
  }
  if (rc != CRL_OK) {
    free_tables(x);
    delete x;
    return rc;
  }
  *out = x;
  return CRL_OK;
}

CRL_API int crl_destroy(crl_ctx* x) {
  if (!x) return CRL_OK;
  free_tables(x);
  delete x;
  return CRL_OK;
}

CRL_API int crl_param_count(const crl_ctx* x, int64_t* n) {
  if (!x || !n) return fail(CRL_EINVAL, "NULL argument");
  *n = x->nparam;
  return CRL_OK;
}

CRL_API int crl_actor_param_count(const crl_ctx* x, int64_t* n) {
  if (!x || !n) return fail(CRL_EINVAL, "NULL argument");
  *n = x->nparam_actor;
  return CRL_OK;
}

CRL_API int crl_layer_layout(const crl_ctx* x, int32_t net, int32_t layer, crl_layer_info* out) {
  if (!x || !out) return fail(CRL_EINVAL, "NULL argument");
  if (net < 0 || net > 2) return fail(CRL_EINVAL, "net must be 0 (phi), 1 (psi) or 2 (policy)");
  if (net == 2 && !x->actor) return fail(CRL_EINVAL, "this context has no actor");
  const Net& N = x->net[net];
  if (layer < 0 || layer > N.L) return fail(CRL_EINVAL, "layer %d out of range [0, %d]", layer, N.L);
  const LayerOff& l = N.lay[layer];
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
  if (ld_sa) *ld_sa = x->net[0].ld_in;
  if (ld_g) *ld_g = x->net[1].ld_in;
  if (ld_sg) *ld_sg = x->ld_sg;
  if (elem_bytes) *elem_bytes = x->esz;
  return CRL_OK;
}

CRL_API int crl_workspace_view(const crl_ctx* x, int32_t which, int64_t* offset, int64_t* bytes) {
  if (!x || !offset || !bytes) return fail(CRL_EINVAL, "NULL argument");
  const int64_t B = x->B, D = x->D;
  if (which >= CRL_WS_POLICY_OUT && which <= CRL_WS_DACTION && !x->actor)
    return fail(CRL_EINVAL, "this context has no actor");
  switch (which) {
    case CRL_WS_PHI: *offset = x->sl[0].out; *bytes = B * D * 4; break;
    case CRL_WS_PSI: *offset = x->sl[1].out; *bytes = B * D * 4; break;
    case CRL_WS_ROW_LSE: *offset = x->r; *bytes = B * 4; break;
    case CRL_WS_COL_LSE: *offset = x->c; *bytes = B * 4; break;
    case CRL_WS_DIAG: *offset = x->diag; *bytes = B * 4; break;
    case CRL_WS_DPHI: *offset = x->sl[0].dout; *bytes = B * D * 4; break;
    case CRL_WS_DPSI: *offset = x->sl[1].dout; *bytes = B * D * 4; break;
    case CRL_WS_LOGITS:
      if (x->fused) return fail(CRL_EUNSUPPORTED, "fused logits are never materialised");
      *offset = x->logits; *bytes = B * x->ldF * 4; break;
    case CRL_WS_POLICY_OUT: *offset = x->sl[2].out; *bytes = B * x->P * 4; break;
    case CRL_WS_NOISE: *offset = x->noise; *bytes = B * x->A * 4; break;
    case CRL_WS_LOG_PI: *offset = x->logpi; *bytes = B * 4; break;
    case CRL_WS_POLICY_ENERGY: *offset = x->fpol; *bytes = B * 4; break;
    case CRL_WS_DACTION: *offset = x->dact; *bytes = B * x->ldd * 4; break;
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
  CRL_TRY(check_device(x));
  CRL_HIP(launch_relabel(obs, act, E, T, x->cfg.obs_dim, x->cfg.act_dim, x->cfg.goal_dim,
                         x->cfg.goal_lo, seed, step, x->d_thr, x->B, idx, x_sa, x->net[0].ld_in,
                         x_g, x->net[1].ld_in, x_sg, x->ld_sg, x->bf16, (hipStream_t)stream),
          "relabel launch");
  return CRL_OK;
}

CRL_API int crl_replay_insert(float* obs, float* act, int32_t* traj, int32_t E, int32_t C,
                              int32_t d_s, int32_t d_a, const float* new_obs,
                              const float* new_act, const int32_t* new_traj, int32_t U,
                              int64_t* count, void* stream) {
  if (!obs || !traj || !new_obs || !new_traj || !count)
    return fail(CRL_EINVAL, "NULL buffer argument");
  if (d_a > 0 && (!act || !new_act)) return fail(CRL_EINVAL, "act is NULL");
  if (E < 1 || C < 2) return fail(CRL_EINVAL, "need num_envs >= 1 and capacity >= 2");
  if (d_s < 1 || d_a < 0) return fail(CRL_EINVAL, "bad row widths %d, %d", d_s, d_a);
  if (U < 1 || U > C) return fail(CRL_EINVAL, "steps %d outside [1, capacity %d]", U, C);
  if ((int64_t)U * E > INT32_MAX / 4 || (int64_t)E * C > INT32_MAX)
    return fail(CRL_EINVAL, "chunk or ring too large");
  CRL_HIP(launch_replay_insert(obs, act, traj, E, C, d_s, d_a, new_obs, new_act, new_traj, U,
                               count, (hipStream_t)stream),
          "replay insert launch");
  return CRL_OK;
}

CRL_API int crl_ring_sample_relabel(crl_ctx* x, const float* obs, const float* act,
                                    const int32_t* traj, int32_t E, int32_t C,
                                    const int64_t* count, uint64_t seed, const int64_t* step,
                                    int32_t* idx, void* x_sa, void* x_g, void* x_sg,
                                    void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!obs || !traj || !count || !step || !idx || !x_sa || !x_g)
    return fail(CRL_EINVAL, "NULL buffer argument");
  if (!act && x->cfg.act_dim > 0) return fail(CRL_EINVAL, "act is NULL");
  if (E < 1 || C < 2) return fail(CRL_EINVAL, "need num_envs >= 1 and capacity >= 2");
  if ((int64_t)E * C > INT32_MAX) return fail(CRL_EINVAL, "ring too large");
  CRL_TRY(check_device(x));
  CRL_HIP(launch_ring_relabel(obs, act, traj, E, C, count, x->cfg.obs_dim, x->cfg.act_dim,
                              x->cfg.goal_dim, x->cfg.goal_lo, seed, step, x->d_thr,
                              x->cfg.max_episode_len - 2, x->B, idx, x_sa, x->net[0].ld_in, x_g,
                              x->net[1].ld_in, x_sg, x->ld_sg, x->bf16, (hipStream_t)stream),
          "ring relabel launch");
  return CRL_OK;
}

CRL_API int crl_critic_fwd(crl_ctx* x, const float* params, const uint16_t* params_bf16,
                           const void* x_sa, const void* x_g, void* ws, float* loss_out,
                           int64_t* advance, void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!params || !x_sa || !x_g || !ws || !loss_out) return fail(CRL_EINVAL, "NULL buffer argument");
  if (reinterpret_cast<uintptr_t>(advance) % alignof(int64_t))
    return fail(CRL_EINVAL, "advance must be 8-byte aligned");
  if (x->bf16 && !params_bf16) return fail(CRL_EINVAL, "BF16 precision needs params_bf16");
  if (!aligned16(params) || !aligned16(x_sa) || !aligned16(x_g) || !aligned16(ws) ||
      (params_bf16 && !aligned16(params_bf16)))
    return fail(CRL_EINVAL, "buffers must be 16-byte aligned");
  CRL_TRY(check_device(x));
  hipStream_t s = (hipStream_t)stream;
  const bf16_t* pb = reinterpret_cast<const bf16_t*>(params_bf16);

  NetCall nc[2] = {{0, x_sa, x->net[0].ld_in, params, pb, nullptr, nullptr, 0, 0, 0},
                   {1, x_g, x->net[1].ld_in, params, pb, nullptr, nullptr, 0, 0, 0}};
  // fused logits: the output layer's split-K sum is taken by the kernel that
  // makes the BF16 copies and norms
  GemmParams top{};
  CRL_TRY(mlp_forward(x, nc, 2, ws, s, x->fused ? &top : nullptr));

  return contrastive_fwd(x, WF(ws, x->sl[0].out), WF(ws, x->sl[1].out), ws, loss_ws(x),
                         loss_out, x->fused ? &top : nullptr, s, advance);
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
  CRL_TRY(check_device(x));
  hipStream_t s = (hipStream_t)stream;
  const bf16_t* pb = reinterpret_cast<const bf16_t*>(params_bf16);
  const float* phi = WF(ws, x->sl[0].out);
  const float* psi = WF(ws, x->sl[1].out);
  float* dphi = WF(ws, x->sl[0].dout);
  float* dpsi = WF(ws, x->sl[1].dout);

  // dL/dphi, dL/dpsi, their storage-type copies and (fused) the output
  // layer's bias partials
  CRL_TRY(contrastive_bwd(x, phi, psi, ws, dphi, dpsi, W(ws, x->sl[0].dout_t),
                          W(ws, x->sl[1].dout_t), true, s));

  NetCall nc[2] = {{0, x_sa, x->net[0].ld_in, params, pb, grads, nullptr, 0, 0, 0},
                   {1, x_g, x->net[1].ld_in, params, pb, grads, nullptr, 0, 0, 0}};
  return mlp_backward(x, nc, 2, ws, s, x->fused);
}

CRL_API int crl_critic_bwd_adam(crl_ctx* x, float* params, uint16_t* params_bf16,
                                const void* x_sa, const void* x_g, void* ws, float* grads,
                                float* m, float* v, const int64_t* step, double lr, double b1,
                                double b2, double eps, void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!params || !x_sa || !x_g || !ws || !m || !v || !step)
    return fail(CRL_EINVAL, "NULL buffer argument");
  if (x->bf16 && !params_bf16) return fail(CRL_EINVAL, "BF16 precision needs params_bf16");
  if (!aligned16(params) || !aligned16(ws) || (grads && !aligned16(grads)) || !aligned16(x_sa) ||
      !aligned16(x_g) || !aligned16(m) || !aligned16(v) ||
      (params_bf16 && !aligned16(params_bf16)))
    return fail(CRL_EINVAL, "buffers must be 16-byte aligned");
  if (!(b1 > 0.0 && b1 < 1.0 && b2 > 0.0 && b2 < 1.0 && eps >= 0.0 && std::isfinite(lr)))
    return fail(CRL_EINVAL, "Adam hyperparameters out of range");
  CRL_TRY(check_device(x));
  hipStream_t s = (hipStream_t)stream;
  AdamArgs A{};
  A.p = params;
  A.m = m;
  A.v = v;
  A.pb = reinterpret_cast<bf16_t*>(params_bf16);
  A.step = step;
  A.c = adam_coef(lr, b1, b2, eps);
  const bf16_t* pb = reinterpret_cast<const bf16_t*>(params_bf16);
  const float* phi = WF(ws, x->sl[0].out);
  const float* psi = WF(ws, x->sl[1].out);
  CRL_TRY(contrastive_bwd(x, phi, psi, ws, WF(ws, x->sl[0].dout), WF(ws, x->sl[1].dout),
                          W(ws, x->sl[0].dout_t), W(ws, x->sl[1].dout_t), true, s));
  NetCall nc[2] = {{0, x_sa, x->net[0].ld_in, params, pb, grads, nullptr, 0, 0, 0},
                   {1, x_g, x->net[1].ld_in, params, pb, grads, nullptr, 0, 0, 0}};
  return mlp_backward(x, nc, 2, ws, s, x->fused, &A);
}

CRL_API int crl_infonce_fwd(crl_ctx* x, const float* phi, const float* psi, void* ws,
                            float* loss_out, void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!phi || !psi || !ws || !loss_out) return fail(CRL_EINVAL, "NULL buffer argument");
  if (!aligned16(phi) || !aligned16(psi) || !aligned16(ws))
    return fail(CRL_EINVAL, "phi, psi and ws must be 16-byte aligned");
  CRL_TRY(check_device(x));
  return contrastive_fwd(x, phi, psi, ws, loss_ws(x), loss_out, nullptr, (hipStream_t)stream);
}

CRL_API int crl_infonce_fwd_noalloc(crl_ctx* x, const float* phi, const float* psi,
                                    float* loss_out, float* r_out, float* c_out,
                                    float* diag_out, void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!phi || !psi || !loss_out) return fail(CRL_EINVAL, "NULL buffer argument");
  if (!aligned16(phi) || !aligned16(psi)) return fail(CRL_EINVAL, "phi and psi must be 16-byte aligned");
  CRL_TRY(check_device(x));
  if (x->na_bytes > (int64_t)CRL_NOALLOC_SCRATCH_BYTES)
    return fail(CRL_EINVAL,
                "the loss of this context (batch %d, repr_dim %d) needs %lld bytes of scratch, "
                "more than the %lld of the static array",
                x->B, x->D, (long long)x->na_bytes, (long long)CRL_NOALLOC_SCRATCH_BYTES);
  if (!x->scratch) return hip_fail(x->scratch_err, "hipGetSymbolAddress(scratch)");
  hipStream_t s = (hipStream_t)stream;
  CRL_TRY(contrastive_fwd(x, phi, psi, x->scratch, x->na, loss_out, nullptr, s));
  const size_t nb = (size_t)x->B * sizeof(float);
  if (r_out)
    CRL_HIP(hipMemcpyAsync(r_out, WF(x->scratch, x->na.r), nb, hipMemcpyDeviceToDevice, s), "copy r");
  if (c_out)
    CRL_HIP(hipMemcpyAsync(c_out, WF(x->scratch, x->na.c), nb, hipMemcpyDeviceToDevice, s), "copy c");
  if (diag_out)
    CRL_HIP(hipMemcpyAsync(diag_out, WF(x->scratch, x->na.diag), nb, hipMemcpyDeviceToDevice, s),
            "copy diag");
  return CRL_OK;
}

CRL_API int crl_infonce_bwd(crl_ctx* x, const float* phi, const float* psi, void* ws,
                            float* dphi, float* dpsi, void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!phi || !psi || !ws || !dphi || !dpsi) return fail(CRL_EINVAL, "NULL buffer argument");
  if (!aligned16(phi) || !aligned16(psi) || !aligned16(ws) || !aligned16(dphi) ||
      !aligned16(dpsi))
    return fail(CRL_EINVAL, "phi, psi, ws, dphi and dpsi must be 16-byte aligned");
  CRL_TRY(check_device(x));
  // the storage-type copies go to the workspace's own slots (FP32: dphi, dpsi)
  void* dphi_t = x->bf16 ? W(ws, x->sl[0].dout_t) : (void*)dphi;
  void* dpsi_t = x->bf16 ? W(ws, x->sl[1].dout_t) : (void*)dpsi;
  return contrastive_bwd(x, phi, psi, ws, dphi, dpsi, dphi_t, dpsi_t, false, (hipStream_t)stream);
}

CRL_API int crl_check_finite(const float* loss_out, void* stream) {
  if (!loss_out) return fail(CRL_EINVAL, "NULL loss_out");
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  CRL_HIP(hipStreamIsCapturing(s, &cs), "hipStreamIsCapturing");
  if (cs != hipStreamCaptureStatusNone)
    return fail(CRL_EINVAL, "crl_check_finite synchronises and cannot run under graph capture");
  float h[8];
  CRL_HIP(hipMemcpyAsync(h, loss_out, sizeof(h), hipMemcpyDeviceToHost, s), "copy loss_out");
  CRL_HIP(hipStreamSynchronize(s), "hipStreamSynchronize");
  if (!std::isfinite(h[0]) || h[6] != 0.f)
    return fail(CRL_ENONFINITE, "non-finite loss (total %g, %g non-finite row/column terms)",
                (double)h[0], (double)h[6]);
  return CRL_OK;
}

// The policy step (both entry points): the arguments are checked by the
// caller; adam, if not NULL, takes the policy gradient into its Adam step as
// the gradient is reduced.
static int actor_step(crl_ctx* x, const float* params, const uint16_t* params_bf16,
                      const float* actor_params, const uint16_t* actor_params_bf16,
                      const float* log_alpha, const void* x_sa, const void* x_g,
                      const void* x_sg, uint64_t seed, const int64_t* step, void* ws,
                      float* actor_grads, float* alpha_grad, float* loss_out,
                      const AdamArgs* adam, hipStream_t s) {
  const int B = x->B;
  const bf16_t* pb = reinterpret_cast<const bf16_t*>(params_bf16);
  const bf16_t* apb = reinterpret_cast<const bf16_t*>(actor_params_bf16);
  void* xsa2 = W(ws, x->xsa2);
  float* eps = WF(ws, x->noise);
  float* logpi = WF(ws, x->logpi);
  float* fpol = WF(ws, x->fpol);
  float* dact = WF(ws, x->dact);
  const float* pout = WF(ws, x->sl[2].out);

  // random goals: the policy and psi see the mixed goals
  if (x->mix_thr > 0) {
    CRL_HIP(launch_goal_mix(x_g, x->net[1].ld_in, x_sg, x->ld_sg, x->cfg.obs_dim,
                            x->cfg.goal_dim, seed, step, x->mix_thr, B, W(ws, x->xg_mix),
                            W(ws, x->xsg_mix), x->bf16, s), "random-goal mix");
    x_g = W(ws, x->xg_mix);
    x_sg = W(ws, x->xsg_mix);
  }
  // policy MLP on [s, g], then the sampled action and log pi
  NetCall pol = {2, x_sg, x->ld_sg, actor_params, apb, actor_grads, nullptr, 0, 0, 0};
  CRL_TRY(mlp_forward(x, &pol, 1, ws, s));
  CRL_HIP(launch_actor_head_fwd(pout, x->P, x->A, seed, step, x_sa, xsa2, x->net[0].ld_in,
                                x->cfg.obs_dim, eps, logpi, B, x->bf16, s), "policy head");
  // frozen critic on (s, a') and g
  NetCall crit[2] = {{0, xsa2, x->net[0].ld_in, params, pb, nullptr, nullptr, 0, 0, 0},
                     {1, x_g, x->net[1].ld_in, params, pb, nullptr, nullptr, 0, 0, 0}};
  CRL_TRY(mlp_forward(x, crit, 2, ws, s));
  CRL_HIP(launch_actor_energy(WF(ws, x->sl[0].out), WF(ws, x->sl[1].out), x->D, x->energy, fpol,
                              W(ws, x->sl[0].dout_t), B, x->bf16, s), "policy energy");
  // d(-mean f)/da' through phi (no parameter gradients)
  NetCall back = {0, xsa2, x->net[0].ld_in, params, pb, nullptr, dact, x->cfg.obs_dim, x->A, x->ldd};
  CRL_TRY(mlp_backward(x, &back, 1, ws, s));
  CRL_HIP(launch_actor_head_bwd(pout, x->P, x->A, eps, dact, x->ldd, log_alpha,
                                WF(ws, x->sl[2].dout), W(ws, x->sl[2].dout_t), B, x->bf16, s),
          "policy head backward");
  CRL_TRY(mlp_backward(x, &pol, 1, ws, s, false, adam));
  CRL_HIP(launch_actor_loss(logpi, fpol, B, log_alpha, x->cfg.target_entropy, loss_out,
                            alpha_grad, s), "actor loss");
  return CRL_OK;
}

CRL_API int crl_actor_step(crl_ctx* x, const float* params, const uint16_t* params_bf16,
                           const float* actor_params, const uint16_t* actor_params_bf16,
                           const float* log_alpha, const void* x_sa, const void* x_g,
                           const void* x_sg, uint64_t seed, const int64_t* step, void* ws,
                           float* actor_grads, float* alpha_grad, float* loss_out,
                           void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!x->actor) return fail(CRL_EINVAL, "this context has no actor (actor_n_hidden = 0)");
  if (!params || !actor_params || !log_alpha || !x_sa || !x_g || !x_sg || !step || !ws ||
      !actor_grads || !alpha_grad || !loss_out)
    return fail(CRL_EINVAL, "NULL buffer argument");
  if (x->bf16 && (!params_bf16 || !actor_params_bf16))
    return fail(CRL_EINVAL, "BF16 precision needs params_bf16 and actor_params_bf16");
  if (!aligned16(params) || !aligned16(actor_params) || !aligned16(x_sa) || !aligned16(x_g) ||
      !aligned16(x_sg) || !aligned16(ws) || !aligned16(actor_grads) ||
      (params_bf16 && !aligned16(params_bf16)) ||
      (actor_params_bf16 && !aligned16(actor_params_bf16)))
    return fail(CRL_EINVAL, "buffers must be 16-byte aligned");
  CRL_TRY(check_device(x));
  return actor_step(x, params, params_bf16, actor_params, actor_params_bf16, log_alpha, x_sa, x_g,
                    x_sg, seed, step, ws, actor_grads, alpha_grad, loss_out, nullptr,
                    (hipStream_t)stream);
}

CRL_API int crl_actor_step_adam(crl_ctx* x, const float* params, const uint16_t* params_bf16,
                                float* actor_params, uint16_t* actor_params_bf16,
                                const float* log_alpha, const void* x_sa, const void* x_g,
                                const void* x_sg, uint64_t seed, const int64_t* step, void* ws,
                                float* actor_grads, float* alpha_grad, float* loss_out,
                                float* actor_m, float* actor_v, const int64_t* adam_step,
                                double lr, double b1, double b2, double eps, void* stream) {
  if (!x) return fail(CRL_EINVAL, "NULL context");
  if (!x->actor) return fail(CRL_EINVAL, "this context has no actor (actor_n_hidden = 0)");
  if (!params || !actor_params || !log_alpha || !x_sa || !x_g || !x_sg || !step || !ws ||
      !alpha_grad || !loss_out || !actor_m || !actor_v || !adam_step)
    return fail(CRL_EINVAL, "NULL buffer argument");
  if (x->bf16 && (!params_bf16 || !actor_params_bf16))
    return fail(CRL_EINVAL, "BF16 precision needs params_bf16 and actor_params_bf16");
  if (!aligned16(params) || !aligned16(actor_params) || !aligned16(x_sa) || !aligned16(x_g) ||
      !aligned16(x_sg) || !aligned16(ws) || (actor_grads && !aligned16(actor_grads)) ||
      !aligned16(actor_m) || !aligned16(actor_v) ||
      (params_bf16 && !aligned16(params_bf16)) ||
      (actor_params_bf16 && !aligned16(actor_params_bf16)))
    return fail(CRL_EINVAL, "buffers must be 16-byte aligned");
  if (!(b1 > 0.0 && b1 < 1.0 && b2 > 0.0 && b2 < 1.0 && eps >= 0.0 && std::isfinite(lr)))
    return fail(CRL_EINVAL, "Adam hyperparameters out of range");
  CRL_TRY(check_device(x));
  AdamArgs A{};
  A.p = actor_params;
  A.m = actor_m;
  A.v = actor_v;
  A.pb = reinterpret_cast<bf16_t*>(actor_params_bf16);
  A.step = adam_step;
  A.c = adam_coef(lr, b1, b2, eps);
  return actor_step(x, params, params_bf16, actor_params, actor_params_bf16, log_alpha, x_sa, x_g,
                    x_sg, seed, step, ws, actor_grads, alpha_grad, loss_out, &A,
                    (hipStream_t)stream);
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
  const AdamCoef c = adam_coef(lr, b1, b2, eps);
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
