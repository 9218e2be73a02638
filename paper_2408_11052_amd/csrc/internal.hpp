// Internal launch wrappers shared by the C-ABI layer (not part of the ABI).
#pragma once

#include "common.hpp"
#include "crl.h"
#include "gemm.hpp"

namespace crl {

// timing.hip: opt-in HIP-event timing of single launches (see crl_timing_*).
struct KTimer {
  bool on;
  int slot;
  hipEvent_t a, b;
  hipStream_t s;
  double flops, bytes;
};
KTimer timing_begin(const char* name, double flops, double bytes, hipStream_t s);
void timing_end(KTimer& t);
#define CRL_TIMED(name, flops, bytes, stream, ...)                   \
  do {                                                               \
    ::crl::KTimer _crl_t = ::crl::timing_begin(name, flops, bytes, stream); \
    __VA_ARGS__;                                                     \
    ::crl::timing_end(_crl_t);                                       \
  } while (0)

// gemm.hip: dispatch on storage type / operand layouts / output type.
hipError_t launch_gemm(GemmParams& P, bool bf16, int la, int lb, bool out_bf16,
                       hipStream_t s);
// One layer's weight gradient (Pw: MC x MC, FP32 out or deferred split-K
// partials) and input gradient (Px: KC x KC, BF16 out, unsplit) in one launch
// of the direct-to-LDS kernel with 128-wide tiles (also for a dW with N <= 64);
// gemm_pair_ok tells whether both launches qualify (BF16 storage, both on the
// direct-to-LDS kernel, dX 128 wide, no split-K reduction left to run).
bool gemm_pair_ok(const GemmParams& Pw, const GemmParams& Px, bool bf16);
hipError_t launch_gemm_dw_dx(GemmParams& Pw, GemmParams& Px, hipStream_t s);
// Split factor and chunk for a batch of problems (fills P.splits, P.k_chunk):
// the largest power of two that keeps the launch within target_wgs workgroups
// and every split at least min_steps K steps deep.
void plan_split_k(GemmParams& P, bool bf16, int target_wgs, int min_steps = 4);
// Column-tile width of the direct-to-LDS kernel for this launch (128 or 64),
// or 0 when the register-staged kernel takes it.  Depends on shapes, leading
// dimensions and pointer alignment only.
int gemm_lds_bn(const GemmParams& P, bool bf16);
// Floats of one split's deferred partial of problem g: the whole 128 x bn
// tiles in fragment order (bn > 0), or the dense M x N block (bn == 0).
int64_t frag_partial_floats(const GemmParams& P, int g, int bn);

// kernels.hip
hipError_t launch_relabel(const float* obs, const float* act, int E, int T,
                          int d_s, int d_a, int d_g, int goal_lo, uint64_t seed,
                          const int64_t* step, const uint64_t* thr, int B,
                          int32_t* idx, void* x_sa, int ld_sa, void* x_g, int ld_g,
                          void* x_sg, int ld_sg, bool bf16, hipStream_t s);

// replay.hip: the ring buffer
hipError_t launch_replay_insert(float* obs, float* act, int32_t* traj, int E, int C, int d_s,
                                int d_a, const float* nobs, const float* nact,
                                const int32_t* ntraj, int U, int64_t* count, hipStream_t s);
hipError_t launch_ring_relabel(const float* obs, const float* act, const int32_t* traj, int E,
                               int C, const int64_t* count, int d_s, int d_a, int d_g,
                               int goal_lo, uint64_t seed, const int64_t* step,
                               const uint64_t* thr, int n_thr, int B, int32_t* idx, void* x_sa,
                               int ld_sa, void* x_g, int ld_g, void* x_sg, int ld_sg, bool bf16,
                               hipStream_t s);

struct LnArgs {
  const void* Z[2];     // [B][N] pre-LN values
  void* H[2];           // [B][N] Swish(LN(z)) out
  float* mu[2];
  float* rstd[2];
  const float* g[2];    // LN scale
  const float* b[2];    // LN offset
  // backward
  const void* dH[2];
  void* dZ[2];
  float* part[2];       // [ceil(B/128)][3][N] column partials
};
hipError_t launch_ln_swish_fwd(const LnArgs& a, int count, int B, int N, float eps,
                               bool bf16, hipStream_t s);
hipError_t launch_ln_swish_bwd(const LnArgs& a, int count, int B, int N, bool bf16,
                               int rows_per_wave, hipStream_t s);
int ln_bwd_partials(int B, int rows_per_wave);

// out[k][n] = sum_w part[w][k][n] for k < nk; the three sums go to out0/1/2.
struct ColReduceArgs {
  const float* part[2];
  float* out[2][3];
};
hipError_t launch_partial_reduce(const ColReduceArgs& a, int count, int nparts, int nk,
                                 int N, hipStream_t s);

// column sums of X [B][N] (FP32 or BF16), written to out[N] (FP32).
struct ColSumArgs {
  const void* X[2];
  float* out[2];
  float* part[2];   // [ceil(B/128)][N]
};
hipError_t launch_colsum(const ColSumArgs& a, int count, int B, int N, int ld,
                         bool bf16, hipStream_t s);
// only the per-chunk partials part[e][ceil(B/128)][N] of launch_colsum
hipError_t launch_colsum_partials(const ColSumArgs& a, int count, int B, int N, int ld,
                                  bool bf16, hipStream_t s);
int colsum_chunks(int B);

// Deferred gradient reductions: g[dst + i] = sum_k part_k[i], part_k at byte
// offset src + 4 k stride in the workspace, i < n, in the order k = 0, 1, ...
// (with four interleaved running sums, combined in a fixed order).  `first`
// is the job's first float4 (few-part jobs) or first 16-output block
// (many-part jobs) in the launch's index space.
// Sum of nparts partial blocks (src + k * stride floats, k = 0..nparts-1, in
// that order) into g + dst.  bn == 0: n contiguous floats.  bn > 0: split-K
// partials of an M x N GEMM in the direct-to-LDS kernel's fragment order
// (128 x bn tiles, tiles_n per row of tiles), scattered into the row-major
// M x N block at dst.
struct RedJob {
  int64_t src;
  int64_t stride;
  int64_t dst;
  int64_t first;
  int64_t first_chunk;  // few-part jobs with the Adam epilogue: first block, in
                        // chunks of kRedChunk4 float4 outputs
  int32_t nparts, n;
  int32_t M, N, tiles_n, bn;
};
// float4 outputs per block of the reduction with the Adam epilogue: a 64 x 64
// block of a fragment-order tile (two of its waves)
constexpr int kRedChunk4 = 1024;
constexpr int kManyCols = 32;  // outputs per workgroup of a many-part reduction job
struct AdamArgs;
// few-part jobs (total4 float4 outputs) and many-part jobs (nblocks blocks of
// 16 outputs) in one launch.  With A, each gradient element goes straight
// into the Adam step of its parameter (g, if not NULL, still receives it).
hipError_t launch_grad_reduce(const char* ws, float* g, const RedJob* few, int nfew,
                              int64_t total4, const RedJob* many, int nmany, int64_t nblocks,
                              double bytes, hipStream_t s, const AdamArgs* A = nullptr);

hipError_t launch_sqnorm(const float* X, float* out, int B, int D, hipStream_t s);
hipError_t launch_cast_bf16(const float* src, bf16_t* dst, int64_t n, hipStream_t s);
// Adam coefficients: 1 - b and log b are formed in double on the host.
struct AdamCoef {
  float lr, b1, b2, omb1, omb2, log_b1, log_b2, eps;
};
hipError_t launch_adam(float* p, const float* g, float* m, float* v, bf16_t* pb,
                       int64_t n, const int64_t* step, const AdamCoef& c, hipStream_t s);
// The optimiser state of a flat vector, for the reduction's Adam epilogue.
struct AdamArgs {
  float* p;
  float* m;
  float* v;
  bf16_t* pb;            // BF16 copy of p, or NULL
  const int64_t* step;   // t (device, read)
  AdamCoef c;
};
hipError_t launch_counter_add(int64_t* c, int64_t inc, hipStream_t s);

// materialised critic matrix (FP32 B x B in the workspace, row stride ld)
hipError_t launch_col_lse_partial(const float* F, int B, int ld, int rchunks, float* pm,
                                  float* ps, hipStream_t s);
// log-sum-exp of (max, sum) partials [nparts][B] per column j, for `count`
// problems in one launch
struct LseMergeArgs {
  const float* pm[2];
  const float* ps[2];
  int nparts[2];
  float* out[2];
};
hipError_t launch_lse_merge(const LseMergeArgs& a, int count, int B, hipStream_t s);
hipError_t launch_lse_merge(const float* pm, const float* ps, int nparts, int B,
                            float* out, hipStream_t s);
// loss_out[8] from r, c, diag and (pairwise objectives) the per-row terms;
// then *advance += 1 if advance is not NULL (one workgroup, so no fence)
hipError_t launch_loss(const float* r, const float* c, const float* diag, const float* term,
                       int B, int loss, float beta, float* loss_out, int64_t* advance,
                       hipStream_t s);
hipError_t launch_l2_fix(float* dX, const float* X, const float* rs, int B, int D,
                         hipStream_t s);

// objectives.hip: energies and objectives on the materialised matrix
hipError_t launch_unit_rows(const float* X, float* U, float* nrm, int B, int D, hipStream_t s);
hipError_t launch_l1_energy(const float* phi, const float* psi, float* F, int B, int D, int ld,
                            hipStream_t s);
hipError_t launch_l1_backward(const float* X, const float* Y, const float* G, int ldg, int trans,
                              float* dX, int B, int D, hipStream_t s);
// r, diag, and for the pairwise objectives the row terms and the sums that
// form dL/dF_ii
hipError_t launch_row_obj(const float* F, int B, int ld, int loss, float* r, float* diag,
                          float* term, float* aux, hipStream_t s);
// in place F -> dL/dF (or H for the distance energies, with its row sums)
hipError_t launch_grad_obj(float* F, int B, int ld, const float* r, const float* c,
                           const float* diag, const float* aux, int loss, int energy, float beta,
                           float* rowsum, hipStream_t s);
hipError_t launch_cos_fix(float* dX, const float* U, const float* nrm, int B, int D, hipStream_t s);

// fused InfoNCE (BF16 tiles, FP32 online LSE)
struct FusedArgs {
  const float* phi;
  const float* psi;
  bf16_t* phi_b;      // BF16 copies written by the prep kernel
  bf16_t* psi_b;
  float* nphi;        // squared norms of the BF16-rounded rows (L2)
  float* npsi;
  float* row_m;       // [S][B]
  float* row_s;
  float* col_m;       // [B/64][B]
  float* col_s;
  float* r;
  float* c;
  float* diag;
  float* dX_part;     // [2][S][B][D] backward partials (rows pass, columns pass)
  float* rs_part;     // [2][S][B]   sum_b H_ab (L2)
  float* dphi;        // [B][D] FP32 out
  float* dpsi;
  void* dphi_t;       // storage-type copies for the encoder GEMMs
  void* dpsi_t;
  float* bias_part[2]; // [chunks][D] column sums of dphi / dpsi per 256/D rows, or nullptr
};
int fused_splits(int B);
int fused_bwd_splits(int B);          // splits of the one-pass backward (D = 64)
int fused_bias_chunks(int B, int D);  // row blocks of the backward reduction
// top: the output layer's deferred split-K launch (phi = d[0].C, psi =
// d[1].C), summed with its bias by the prep kernel; nullptr: phi and psi are
// final already.
// energy: CRL_ENERGY_DOT, _L2, _COS (unit rows, dot product) or _L2SQ
hipError_t launch_fused_fwd(const FusedArgs& a, int B, int D, int energy, const GemmParams* top,
                            hipStream_t s);
// loss: CRL_LOSS_FWD, _SYM, _BWD, _FLATNCE_FWD or _FLATNCE_BWD
hipError_t launch_fused_bwd(const FusedArgs& a, int B, int D, int energy, int loss, float beta,
                            bool out_bf16, hipStream_t s);
// whether the backward takes the one-pass kernel (D = 64, at most 16 row
// blocks of 256), whose partials are indexed by 256-row blocks
bool fused_bwd_one_pass(int B, int D);

// actor.hip: the policy step's elementwise/row kernels
hipError_t launch_actor_head_fwd(const float* out, int ldo, int A, uint64_t seed,
                                 const int64_t* step, const void* x_sa, void* x_sa2, int ld,
                                 int d_s, float* eps, float* logpi, int B, bool bf16,
                                 hipStream_t s);
// f_b = energy(phi_b, psi_b) (CRL_ENERGY_*) and d(-mean f)/dphi
hipError_t launch_actor_energy(const float* phi, const float* psi, int D, int energy, float* f,
                               void* dphi, int B, bool bf16, hipStream_t s);
hipError_t launch_actor_head_bwd(const float* out, int ldo, int A, const float* eps,
                                 const float* da, int ldd, const float* log_alpha, float* dout,
                                 void* dout_t, int B, bool bf16, hipStream_t s);
// random goals: xg_out[b] = x_g[j], xsg_out[b] = [x_sg[b][0:d_s], x_g[j], 0...]
// with j the partner drawn for b (j = b when b is not mixed)
hipError_t launch_goal_mix(const void* x_g, int ld_g, const void* x_sg, int ld_sg, int d_s,
                           int d_g, uint64_t seed, const int64_t* step, uint64_t thr53, int B,
                           void* xg_out, void* xsg_out, bool bf16, hipStream_t s);
hipError_t launch_actor_loss(const float* logpi, const float* f, int B, const float* log_alpha,
                             float target_entropy, float* loss_out, float* alpha_grad,
                             hipStream_t s);

}  // namespace crl
