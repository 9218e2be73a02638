/*
 * crl.h -- C ABI of the contrastive-RL (CRL) update hot path on MI355X (gfx950).
 *
 * One critic update of contrastive RL (Algorithm 1, the update loop):
 *   1. draw a batch of (s, a) uniformly from a GPU-resident replay buffer and
 *      relabel each goal to a future state of the same trajectory at a
 *      geometric offset (Section 3.2 "Policy Learning"; Preliminaries, the
 *      discounted state-visitation law; Appendix D)        -> crl_sample_relabel
 *   2. run the encoders phi(s, a) and psi(g), form the B x B critic matrix
 *      with the dot or L2 energy (Section 3.1; Appendix A.2 energy table), and
 *      the InfoNCE loss with the logsumexp penalty (Section 3.1 critic
 *      objective; Appendix A.2 InfoNCE-forward/backward/symmetric)
 *                                                          -> crl_critic_fwd
 *   3. the gradient of that loss w.r.t. every encoder parameter
 *                                                          -> crl_critic_bwd
 *   4. the optimiser step on the flat parameter vector     -> crl_adam_step
 * and, when the context has a policy, the policy step that follows the critic
 * step on the same batch (Section 3.2 policy learning; Algorithm 1, policy
 * update; Section 5.1 setup, tunable entropy coefficient)   -> crl_actor_step
 *
 * Conventions shared by every call
 *  - Pointers named "device" point to device memory on the current HIP device;
 *    the caller owns every buffer (inputs, outputs, parameters, optimiser
 *    state and the workspace).  The compute calls allocate nothing; only
 *    crl_create allocates (small device tables) and crl_destroy frees them.
 *  - All compute calls are asynchronous and ordered on the `stream` argument
 *    (a hipStream_t passed as void*; NULL is the legacy default stream).  No
 *    call synchronises with the host, so every call may be captured into a
 *    HIP graph.
 *  - Return value: CRL_OK (0) or a negative crl_status.  Arguments are checked
 *    on the host before anything is launched: a bad argument launches nothing
 *    and returns CRL_EINVAL / CRL_EUNSUPPORTED; a failed launch returns
 *    CRL_EHIP.  crl_last_error() then holds a message (thread-local).
 *  - Matrices are row-major.  BF16 values are stored as uint16 bit patterns
 *    (round-to-nearest-even from FP32).
 *
 * Flat parameter layout (crl_param_count / crl_layer_layout): phi's layers
 * first, then psi's; each layer holds W [fan_in][fan_out], b [fan_out] and,
 * for LayerNorm layers, ln_g [fan_out] and ln_b [fan_out].  Every tensor
 * starts at an element offset that is a multiple of 64; the gaps are padding
 * whose gradient is written as 0.  The policy's layers live in a second flat
 * vector of the same form (crl_actor_param_count), since they have their own
 * optimiser state and learning rate.
 */
#ifndef CRL_H
#define CRL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CRL_API __attribute__((visibility("default")))

typedef enum {
  CRL_OK = 0,
  CRL_EINVAL = -1,        /* bad argument (null pointer, size, alignment) */
  CRL_EUNSUPPORTED = -2,  /* valid but not supported by this build */
  CRL_EHIP = -3,          /* a HIP runtime call or launch failed */
  CRL_ENONFINITE = -4     /* crl_check_finite: the loss or a row term is not finite */
} crl_status;

enum { CRL_ACT_RELU = 0, CRL_ACT_LN_SWISH = 1 };
/* Energies of Appendix A.2: <phi, psi>; -||phi - psi||_2; the cosine
 * <phi, psi> / (||phi|| ||psi||) (0 where a norm is 0); -||phi - psi||_2^2
 * ("L2 without the square root"); -||phi - psi||_1. */
enum { CRL_ENERGY_DOT = 0, CRL_ENERGY_L2 = 1, CRL_ENERGY_COS = 2, CRL_ENERGY_L2SQ = 3,
       CRL_ENERGY_L1 = 4 };
/* Contrastive objectives of Appendix A.2 (every one with the logsumexp
 * penalty beta * mean_i r_i^2, Section 5.3), averaged over the positives i,
 * sums over j over the whole batch; r_i = LSE_j F_ij, c_j = LSE_i F_ij:
 *   FWD   InfoNCE-forward   mean_i (r_i - F_ii)
 *   SYM   InfoNCE-symmetric FWD + BWD
 *   BWD   InfoNCE-backward  mean_j (c_j - F_jj)
 *   FLATNCE_FWD / _BWD      mean_i S_i / stopgrad(S_i), S_i = sum_j
 *                           exp(F_ij - F_ii) (rows) or sum_j exp(F_ji - F_ii)
 *                           (columns): value 1, the gradient of mean log S
 *   FB    Forward-Backward  mean_i [-exp(F_ii) + sum_{j!=i} exp(2 F_ij) / (2(B-1))]
 *   DPO   mean_i sum_j -log sigmoid(F_ii - F_ij)
 *   IPO   mean_i sum_j (F_ii - F_ij - 1)^2
 *   SPPO  mean_i sum_j [(F_ii - 1)^2 + (F_ij + 1)^2] */
enum { CRL_LOSS_FWD = 0, CRL_LOSS_SYM = 1, CRL_LOSS_BWD = 2, CRL_LOSS_FLATNCE_FWD = 3,
       CRL_LOSS_FLATNCE_BWD = 4, CRL_LOSS_FB = 5, CRL_LOSS_DPO = 6, CRL_LOSS_IPO = 7,
       CRL_LOSS_SPPO = 8 };
enum { CRL_PREC_FP32 = 0, CRL_PREC_BF16 = 1 };
/* materialised: the B x B critic matrix is written to the workspace (FP32);
 * fused: online log-sum-exp over tiles, the matrix never exists in memory. */
enum { CRL_LOGITS_MATERIALISED = 0, CRL_LOGITS_FUSED = 1 };

typedef struct crl_config {
  int32_t batch;          /* B >= 1 */
  int32_t obs_dim;        /* d_s: state features per buffer row */
  int32_t act_dim;        /* d_a */
  int32_t goal_dim;       /* d_g: goal = obs[goal_lo : goal_lo + d_g] */
  int32_t goal_lo;
  int32_t n_hidden;       /* hidden layers per encoder (>= 1) */
  int32_t hidden;         /* hidden width (multiple of 8, at most 1024) */
  int32_t repr_dim;       /* D, multiple of 8 (fused logits: 32, 64, 128 or 256;
                             L1 energy: at most 256) */
  int32_t activation;     /* CRL_ACT_* : ReLU, or LayerNorm then Swish */
  int32_t energy;         /* CRL_ENERGY_* (fused logits: DOT, L2, COS, L2SQ) */
  int32_t loss;           /* CRL_LOSS_* (fused logits: FWD, SYM, BWD, FLATNCE_*) */
  int32_t precision;      /* CRL_PREC_*: arithmetic of GEMM and logit tiles */
  int32_t logits;         /* CRL_LOGITS_* */
  float logsumexp_penalty;/* beta of beta * mean_i (LSE_j F_ij)^2 */
  float ln_eps;           /* LayerNorm epsilon (added to the variance) */
  double discount;        /* gamma in (0,1) of the relabel offset law */
  int32_t max_episode_len;/* longest episode crl_sample_relabel will see */
  int32_t actor_n_hidden; /* hidden layers of the policy MLP; 0 = no policy */
  int32_t actor_hidden;   /* its width (multiple of 8, at most 1024); 0 without */
  float target_entropy;   /* H of the entropy-coefficient objective (-act_dim
                             is the usual choice); used with a policy only */
  double random_goal_ratio;/* share of the policy step's goals replaced by
                             another sample's (Appendix C random goals), in
                             [0, 1]; 0 = none.  Used with a policy only. */
  int32_t reserved[2];    /* must be zero */
} crl_config;

typedef struct crl_ctx crl_ctx;

typedef struct crl_layer_info {
  int64_t w, b, ln_g, ln_b; /* element offsets in the flat vector, -1 if absent */
  int32_t fan_in, fan_out;
} crl_layer_info;

/* Create a context on the current HIP device: validates the configuration,
 * plans the workspace and uploads the geometric-offset threshold table for
 * `discount` (see crl_sample_relabel) and the job tables of the gradient
 * reductions.  On success *out owns those tables. */
CRL_API int crl_create(const crl_config* cfg, crl_ctx** out);
CRL_API int crl_destroy(crl_ctx* ctx);

/* Number of floats of the flat parameter (and gradient, Adam m, v) vector. */
CRL_API int crl_param_count(const crl_ctx* ctx, int64_t* n);
/* Number of floats of the policy's flat parameter vector (0 without one). */
CRL_API int crl_actor_param_count(const crl_ctx* ctx, int64_t* n);
/* Offsets of layer `layer` (0 = first) of net 0 (phi) or 1 (psi), in the
 * critic vector, or of net 2 (the policy), in the policy vector.  The policy's
 * output layer has fan_out = 2 act_dim rounded up to a multiple of 64: columns
 * [0, act_dim) are the mean, [act_dim, 2 act_dim) the scale pre-activation,
 * the rest padding whose gradient is 0 (zero-initialised, it stays 0). */
CRL_API int crl_layer_layout(const crl_ctx* ctx, int32_t net, int32_t layer,
                             crl_layer_info* out);
/* Bytes of the device workspace that crl_critic_fwd / _bwd and crl_actor_step
 * use (256-aligned). */
CRL_API int crl_workspace_size(const crl_ctx* ctx, int64_t* bytes);
/* Row strides (elements) of the encoder inputs x_sa [B][ld_sa], x_g [B][ld_g],
 * x_sg [B][ld_sg], and their element size: 4 (FP32) or 2 (BF16).  Columns
 * past the real width are zero. */
CRL_API int crl_input_layout(const crl_ctx* ctx, int32_t* ld_sa, int32_t* ld_g,
                             int32_t* ld_sg, int32_t* elem_bytes);

/* Step 1: sample and relabel one batch (Section 3.2; Algorithm 1, batch
 * sampling "with discount"; Preliminaries: the offset T ~ Geom(1 - gamma)).
 *   obs    device FP32 [num_envs][episode_len][obs_dim], one episode per row
 *   act    device FP32 [num_envs][episode_len][act_dim]
 *   seed   Philox key word 0 (key = (seed, 0))
 *   step   device int64: the batch counter n (read, not modified)
 *   idx    device int32 [B][3] out: (e, t, t_g)
 *   x_sa   device out [B][ld_sa]: [obs[e,t,:], act[e,t,:], 0...]
 *   x_g    device out [B][ld_g]:  [obs[e,t_g,goal_lo:goal_lo+d_g], 0...]
 *   x_sg   device out [B][ld_sg] or NULL: [obs[e,t,:], goal, 0...]
 * For sample b, Philox4x64-10 with counter (b, n, 0, 0) gives words w0..w3:
 *   e = floor(w0 * E / 2^64), t = floor(w1 * (T-1) / 2^64),
 *   k = 1 + #{m >= 1 : w2 < thr[m]}, thr[1] = G = floor(gamma * 2^64),
 *   thr[m] = floor(thr[m-1] * G / 2^64), and t_g = min(t + k, T - 1),
 * so k is geometric on {1, 2, ...} with P(k) ~ (1-gamma) gamma^(k-1) and the
 * goal is a strictly future state clipped to the episode end.
 * Requires 2 <= episode_len <= cfg.max_episode_len, num_envs >= 1. */
CRL_API int crl_sample_relabel(crl_ctx* ctx, const float* obs, const float* act,
                               int32_t num_envs, int32_t episode_len,
                               uint64_t seed, const int64_t* step, int32_t* idx,
                               void* x_sa, void* x_g, void* x_sg, void* stream);

/* The replay buffer as a ring of steps per environment (Algorithm 1: each
 * iteration's unroll of every environment is appended to the buffer D, a new
 * trajectory starting after each terminal step; Appendix B, benchmark
 * parameters: the buffer keeps max_replay_size steps per environment and
 * each iteration appends unroll_length steps of every environment).
 *   obs    device FP32 [num_envs][capacity][obs_dim] ring (written)
 *   act    device FP32 [num_envs][capacity][act_dim] ring (written; may be
 *          NULL with new_act when act_dim == 0)
 *   traj   device int32 [num_envs][capacity]: the trajectory id of each
 *          stored step (written).  Within one environment a trajectory is a
 *          maximal run of equal ids in append order; ids that never repeat
 *          after changing (an episode counter) are the intended use.
 *   new_obs  device FP32 [steps][num_envs][obs_dim], time-major as a
 *          vectorised simulator emits them; new_act [steps][num_envs][act_dim];
 *          new_traj device int32 [steps][num_envs]
 *   count  device int64: steps appended per environment so far.  Read, then
 *          advanced by `steps` on the stream (a second, one-thread launch),
 *          so a captured graph appends a fresh chunk on every replay.
 * Step u of the chunk lands in ring row (count + u) mod capacity, so the
 * ring holds the last min(count, capacity) steps of every environment.
 * Requires 1 <= steps <= capacity, num_envs >= 1, capacity >= 2.  Nothing
 * is allocated; the caller owns every buffer. */
CRL_API int crl_replay_insert(float* obs, float* act, int32_t* traj, int32_t num_envs,
                              int32_t capacity, int32_t obs_dim, int32_t act_dim,
                              const float* new_obs, const float* new_act,
                              const int32_t* new_traj, int32_t steps, int64_t* count,
                              void* stream);

/* Step 1 on the ring buffer: crl_sample_relabel with goals that never leave
 * the trajectory of the drawn step (Section 3.2: the goal is a state that
 * follows s in the same trajectory).  With size = min(*count, capacity)
 * steps stored and logical index i in [0, size) at ring row
 * (*count - size + i) mod capacity (0 = oldest), sample b draws, from the
 * same Philox4x64-10 block as crl_sample_relabel (counter (b, n, 0, 0)):
 *   e = floor(w0 * E / 2^64), i = floor(w1 * (size - 1) / 2^64),
 *   k = 1 + #{m in [1, L - 2] : w2 < thr[m]}  (L = cfg.max_episode_len),
 *   t_g = min(i + k, end(i)), end(i) the last logical index of the run of
 *   i's trajectory id inside the buffer (a step that ends its trajectory
 *   takes itself as goal).
 *   idx   device int32 [B][3] out: (e, ring row of i, ring row of t_g)
 *   x_sa, x_g, x_sg as crl_sample_relabel, gathered from those rows.
 * With fewer than two steps stored nothing is drawn: idx rows are
 * (-1, -1, -1) and the input rows are 0.  The buffer arguments are those of
 * crl_replay_insert; obs_dim and act_dim are the context's. */
CRL_API int crl_ring_sample_relabel(crl_ctx* ctx, const float* obs, const float* act,
                                    const int32_t* traj, int32_t num_envs, int32_t capacity,
                                    const int64_t* count, uint64_t seed, const int64_t* step,
                                    int32_t* idx, void* x_sa, void* x_g, void* x_sg,
                                    void* stream);

/* Step 2: encoders, critic matrix and loss (Section 3.1 objective; Appendix A.2
 * energies and InfoNCE variants; Algorithm 1 critic update with the
 * logsumexp penalty).
 *   params       device FP32 flat parameters (layout above)
 *   params_bf16  device BF16 copy of params (same layout); required when
 *                precision is BF16, ignored for FP32
 *   x_sa, x_g    device inputs as written by crl_sample_relabel
 *   ws           device workspace of crl_workspace_size bytes; keeps the
 *                activations that crl_critic_bwd needs
 *   loss_out     device FP32 [8] out: {total, L_fwd, L_bwd, L_pen,
 *                mean_i r_i, mean_j c_j, #non-finite row/col terms, L_obj}
 *   advance      device int64 (8-byte aligned) or NULL: if given, *advance
 *                is incremented by 1 on the stream after everything above
 *                has read its inputs, in the forward's last kernel (the
 *                update's step counter without a crl_counter_add launch)
 * with F_ij = energy(phi_i, psi_j) (CRL_ENERGY_*), r_i = LSE_j F_ij,
 * c_j = LSE_i F_ij, L_fwd = mean_i (r_i - F_ii), L_bwd = mean_j (c_j - F_jj)
 * (the two InfoNCE directions, reported for every objective),
 * L_pen = beta * mean_i r_i^2, L_obj the objective (CRL_LOSS_*) and
 * total = L_obj + L_pen. */
CRL_API int crl_critic_fwd(crl_ctx* ctx, const float* params,
                           const uint16_t* params_bf16, const void* x_sa,
                           const void* x_g, void* ws, float* loss_out,
                           int64_t* advance, void* stream);

/* Step 3: gradient of loss_out[0] w.r.t. every parameter, written (not
 * accumulated) into grads (device FP32, crl_param_count floats, padding set
 * to 0), by the chain rule through the loss, the energy and both MLPs.  Uses
 * the activations crl_critic_fwd left in ws, so it must follow a
 * crl_critic_fwd with the same params, x_sa, x_g and ws on the same stream. */
CRL_API int crl_critic_bwd(crl_ctx* ctx, const float* params,
                           const uint16_t* params_bf16, const void* x_sa,
                           const void* x_g, void* ws, float* grads,
                           void* stream);

/* Steps 3 and 4 in one call (Algorithm 1, the critic's gradient step): the
 * gradient of crl_critic_bwd, each element fed to the Adam step of
 * crl_adam_step as it is formed (the gradient vector is not read back).
 *   params, params_bf16  updated in place (params_bf16 may be NULL for FP32)
 *   grads                device FP32 [crl_param_count] out, or NULL: then
 *                        the gradient is not kept
 *   m, v, step, lr, b1, b2, eps   as for crl_adam_step, over the whole vector
 * Other arguments as for crl_critic_bwd.  params, m, v and params_bf16 come
 * out bit-identical to crl_critic_bwd followed by crl_adam_step (grads equal
 * as values); the same alignment rules apply. */
CRL_API int crl_critic_bwd_adam(crl_ctx* ctx, float* params,
                                uint16_t* params_bf16, const void* x_sa,
                                const void* x_g, void* ws, float* grads,
                                float* m, float* v, const int64_t* step,
                                double lr, double b1, double b2, double eps,
                                void* stream);

/* The critic matrix and the loss alone, from given representations: the
 * energy and objective steps of crl_critic_fwd / crl_critic_bwd (Section 3.1
 * objective; Appendix A.2 energies and objectives; the logsumexp penalty of
 * Algorithm 1) with phi and psi supplied by the caller instead of the
 * encoders, for tests of the loss on chosen logits (all-zero logits, logits
 * whose row log-sum-exps vanish, B = 1 or 2, large |F|).
 *   phi, psi   device FP32 [B][repr_dim] (read; BF16 precision rounds them
 *              to BF16 tiles as the encoder outputs are)
 *   ws         the context's workspace (r, c and F_ii land in the views
 *              CRL_WS_ROW_LSE, CRL_WS_COL_LSE, CRL_WS_DIAG)
 *   loss_out   device FP32 [8] out, as crl_critic_fwd's
 * crl_infonce_bwd must follow crl_infonce_fwd on the same phi, psi, ws and
 * stream; it writes dL/dphi and dL/dpsi (device FP32 [B][repr_dim], caller
 * owned, not accumulated).  Arguments as for crl_critic_fwd; 16-byte aligned
 * pointers.  Nothing is allocated. */
CRL_API int crl_infonce_fwd(crl_ctx* ctx, const float* phi, const float* psi, void* ws,
                            float* loss_out, void* stream);
CRL_API int crl_infonce_bwd(crl_ctx* ctx, const float* phi, const float* psi, void* ws,
                            float* dphi, float* dpsi, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * crl_infonce_fwd without the workspace argument.  The same kernels run on a
 * static device array of CRL_NOALLOC_SCRATCH_BYTES instead, one per device,
 * which the library holds from its first crl_create on that device until the
 * process ends.  Nothing is allocated or freed by this call (with kernel
 * timing off, the default).
 *   phi, psi    device FP32 [B][repr_dim], 16-byte aligned (read)
 *   loss_out    device FP32 [8] out, as crl_critic_fwd's
 *   r_out, c_out, diag_out   device FP32 [B] out, or NULL: r_i, c_j, F_ii
 * Returns CRL_EINVAL, launching nothing, when the context's loss step needs
 * more scratch than the array holds.  Bytes needed, each buffer rounded up
 * to 256: fused logits 4 B D (BF16 rows) + 8 B (S + ceil(B / 64)) (log-sum-exp
 * partials, S <= 16 column splits) + 28 B (B = 16384 with D = 256 fits);
 * materialised 4 B ldF + 512 B + 28 B, + 8 B D for the cosine energy
 * (B = 2048 fits, B = 4096 does not).  Every call on a device shares its array
 * and leaves its contents there; nothing in it needs to start at zero (every
 * value is written before it is read).  Calls that overlap in time on one
 * device (other streams, other threads) race on the array and must not be
 * issued. */
#define CRL_NOALLOC_SCRATCH_BYTES (64u << 20)
CRL_API int crl_infonce_fwd_noalloc(crl_ctx* ctx, const float* phi, const float* psi,
                                    float* loss_out, float* r_out, float* c_out,
                                    float* diag_out, void* stream);

/* Reads loss_out [8] as a forward left it (crl_critic_fwd, crl_infonce_fwd)
 * after waiting for `stream`: CRL_ENONFINITE if the total is not finite or
 * any row / column term was (loss_out[6] > 0), else CRL_OK.  This call
 * synchronises with the host, so it must not be captured into a graph
 * (CRL_EINVAL while the stream is capturing). */
CRL_API int crl_check_finite(const float* loss_out, void* stream);

/* Policy step (Section 3.2, the policy objective; Algorithm 1 takes it after
 * the critic update, on the same batch; Section 5.1 setup, SAC-style tunable
 * entropy coefficient).  With the critic frozen at `params`:
 *   o = pi_MLP(x_sg) = [mu | rho | pad],  sigma = softplus(rho) + 1e-3,
 *   u = mu + sigma eps,  a' = tanh(u),
 *   log pi = sum_k [log N(u_k; mu_k, sigma_k) - log(1 - tanh^2 u_k)]
 *            (the second term evaluated as 2 (log 2 - u - softplus(-2u))),
 *   f_b = energy(phi(s_b, a'_b), psi(g_b))   (the diagonal of the critic),
 *   L_pi = mean_b [alpha log pi_b - f_b],  alpha = exp(*log_alpha),
 *   L_alpha = -log alpha * (mean_b log pi_b + target_entropy).
 * With cfg.random_goal_ratio = r > 0 (Appendix C, random goals: the policy
 * objective (1 - r) E f(s, a', g) + r E f(s, a', g-) with g- a goal from
 * the buffer's marginal), sample b's goal g (in the policy input [s, g] and
 * in psi(g)) is first replaced by the goal of sample
 * j = (b + 1 + floor(v1 (B - 1) / 2^64)) mod B when
 * floor(v0 / 2^11) < floor(r 2^53), v0, v1 the first two words of the
 * Philox4x64-10 block with counter (b, n, 2, 0), key (seed, 0); with B = 1
 * nothing is replaced.  The goals of a batch are independent draws of the
 * marginal, so the step's estimate is unbiased for the mixed objective. 
 * eps is standard normal from Box-Muller on the Philox4x64-10 stream 1: for
 * sample b the block with counter (b, n, 1, j), key (seed, 0), gives words
 * w0..w3; each word w becomes the uniform (2 floor(w / 2^41) + 1) / 2^24,
 * (w0, w1) and (w2, w3) make the Box-Muller pairs sqrt(-2 ln u1) cos(2 pi u2),
 * sqrt(-2 ln u1) sin(2 pi u2), and coordinates 4j .. 4j+3 take them in order.
 *   params, params_bf16   critic vector (after its Adam step) and BF16 copy
 *   actor_params, actor_params_bf16   policy vector and BF16 copy (BF16 copy
 *                         required when precision is BF16)
 *   log_alpha     device FP32 [1], read
 *   x_sa, x_g, x_sg   the batch as crl_sample_relabel wrote it (x_sg needed);
 *                 the state columns of x_sa are reused for phi(s, a')
 *   seed, step    Philox key word 0 and device batch counter n (read)
 *   ws            the workspace; this call overwrites the critic's saved
 *                 activations, so it must come after crl_critic_bwd
 *   actor_grads   device FP32 out, crl_actor_param_count floats, written (not
 *                 accumulated): dL_pi / d(policy parameters), padding 0
 *   alpha_grad    device FP32 [1] out: dL_alpha / dlog alpha
 *   loss_out      device FP32 [4] out: {L_pi, mean log pi, L_alpha, mean f}
 * EINVAL when the context was created without a policy. */
CRL_API int crl_actor_step(crl_ctx* ctx, const float* params,
                           const uint16_t* params_bf16, const float* actor_params,
                           const uint16_t* actor_params_bf16,
                           const float* log_alpha, const void* x_sa,
                           const void* x_g, const void* x_sg, uint64_t seed,
                           const int64_t* step, void* ws, float* actor_grads,
                           float* alpha_grad, float* loss_out, void* stream);

/* The policy's gradient step in one call (Algorithm 1, the policy update):
 * crl_actor_step with each element of the policy gradient fed to the Adam
 * step of crl_adam_step as it is formed (the gradient vector is not read
 * back).
 *   actor_params, actor_params_bf16   updated in place (the BF16 copy may be
 *                 NULL for FP32)
 *   actor_grads   device FP32 [crl_actor_param_count] out, or NULL: then the
 *                 gradient is not kept
 *   actor_m, actor_v, adam_step, lr, b1, b2, eps   as for crl_adam_step, over
 *                 the whole policy vector (adam_step is the Adam step count t,
 *                 step the batch counter n of the noise draw)
 * Other arguments as for crl_actor_step.  actor_params, actor_m, actor_v and
 * the BF16 copy come out bit-identical to crl_actor_step followed by
 * crl_adam_step on the policy vector; alpha_grad is written as there (the
 * temperature's one-element Adam step stays with crl_adam_step). */
CRL_API int crl_actor_step_adam(crl_ctx* ctx, const float* params,
                                const uint16_t* params_bf16, float* actor_params,
                                uint16_t* actor_params_bf16,
                                const float* log_alpha, const void* x_sa,
                                const void* x_g, const void* x_sg, uint64_t seed,
                                const int64_t* step, void* ws, float* actor_grads,
                                float* alpha_grad, float* loss_out, float* actor_m,
                                float* actor_v, const int64_t* adam_step, double lr,
                                double b1, double b2, double eps, void* stream);

/* Step 4: Adam (Kingma & Ba) on n floats, the optimiser read into the
 * gradient steps of Algorithm 1:
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   p -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * with t = *step (device int64, t >= 1, read only).  The hyperparameters
 * are given in double; 1 - b1, 1 - b2 and log b1, log b2 are formed on the
 * host in double and used in FP32 on the device, so (1 - b2) carries no FP32
 * representation error of b2.  If p_bf16 is not NULL the BF16 copy of the new
 * p is written there too.  p, g, m, v, p_bf16 must
 * be 16-byte aligned. */
CRL_API int crl_adam_step(float* p, const float* g, float* m, float* v,
                          uint16_t* p_bf16, int64_t n, const int64_t* step,
                          double lr, double b1, double b2, double eps,
                          void* stream);

/* *counter += inc on the device (stream-ordered; for step counters that a
 * captured graph advances on every replay). */
CRL_API int crl_counter_add(int64_t* counter, int64_t inc, void* stream);

/* dst[i] = BF16(src[i]) (round to nearest even), n floats, device pointers. */
CRL_API int crl_cast_bf16(const float* src, uint16_t* dst, int64_t n,
                          void* stream);

/* Location of intermediate results inside the workspace, for inspection:
 * byte offset and size of the buffer `which` (CRL_WS_*).  FP32 unless noted. */
enum {
  CRL_WS_PHI = 0,     /* [B][D] phi(s, a) */
  CRL_WS_PSI = 1,     /* [B][D] psi(g) */
  CRL_WS_ROW_LSE = 2, /* [B] r_i */
  CRL_WS_COL_LSE = 3, /* [B] c_j */
  CRL_WS_DIAG = 4,    /* [B] F_ii */
  CRL_WS_DPHI = 5,    /* [B][D] dL/dphi (after crl_critic_bwd) */
  CRL_WS_DPSI = 6,    /* [B][D] dL/dpsi */
  CRL_WS_LOGITS = 7,  /* [B][ldF] F, ldF = B rounded up to a multiple of 8
                         (materialised logits only) */
  /* after crl_actor_step (contexts with a policy only): */
  CRL_WS_POLICY_OUT = 8,    /* [B][P] policy MLP output [mu | rho | pad] */
  CRL_WS_NOISE = 9,         /* [B][act_dim] eps */
  CRL_WS_LOG_PI = 10,       /* [B] log pi */
  CRL_WS_POLICY_ENERGY = 11,/* [B] f_b */
  CRL_WS_DACTION = 12       /* [B][ldd] d(-mean f)/da', ldd = act_dim rounded
                               up to a multiple of 8 */
};
CRL_API int crl_workspace_view(const crl_ctx* ctx, int32_t which,
                               int64_t* offset, int64_t* bytes);

/* Opt-in kernel timing, for measurement.  While enabled, every kernel that
 * the calls above launch outside graph capture is bracketed by HIP events on
 * its own stream and accounted under the kernel's name together with its
 * algorithmic FLOPs and HBM bytes (the minimum the operation must move).
 * crl_timing_read waits for the recorded events (it synchronises with them);
 * nothing else here synchronises.  Process-wide state, guarded by a mutex. */
CRL_API int crl_timing_enable(int32_t enable);
CRL_API int crl_timing_reset(void);
CRL_API int crl_timing_count(int32_t* n);
CRL_API int crl_timing_read(int32_t index, char* name, int32_t name_len,
                            int64_t* launches, double* ms, double* flops,
                            double* bytes);

/* Measured issue rate of one instruction kind on the current device, for
 * the rooflines of kernels bound by it rather than by MFMA or HBM:
 * CRL_RATE_EXP counts v_exp_f32 (the exponential of the log-sum-exp and
 * softmax terms) per second, CRL_RATE_FMA32 FP32 fused multiply-adds per
 * second (unpacked, as this library's vector code issues them).  Runs
 * CRL_RATE_PROBE_BLOCKS workgroups of 256 lanes, each lane 8 independent
 * chains of 4096 instructions, three times on `stream`, and reports the
 * fastest; waits for the stream (not graph-capturable).  scratch: device
 * FP32 [CRL_RATE_PROBE_BLOCKS * 256], overwritten. */
enum { CRL_RATE_EXP = 0, CRL_RATE_FMA32 = 1 };
#define CRL_RATE_PROBE_BLOCKS 8192
CRL_API int crl_peak_rate(int32_t which, float* scratch, double* per_second, void* stream);

/* Message for the last non-OK status returned on this thread. */
CRL_API const char* crl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CRL_H */
