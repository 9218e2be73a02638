"""Workload descriptions for the contrastive-RL critic update.

Each workload fixes the replay-buffer shape, the synthetic state process, the
batch size and the encoder architecture.  These are plain records: nothing
here computes any part of the method.  Field names follow the hyperparameter
table of the paper (Appendix B.3, "Benchmark parameters": ``batch_size``,
``discounting``, ``energy_function``, ``contrastive_loss_function``,
``logsumexp_penalty``, hidden layers, representation dimension).
"""
from __future__ import annotations

from dataclasses import dataclass, replace
from typing import Tuple


@dataclass(frozen=True)
class Workload:
    name: str
    # replay buffer: E environments x T steps, one episode per env row
    num_envs: int
    episode_len: int
    obs_dim: int
    act_dim: int
    goal_dim: int
    goal_lo: int
    states: str              # "random_walk" | "ar1"
    # batch and networks
    batch_size: int
    hidden: Tuple[int, ...]  # hidden widths of each encoder
    activation: str          # "relu" | "ln_swish"
    repr_dim: int
    energy_function: str     # "dot" | "l2" | "cos" | "l2sq" | "l1"
    # "fwd_infonce" | "symmetric_infonce" | "bwd_infonce" | "flatnce_fwd" |
    # "flatnce_bwd" | "fb" | "dpo" | "ipo" | "sppo"
    contrastive_loss_function: str
    logsumexp_penalty: float = 0.1
    discounting: float = 0.99
    precision: str = "fp32"  # arithmetic of the GEMM/logit tiles: "fp32" | "bf16"
    logits: str = "materialised"  # "materialised" | "fused"
    critic_lr: float = 3e-4
    policy_lr: float = 6e-4
    ln_eps: float = 1e-6
    # state processes
    rw_std: float = 0.1
    ar_rho: float = 0.99
    ar_std: float = 0.05
    # actor (full update only)
    actor_hidden: Tuple[int, ...] = ()
    alpha_lr: float = 3e-4
    # share of the policy's goals replaced by another sample's (0 = none)
    random_goal_ratio: float = 0.0

    @property
    def in_sa(self) -> int:
        return self.obs_dim + self.act_dim

    @property
    def in_sg(self) -> int:
        return self.obs_dim + self.goal_dim

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# 256 envs x 1001 steps random walk, B=256, [256,256] ReLU, L2, symmetric.
SMALL_RELU = Workload(
    name="b256_relu2x256_l2_sym", num_envs=256, episode_len=1001, obs_dim=29,
    act_dim=8, goal_dim=2, goal_lo=0, states="random_walk", batch_size=256,
    hidden=(256, 256), activation="relu", repr_dim=64, energy_function="l2",
    contrastive_loss_function="symmetric_infonce", precision="fp32")

# 1024 envs x 1001 steps, B=1024, 4x1024 LN+Swish, L2, forward InfoNCE, FP32.
LN_FWD_FP32 = Workload(
    name="b1024_lnswish4x1024_l2_fwd", num_envs=1024, episode_len=1001,
    obs_dim=29, act_dim=8, goal_dim=2, goal_lo=0, states="random_walk",
    batch_size=1024, hidden=(1024,) * 4, activation="ln_swish", repr_dim=64,
    energy_function="l2", contrastive_loss_function="fwd_infonce",
    precision="fp32")

# 4096 envs x 1000 steps AR(1) states of dim 268, B=4096, 4x1024 LN+Swish,
# dot energy, symmetric InfoNCE, BF16 tiles.  The headline workload.
DOT_B4096_BF16 = Workload(
    name="b4096_lnswish4x1024_dot_sym", num_envs=4096, episode_len=1000,
    obs_dim=268, act_dim=17, goal_dim=3, goal_lo=0, states="ar1",
    batch_size=4096, hidden=(1024,) * 4, activation="ln_swish", repr_dim=64,
    energy_function="dot", contrastive_loss_function="symmetric_infonce",
    precision="bf16", logits="fused")

# The same workload on the plain path: FP32 tiles, B x B logits materialised.
DOT_B4096_FP32 = DOT_B4096_BF16.with_(
    name="b4096_lnswish4x1024_dot_sym_fp32", precision="fp32",
    logits="materialised")

# Large-batch fused path: B=16384, D=256, 2x1024, L2, symmetric.
L2_B16384_FUSED = Workload(
    name="b16384_lnswish2x1024_d256_l2_sym", num_envs=2048, episode_len=1000,
    obs_dim=67, act_dim=8, goal_dim=2, goal_lo=0, states="random_walk",
    batch_size=16384, hidden=(1024,) * 2, activation="ln_swish", repr_dim=256,
    energy_function="l2", contrastive_loss_function="symmetric_infonce",
    precision="bf16", logits="fused")

# Full update: the B=4096 critic plus a 4x1024 tanh-Gaussian actor.
FULL_UPDATE_B4096 = DOT_B4096_BF16.with_(
    name="b4096_full_update_actor4x1024", actor_hidden=(1024,) * 4)

ALL = {w.name: w for w in (SMALL_RELU, LN_FWD_FP32, DOT_B4096_BF16,
                           DOT_B4096_FP32, L2_B16384_FUSED, FULL_UPDATE_B4096)}
