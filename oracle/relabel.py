"""Hindsight future-state relabeling, written from the paper's definitions.

Preliminaries: the discounted state-visitation distribution is the law of the
state T steps ahead with T ~ Geom(1 - gamma), and it equals the Q-function of
the goal-reaching reward (Appendix D, "Q-function is probability").
Section 3.2 ("Policy Learning") and Algorithm 1 ("Contrastive Reinforcement
Learning", the update loop) form a batch by drawing (s, a) uniformly from the
buffer and a goal from the *future* of the same trajectory, sampled with
discount.

Readings where the paper is silent (each also listed in the design notes):

* the offset k counts strictly future steps: k in {1, 2, ...} with
  P(k) = (1 - gamma) gamma^(k-1);
* t is uniform on [0, T-2] (the steps that have a future), e uniform on [0, E);
* the goal step is clipped to the episode end: t_g = min(t + k, T - 1);
* the random words come from Philox4x64-10 with key (seed, 0) and counter
  (b, step, stream, 0); word 0 picks e, word 1 picks t, word 2 picks k;
* a word is mapped onto [0, n) by the multiply-high map floor(w n / 2^64);
* k is drawn without floating point: with G = floor(gamma_hat 2^64)
  (gamma_hat the binary64 value of gamma), thr[1] = G and
  thr[m] = floor(thr[m-1] G / 2^64); then k = 1 + #{m >= 1 : w2 < thr[m]},
  so P(k > m) = thr[m] / 2^64 ~ gamma^m.

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

from fractions import Fraction
from typing import List

import numpy as np

from .philox import philox4x64_10, mulhi64

TWO64 = 1 << 64


def geometric_thresholds(gamma: float, count: int) -> List[int]:
    """[thr[1], ..., thr[count]] as Python ints (thr[0] = 2^64 is implicit)."""
    if not (0.0 < gamma < 1.0):
        raise ValueError("gamma must lie in (0, 1)")
    G = int(Fraction(float(gamma)) * TWO64)  # exact floor of gamma_hat * 2^64
    thr = []
    cur = TWO64
    for _ in range(count):
        cur = (cur * G) >> 64
        thr.append(cur)
    return thr


def geometric_offset(w2: int, thr: List[int]) -> int:
    """k = 1 + #{m >= 1 : w2 < thr[m]}, scanning the decreasing table."""
    k = 1
    while k - 1 < len(thr) and w2 < thr[k - 1]:
        k += 1
    return k


def relabel_indices(num_envs: int, episode_len: int, batch: int, gamma: float,
                    seed: int, step: int, stream: int = 0) -> np.ndarray:
    """idx[b] = (e, t, t_g) for b in [0, batch), as int64 [batch, 3]."""
    E, T = int(num_envs), int(episode_len)
    if E < 1 or T < 2:
        raise ValueError("need at least one env and two steps per episode")
    thr = geometric_thresholds(gamma, T - 2)
    idx = np.empty((batch, 3), dtype=np.int64)
    for b in range(batch):
        w0, w1, w2, _ = philox4x64_10((b, step, stream, 0), (seed, 0))
        e = mulhi64(w0, E)
        t = mulhi64(w1, T - 1)
        k = geometric_offset(w2, thr)
        idx[b] = (e, t, min(t + k, T - 1))
    return idx


def gather(obs: np.ndarray, act: np.ndarray, idx: np.ndarray, goal_lo: int,
           goal_dim: int):
    """x_sa = [s_t, a_t], x_g = s_{t_g}[lo:lo+d_g], x_sg = [s_t, x_g] in FP64."""
    e, t, tg = idx[:, 0], idx[:, 1], idx[:, 2]
    s = obs[e, t, :].astype(np.float64)
    a = act[e, t, :].astype(np.float64)
    g = obs[e, tg, goal_lo:goal_lo + goal_dim].astype(np.float64)
    return np.concatenate([s, a], axis=1), g, np.concatenate([s, g], axis=1)


def sample_relabel(obs, act, batch, gamma, seed, step, goal_lo, goal_dim,
                   stream: int = 0):
    """Relabel indices and the gathered encoder inputs for one batch."""
    E, T = obs.shape[0], obs.shape[1]
    idx = relabel_indices(E, T, batch, gamma, seed, step, stream)
    x_sa, x_g, x_sg = gather(obs, act, idx, goal_lo, goal_dim)
    return idx, x_sa, x_g, x_sg


def goal_step_pmf(gamma: float, episode_len: int, t: int) -> dict:
    """Exact law of t_g given t under the threshold table, as Fractions.

    P(k > m) = thr[m] / 2^64 (thr[0] = 2^64); t_g = t + k below the last
    step, and every k >= T-1-t lands on T-1.
    """
    T = int(episode_len)
    thr = [TWO64] + geometric_thresholds(gamma, T - 2)
    pmf = {}
    for j in range(t + 1, T - 1):
        k = j - t
        pmf[j] = Fraction(thr[k - 1] - thr[k], TWO64)
    pmf[T - 1] = Fraction(thr[T - 2 - t], TWO64)
    return pmf
