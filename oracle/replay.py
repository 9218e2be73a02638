"""The replay buffer as a ring of trajectory steps, and hindsight relabeling
inside it, written from the paper's description.

Algorithm 1 ("Contrastive Reinforcement Learning"): every environment appends
its (s, a) steps to its current trajectory, a terminal step starts a new one,
and the buffer D keeps what was stored.  The benchmark parameters (Appendix B,
"Benchmark parameters", the hyperparameter table) bound the buffer per
environment (max_replay_size steps) and append unroll_length steps of every
environment at a time.  Section 3.2 ("Policy Learning") draws (s, a)
uniformly and the goal from the states after s *in the same trajectory*.

Readings where the paper is silent (each also listed in the design notes):

* storage: per environment e, a ring of `capacity` steps; after n steps per
  environment have been appended (all environments append together), the
  buffer holds the last size = min(n, capacity) of them, absolute step a at
  ring row a mod capacity.  Logical index i in [0, size) is absolute step
  n - size + i (0 = oldest);
* every step carries a trajectory id; within one environment the ids never
  decrease in append order, and a trajectory is a maximal run of equal ids;
* e is uniform on [0, E) (word 0), the logical index i uniform on
  [0, size - 2] (word 1; the newest step has no successor in the buffer);
* k = 1 + #{m in [1, L-2] : w2 < thr[m]} with the threshold table of
  ``relabel.geometric_thresholds`` (L the longest episode the sampler is set
  up for, so k <= L - 1), and the goal step is clipped to the end of i's
  trajectory inside the buffer: t_g = min(i + k, end(i)), end(i) the last
  logical index of the run of i's id.  A step that ends its trajectory gets
  t_g = i;
* with fewer than two steps stored nothing is drawn: the index rows are
  (-1, -1, -1) and the gathered rows are zero.

With one trajectory per environment and n <= capacity this is exactly the
single-episode law of ``relabel.relabel_indices`` (end(i) = T - 1).

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import numpy as np

from .philox import mulhi64, philox4x64_10
from .relabel import geometric_offset, geometric_thresholds


class RingBuffer:
    """obs [E][C][d_s], act [E][C][d_a] (float32) and traj [E][C] (int32)."""

    def __init__(self, num_envs: int, capacity: int, obs_dim: int, act_dim: int):
        if num_envs < 1 or capacity < 2:
            raise ValueError("need at least one env and a capacity of two steps")
        self.E, self.C = int(num_envs), int(capacity)
        self.obs = np.zeros((self.E, self.C, obs_dim), np.float32)
        self.act = np.zeros((self.E, self.C, act_dim), np.float32)
        self.traj = np.zeros((self.E, self.C), np.int32)
        self.count = 0  # steps appended per environment so far

    def insert(self, new_obs, new_act, new_traj):
        """Append U steps of every environment: new_* are [U][E][...] (time-major)."""
        U = new_obs.shape[0]
        if not (1 <= U <= self.C):
            raise ValueError("a chunk holds 1..capacity steps")
        for u in range(U):
            row = (self.count + u) % self.C
            self.obs[:, row, :] = new_obs[u]
            self.act[:, row, :] = new_act[u]
            self.traj[:, row] = new_traj[u]
        self.count += U

    @property
    def size(self) -> int:
        return min(self.count, self.C)

    def row_of(self, i: int) -> int:
        """Ring row of logical index i (0 = oldest stored step)."""
        return (self.count - self.size + i) % self.C


def trajectory_end(traj_e, buf: RingBuffer, i: int) -> int:
    """Last logical index j >= i with the same trajectory id on every step of [i, j]."""
    tid = traj_e[buf.row_of(i)]
    j = i
    while j + 1 < buf.size and traj_e[buf.row_of(j + 1)] == tid:
        j += 1
    return j


def ring_relabel_indices(buf: RingBuffer, batch: int, gamma: float, max_episode_len: int,
                         seed: int, step: int, stream: int = 0) -> np.ndarray:
    """idx[b] = (e, ring row of i, ring row of t_g), int64 [batch, 3]."""
    size = buf.size
    idx = np.full((batch, 3), -1, dtype=np.int64)
    if size < 2:
        return idx
    thr = geometric_thresholds(gamma, max(0, int(max_episode_len) - 2))
    for b in range(batch):
        w0, w1, w2, _ = philox4x64_10((b, step, stream, 0), (seed, 0))
        e = mulhi64(w0, buf.E)
        i = mulhi64(w1, size - 1)
        k = geometric_offset(w2, thr)
        tg = min(i + k, trajectory_end(buf.traj[e], buf, i))
        idx[b] = (e, buf.row_of(i), buf.row_of(tg))
    return idx


def ring_sample_relabel(buf: RingBuffer, batch: int, gamma: float, max_episode_len: int,
                        seed: int, step: int, goal_lo: int, goal_dim: int):
    """Indices and the gathered encoder inputs x_sa, x_g, x_sg (FP64)."""
    idx = ring_relabel_indices(buf, batch, gamma, max_episode_len, seed, step)
    d_s, d_a = buf.obs.shape[2], buf.act.shape[2]
    x_sa = np.zeros((batch, d_s + d_a))
    x_g = np.zeros((batch, goal_dim))
    ok = idx[:, 0] >= 0
    e, r, rg = idx[ok, 0], idx[ok, 1], idx[ok, 2]
    x_sa[ok, :d_s] = buf.obs[e, r, :]
    x_sa[ok, d_s:] = buf.act[e, r, :]
    x_g[ok] = buf.obs[e, rg, goal_lo:goal_lo + goal_dim]
    x_sg = np.concatenate([x_sa[:, :d_s], x_g], axis=1)
    return idx, x_sa, x_g, x_sg
