"""Device-resident ring replay buffer: argument marshalling only.

Appending runs ``crl_replay_insert``, sampling ``crl_ring_sample_relabel``
(include/crl.h).  The ring keeps the last `capacity` steps of every
environment (Algorithm 1's buffer; Appendix B: max_replay_size steps per
environment, unroll_length steps of every environment per append), with the
trajectory id of each step so that relabelled goals stay inside the
trajectory of the drawn step (Section 3.2).
"""
from __future__ import annotations

import torch

from .critic import Critic, crl_replay_insert


class ReplayRing:
    """obs [E][C][d_s], act [E][C][d_a] (FP32), traj [E][C] (int32) and the
    per-environment step count (device int64), all in device memory."""

    def __init__(self, num_envs: int, capacity: int, obs_dim: int, act_dim: int,
                 device="cuda:0"):
        dev = torch.device(device)
        self.E, self.C = int(num_envs), int(capacity)
        self.obs = torch.zeros(self.E, self.C, obs_dim, dtype=torch.float32, device=dev)
        self.act = torch.zeros(self.E, self.C, act_dim, dtype=torch.float32, device=dev)
        self.traj = torch.zeros(self.E, self.C, dtype=torch.int32, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)

    def insert(self, new_obs, new_act, new_traj, stream=None):
        """Append U steps of every environment: new_obs [U][E][d_s], new_act
        [U][E][d_a], new_traj [U][E] (device, time-major)."""
        crl_replay_insert(self.obs, self.act, self.traj, new_obs, new_act, new_traj, self.count,
                          stream)

    def sample_relabel(self, crit: Critic, seed: int, step, idx, x_sa, x_g, x_sg=None,
                       stream=None):
        crit.crl_ring_sample_relabel(self.obs, self.act, self.traj, self.count, seed, step, idx,
                                     x_sa, x_g, x_sg, stream)
