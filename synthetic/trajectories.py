"""Seeded synthetic environment steps, time-major, with episode boundaries.

Stands in for the simulator's unrolls (the paper's environments run in
Brax / MJX, which are not available): a stream of `n_steps` steps of every
environment, obs [n][E][d_s], act [n][E][d_a] (float32) and the trajectory
id of each step, traj [n][E] (int32).  Each environment runs episodes one
after the other; an episode's states are a random walk that restarts from
N(0, I) at its first step, actions are i.i.d. uniform on [-1, 1], and the
trajectory id counts the environment's episodes (so it never decreases).

Episode lengths: `episode_len` fixed (an int), with each environment's first
episode cut to a uniform length in [1, episode_len] so that resets are
staggered across environments as in a vectorised simulator; or drawn
uniformly from [lo, hi] for every episode (a tuple).  Nothing here computes
any part of the method.
"""
from __future__ import annotations

import numpy as np


def unroll_stream(num_envs: int, n_steps: int, obs_dim: int, act_dim: int, episode_len,
                  seed: int = 0, rw_std: float = 0.1):
    rng = np.random.default_rng(seed)
    E, n = int(num_envs), int(n_steps)
    fixed = isinstance(episode_len, (int, np.integer))
    # episode starts: start[t, e] is True where step t opens an episode of env e
    start = np.zeros((n, E), bool)
    for e in range(E):
        t = 0
        first = True
        while t < n:
            start[t, e] = True
            if fixed:
                L = int(rng.integers(1, episode_len + 1)) if first else int(episode_len)
            else:
                L = int(rng.integers(episode_len[0], episode_len[1] + 1))
            t += L
            first = False
    traj = (np.cumsum(start, axis=0) - 1).astype(np.int32)
    noise = rng.standard_normal((n, E, obs_dim), dtype=np.float32)
    # random walk restarted at each episode start: s_t = sum of the episode's
    # increments so far (the first one is the N(0, I) start state)
    inc = noise * np.float32(rw_std)
    inc[start] = noise[start]
    csum = np.cumsum(inc, axis=0, dtype=np.float32)
    t_idx = np.arange(n)[:, None]
    seg0 = np.maximum.accumulate(np.where(start, t_idx, 0), axis=0)   # first step of each step's episode
    base = csum[np.maximum(seg0 - 1, 0), np.arange(E)[None, :]]       # [n][E][d_s]
    base[seg0 == 0] = 0.0
    obs = (csum - base).astype(np.float32)
    act = (rng.random((n, E, act_dim), dtype=np.float32) * np.float32(2.0)
           - np.float32(1.0))
    return obs, act, traj
