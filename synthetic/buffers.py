"""Seeded synthetic replay buffers.

The paper's buffers hold simulator trajectories (Brax / MJX), which are not
available; these generators stand in for them with trajectories of the same
shape: ``obs[E][T][d_s]`` and ``act[E][T][d_a]``, FP32, row-major, one episode
per environment row.  Two state processes are provided:

* ``random_walk``: s_0 ~ N(0, I), s_{t+1} = s_t + std * N(0, I)
* ``ar1``:         s_0 ~ N(0, std^2 / (1 - rho^2) I) (the stationary law),
                   s_{t+1} = rho * s_t + std * N(0, I)

Actions are i.i.d. uniform on [-1, 1].  Everything is drawn from
``numpy.random.default_rng(seed)`` in fixed env chunks, so a buffer is a pure
function of (shape, process, seed).
"""
from __future__ import annotations

import numpy as np

from .workloads import Workload

_CHUNK = 128


def make_buffer(num_envs: int, episode_len: int, obs_dim: int, act_dim: int,
                states: str = "random_walk", seed: int = 0, rw_std: float = 0.1,
                ar_rho: float = 0.99, ar_std: float = 0.05):
    """Return (obs, act) as C-contiguous float32 arrays [E,T,d_s], [E,T,d_a]."""
    E, T = int(num_envs), int(episode_len)
    rng = np.random.default_rng(seed)
    obs = np.empty((E, T, obs_dim), dtype=np.float32)
    act = np.empty((E, T, act_dim), dtype=np.float32)
    for e0 in range(0, E, _CHUNK):
        e1 = min(E, e0 + _CHUNK)
        n = e1 - e0
        noise = rng.standard_normal((n, T, obs_dim), dtype=np.float32)
        if states == "random_walk":
            noise[:, 1:, :] *= np.float32(rw_std)
            np.cumsum(noise, axis=1, out=obs[e0:e1])
        elif states == "ar1":
            rho = np.float32(ar_rho)
            std = np.float32(ar_std)
            s = noise[:, 0, :] * np.float32(ar_std / np.sqrt(1.0 - ar_rho * ar_rho))
            obs[e0:e1, 0, :] = s
            for t in range(1, T):
                s = rho * s + std * noise[:, t, :]
                obs[e0:e1, t, :] = s
        else:
            raise ValueError(f"unknown state process {states!r}")
        u = rng.random((n, T, act_dim), dtype=np.float32)
        act[e0:e1] = u * np.float32(2.0) - np.float32(1.0)
    return obs, act


def buffer_for(w: Workload, seed: int = 0, num_envs: int | None = None,
               episode_len: int | None = None):
    """Buffer of a workload's shape (optionally with fewer envs / steps)."""
    return make_buffer(num_envs or w.num_envs, episode_len or w.episode_len,
                       w.obs_dim, w.act_dim, states=w.states, seed=seed,
                       rw_std=w.rw_std, ar_rho=w.ar_rho, ar_std=w.ar_std)
