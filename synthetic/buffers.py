"""Seeded synthetic replay buffers.

The paper's buffers hold simulator trajectories (Brax / MJX), which are not
available; these generators stand in for them with trajectories of the same
shape: ``obs[E][T][d_s]`` and ``act[E][T][d_a]``, FP32, row-major, one episode
per environment row.  Two state processes are provided:

* ``random_walk``: s_0 ~ N(0, I), s_{t+1} = s_t + std * N(0, I)
* ``ar1``:         s_0 ~ N(0, std^2 / (1 - rho^2) I) (the stationary law),
                   s_{t+1} = rho * s_t + std * N(0, I)

Actions are i.i.d. uniform on [-1, 1].  Everything is drawn from
``numpy.random.default_rng`` streams spawned from ``SeedSequence(seed)``, one
per fixed chunk of envs, so a buffer is a pure function of (shape, process,
seed).
"""
from __future__ import annotations

from concurrent.futures import ThreadPoolExecutor

import numpy as np

from .workloads import Workload

_CHUNK = 256


def _fill_chunk(obs, act, e0, e1, seq, states, rw_std, ar_rho, ar_std):
    rng = np.random.default_rng(seq)
    n, T, obs_dim = e1 - e0, obs.shape[1], obs.shape[2]
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
    u = rng.random((n, T, act.shape[2]), dtype=np.float32)
    act[e0:e1] = u * np.float32(2.0) - np.float32(1.0)


def make_buffer(num_envs: int, episode_len: int, obs_dim: int, act_dim: int,
                states: str = "random_walk", seed: int = 0, rw_std: float = 0.1,
                ar_rho: float = 0.99, ar_std: float = 0.05, threads: int = 8):
    """Return (obs, act) as C-contiguous float32 arrays [E,T,d_s], [E,T,d_a].

    Env chunk c draws from its own child of SeedSequence(seed), so the result
    does not depend on how many threads fill the chunks.
    """
    E, T = int(num_envs), int(episode_len)
    if states not in ("random_walk", "ar1"):
        raise ValueError(f"unknown state process {states!r}")
    obs = np.empty((E, T, obs_dim), dtype=np.float32)
    act = np.empty((E, T, act_dim), dtype=np.float32)
    starts = list(range(0, E, _CHUNK))
    seqs = np.random.SeedSequence(seed).spawn(len(starts))
    jobs = [(obs, act, e0, min(E, e0 + _CHUNK), sq, states, rw_std, ar_rho, ar_std)
            for e0, sq in zip(starts, seqs)]
    if threads > 1 and len(jobs) > 1:
        with ThreadPoolExecutor(max_workers=min(threads, len(jobs))) as ex:
            list(ex.map(lambda j: _fill_chunk(*j), jobs))
    else:
        for j in jobs:
            _fill_chunk(*j)
    return obs, act


def buffer_for(w: Workload, seed: int = 0, num_envs: int | None = None,
               episode_len: int | None = None):
    """Buffer of a workload's shape (optionally with fewer envs / steps)."""
    return make_buffer(num_envs or w.num_envs, episode_len or w.episode_len,
                       w.obs_dim, w.act_dim, states=w.states, seed=seed,
                       rw_std=w.rw_std, ar_rho=w.ar_rho, ar_std=w.ar_std)
