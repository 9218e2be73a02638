"""One contrastive-RL critic update as a sequence of C-ABI calls.

Algorithm 1 (the update loop): sample a batch with hindsight goals, take the
critic gradient step on the InfoNCE + logsumexp objective.  The batch counter
n (the Philox counter word) and the Adam step t live in device memory and are
advanced by the library on the stream, so the same enqueued sequence can be
captured once into a HIP graph and replayed for consecutive updates.
"""
from __future__ import annotations

import torch

from .critic import Critic, crl_adam_step, crl_cast_bf16, crl_counter_add


class CriticUpdate:
    """Device state of the critic update: parameters, Adam moments, batch."""

    def __init__(self, w, obs: torch.Tensor, act: torch.Tensor, phi_layers, psi_layers,
                 seed: int = 2, lr: float | None = None, device="cuda:0"):
        self.w = w
        self.dev = torch.device(device)
        self.obs, self.act = obs, act
        self.seed = int(seed)
        self.lr = float(w.critic_lr if lr is None else lr)
        self.crit = Critic(w, max_episode_len=obs.shape[1])
        c = self.crit
        self.params = torch.from_numpy(c.pack(phi_layers, psi_layers)).to(self.dev)
        self.pbf = None
        if w.precision == "bf16":
            self.pbf = torch.empty(c.nparam, dtype=torch.bfloat16, device=self.dev)
            crl_cast_bf16(self.params, self.pbf)
        self.grads = torch.zeros(c.nparam, dtype=torch.float32, device=self.dev)
        self.m = torch.zeros_like(self.grads)
        self.v = torch.zeros_like(self.grads)
        self.x_sa, self.x_g, self.x_sg = c.inputs(self.dev)
        self.idx = torch.zeros(w.batch_size, 3, dtype=torch.int32, device=self.dev)
        self.ws = c.workspace(self.dev)
        self.loss = torch.zeros(8, dtype=torch.float32, device=self.dev)
        self.n = torch.zeros(1, dtype=torch.int64, device=self.dev)  # batch counter
        self.t = torch.zeros(1, dtype=torch.int64, device=self.dev)  # Adam step

    def enqueue(self):
        """Enqueue one full update on the current stream (no host sync)."""
        c = self.crit
        c.crl_sample_relabel(self.obs, self.act, self.seed, self.n, self.idx, self.x_sa,
                             self.x_g, None)
        c.crl_critic_fwd(self.params, self.pbf, self.x_sa, self.x_g, self.ws, self.loss)
        c.crl_critic_bwd(self.params, self.pbf, self.x_sa, self.x_g, self.ws, self.grads)
        crl_counter_add(self.t, 1)
        crl_adam_step(self.params, self.grads, self.m, self.v, self.pbf, self.t, self.lr)
        crl_counter_add(self.n, 1)

    def capture(self, steps: int = 1) -> torch.cuda.CUDAGraph:
        """A HIP graph of `steps` consecutive updates (replay advances n, t)."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for _ in range(steps):
                    self.enqueue()
        torch.cuda.current_stream().wait_stream(s)
        return g

    def close(self):
        self.crit.close()


def critic_step_flops(w) -> dict:
    """Algorithmic FLOPs of one critic update (2 per multiply-add).

    Encoders: forward x W per layer; backward dW for every layer and dX for
    every layer but the first.  Critic matrix: 2 B^2 D forward, 4 B^2 D
    backward (dphi and dpsi); tile recomputation is not counted.
    """
    B, D = w.batch_size, w.repr_dim
    fwd = bwd = 0
    for fan0 in (w.in_sa, w.goal_dim):
        dims = [fan0, *w.hidden, D]
        macs = [dims[i] * dims[i + 1] for i in range(len(dims) - 1)]
        fwd += 2 * B * sum(macs)
        bwd += 2 * B * sum(macs) + 2 * B * sum(macs[1:])
    logits_f = 2 * B * B * D
    logits_b = 4 * B * B * D
    return {"enc_fwd": fwd, "enc_bwd": bwd, "logits_fwd": logits_f, "logits_bwd": logits_b,
            "total": fwd + bwd + logits_f + logits_b}


def adam_bytes(nparam: int, shadow: bool) -> int:
    return nparam * (28 + (2 if shadow else 0))
