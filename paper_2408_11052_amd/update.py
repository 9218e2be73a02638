"""One contrastive-RL update as a sequence of C-ABI calls.

Algorithm 1 (the update loop): sample a batch with hindsight goals, take the
critic gradient step on the InfoNCE + logsumexp objective, then (FullUpdate)
the policy step on the same batch with the updated critic, and the step of
the entropy coefficient.  The batch counter
n (the Philox counter word) and the Adam step t live in device memory and are
advanced by the library on the stream, so the same enqueued sequence can be
captured once into a HIP graph and replayed for consecutive updates.  In the
critic-only update t is n itself: the critic forward's last kernel advances n
after the relabelling has read it, so the Adam step of update k sees k + 1, as
a separate step counter would (the full update's forward advances its own t).

The batch comes either from a static buffer of one episode per environment
row, or from a ReplayRing; with a ring, ``capture_iteration`` records one
training iteration of Algorithm 1's outer loop as a graph: the append of a
freshly unrolled chunk of every environment's steps followed by a given
number of updates on the grown buffer (the update-to-data ratio).
"""
from __future__ import annotations

import torch

from .critic import Critic, crl_adam_step, crl_cast_bf16, crl_counter_add
from .replay import ReplayRing


class CriticUpdate:
    """Device state of the critic update: parameters, Adam moments, batch."""

    def __init__(self, w, obs, act, phi_layers, psi_layers,
                 seed: int = 2, lr: float | None = None, device="cuda:0",
                 keep_grads: bool = True):
        """obs, act: the static buffer [E][T][d] (one episode per row), or
        obs a ReplayRing and act None (goals clipped to the longest episode
        w.episode_len and to the end of the drawn step's trajectory).
        keep_grads: also store each update's critic gradient in self.grads
        (the Adam step takes it as it is formed either way)."""
        self.w = w
        self.keep_grads = bool(keep_grads)
        self.dev = torch.device(device)
        self.ring = obs if isinstance(obs, ReplayRing) else None
        self.obs, self.act = (None, None) if self.ring is not None else (obs, act)
        self.seed = int(seed)
        self.lr = float(w.critic_lr if lr is None else lr)
        max_len = w.episode_len if self.ring is not None else obs.shape[1]
        self.crit = Critic(w, max_episode_len=max_len)
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
        self.t = self.n  # Adam step (the full update keeps its own)

    def _critic_fwd(self, x_sg, advance):
        """Relabel (reads n), then the critic forward, whose last kernel
        advances the counter `advance`."""
        c = self.crit
        if self.ring is not None:
            self.ring.sample_relabel(c, self.seed, self.n, self.idx, self.x_sa, self.x_g, x_sg)
        else:
            c.crl_sample_relabel(self.obs, self.act, self.seed, self.n, self.idx, self.x_sa,
                                 self.x_g, x_sg)
        c.crl_critic_fwd(self.params, self.pbf, self.x_sa, self.x_g, self.ws, self.loss, advance)

    def _critic_step(self):
        """The critic gradient fed into its Adam step (step t)."""
        self.crit.crl_critic_bwd_adam(self.params, self.pbf, self.x_sa, self.x_g, self.ws,
                                      self.grads if self.keep_grads else None, self.m, self.v,
                                      self.t, self.lr)

    def enqueue(self):
        """Enqueue one critic update on the current stream (no host sync)."""
        self._critic_fwd(None, self.n)  # n is also the Adam step
        self._critic_step()

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

    def enqueue_iteration(self, new_obs, new_act, new_traj, updates: int):
        """Append one chunk ([U][E][...], time-major) to the ring, then
        `updates` consecutive updates on the grown buffer."""
        if self.ring is None:
            raise ValueError("iterations need a ReplayRing buffer")
        self.ring.insert(new_obs, new_act, new_traj)
        for _ in range(updates):
            self.enqueue()

    def capture_iteration(self, new_obs, new_act, new_traj, updates: int,
                          iterations: int = 1) -> torch.cuda.CUDAGraph:
        """A HIP graph of `iterations` x (append the chunk held in new_*,
        then `updates` updates).  The chunk buffers are read at replay time,
        so the caller refills them between replays as the environments
        produce steps; the ring's count, n and t advance on the device."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                for _ in range(iterations):
                    self.enqueue_iteration(new_obs, new_act, new_traj, updates)
        torch.cuda.current_stream().wait_stream(s)
        return g

    def close(self):
        self.crit.close()


class FullUpdate(CriticUpdate):
    """Critic update, then the policy and entropy-coefficient steps (the
    policy's Adam step taken inside its gradient reduction; with keep_grads
    the policy gradient is stored in self.agrads as well).

    log alpha and its Adam moments are 4-float vectors so that they meet the
    16-byte alignment of crl_adam_step; only element 0 is used (the others
    have zero gradient and stay 0).
    """

    def __init__(self, w, obs, act, phi_layers, psi_layers, actor_layers, seed: int = 2,
                 log_alpha: float = 0.0, device="cuda:0", keep_grads: bool = True):
        super().__init__(w, obs, act, phi_layers, psi_layers, seed=seed, device=device,
                         keep_grads=keep_grads)
        c = self.crit
        if not c.has_actor:
            raise ValueError("the workload has no policy (actor_hidden is empty)")
        self.policy_lr = float(w.policy_lr)
        self.alpha_lr = float(w.alpha_lr)
        self.aparams = torch.from_numpy(c.pack_actor(actor_layers)).to(self.dev)
        self.apbf = None
        if w.precision == "bf16":
            self.apbf = torch.empty(c.nparam_actor, dtype=torch.bfloat16, device=self.dev)
            crl_cast_bf16(self.aparams, self.apbf)
        self.agrads = torch.zeros_like(self.aparams)
        self.am = torch.zeros_like(self.aparams)
        self.av = torch.zeros_like(self.aparams)
        self.log_alpha = torch.zeros(4, dtype=torch.float32, device=self.dev)
        self.log_alpha[0] = float(log_alpha)
        self.alpha_grad = torch.zeros(4, dtype=torch.float32, device=self.dev)
        self.m_alpha = torch.zeros(4, dtype=torch.float32, device=self.dev)
        self.v_alpha = torch.zeros(4, dtype=torch.float32, device=self.dev)
        self.actor_loss = torch.zeros(4, dtype=torch.float32, device=self.dev)
        # the policy step reads n after the critic's Adam step: t is its own counter
        self.t = torch.zeros(1, dtype=torch.int64, device=self.dev)

    def enqueue(self):
        """Enqueue one full update (critic, policy, alpha) on the current stream."""
        c = self.crit
        self._critic_fwd(self.x_sg, self.t)
        self._critic_step()
        c.crl_actor_step_adam(self.params, self.pbf, self.aparams, self.apbf, self.log_alpha,
                              self.x_sa, self.x_g, self.x_sg, self.seed, self.n, self.ws,
                              self.agrads if self.keep_grads else None, self.alpha_grad,
                              self.actor_loss, self.am, self.av, self.t, self.policy_lr)
        crl_adam_step(self.log_alpha, self.alpha_grad, self.m_alpha, self.v_alpha, None,
                      self.t, self.alpha_lr)
        crl_counter_add(self.n, 1)


def _mlp_macs(dims) -> list:
    return [dims[i] * dims[i + 1] for i in range(len(dims) - 1)]


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


def actor_step_flops(w) -> dict:
    """Algorithmic FLOPs of one policy step (2 per multiply-add).

    Policy MLP forward and backward (dW every layer, dX all but the first);
    the frozen critic's phi and psi forward on (s, a') and g; the input
    gradient of phi down to the action columns.
    """
    B, D, A = w.batch_size, w.repr_dim, w.act_dim
    pol = _mlp_macs([w.in_sg, *w.actor_hidden, 2 * A])
    phi = _mlp_macs([w.in_sa, *w.hidden, D])
    psi = _mlp_macs([w.goal_dim, *w.hidden, D])
    pol_f = 2 * B * sum(pol)
    pol_b = 2 * B * sum(pol) + 2 * B * sum(pol[1:])
    crit_f = 2 * B * (sum(phi) + sum(psi))
    phi_dx = 2 * B * sum(phi[1:]) + 2 * B * w.hidden[0] * A
    return {"policy_fwd": pol_f, "policy_bwd": pol_b, "critic_fwd": crit_f,
            "phi_input_grad": phi_dx, "total": pol_f + pol_b + crit_f + phi_dx}


def adam_bytes(nparam: int, shadow: bool) -> int:
    return nparam * (28 + (2 if shadow else 0))
