"""One full contrastive-RL update in FP64: critic step, then actor step, then
the entropy-coefficient step (Algorithm 1: sample a batch with hindsight
goals, update the critic, update the policy; the policy step uses the critic
after its update).  With a random-goal ratio the policy step takes the goals
mixed as in ``actor.random_goal_mix`` (Appendix C).

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import math

import numpy as np

from . import actor as A
from . import adam as AD
from . import critic as C
from . import relabel as R


def _to64(layers):
    return [{k: np.asarray(v, np.float64).copy() for k, v in L.items()} for L in layers]


class FullUpdate:
    """Parameters and Adam state of critic, actor and log alpha."""

    def __init__(self, w, phi, psi, actor, seed: int = 2, log_alpha: float = 0.0):
        self.w = w
        self.phi, self.psi, self.actor = _to64(phi), _to64(psi), _to64(actor)
        self.seed = seed
        self.log_alpha = float(log_alpha)
        self.mc = [[{k: np.zeros_like(v) for k, v in L.items()} for L in g]
                   for g in (self.phi, self.psi)]
        self.vc = [[{k: np.zeros_like(v) for k, v in L.items()} for L in g]
                   for g in (self.phi, self.psi)]
        self.ma = [{k: np.zeros_like(v) for k, v in L.items()} for L in self.actor]
        self.va = [{k: np.zeros_like(v) for k, v in L.items()} for L in self.actor]
        self.m_alpha = 0.0
        self.v_alpha = 0.0
        self.t = 0

    def step(self, obs, act, n: int):
        w = self.w
        self.t += 1
        _, x_sa, x_g, x_sg = R.sample_relabel(obs, act, w.batch_size, w.discounting, self.seed,
                                              n, w.goal_lo, w.goal_dim)
        crit = C.critic_loss_and_grads(self.phi, self.psi, x_sa, x_g, w)
        for gi, (layers, grads) in enumerate(((self.phi, crit["g_phi"]),
                                              (self.psi, crit["g_psi"]))):
            for l, L in enumerate(layers):
                for k in L:
                    L[k], self.mc[gi][l][k], self.vc[gi][l][k] = AD.adam_step(
                        L[k], grads[l][k], self.mc[gi][l][k], self.vc[gi][l][k], self.t,
                        w.critic_lr)
        eps = A.box_muller_noise(self.seed, n, w.batch_size, w.act_dim)
        obs_t = x_sa[:, :w.obs_dim]
        ratio = float(getattr(w, "random_goal_ratio", 0.0))
        if ratio > 0.0:  # Appendix C: the policy's goals mixed with random ones
            x_sg, x_g, _, _ = A.random_goal_mix(x_sg, x_g, w.obs_dim, ratio, self.seed, n)
        la_used = self.log_alpha
        act_out = A.actor_loss_and_grads(self.actor, self.phi, self.psi, x_sg, x_g, obs_t, eps,
                                         la_used, w)
        for l, L in enumerate(self.actor):
            for k in L:
                L[k], self.ma[l][k], self.va[l][k] = AD.adam_step(
                    L[k], act_out["g_actor"][l][k], self.ma[l][k], self.va[l][k], self.t,
                    w.policy_lr)
        la, m, v = AD.adam_step(np.array([self.log_alpha]), np.array([act_out["d_log_alpha"]]),
                                np.array([self.m_alpha]), np.array([self.v_alpha]), self.t,
                                w.alpha_lr)
        self.log_alpha, self.m_alpha, self.v_alpha = float(la[0]), float(m[0]), float(v[0])
        return {"critic": crit["total"], "actor": act_out["loss"],
                "mean_log_pi": act_out["mean_log_pi"], "mean_f": float(np.mean(act_out["f"])),
                "alpha": math.exp(la_used), "log_alpha": self.log_alpha}
