"""Pin for the oracle's full update (no GPU).

``oracle.update.FullUpdate`` composes the pinned pieces in the order of
Algorithm 1 (Appendix F, "Pseudocode"): sample a batch with hindsight goals,
take the critic step, then the policy step on the *updated* critic, then the
entropy-coefficient step.  Here the same three steps are written again with
torch float64 autograd and one ``torch.optim.Adam`` per parameter set
(critic 3e-4, policy 6e-4, log alpha 3e-4), sharing nothing with the oracle
but the batch indices and the Gaussian noise (both pinned on their own).

A mistake in the composition fails these tests: the policy step seeing the
critic before its Adam step, L_pi using the alpha after its step, swapped
learning rates, or a step number t that is not shared by the three Adams.
"""
import math

import numpy as np
import pytest
import torch

from oracle import actor as OA
from oracle import relabel as OR
from oracle.update import FullUpdate
from synthetic import Workload, actor_params, critic_params, make_buffer

W = Workload(name="tiny_full_update", num_envs=5, episode_len=24, obs_dim=5, act_dim=3,
             goal_dim=2, goal_lo=0, states="random_walk", batch_size=12, hidden=(16, 16),
             activation="ln_swish", repr_dim=4, energy_function="dot",
             contrastive_loss_function="symmetric_infonce", actor_hidden=(16, 16))


def _mlp(layers, x, w):
    h = x
    for i, L in enumerate(layers):
        z = h @ L["W"] + L["b"]
        if i == len(layers) - 1:
            return z
        if w.activation == "relu":
            h = torch.relu(z)
        else:
            y = torch.nn.functional.layer_norm(z, (z.shape[1],), L["ln_g"], L["ln_b"],
                                               eps=w.ln_eps)
            h = torch.nn.functional.silu(y)
    raise AssertionError


def _energy(p, q, kind):
    if kind == "dot":
        return p @ q.T
    return -torch.cdist(p, q, compute_mode="donot_use_mm_for_euclid_dist")


def _critic_loss(F, w):
    B = F.shape[0]
    r = torch.logsumexp(F, 1)
    c = torch.logsumexp(F, 0)
    d = torch.diagonal(F)
    loss = (r - d).sum() / B
    if w.contrastive_loss_function == "symmetric_infonce":
        loss = loss + (c - d).sum() / B
    return loss + w.logsumexp_penalty * (r * r).sum() / B


class TorchFullUpdate:
    """Algorithm 1's update with autograd and torch.optim.Adam."""

    def __init__(self, w, phi, psi, actor, seed, log_alpha=0.0):
        T = lambda a: torch.tensor(np.asarray(a, np.float64), requires_grad=True)
        self.w, self.seed = w, seed
        self.phi = [{k: T(v) for k, v in L.items()} for L in phi]
        self.psi = [{k: T(v) for k, v in L.items()} for L in psi]
        self.actor = [{k: T(v) for k, v in L.items()} for L in actor]
        self.log_alpha = torch.tensor([float(log_alpha)], dtype=torch.float64,
                                      requires_grad=True)
        crit = [t for L in self.phi + self.psi for t in L.values()]
        act = [t for L in self.actor for t in L.values()]
        self.opt_c = torch.optim.Adam(crit, lr=w.critic_lr, betas=(0.9, 0.999), eps=1e-8)
        self.opt_a = torch.optim.Adam(act, lr=w.policy_lr, betas=(0.9, 0.999), eps=1e-8)
        self.opt_l = torch.optim.Adam([self.log_alpha], lr=w.alpha_lr, betas=(0.9, 0.999),
                                      eps=1e-8)

    def step(self, obs, act, n):
        w = self.w
        _, x_sa, x_g, x_sg = OR.sample_relabel(obs, act, w.batch_size, w.discounting,
                                               self.seed, n, w.goal_lo, w.goal_dim)
        x_sa, x_g, x_sg = (torch.tensor(v, dtype=torch.float64) for v in (x_sa, x_g, x_sg))
        # critic step
        self.opt_c.zero_grad()
        F = _energy(_mlp(self.phi, x_sa, w), _mlp(self.psi, x_g, w), w.energy_function)
        lc = _critic_loss(F, w)
        lc.backward()
        self.opt_c.step()
        # random goals (Appendix C) for the policy step only; the mixing draw
        # is pinned on its own
        if w.random_goal_ratio > 0:
            sg, g, _, _ = OA.random_goal_mix(x_sg.numpy(), x_g.numpy(), w.obs_dim,
                                             w.random_goal_ratio, self.seed, n)
            x_sg, x_g = torch.tensor(sg), torch.tensor(g)
        # policy step on the updated, frozen critic, with alpha before its step
        alpha = torch.exp(self.log_alpha.detach())[0]
        eps = torch.tensor(OA.box_muller_noise(self.seed, n, w.batch_size, w.act_dim))
        self.opt_a.zero_grad()
        o = _mlp(self.actor, x_sg, w)
        A = w.act_dim
        mu, rho = o[:, :A], o[:, A:2 * A]
        sigma = torch.nn.functional.softplus(rho) + OA.SIGMA_MIN
        u = mu + sigma * eps
        logp = (torch.distributions.Normal(mu, sigma).log_prob(u)
                - torch.log1p(-torch.tanh(u) ** 2)).sum(1)
        frozen = lambda layers: [{k: t.detach() for k, t in L.items()} for L in layers]
        p = _mlp(frozen(self.phi), torch.cat([x_sa[:, :w.obs_dim], torch.tanh(u)], 1), w)
        q = _mlp(frozen(self.psi), x_g, w)
        f = torch.diagonal(_energy(p, q, w.energy_function))
        la = (alpha * logp - f).mean()
        la.backward()
        self.opt_a.step()
        # entropy coefficient, log pi detached, target entropy -|A|
        self.opt_l.zero_grad()
        lal = -(self.log_alpha[0] * (logp.detach() + (-float(A)))).mean()
        lal.backward()
        self.opt_l.step()
        return {"critic": lc.item(), "actor": la.item(), "mean_log_pi": logp.mean().item(),
                "mean_f": f.mean().item(), "log_alpha": self.log_alpha.item()}


def _setup(energy, act_fn):
    w = W.with_(energy_function=energy, activation=act_fn)
    ln = act_fn == "ln_swish"
    phi, psi = critic_params(w.in_sa, w.goal_dim, w.hidden, w.repr_dim, ln, seed=1,
                             perturb=0.2)
    actor = actor_params(w.in_sg, w.actor_hidden, w.act_dim, ln, seed=3, perturb=0.2)
    obs, act = make_buffer(w.num_envs, w.episode_len, w.obs_dim, w.act_dim, seed=0)
    return w, phi, psi, actor, obs, act


def _rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-30))


@pytest.mark.parametrize("energy,act_fn,ratio", [("dot", "ln_swish", 0.0),
                                                 ("l2", "ln_swish", 0.0), ("l2", "relu", 0.0),
                                                 ("dot", "ln_swish", 0.5)])
def test_full_update_matches_torch_autograd_and_adam(energy, act_fn, ratio):
    w, phi, psi, actor, obs, act = _setup(energy, act_fn)
    w = w.with_(random_goal_ratio=ratio)
    o = FullUpdate(w, phi, psi, actor, seed=2, log_alpha=0.1)
    t = TorchFullUpdate(w, phi, psi, actor, seed=2, log_alpha=0.1)
    for n in range(3):
        a = o.step(obs, act, n)
        b = t.step(obs, act, n)
        for k in ("critic", "actor", "mean_log_pi", "mean_f"):
            assert a[k] == pytest.approx(b[k], rel=1e-10, abs=1e-12), (n, k, a[k], b[k])
        assert a["log_alpha"] == pytest.approx(b["log_alpha"], rel=1e-10, abs=1e-14)
        for ours, theirs in ((o.phi, t.phi), (o.psi, t.psi), (o.actor, t.actor)):
            for L, M in zip(ours, theirs):
                for k in L:
                    assert _rel(L[k], M[k].detach().numpy()) <= 1e-10, (n, k)


def _step_with(o, obs, act, n, *, stale_critic=False, post_alpha=False, swap_lr=False):
    """FullUpdate.step with one composition mistake planted (CPU, oracle side)."""
    from oracle import adam as AD
    from oracle import critic as C
    w = o.w
    o.t += 1
    _, x_sa, x_g, x_sg = OR.sample_relabel(obs, act, w.batch_size, w.discounting, o.seed, n,
                                           w.goal_lo, w.goal_dim)
    before = ([{k: v.copy() for k, v in L.items()} for L in o.phi],
              [{k: v.copy() for k, v in L.items()} for L in o.psi])
    crit = C.critic_loss_and_grads(o.phi, o.psi, x_sa, x_g, w)
    for gi, (layers, grads) in enumerate(((o.phi, crit["g_phi"]), (o.psi, crit["g_psi"]))):
        for l, L in enumerate(layers):
            for k in L:
                L[k], o.mc[gi][l][k], o.vc[gi][l][k] = AD.adam_step(
                    L[k], grads[l][k], o.mc[gi][l][k], o.vc[gi][l][k], o.t, w.critic_lr)
    eps = OA.box_muller_noise(o.seed, n, w.batch_size, w.act_dim)
    lr_pol, lr_alpha = (w.alpha_lr, w.policy_lr) if swap_lr else (w.policy_lr, w.alpha_lr)
    la_used = o.log_alpha
    if post_alpha:  # alpha stepped first from a detached policy pass
        pre = OA.actor_loss_and_grads(o.actor, o.phi, o.psi, x_sg, x_g, x_sa[:, :w.obs_dim],
                                      eps, o.log_alpha, w)
        la, _, _ = AD.adam_step(np.array([o.log_alpha]), np.array([pre["d_log_alpha"]]),
                                np.array([o.m_alpha]), np.array([o.v_alpha]), o.t, lr_alpha)
        la_used = float(la[0])
    cphi, cpsi = before if stale_critic else (o.phi, o.psi)
    out = OA.actor_loss_and_grads(o.actor, cphi, cpsi, x_sg, x_g, x_sa[:, :w.obs_dim], eps,
                                  la_used, w)
    for l, L in enumerate(o.actor):
        for k in L:
            L[k], o.ma[l][k], o.va[l][k] = AD.adam_step(L[k], out["g_actor"][l][k], o.ma[l][k],
                                                        o.va[l][k], o.t, lr_pol)
    la, m, v = AD.adam_step(np.array([o.log_alpha]), np.array([out["d_log_alpha"]]),
                            np.array([o.m_alpha]), np.array([o.v_alpha]), o.t, lr_alpha)
    o.log_alpha, o.m_alpha, o.v_alpha = float(la[0]), float(m[0]), float(v[0])
    return {"actor": out["loss"], "log_alpha": o.log_alpha}


@pytest.mark.parametrize("mistake", ["stale_critic", "post_alpha", "swap_lr"])
def test_planted_composition_mistakes_are_caught(mistake):
    """Each plausible ordering mistake moves the result far beyond 1e-10."""
    w, phi, psi, actor, obs, act = _setup("dot", "ln_swish")
    bad = FullUpdate(w, phi, psi, actor, seed=2, log_alpha=0.1)
    t = TorchFullUpdate(w, phi, psi, actor, seed=2, log_alpha=0.1)
    worst = 0.0
    for n in range(3):
        a = _step_with(bad, obs, act, n, **{mistake: True})
        b = t.step(obs, act, n)
        worst = max(worst, abs(a["actor"] - b["actor"]) / abs(b["actor"]),
                    abs(a["log_alpha"] - b["log_alpha"]) / max(abs(b["log_alpha"]), 1e-3))
        for L, M in zip(bad.actor, t.actor):
            for k in L:
                worst = max(worst, _rel(L[k], M[k].detach().numpy()))
    assert worst > 1e-7, (mistake, worst)
