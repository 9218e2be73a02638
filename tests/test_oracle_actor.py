"""Pins for the oracle's policy step (no GPU)."""
import math

import numpy as np
import pytest
import torch
from scipy import stats

from oracle import actor as A
from oracle import critic as C
from oracle.philox import philox4x64_10
from synthetic import Workload, actor_params, critic_params

W = Workload(name="tiny_actor", num_envs=4, episode_len=20, obs_dim=5, act_dim=3, goal_dim=2,
             goal_lo=0, states="random_walk", batch_size=10, hidden=(16, 16),
             activation="ln_swish", repr_dim=4, energy_function="dot",
             contrastive_loss_function="symmetric_infonce", actor_hidden=(16, 16))


def _setup(energy="dot", seed=0):
    w = W.with_(energy_function=energy)
    phi, psi = critic_params(w.in_sa, w.goal_dim, w.hidden, w.repr_dim, True, seed=1,
                             perturb=0.2)
    actor = actor_params(w.in_sg, w.actor_hidden, w.act_dim, True, seed=3, perturb=0.2)
    rng = np.random.default_rng(seed)
    B = w.batch_size
    obs_t = rng.standard_normal((B, w.obs_dim))
    g = rng.standard_normal((B, w.goal_dim))
    x_sg = np.concatenate([obs_t, g], axis=1)
    eps = A.box_muller_noise(7, 3, B, w.act_dim)
    return w, phi, psi, actor, x_sg, g, obs_t, eps


def test_uniforms_are_exact_and_inside_unit_interval():
    assert A.uniform23(0) == 2.0 ** -24
    assert A.uniform23((1 << 64) - 1) == 1.0 - 2.0 ** -24
    for w in philox4x64_10((1, 2, 1, 0), (7, 0)):
        u = A.uniform23(w)
        assert 0.0 < u < 1.0
        assert np.float32(u) == u  # exactly representable in FP32


def test_box_muller_pairs_have_the_radius_of_u1():
    # z0^2 + z1^2 = -2 ln u1 for each Box-Muller pair
    eps = A.box_muller_noise(5, 0, 3, 4)
    for b in range(3):
        w = philox4x64_10((b, 0, 1, 0), (5, 0))
        for p in range(2):
            u1 = A.uniform23(w[2 * p])
            z0, z1 = eps[b, 2 * p], eps[b, 2 * p + 1]
            assert z0 * z0 + z1 * z1 == pytest.approx(-2.0 * math.log(u1), rel=1e-14)


def test_box_muller_noise_is_standard_normal():
    eps = A.box_muller_noise(11, 4, 3000, 7).ravel()
    assert abs(eps.mean()) < 5 / math.sqrt(eps.size)
    assert abs(eps.var() - 1.0) < 5 * math.sqrt(2.0 / eps.size)
    assert stats.kstest(eps, "norm").pvalue > 1e-3


def test_log_pi_matches_torch_tanh_gaussian():
    rng = np.random.default_rng(3)
    out = rng.standard_normal((12, 8)) * 0.7
    eps = rng.standard_normal((12, 4)) * 0.7
    mu, rho, sigma, u, a, log_pi = A.policy_head(out, eps, 4)
    base = torch.distributions.Normal(torch.tensor(mu), torch.tensor(sigma))
    dist = torch.distributions.TransformedDistribution(
        base, [torch.distributions.transforms.TanhTransform()])
    ref = dist.log_prob(torch.tanh(torch.tensor(u))).sum(-1).numpy()
    # torch evaluates the density at tanh(u); far in the tails atanh(tanh u)
    # loses precision, so compare where |u| is moderate
    ok = np.all(np.abs(u) < 3.0, axis=1)
    assert ok.sum() >= 3
    assert np.allclose(log_pi[ok], ref[ok], rtol=1e-9, atol=1e-9)
    # and exactly against the plain formula with log(1 - tanh^2 u)
    plain = (-0.5 * eps ** 2 - np.log(sigma) - 0.5 * math.log(2 * math.pi)
             - np.log(1 - np.tanh(u) ** 2)).sum(1)
    assert np.allclose(log_pi[ok], plain[ok], rtol=1e-12)


@pytest.mark.parametrize("energy", ["dot", "l2", "cos", "l2sq", "l1"])
def test_actor_gradients_central_differences(energy):
    w, phi, psi, actor, x_sg, g, obs_t, eps = _setup(energy)
    actor = [{k: v.astype(np.float64) for k, v in L.items()} for L in actor]
    la = 0.3
    out = A.actor_loss_and_grads(actor, phi, psi, x_sg, g, obs_t, eps, la, w)
    assert out["loss"] == pytest.approx(
        A.actor_loss_only(actor, phi, psi, x_sg, g, obs_t, eps, la, w), rel=1e-14)
    rng = np.random.default_rng(4)
    keys = [(l, k) for l, L in enumerate(actor) for k in L]
    e = 1e-6
    for _ in range(48):
        l, k = keys[rng.integers(len(keys))]
        arr = actor[l][k]
        j = tuple(int(rng.integers(s)) for s in arr.shape)
        old = arr[j]
        arr[j] = old + e
        lp = A.actor_loss_only(actor, phi, psi, x_sg, g, obs_t, eps, la, w)
        arr[j] = old - e
        lm = A.actor_loss_only(actor, phi, psi, x_sg, g, obs_t, eps, la, w)
        arr[j] = old
        fd = (lp - lm) / (2 * e)
        gg = out["g_actor"][l][k][j]
        assert abs(fd - gg) <= 1e-6 * max(abs(gg), 1e-3), (l, k, j, fd, gg)
    # d L_alpha / d log alpha
    H = -w.act_dim
    lam = lambda x: -x * np.mean(out["log_pi"] + H)
    fd = (lam(la + 1e-6) - lam(la - 1e-6)) / 2e-6
    assert out["d_log_alpha"] == pytest.approx(fd, rel=1e-8)


def _torch_pair_energy(p, q, kind):
    if kind == "dot":
        return (p * q).sum(1)
    if kind == "l2":
        return -torch.linalg.vector_norm(p - q, dim=1)
    if kind == "l2sq":
        return -((p - q) ** 2).sum(1)
    if kind == "l1":
        return -(p - q).abs().sum(1)
    return torch.nn.functional.cosine_similarity(p, q, dim=1, eps=1e-300)


@pytest.mark.parametrize("energy", ["dot", "l2", "cos", "l2sq", "l1"])
def test_actor_gradients_match_torch_autograd(energy):
    w, phi, psi, actor, x_sg, g, obs_t, eps = _setup(energy)
    out = A.actor_loss_and_grads(actor, phi, psi, x_sg, g, obs_t, eps, -0.2, w)
    T = lambda a, rg=False: torch.tensor(np.asarray(a, np.float64), requires_grad=rg)
    ta = [{k: T(v, True) for k, v in L.items()} for L in actor]

    def mlp(layers, x):
        h = x
        for i, L in enumerate(layers):
            z = h @ L["W"] + L["b"]
            if i == len(layers) - 1:
                return z
            y = torch.nn.functional.layer_norm(z, (z.shape[1],), L["ln_g"], L["ln_b"],
                                               eps=w.ln_eps)
            h = torch.nn.functional.silu(y)

    o = mlp(ta, T(x_sg))
    Ad = w.act_dim
    mu, rho = o[:, :Ad], o[:, Ad:2 * Ad]
    sigma = torch.nn.functional.softplus(rho) + A.SIGMA_MIN
    u = mu + sigma * T(eps)
    base = torch.distributions.Normal(mu, sigma)
    logp = (base.log_prob(u) - torch.log1p(-torch.tanh(u) ** 2)).sum(-1)
    tphi = [{k: T(v) for k, v in L.items()} for L in phi]
    tpsi = [{k: T(v) for k, v in L.items()} for L in psi]
    p = mlp(tphi, torch.cat([T(obs_t), torch.tanh(u)], 1))
    q = mlp(tpsi, T(g))
    f = _torch_pair_energy(p, q, w.energy_function)
    loss = (math.exp(-0.2) * logp - f).mean()
    loss.backward()
    assert out["loss"] == pytest.approx(loss.item(), rel=1e-12)
    for l, L in enumerate(ta):
        for k, t in L.items():
            assert np.allclose(out["g_actor"][l][k], t.grad.numpy(), rtol=1e-9, atol=1e-12)
