"""Pins for the oracle's critic loss and gradients (no GPU).

Every check is a closed form, an invariant, an independent library (torch
float64 autograd on the CPU) or central finite differences.
"""
import math

import numpy as np
import pytest
import torch

from oracle import critic, adam
from synthetic import Workload, critic_params

W0 = Workload(name="tiny", num_envs=4, episode_len=10, obs_dim=5, act_dim=3,
              goal_dim=2, goal_lo=0, states="random_walk", batch_size=8,
              hidden=(16, 16), activation="ln_swish", repr_dim=4,
              energy_function="l2", contrastive_loss_function="symmetric_infonce")

VARIANTS = [(a, e, l) for a in ("relu", "ln_swish") for e in ("dot", "l2")
            for l in ("symmetric_infonce", "fwd_infonce")]


def _setup(act, energy, loss, B=8, seed=0, perturb=0.2):
    w = W0.with_(activation=act, energy_function=energy,
                 contrastive_loss_function=loss, batch_size=B)
    phi, psi = critic_params(w.in_sa, w.goal_dim, w.hidden, w.repr_dim,
                             act == "ln_swish", seed=seed + 1, perturb=perturb)
    rng = np.random.default_rng(seed)
    x_sa = rng.standard_normal((B, w.in_sa))
    x_g = rng.standard_normal((B, w.goal_dim))
    return w, phi, psi, x_sa, x_g


# ---------------------------------------------------------------- loss values
@pytest.mark.parametrize("B", [1, 2, 7, 256])
def test_zero_logits_give_log_b(B):
    F = np.zeros((B, B))
    out = critic.infonce_loss(F, "fwd_infonce", beta=0.0)
    assert out["fwd"] == pytest.approx(math.log(B), abs=1e-15)
    assert out["bwd"] == pytest.approx(math.log(B), abs=1e-15)
    sym = critic.infonce_loss(F, "symmetric_infonce", beta=0.1)
    assert sym["total"] == pytest.approx(2 * math.log(B) + 0.1 * math.log(B) ** 2,
                                         abs=1e-14)


@pytest.mark.parametrize("energy", ["dot", "l2"])
def test_zeroed_output_layers_give_log_b(energy):
    w, phi, psi, x_sa, x_g = _setup("ln_swish", energy, "symmetric_infonce", B=16)
    for L in (phi[-1], psi[-1]):
        L["W"][:] = 0
        L["b"][:] = 0
    out = critic.critic_forward(phi, psi, x_sa, x_g, w.with_(logsumexp_penalty=0.0))
    assert out["fwd"] == pytest.approx(math.log(16), abs=1e-14)
    assert out["total"] == pytest.approx(2 * math.log(16), abs=1e-14)


def test_normalised_logits_zero_penalty():
    B, D = 9, 4
    phi = np.zeros((B, D)); phi[:, 0] = 1.0
    psi = np.zeros((B, D)); psi[:, 0] = -math.log(B)
    F = critic.energy_matrix(phi, psi, "dot")
    out = critic.infonce_loss(F, "symmetric_infonce", beta=0.1)
    assert np.max(np.abs(out["r"])) < 1e-15
    assert out["pen"] == pytest.approx(0.0, abs=1e-28)
    g1 = critic.infonce_grad(F, out["r"], out["c"], "symmetric_infonce", 0.1)
    g0 = critic.infonce_grad(F, out["r"], out["c"], "symmetric_infonce", 0.0)
    assert np.max(np.abs(g1 - g0)) < 1e-16


def test_batch_of_one():
    F = np.array([[1.7]])
    out = critic.infonce_loss(F, "symmetric_infonce", beta=0.1)
    assert out["fwd"] == 0.0 and out["bwd"] == 0.0
    assert out["pen"] == pytest.approx(0.1 * 1.7 ** 2, rel=1e-15)


def test_batch_of_two_by_hand():
    F = np.array([[0.3, -1.2], [2.0, 0.5]])
    out = critic.infonce_loss(F, "fwd_infonce", beta=0.0)
    hand = 0.5 * (math.log1p(math.exp(-1.2 - 0.3)) + math.log1p(math.exp(2.0 - 0.5)))
    assert out["fwd"] == pytest.approx(hand, rel=1e-15)
    handc = 0.5 * (math.log1p(math.exp(2.0 - 0.3)) + math.log1p(math.exp(-1.2 - 0.5)))
    assert out["bwd"] == pytest.approx(handc, rel=1e-15)


def test_l2_energy_direct_vs_norm_expansion_and_scipy():
    from scipy.spatial.distance import cdist
    rng = np.random.default_rng(1)
    phi, psi = rng.standard_normal((13, 6)), rng.standard_normal((11, 6))
    F = critic.energy_matrix(phi, psi, "l2", block=4)
    assert np.allclose(F, -cdist(phi, psi), rtol=1e-14, atol=1e-14)
    assert np.allclose(critic.energy_row(phi[3], psi, "l2"), F[3], rtol=0, atol=0)
    assert np.allclose(critic.energy_row(phi[3], psi, "dot"), (phi @ psi.T)[3])


def test_logsumexp_matches_scipy():
    from scipy.special import logsumexp
    rng = np.random.default_rng(2)
    F = 30 * rng.standard_normal((7, 9))
    assert np.allclose(critic.logsumexp(F, 1), logsumexp(F, axis=1), rtol=1e-15)
    assert np.allclose(critic.logsumexp(F, 0), logsumexp(F, axis=0), rtol=1e-15)


# ---------------------------------------------------------------- invariances
def test_joint_permutation_invariance():
    w, phi, psi, x_sa, x_g = _setup("ln_swish", "l2", "symmetric_infonce", B=12)
    perm = np.random.default_rng(3).permutation(12)
    a = critic.critic_loss_and_grads(phi, psi, x_sa, x_g, w)
    b = critic.critic_loss_and_grads(phi, psi, x_sa[perm], x_g[perm], w)
    assert b["total"] == pytest.approx(a["total"], rel=1e-13)
    assert np.allclose(b["dphi"], a["dphi"][perm], rtol=1e-11, atol=1e-15)
    for ga, gb in zip(a["g_phi"], b["g_phi"]):
        for k in ga:
            assert np.allclose(ga[k], gb[k], rtol=1e-10, atol=1e-14)


def test_shift_invariance():
    rng = np.random.default_rng(4)
    F = rng.standard_normal((10, 10))
    a = critic.infonce_loss(F, "symmetric_infonce", 0.1)
    b = critic.infonce_loss(F + 2.5, "symmetric_infonce", 0.1)
    assert b["fwd"] == pytest.approx(a["fwd"], rel=1e-13)
    assert b["bwd"] == pytest.approx(a["bwd"], rel=1e-13)
    assert b["pen"] == pytest.approx(0.1 * np.mean((a["r"] + 2.5) ** 2), rel=1e-13)


def test_dot_symmetric_swap():
    rng = np.random.default_rng(5)
    phi, psi = rng.standard_normal((10, 3)), rng.standard_normal((10, 3))
    Fa = critic.energy_matrix(phi, psi, "dot")
    Fb = critic.energy_matrix(psi, phi, "dot")
    a = critic.infonce_loss(Fa, "symmetric_infonce", 0.0)
    b = critic.infonce_loss(Fb, "symmetric_infonce", 0.0)
    assert b["total"] == pytest.approx(a["total"], rel=1e-14)


def test_gradient_row_and_column_sums():
    rng = np.random.default_rng(6)
    F = rng.standard_normal((10, 10))
    out = critic.infonce_loss(F, "symmetric_infonce", 0.0)
    Gf = critic.infonce_grad(F, out["r"], out["c"], "fwd_infonce", 0.0)
    assert np.max(np.abs(Gf.sum(axis=1))) < 1e-15
    Gs = critic.infonce_grad(F, out["r"], out["c"], "symmetric_infonce", 0.0)
    Gb = Gs - Gf
    assert np.max(np.abs(Gb.sum(axis=0))) < 1e-15


# ---------------------------------------------------------------- gradients
def _flat(phi, psi):
    return [(side, i, k) for side, layers in (("phi", phi), ("psi", psi))
            for i, L in enumerate(layers) for k in L]


@pytest.mark.parametrize("act,energy,loss", VARIANTS)
def test_gradients_central_differences(act, energy, loss):
    w, phi, psi, x_sa, x_g = _setup(act, energy, loss)
    phi = [{k: v.astype(np.float64) for k, v in L.items()} for L in phi]
    psi = [{k: v.astype(np.float64) for k, v in L.items()} for L in psi]
    out = critic.critic_loss_and_grads(phi, psi, x_sa, x_g, w)
    rng = np.random.default_rng(7)
    eps = 1e-6
    keys = _flat(phi, psi)
    checked = 0
    while checked < 64:
        side, i, k = keys[rng.integers(len(keys))]
        layers = phi if side == "phi" else psi
        arr = layers[i][k]
        j = tuple(rng.integers(s) for s in arr.shape)
        g = out["g_" + side][i][k][j]
        old = arr[j]
        arr[j] = old + eps
        lp = critic.loss_only(phi, psi, x_sa, x_g, w)
        arr[j] = old - eps
        lm = critic.loss_only(phi, psi, x_sa, x_g, w)
        arr[j] = old
        fd = (lp - lm) / (2 * eps)
        if act == "relu":
            # a ReLU kink inside [old-eps, old+eps] makes FD meaningless
            arr[j] = old + 3 * eps
            l3 = critic.loss_only(phi, psi, x_sa, x_g, w)
            arr[j] = old
            if abs((l3 - lp) / (2 * eps) - fd) > 1e-5 * (abs(fd) + 1e-3):
                continue
        assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3), (side, i, k, j, fd, g)
        checked += 1


def _torch_loss(phi, psi, x_sa, x_g, w):
    def mlp(layers, x):
        h = x
        for i, L in enumerate(layers):
            z = h @ L["W"] + L["b"]
            if i == len(layers) - 1:
                return z
            if w.activation == "relu":
                h = torch.relu(z)
            else:
                y = torch.nn.functional.layer_norm(z, (z.shape[1],), L["ln_g"],
                                                   L["ln_b"], eps=w.ln_eps)
                h = torch.nn.functional.silu(y)
    p = mlp(phi, x_sa)
    q = mlp(psi, x_g)
    if w.energy_function == "dot":
        F = p @ q.T
    else:
        F = -torch.cdist(p, q)
    B = F.shape[0]
    r = torch.logsumexp(F, 1)
    c = torch.logsumexp(F, 0)
    d = torch.diagonal(F)
    L = (r - d).mean()
    if w.contrastive_loss_function == "symmetric_infonce":
        L = L + (c - d).mean()
    return L + w.logsumexp_penalty * (r * r).mean()


@pytest.mark.parametrize("act,energy,loss", VARIANTS)
def test_gradients_match_torch_autograd(act, energy, loss):
    w, phi, psi, x_sa, x_g = _setup(act, energy, loss, B=10)
    out = critic.critic_loss_and_grads(phi, psi, x_sa, x_g, w)
    tphi = [{k: torch.tensor(v, dtype=torch.float64, requires_grad=True)
             for k, v in L.items()} for L in phi]
    tpsi = [{k: torch.tensor(v, dtype=torch.float64, requires_grad=True)
             for k, v in L.items()} for L in psi]
    L = _torch_loss(tphi, tpsi, torch.tensor(x_sa), torch.tensor(x_g), w)
    L.backward()
    assert out["total"] == pytest.approx(L.item(), rel=1e-13)
    for side, tl in (("phi", tphi), ("psi", tpsi)):
        for i, TL in enumerate(tl):
            for k, t in TL.items():
                ref = t.grad.numpy()
                got = out["g_" + side][i][k]
                assert np.allclose(got, ref, rtol=1e-10, atol=1e-13), (side, i, k)


# ---------------------------------------------------------------- Adam
def test_adam_first_step_closed_form():
    rng = np.random.default_rng(8)
    p0, g = rng.standard_normal(100), rng.standard_normal(100)
    p1, m, v = adam.adam_step(p0, g, np.zeros(100), np.zeros(100), 1, lr=3e-4)
    assert np.allclose(p1, p0 - 3e-4 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(9)
    p0 = rng.standard_normal(50)
    tp = torch.tensor(p0, requires_grad=True)
    opt = torch.optim.Adam([tp], lr=6e-4, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        g = rng.standard_normal(50)
        tp.grad = torch.tensor(g)
        opt.step()
        p, m, v = adam.adam_step(p, g, m, v, t, lr=6e-4)
        assert np.allclose(p, tp.detach().numpy(), rtol=0, atol=1e-14)
