"""Pins for the oracle's other energies and contrastive objectives (no GPU).

Energies (Appendix A.2): cosine, L1, L2 without the square root, checked
against scipy's distance routines; their backward against torch float64
autograd.  Objectives (Appendix A.2; readings in ``oracle/objectives.py``):
closed forms at zero logits, B = 1 and B = 2 by hand, the transpose relation
between the two directions, and the hand-derived gradients against torch
float64 autograd of the loss; finally the whole critic (MLPs, energy,
objective) against central finite differences and autograd.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.distance import cdist

from oracle import critic, objectives
from synthetic import Workload, critic_params

ENERGIES = ["dot", "cos", "l1", "l2", "l2sq"]
LOSSES = list(objectives.ALL)


# ---------------------------------------------------------------- energies
def test_energies_match_scipy_distances():
    rng = np.random.default_rng(11)
    phi, psi = rng.standard_normal((13, 6)), rng.standard_normal((11, 6))
    assert np.allclose(critic.energy_matrix(phi, psi, "cos"), 1.0 - cdist(phi, psi, "cosine"),
                       rtol=1e-13, atol=1e-14)
    assert np.allclose(critic.energy_matrix(phi, psi, "l1", block=4),
                       -cdist(phi, psi, "cityblock"), rtol=1e-14, atol=1e-14)
    assert np.allclose(critic.energy_matrix(phi, psi, "l2sq", block=5),
                       -cdist(phi, psi, "sqeuclidean"), rtol=1e-13, atol=1e-13)
    for kind in ENERGIES:
        F = critic.energy_matrix(phi, psi, kind)
        assert np.allclose(critic.energy_row(phi[4], psi, kind), F[4], rtol=1e-14, atol=1e-14)


def test_cosine_energy_is_scale_free_and_zero_rows_give_zero():
    rng = np.random.default_rng(12)
    phi, psi = rng.standard_normal((5, 4)), rng.standard_normal((6, 4))
    F = critic.energy_matrix(phi, psi, "cos")
    assert np.allclose(critic.energy_matrix(3.0 * phi, 0.5 * psi, "cos"), F, rtol=1e-14)
    assert np.all(np.abs(F) <= 1.0 + 1e-15)
    phi[2] = 0.0
    assert np.all(critic.energy_matrix(phi, psi, "cos")[2] == 0.0)


def _torch_energy(p, q, kind):
    if kind == "dot":
        return p @ q.T
    if kind == "cos":
        return torch.nn.functional.cosine_similarity(p[:, None, :], q[None, :, :], dim=2,
                                                     eps=1e-300)
    if kind == "l1":
        return -torch.cdist(p, q, p=1.0)
    if kind == "l2":
        return -torch.cdist(p, q, compute_mode="donot_use_mm_for_euclid_dist")
    return -((p[:, None, :] - q[None, :, :]) ** 2).sum(2)


@pytest.mark.parametrize("kind", ENERGIES)
def test_energy_backward_matches_torch_autograd(kind):
    rng = np.random.default_rng(13)
    phi, psi = rng.standard_normal((9, 5)), rng.standard_normal((9, 5))
    G = rng.standard_normal((9, 9))
    F = critic.energy_matrix(phi, psi, kind)
    dphi, dpsi = critic.energy_backward(phi, psi, F, G, kind)
    tp = torch.tensor(phi, requires_grad=True)
    tq = torch.tensor(psi, requires_grad=True)
    TF = _torch_energy(tp, tq, kind)
    assert np.allclose(TF.detach().numpy(), F, rtol=1e-12, atol=1e-13)
    (TF * torch.tensor(G)).sum().backward()
    assert np.allclose(dphi, tp.grad.numpy(), rtol=1e-10, atol=1e-12)
    assert np.allclose(dpsi, tq.grad.numpy(), rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------- objectives
@pytest.mark.parametrize("B", [1, 2, 5, 64])
def test_zero_logits_closed_forms(B):
    F = np.zeros((B, B))
    lb = math.log(B)
    expect = {"fwd_infonce": lb, "symmetric_infonce": 2 * lb, "bwd_infonce": lb,
              "flatnce_fwd": 1.0, "flatnce_bwd": 1.0,
              "fb": -1.0 + (0.5 if B > 1 else 0.0),
              "dpo": B * math.log(2.0), "ipo": float(B), "sppo": 2.0 * B}
    for loss, obj in expect.items():
        out = objectives.contrastive_loss(F, loss, beta=0.1)
        assert out["obj"] == pytest.approx(obj, rel=1e-14, abs=1e-14), loss
        assert out["pen"] == pytest.approx(0.1 * lb * lb, rel=1e-14, abs=1e-300), loss
        assert out["total"] == pytest.approx(obj + 0.1 * lb * lb, rel=1e-14, abs=1e-14), loss


def test_batch_of_two_by_hand():
    a, b, c, d = 0.3, -1.2, 2.0, 0.5          # F = [[a, b], [c, d]]
    F = np.array([[a, b], [c, d]])
    sp = lambda x: math.log1p(math.exp(x))
    got = {k: objectives.contrastive_loss(F, k, 0.0)["obj"] for k in LOSSES}
    assert got["bwd_infonce"] == pytest.approx(0.5 * (sp(c - a) + sp(b - d)), rel=1e-15)
    assert got["fb"] == pytest.approx(0.5 * (-math.exp(a) - math.exp(d)
                                             + 0.5 * math.exp(2 * b) + 0.5 * math.exp(2 * c)),
                                      rel=1e-15)
    assert got["dpo"] == pytest.approx(0.5 * (2 * math.log(2) + sp(b - a) + sp(c - d)),
                                       rel=1e-15)
    assert got["ipo"] == pytest.approx(0.5 * (2 + (a - b - 1) ** 2 + (d - c - 1) ** 2),
                                       rel=1e-15)
    assert got["sppo"] == pytest.approx(
        0.5 * (2 * (a - 1) ** 2 + (a + 1) ** 2 + (b + 1) ** 2
               + 2 * (d - 1) ** 2 + (c + 1) ** 2 + (d + 1) ** 2), rel=1e-15)


def test_batch_of_one():
    f = 0.7
    F = np.array([[f]])
    got = {k: objectives.contrastive_loss(F, k, 0.0)["obj"] for k in LOSSES}
    assert got["bwd_infonce"] == 0.0 and got["flatnce_fwd"] == 1.0
    assert got["fb"] == pytest.approx(-math.exp(f), rel=1e-15)
    assert got["dpo"] == pytest.approx(math.log(2.0), rel=1e-15)
    assert got["ipo"] == 1.0
    assert got["sppo"] == pytest.approx((f - 1) ** 2 + (f + 1) ** 2, rel=1e-15)


def test_backward_direction_is_forward_of_transpose():
    rng = np.random.default_rng(14)
    F = rng.standard_normal((9, 9))
    a = objectives.contrastive_loss(F, "bwd_infonce", 0.0)
    b = critic.infonce_loss(F.T, "fwd_infonce", 0.0)
    assert a["obj"] == pytest.approx(b["fwd"], rel=1e-14)
    Ga = objectives.contrastive_grad(F, a["r"], a["c"], "bwd_infonce", 0.0)
    Gb = critic.infonce_grad(F.T, b["r"], b["c"], "fwd_infonce", 0.0)
    assert np.allclose(Ga, Gb.T, rtol=1e-14, atol=1e-16)


def _torch_objective(F, loss, beta):
    B = F.shape[0]
    eye = torch.eye(B, dtype=F.dtype)
    off = 1.0 - eye
    r = torch.logsumexp(F, 1)
    c = torch.logsumexp(F, 0)
    d = torch.diagonal(F)
    if loss == "fwd_infonce":
        obj = (r - d).mean()
    elif loss == "symmetric_infonce":
        obj = (r - d).mean() + (c - d).mean()
    elif loss == "bwd_infonce":
        obj = (c - d).mean()
    elif loss in ("flatnce_fwd", "flatnce_bwd"):
        X = F - d[:, None] if loss == "flatnce_fwd" else F - d[None, :]
        logS = torch.logsumexp(X, 1 if loss == "flatnce_fwd" else 0)
        obj = torch.exp(logS - logS.detach()).mean()
    elif loss == "fb":
        scale = 1.0 / (2.0 * (B - 1)) if B > 1 else 0.0
        obj = (-torch.exp(d) + scale * (off * torch.exp(F) ** 2).sum(1)).mean()
    elif loss == "dpo":
        obj = (-torch.nn.functional.logsigmoid(d[:, None] - F)).sum(1).mean()
    elif loss == "ipo":
        obj = (((d[:, None] - F) - 1.0) ** 2).sum(1).mean()
    elif loss == "sppo":
        obj = (((d[:, None] - 1.0) ** 2) + (F + 1.0) ** 2).sum(1).mean()
    else:
        raise ValueError(loss)
    return obj + beta * (r * r).mean()


@pytest.mark.parametrize("loss", LOSSES)
@pytest.mark.parametrize("B", [1, 2, 11])
def test_objective_gradients_match_torch_autograd(loss, B):
    rng = np.random.default_rng(15 + B)
    F = 1.5 * rng.standard_normal((B, B))
    out = objectives.contrastive_loss(F, loss, 0.1)
    G = objectives.contrastive_grad(F, out["r"], out["c"], loss, 0.1)
    TF = torch.tensor(F, requires_grad=True)
    L = _torch_objective(TF, loss, 0.1)
    L.backward()
    assert out["total"] == pytest.approx(L.item(), rel=1e-13, abs=1e-14)
    assert np.allclose(G, TF.grad.numpy(), rtol=1e-11, atol=1e-14)


def test_flatnce_has_the_gradient_of_infonce():
    rng = np.random.default_rng(16)
    F = rng.standard_normal((8, 8))
    out = objectives.contrastive_loss(F, "flatnce_fwd", 0.0)
    Gf = objectives.contrastive_grad(F, out["r"], out["c"], "flatnce_fwd", 0.0)
    Gi = critic.infonce_grad(F, out["r"], out["c"], "fwd_infonce", 0.0)
    assert out["obj"] == 1.0
    assert np.allclose(Gf, Gi, rtol=0, atol=1e-17)


# ---------------------------------------------------------------- whole critic
W0 = Workload(name="tiny_obj", num_envs=4, episode_len=10, obs_dim=5, act_dim=3,
              goal_dim=2, goal_lo=0, states="random_walk", batch_size=7, hidden=(12, 12),
              activation="ln_swish", repr_dim=4, energy_function="l2",
              contrastive_loss_function="symmetric_infonce")


def _setup(energy, loss, B=7, seed=0):
    w = W0.with_(energy_function=energy, contrastive_loss_function=loss, batch_size=B)
    phi, psi = critic_params(w.in_sa, w.goal_dim, w.hidden, w.repr_dim, True, seed=seed + 1,
                             perturb=0.2)
    phi = [{k: v.astype(np.float64) for k, v in L.items()} for L in phi]
    psi = [{k: v.astype(np.float64) for k, v in L.items()} for L in psi]
    rng = np.random.default_rng(seed)
    return w, phi, psi, rng.standard_normal((B, w.in_sa)), rng.standard_normal((B, w.goal_dim))


def _torch_critic(phi, psi, x_sa, x_g, w):
    def mlp(layers, x):
        h = x
        for i, L in enumerate(layers):
            z = h @ L["W"] + L["b"]
            if i == len(layers) - 1:
                return z
            y = torch.nn.functional.layer_norm(z, (z.shape[1],), L["ln_g"], L["ln_b"],
                                               eps=w.ln_eps)
            h = torch.nn.functional.silu(y)
    F = _torch_energy(mlp(phi, x_sa), mlp(psi, x_g), w.energy_function)
    return _torch_objective(F, w.contrastive_loss_function, w.logsumexp_penalty)


@pytest.mark.parametrize("energy", ENERGIES)
@pytest.mark.parametrize("loss", LOSSES)
def test_critic_gradients_match_torch_autograd(energy, loss):
    w, phi, psi, x_sa, x_g = _setup(energy, loss)
    out = critic.critic_loss_and_grads(phi, psi, x_sa, x_g, w)
    T = lambda a: torch.tensor(a, dtype=torch.float64, requires_grad=True)
    tphi = [{k: T(v) for k, v in L.items()} for L in phi]
    tpsi = [{k: T(v) for k, v in L.items()} for L in psi]
    L = _torch_critic(tphi, tpsi, torch.tensor(x_sa), torch.tensor(x_g), w)
    L.backward()
    assert out["total"] == pytest.approx(L.item(), rel=1e-12, abs=1e-13)
    for side, tl in (("phi", tphi), ("psi", tpsi)):
        for i, TL in enumerate(tl):
            for k, t in TL.items():
                assert np.allclose(out["g_" + side][i][k], t.grad.numpy(), rtol=1e-9,
                                   atol=1e-12), (side, i, k)


@pytest.mark.parametrize("energy,loss", [("cos", "symmetric_infonce"), ("l1", "dpo"),
                                         ("l2sq", "ipo"), ("dot", "fb"), ("l2", "sppo"),
                                         ("l2", "bwd_infonce"), ("cos", "fwd_infonce")])
def test_critic_gradients_central_differences(energy, loss):
    # (FlatNCE's value is 1 whatever the parameters, by its stop-gradient, so
    # finite differences cannot see its gradient; autograd checks it above)
    w, phi, psi, x_sa, x_g = _setup(energy, loss, seed=3)
    out = critic.critic_loss_and_grads(phi, psi, x_sa, x_g, w)
    rng = np.random.default_rng(17)
    keys = [(side, i, k) for side, layers in (("phi", phi), ("psi", psi))
            for i, L in enumerate(layers) for k in L]
    e = 1e-6
    checked = 0
    while checked < 32:
        side, i, k = keys[rng.integers(len(keys))]
        arr = (phi if side == "phi" else psi)[i][k]
        j = tuple(int(rng.integers(s)) for s in arr.shape)
        old = arr[j]
        arr[j] = old + e
        lp = critic.loss_only(phi, psi, x_sa, x_g, w)
        arr[j] = old - e
        lm = critic.loss_only(phi, psi, x_sa, x_g, w)
        arr[j] = old
        fd = (lp - lm) / (2 * e)
        if energy == "l1":   # an |x| kink inside the FD interval makes FD meaningless
            arr[j] = old + 3 * e
            l3 = critic.loss_only(phi, psi, x_sa, x_g, w)
            arr[j] = old
            if abs((l3 - lp) / (2 * e) - fd) > 1e-5 * (abs(fd) + 1e-3):
                continue
        g = out["g_" + side][i][k][j]
        assert abs(fd - g) <= 1e-6 * max(abs(g), 1e-3), (side, i, k, j, fd, g)
        checked += 1
