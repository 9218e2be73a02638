"""Policy (actor) step of contrastive RL, in FP64 numpy.

What is computed (Section 3.2 "Policy Learning", the DDPG-style policy
objective; Section 5.1 setup: SAC-style tunable entropy coefficient; Algorithm 1,
policy update after the critic update):

* the policy pi(a | s, g) is a tanh-squashed Gaussian: an MLP on [s, g]
  outputs the mean mu and a pre-scale rho; sigma = softplus(rho) + 1e-3,
  u = mu + sigma * eps with eps ~ N(0, I) (reparameterised), a' = tanh(u);
* log pi(a'|s,g) = sum_k [log N(u_k; mu_k, sigma_k) - log(1 - tanh^2 u_k)],
  the tanh correction written stably as 2 (log 2 - u - softplus(-2u));
* the actor loss is L_pi = mean_i [alpha log pi_i - f(phi(s_i, a'_i), psi(g_i))]
  with the critic phi, psi frozen (their parameters after the critic update),
  f any of the critic's energies;
  maximising the energy of the policy's action is the objective of the
  policy-learning section;
* the entropy coefficient: L_alpha = -mean_i [log alpha (log pi_i + H)] with
  log pi detached and target entropy H = -|A|, optimised in log alpha.

Random goals (Appendix C): the policy objective generalised with a ratio
alpha_rand in [0, 1], (1 - alpha_rand) E[f(s, a', g)] with g from the future
of s's trajectory plus alpha_rand E[f(s, a', g-)] with g- drawn from the
goal marginal of the buffer.  Reading: each sample's goal is replaced, with
probability alpha_rand, by the relabelled goal of another sample of the same
batch (the batch goals are independent draws of that marginal), for both
the policy input [s, g] and the critic's psi(g); the estimate is unbiased
for the mixed objective.  The draw uses Philox4x64-10 stream 2: counter
(b, step, 2, 0), key (seed, 0), words w0, w1; sample b is mixed iff
floor(w0 / 2^11) < floor(alpha_rand * 2^53) (so P = that floor / 2^53) and
takes the goal of j = (b + 1 + floor(w1 (B - 1) / 2^64)) mod B, uniform over
the other samples; with B = 1 nothing is mixed.

The Gaussian noise is drawn without any floating-point step in the random
stream itself: Philox4x64-10 with key (seed, 0) and counter (b, step, 1, j)
gives four 64-bit words; each word w becomes u = (2 floor(w / 2^41) + 1) / 2^24
(23-bit uniforms, exact in FP32 and FP64); consecutive uniform pairs
(u1, u2) become Box-Muller normals sqrt(-2 ln u1) cos(2 pi u2),
sqrt(-2 ln u1) sin(2 pi u2), used for action coordinates in order.

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import math

import numpy as np

from . import critic as C
from fractions import Fraction

from .philox import mulhi64, philox4x64_10

SIGMA_MIN = 1e-3
LOG_2PI = math.log(2.0 * math.pi)


def uniform23(w: int) -> float:
    return (2 * (int(w) >> 41) + 1) / float(1 << 24)


def box_muller_noise(seed: int, step: int, batch: int, act_dim: int, stream: int = 1):
    """eps [batch, act_dim] in FP64 from the counter-based stream."""
    eps = np.empty((batch, act_dim))
    n_pairs = (act_dim + 1) // 2
    n_blocks = (n_pairs + 1) // 2
    for b in range(batch):
        z = []
        for j in range(n_blocks):
            w = philox4x64_10((b, step, stream, j), (seed, 0))
            for p in range(2):
                u1, u2 = uniform23(w[2 * p]), uniform23(w[2 * p + 1])
                r = math.sqrt(-2.0 * math.log(u1))
                z.append(r * math.cos(2.0 * math.pi * u2))
                z.append(r * math.sin(2.0 * math.pi * u2))
        eps[b] = z[:act_dim]
    return eps


def random_goal_mix(x_sg, x_g, obs_dim: int, ratio: float, seed: int, step: int,
                    stream: int = 2):
    """(x_sg', x_g', mixed [B] bool, partner [B]) of the random-goal reading above."""
    x_sg = np.asarray(x_sg, np.float64)
    x_g = np.asarray(x_g, np.float64)
    B, d_g = x_g.shape
    R = int(Fraction(float(ratio)) * (1 << 53))  # floor, ratio >= 0
    partner = np.arange(B)
    mixed = np.zeros(B, bool)
    for b in range(B if B >= 2 else 0):
        w0, w1, _, _ = philox4x64_10((b, step, stream, 0), (seed, 0))
        if (w0 >> 11) < R:
            mixed[b] = True
            partner[b] = (b + 1 + mulhi64(w1, B - 1)) % B
    g = x_g[partner].copy()
    sg = x_sg.copy()
    sg[:, obs_dim:obs_dim + d_g] = g
    return sg, g, mixed, partner


def softplus(x):
    return np.logaddexp(0.0, x)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def policy_head(out, eps, act_dim: int):
    """(mu, rho, sigma, u, a, log_pi) from the policy MLP output."""
    mu = out[:, :act_dim]
    rho = out[:, act_dim:2 * act_dim]
    sigma = softplus(rho) + SIGMA_MIN
    u = mu + sigma * eps
    a = np.tanh(u)
    log_n = -0.5 * eps * eps - np.log(sigma) - 0.5 * LOG_2PI
    log_det = 2.0 * (math.log(2.0) - u - softplus(-2.0 * u))  # log(1 - tanh^2 u)
    log_pi = (log_n - log_det).sum(axis=1)
    return mu, rho, sigma, u, a, log_pi


def actor_loss_and_grads(actor_layers, phi_layers, psi_layers, x_sg, x_g, obs_t, eps,
                         log_alpha: float, w, target_entropy: float | None = None):
    """Actor loss, its gradients (per actor layer) and d L_alpha / d log alpha.

    x_sg = [s, g] (policy input), x_g = g (critic goal input), obs_t = s.
    The critic (phi, psi) is frozen.
    """
    A = w.act_dim
    B = x_sg.shape[0]
    H = -float(A) if target_entropy is None else target_entropy
    alpha = math.exp(log_alpha)
    out, c_act = C.mlp_forward(actor_layers, x_sg, w.activation, w.ln_eps)
    mu, rho, sigma, u, a, log_pi = policy_head(out, eps, A)
    x_sa = np.concatenate([np.asarray(obs_t, np.float64), a], axis=1)
    phi, c_phi = C.mlp_forward(phi_layers, x_sa, w.activation, w.ln_eps)
    psi, _ = C.mlp_forward(psi_layers, x_g, w.activation, w.ln_eps)
    f, df = C.pair_energy(phi, psi, w.energy_function)
    dphi = -df / B                           # d(-mean f)/d phi
    loss = math.fsum((alpha * log_pi - f).tolist()) / B
    # through the frozen critic to the action input
    _, dx = C.mlp_backward(phi_layers, c_phi, dphi, w.activation)
    da = dx[:, obs_t.shape[1]:obs_t.shape[1] + A]
    t = np.tanh(u)
    dlogpi_du = 2.0 * t                       # d/du of -log(1 - tanh^2 u)
    gu = (alpha / B) * dlogpi_du + da * (1.0 - t * t)
    g_mu = gu
    g_sigma = (alpha / B) * (-1.0 / sigma) + gu * eps
    g_rho = g_sigma * sigmoid(rho)
    dout = np.zeros_like(out)
    dout[:, :A] = g_mu
    dout[:, A:2 * A] = g_rho
    g_actor, _ = C.mlp_backward(actor_layers, c_act, dout, w.activation)
    d_log_alpha = -math.fsum((log_pi + H).tolist()) / B
    return {"loss": loss, "log_pi": log_pi, "f": f, "a": a, "u": u, "g_actor": g_actor,
            "d_log_alpha": d_log_alpha, "mean_log_pi": float(np.mean(log_pi)),
            "alpha_loss": -log_alpha * (math.fsum((log_pi + H).tolist()) / B)}


def actor_loss_only(actor_layers, phi_layers, psi_layers, x_sg, x_g, obs_t, eps, log_alpha, w):
    A = w.act_dim
    B = x_sg.shape[0]
    out, _ = C.mlp_forward(actor_layers, x_sg, w.activation, w.ln_eps)
    _, _, _, _, a, log_pi = policy_head(out, eps, A)
    x_sa = np.concatenate([np.asarray(obs_t, np.float64), a], axis=1)
    phi, _ = C.mlp_forward(phi_layers, x_sa, w.activation, w.ln_eps)
    psi, _ = C.mlp_forward(psi_layers, x_g, w.activation, w.ln_eps)
    # the loss alone evaluates f row by row from the energy definitions
    f = np.array([C.energy_row(phi[b], psi[b:b + 1], w.energy_function)[0] for b in range(B)])
    return math.fsum((math.exp(log_alpha) * log_pi - f).tolist()) / B
