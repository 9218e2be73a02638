"""Pins for the random-goal mixing of the policy step (Appendix C), no GPU.

The mixing draw is checked against its definition in exact rational
arithmetic (a Bernoulli(ratio) decision on the uniform w0 / 2^64), the
degenerate ratios 0 and 1 and B = 1, the uniformity of the partner over the
other samples, the rows it writes, and, through the oracle's policy loss,
that the estimate's expectation is Appendix C's mixed objective
(1 - ratio) E[f(s, a', g)] + ratio E[f(s, a', g-)].
"""
import math
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from oracle import actor as A
from oracle.philox import philox4x64_10
from synthetic import Workload, actor_params, critic_params_for


def _batch(B, d_s=4, d_g=2, seed=0):
    rng = np.random.default_rng(seed)
    x_g = rng.standard_normal((B, d_g))
    s = rng.standard_normal((B, d_s))
    return np.concatenate([s, x_g], axis=1), x_g


@pytest.mark.parametrize("ratio", [0.0, 0.25, 0.3, 0.5, 1.0])
def test_decision_is_bernoulli_of_the_uniform_word(ratio):
    B = 64
    x_sg, x_g = _batch(B)
    for step in (0, 5, 2**33 + 1):
        _, _, mixed, partner = A.random_goal_mix(x_sg, x_g, 4, ratio, seed=7, step=step)
        for b in range(B):
            w0 = philox4x64_10((b, step, 2, 0), (7, 0))[0]
            assert mixed[b] == (Fraction(w0, 2**64) < Fraction(ratio))
            assert (partner[b] != b) == mixed[b]


def test_ratio_zero_is_the_identity_and_one_mixes_every_sample():
    x_sg, x_g = _batch(50)
    sg, g, mixed, _ = A.random_goal_mix(x_sg, x_g, 4, 0.0, seed=2, step=3)
    assert not mixed.any() and np.array_equal(sg, x_sg) and np.array_equal(g, x_g)
    sg, g, mixed, partner = A.random_goal_mix(x_sg, x_g, 4, 1.0, seed=2, step=3)
    assert mixed.all() and (partner != np.arange(50)).all()
    # one sample alone has no other goal to take
    sg, g, mixed, _ = A.random_goal_mix(x_sg[:1], x_g[:1], 4, 1.0, seed=2, step=3)
    assert not mixed.any() and np.array_equal(g, x_g[:1])


def test_mixed_rows_take_the_partner_goal_and_keep_their_state():
    x_sg, x_g = _batch(40, d_s=5, d_g=3, seed=4)
    sg, g, mixed, partner = A.random_goal_mix(x_sg, x_g, 5, 0.5, seed=3, step=11)
    assert 0 < mixed.sum() < 40
    assert np.array_equal(sg[:, :5], x_sg[:, :5])
    assert np.array_equal(g, x_g[partner])
    assert np.array_equal(sg[:, 5:], x_g[partner])


def test_rate_and_partner_law():
    B, ratio = 7, 0.3
    x_sg, x_g = _batch(B)
    n_mixed, offsets, total = 0, [], 0
    for step in range(3000):
        _, _, mixed, partner = A.random_goal_mix(x_sg, x_g, 4, ratio, seed=9, step=step)
        n_mixed += int(mixed.sum())
        total += B
        offsets += [int((partner[b] - b) % B) for b in np.flatnonzero(mixed)]
    sd = math.sqrt(total * ratio * (1 - ratio))
    assert abs(n_mixed - total * ratio) < 5 * sd
    counts = np.bincount(offsets, minlength=B)
    assert counts[0] == 0                      # never the sample itself
    chi2 = stats.chisquare(counts[1:])         # uniform over the B - 1 others
    assert chi2.pvalue > 1e-4


def test_expected_policy_objective_is_the_mixed_objective():
    """Averaged over the mixing draw (fixed noise and parameters), the
    per-sample energy term tends to (1 - r) f(s_b, a'_b, g_b)
    + r mean_{j != b} f(s_b, a'_b(g_j), g_j): Appendix C's objective."""
    w = Workload(name="rg", num_envs=4, episode_len=20, obs_dim=5, act_dim=2, goal_dim=2,
                 goal_lo=0, states="random_walk", batch_size=4, hidden=(16,),
                 activation="relu", repr_dim=8, energy_function="dot",
                 contrastive_loss_function="symmetric_infonce", actor_hidden=(16,))
    phi, psi = critic_params_for(w, seed=1, perturb=0.1)
    pol = actor_params(w.in_sg, w.actor_hidden, w.act_dim, False, seed=3, perturb=0.1)
    to64 = lambda layers: [{k: np.asarray(v, np.float64) for k, v in L.items()} for L in layers]
    phi, psi, pol = to64(phi), to64(psi), to64(pol)
    B, r = 4, 0.4
    x_sg, x_g = _batch(B, d_s=5, d_g=2, seed=8)
    s = x_sg[:, :5]
    eps = np.random.default_rng(5).standard_normal((B, 2))

    def energies(sg, g):
        out = A.actor_loss_and_grads(pol, phi, psi, sg, g, s, eps, 0.0, w)
        return out["f"]

    f_pos = energies(x_sg, x_g)
    f_neg = np.zeros(B)
    spread = np.zeros(B)
    for b in range(B):
        vals = []
        for j in range(B):
            if j == b:
                continue
            sg = x_sg.copy()
            sg[b, 5:] = x_g[j]
            g = x_g.copy()
            g[b] = x_g[j]
            vals.append(energies(sg, g)[b])
        f_neg[b] = np.mean(vals)
        spread[b] = max(abs(v - f_pos[b]) for v in vals)
    target = (1 - r) * f_pos + r * f_neg
    N = 3000
    acc = np.zeros(B)
    for step in range(N):
        sg, g, _, _ = A.random_goal_mix(x_sg, x_g, 5, r, seed=1, step=step)
        acc += energies(sg, g)
    err = np.abs(acc / N - target) / spread
    assert (err < 0.05).all(), err
