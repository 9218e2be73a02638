"""GPU: Adam, device counters, determinism, graph replay == eager, the
autograd Function, and short update trajectories against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import adam as oadam
from oracle import critic as ocritic
from oracle import relabel as orelabel
from synthetic import workloads as WL
from tests.gpu_helpers import cosine, log, setup

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def test_adam_matches_oracle_and_shadow_is_rne():
    from paper_2408_11052_amd import crl_adam_step, crl_counter_add
    rng = np.random.default_rng(0)
    n = 4099  # ragged: not a multiple of the 4-wide vectors
    p0 = rng.standard_normal(n).astype(np.float32)
    p = torch.from_numpy(p0).to(DEV)
    m = torch.zeros(n, device=DEV)
    v = torch.zeros(n, device=DEV)
    pb = torch.zeros(n, dtype=torch.bfloat16, device=DEV)
    t = torch.zeros(1, dtype=torch.int64, device=DEV)
    rp, rm, rv = p0.astype(np.float64), np.zeros(n), np.zeros(n)
    # FP32 rounding bound of m = b1 m + (1 - b1) g, propagated over the steps
    # (the two terms can cancel, so the bound is relative to the terms)
    em = np.zeros(n)
    for step in range(1, 6):
        g0 = (rng.standard_normal(n) * 10.0 ** rng.uniform(-3, 1, n)).astype(np.float32)
        g = torch.from_numpy(g0).to(DEV)
        crl_counter_add(t, 1)
        crl_adam_step(p, g, m, v, pb, t, 3e-4)
        em = 0.9 * em + 2.0 ** -22 * (0.9 * np.abs(rm) + 0.1 * np.abs(g0))
        rp, rm, rv = oadam.adam_step(rp, g0.astype(np.float64), rm, rv, step, 3e-4)
        torch.cuda.synchronize()
        assert int(t.item()) == step
        got_m, got_v, got_p = m.cpu().numpy(), v.cpu().numpy(), p.cpu().numpy()
        assert np.all(np.abs(got_m - rm) <= em + 1e-30)
        assert np.allclose(got_v, rv, rtol=1e-5, atol=1e-16)
        # the step size is at most lr; FP32 error of the update is ~1e-7 lr
        assert np.max(np.abs(got_p - rp)) < 3e-4 * 1e-3 * step + 1e-6
        assert torch.equal(pb, p.bfloat16())
    log(f"[adam] max |p - oracle| after 5 steps: {np.max(np.abs(got_p - rp)):.3e}")


def _small_bf16():
    return WL.DOT_B4096_BF16.with_(name="upd_bf16", batch_size=320, hidden=(256,) * 2,
                                   num_envs=32, episode_len=64)


def _make_update(w, seed=2):
    from paper_2408_11052_amd.update import CriticUpdate
    obs, act, phi, psi = setup(w, perturb=0.0)
    return CriticUpdate(w, torch.from_numpy(obs).to(DEV), torch.from_numpy(act).to(DEV),
                        phi, psi, seed=seed), (obs, act, phi, psi)


def test_two_runs_are_bit_identical():
    w = _small_bf16()
    outs = []
    for _ in range(2):
        u, _ = _make_update(w)
        for _ in range(3):
            u.enqueue()
        torch.cuda.synchronize()
        outs.append((u.params.clone(), u.grads.clone(), u.loss.clone()))
        u.close()
    for a, b in zip(*outs):
        assert torch.equal(a, b)


@pytest.mark.parametrize("wname", ["bf16", "fp32"])
def test_graph_replay_equals_eager(wname):
    w = _small_bf16() if wname == "bf16" else WL.LN_FWD_FP32.with_(
        name="upd_fp32", batch_size=256, hidden=(256,) * 2, num_envs=32, episode_len=64)
    ue, _ = _make_update(w)
    ug, _ = _make_update(w)
    g = ug.capture(1)
    for step in range(4):
        ue.enqueue()
        g.replay()
        torch.cuda.synchronize()
        # some eager work of the program between replays
        _ = (ue.params * 2).sum().item()
        assert torch.equal(ue.loss, ug.loss), step
        assert torch.equal(ue.params, ug.params), step
        assert torch.equal(ue.idx, ug.idx), step
    assert int(ug.n.item()) == 4 and int(ug.t.item()) == 4
    ue.close()
    ug.close()


def test_update_trajectory_matches_oracle_fp32():
    """Five full updates (relabel, critic, Adam) against the FP64 oracle."""
    w = WL.SMALL_RELU.with_(name="traj_relu", batch_size=192, hidden=(128, 128),
                            num_envs=24, episode_len=80, energy_function="l2")
    u, (obs, act, phi, psi) = _make_update(w)
    P = [{k: a.astype(np.float64) for k, a in L.items()} for L in phi]
    Q = [{k: a.astype(np.float64) for k, a in L.items()} for L in psi]
    keys = [(s, l, k) for s, layers in (("phi", P), ("psi", Q)) for l, L in enumerate(layers)
            for k in L]
    mom = {key: (0.0, 0.0) for key in keys}
    for step in range(5):
        u.enqueue()
        torch.cuda.synchronize()
        _, x_sa, x_g, _ = orelabel.sample_relabel(obs, act, w.batch_size, w.discounting, 2,
                                                  step, w.goal_lo, w.goal_dim)
        out = ocritic.critic_loss_and_grads(P, Q, x_sa, x_g, w)
        got = float(u.loss[0])
        log(f"[traj] step {step}: loss gpu {got:.7f} oracle {out['total']:.7f}")
        assert abs(got - out["total"]) <= 1e-5 * abs(out["total"])
        for (s, l, k) in keys:
            layers = P if s == "phi" else Q
            m, v = mom[(s, l, k)]
            layers[l][k], m, v = oadam.adam_step(layers[l][k], out["g_" + s][l][k], m, v,
                                                 step + 1, w.critic_lr)
            mom[(s, l, k)] = (m, v)
    gp, gq = u.crit.unpack(u.params.cpu().numpy())
    worst = 0.0
    for a, b in zip(gp + gq, P + Q):
        for k in b:
            worst = max(worst, float(np.max(np.abs(a[k] - b[k]))))
    log(f"[traj] max |param - oracle| after 5 Adam steps: {worst:.3e}")
    # each Adam step moves a parameter by <= lr; sign flips of near-zero
    # gradients can cost at most 2 lr per step
    assert worst <= 2 * 5 * w.critic_lr
    u.close()


def test_autograd_function_matches_oracle_finite_differences():
    """The hand-written backward (CriticLoss) on the FP32 path against central
    differences of the FP64 oracle loss on 64 random coordinates, eps = 1e-3."""
    from paper_2408_11052_amd import Critic, CriticLoss
    w = WL.LN_FWD_FP32.with_(name="fd_ln_l2_fwd", batch_size=96, hidden=(64,) * 4,
                             num_envs=16, episode_len=40)
    obs, act, phi, psi = setup(w, perturb=0.1)
    crit = Critic(w, max_episode_len=obs.shape[1])
    params = torch.from_numpy(crit.pack(phi, psi)).to(DEV).requires_grad_(True)
    x_sa, x_g, _ = crit.inputs(DEV)
    idx = torch.zeros(w.batch_size, 3, dtype=torch.int32, device=DEV)
    step = torch.zeros(1, dtype=torch.int64, device=DEV)
    crit.crl_sample_relabel(torch.from_numpy(obs).to(DEV), torch.from_numpy(act).to(DEV), 2,
                            step, idx, x_sa, x_g)
    ws = crit.workspace(DEV)
    loss = CriticLoss.apply(params, crit, None, x_sa, x_g, ws)
    loss.backward()
    g = params.grad.detach().cpu().numpy().astype(np.float64)
    _, ox_sa, ox_g, _ = orelabel.sample_relabel(obs, act, w.batch_size, w.discounting, 2, 0,
                                                w.goal_lo, w.goal_dim)
    P = [{k: a.astype(np.float64) for k, a in L.items()} for L in phi]
    Q = [{k: a.astype(np.float64) for k, a in L.items()} for L in psi]
    assert abs(float(loss) - ocritic.loss_only(P, Q, ox_sa, ox_g, w)) < 1e-5 * abs(float(loss))
    rng = np.random.default_rng(11)
    keys = [(side, l, k) for side, layers in (("phi", P), ("psi", Q))
            for l, L in enumerate(layers) for k in L]
    eps, worst = 1e-3, 0.0
    for _ in range(64):
        side, l, k = keys[rng.integers(len(keys))]
        layers = P if side == "phi" else Q
        arr = layers[l][k]
        j = tuple(int(rng.integers(s)) for s in arr.shape)
        old = arr[j]
        arr[j] = old + eps
        lp = ocritic.loss_only(P, Q, ox_sa, ox_g, w)
        arr[j] = old - eps
        lm = ocritic.loss_only(P, Q, ox_sa, ox_g, w)
        arr[j] = old
        fd = (lp - lm) / (2 * eps)
        info = crit.layers[0 if side == "phi" else 1][l]
        base = {"W": info.w, "b": info.b, "ln_g": info.ln_g, "ln_b": info.ln_b}[k]
        flat = base + (j[0] * info.fan_out + j[1] if k == "W" else j[0])
        err = abs(g[flat] - fd)
        # FD truncation at eps = 1e-3 is O(eps^2) relative; FP32 gradient ~1e-6
        tol = 2e-3 * abs(fd) + 2e-6
        worst = max(worst, err / (abs(fd) + 1e-6))
        assert err <= tol, (side, l, k, j, g[flat], fd)
    log(f"[fd] 64 coordinates, worst relative deviation {worst:.2e}")
    crit.close()


def _bwd_adam_case(case):
    if case == "bf16_unsplit":   # B < 1024: every dW is one whole-K launch
        return _small_bf16()
    if case == "bf16_split":
        return WL.DOT_B4096_BF16.with_(name="bwdadam_bf16", batch_size=2048,
                                       hidden=(256,) * 2, num_envs=64, episode_len=64)
    if case == "bf16_materialised_relu":
        return WL.DOT_B4096_BF16.with_(name="bwdadam_relu", batch_size=520, hidden=(128,) * 3,
                                       activation="relu", logits="materialised",
                                       num_envs=32, episode_len=64)
    if case == "fp32_unsplit":
        return WL.LN_FWD_FP32.with_(name="bwdadam_fp32", batch_size=200, hidden=(96,) * 2,
                                    num_envs=16, episode_len=40)
    return WL.LN_FWD_FP32.with_(name="bwdadam_fp32s", batch_size=1024, hidden=(128,) * 2,
                                num_envs=32, episode_len=64)


@pytest.mark.parametrize("case", ["bf16_unsplit", "bf16_split", "bf16_materialised_relu",
                                  "fp32_unsplit", "fp32_split"])
def test_bwd_adam_equals_bwd_then_adam(case):
    """crl_critic_bwd_adam against crl_critic_bwd followed by crl_adam_step on
    the same batch: parameters, BF16 copy, m and v bit for bit over three
    steps, the gradient (when kept) equal as values; the second forward also
    advances a step counter (advance=), once per call, with the same loss."""
    from paper_2408_11052_amd import Critic, crl_adam_step, crl_cast_bf16
    w = _bwd_adam_case(case)
    obs, act, phi, psi = setup(w, perturb=0.1)
    log(f"[bwd_adam] {case}: B={w.batch_size} hidden={w.hidden} prec={w.precision}")
    crit = Critic(w, max_episode_len=obs.shape[1])
    d_obs, d_act = torch.from_numpy(obs).to(DEV), torch.from_numpy(act).to(DEV)
    packed = torch.from_numpy(crit.pack(phi, psi)).to(DEV)

    def state():
        s = {"p": packed.clone(), "pb": None, "m": torch.zeros_like(packed),
             "v": torch.zeros_like(packed),
             "g": torch.full_like(packed, float("nan"))}
        if w.precision == "bf16":
            s["pb"] = torch.empty(crit.nparam, dtype=torch.bfloat16, device=DEV)
            crl_cast_bf16(s["p"], s["pb"])
        return s

    a, b = state(), state()
    x_sa, x_g, x_sg = crit.inputs(DEV)
    ws = crit.workspace(DEV)
    idx = torch.zeros(w.batch_size, 3, dtype=torch.int32, device=DEV)
    loss = torch.zeros(8, dtype=torch.float32, device=DEV)
    loss_b = torch.zeros(8, dtype=torch.float32, device=DEV)
    t = torch.zeros(1, dtype=torch.int64, device=DEV)
    adv = torch.full((1,), 40, dtype=torch.int64, device=DEV)  # advanced by b's forward
    lr = 3e-4
    bits = lambda x: x.view(torch.int32) if x.dtype == torch.float32 else x.view(torch.int16)
    for step in range(3):
        d_step = torch.tensor([step], dtype=torch.int64, device=DEV)
        t.fill_(step + 1)
        keep = step != 1
        crit.crl_sample_relabel(d_obs, d_act, 2, d_step, idx, x_sa, x_g, x_sg)
        crit.crl_critic_fwd(a["p"], a["pb"], x_sa, x_g, ws, loss)
        crit.crl_critic_bwd(a["p"], a["pb"], x_sa, x_g, ws, a["g"])
        crl_adam_step(a["p"], a["g"], a["m"], a["v"], a["pb"], t, lr)
        crit.crl_sample_relabel(d_obs, d_act, 2, d_step, idx, x_sa, x_g, x_sg)
        crit.crl_critic_fwd(b["p"], b["pb"], x_sa, x_g, ws, loss_b, advance=adv)
        crit.crl_critic_bwd_adam(b["p"], b["pb"], x_sa, x_g, ws, b["g"] if keep else None,
                                 b["m"], b["v"], t, lr)
        torch.cuda.synchronize()
        assert torch.equal(bits(loss), bits(loss_b)), step
        assert int(adv.item()) == 41 + step  # one increment per forward
        if keep:
            assert torch.equal(a["g"], b["g"]), step
        for k in ("p", "m", "v", "pb"):
            if a[k] is not None:
                assert torch.equal(bits(a[k]), bits(b[k])), (step, k)
    assert float(a["m"].abs().max()) > 0.0
    crit.close()
