"""GPU: the policy step (crl_actor_step) and the full update (critic, policy,
entropy coefficient) against the FP64 oracle, graph replay == eager."""
import math

import numpy as np
import pytest
import torch

from oracle import actor as oactor
from oracle import relabel as orelabel
from oracle.update import FullUpdate as OracleUpdate
from synthetic import Workload, actor_params
from synthetic import workloads as WL
from tests.gpu_helpers import SEED_PHILOX, cosine, log, rel_l2, setup

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")

SMALL = Workload(name="actor_small", num_envs=24, episode_len=60, obs_dim=13, act_dim=5,
                 goal_dim=3, goal_lo=1, states="random_walk", batch_size=200,
                 hidden=(64, 64), activation="ln_swish", repr_dim=32, energy_function="dot",
                 contrastive_loss_function="symmetric_infonce", actor_hidden=(48, 48))


def _actor_layers(w, perturb=0.1):
    return actor_params(w.in_sg, w.actor_hidden, w.act_dim, w.activation == "ln_swish",
                        seed=3, perturb=perturb)


def _to64(layers):
    return [{k: np.asarray(v, np.float64) for k, v in L.items()} for L in layers]


def _gpu_actor_step(w, obs, act, phi, psi, actor, log_alpha, step):
    from paper_2408_11052_amd import Critic, crl_cast_bf16
    crit = Critic(w, max_episode_len=obs.shape[1])
    log(f"[actor] {w.name} B={w.batch_size} prec={w.precision} energy={w.energy_function} "
        f"act={w.activation} step={step}")
    params = torch.from_numpy(crit.pack(phi, psi)).to(DEV)
    aparams = torch.from_numpy(crit.pack_actor(actor)).to(DEV)
    pbf = apbf = None
    if w.precision == "bf16":
        pbf = torch.empty(crit.nparam, dtype=torch.bfloat16, device=DEV)
        apbf = torch.empty(crit.nparam_actor, dtype=torch.bfloat16, device=DEV)
        crl_cast_bf16(params, pbf)
        crl_cast_bf16(aparams, apbf)
    x_sa, x_g, x_sg = crit.inputs(DEV)
    idx = torch.zeros(w.batch_size, 3, dtype=torch.int32, device=DEV)
    n = torch.tensor([step], dtype=torch.int64, device=DEV)
    ws = crit.workspace(DEV)
    la = torch.tensor([log_alpha, 0, 0, 0], dtype=torch.float32, device=DEV)
    agrads = torch.full((crit.nparam_actor,), float("nan"), device=DEV)
    ag = torch.zeros(4, device=DEV)
    loss = torch.zeros(4, device=DEV)
    crit.crl_sample_relabel(torch.from_numpy(obs).to(DEV), torch.from_numpy(act).to(DEV),
                            SEED_PHILOX, n, idx, x_sa, x_g, x_sg)
    crit.crl_actor_step(params, pbf, aparams, apbf, la, x_sa, x_g, x_sg, SEED_PHILOX, n, ws,
                        agrads, ag, loss)
    torch.cuda.synchronize()
    out = {"loss": loss.cpu().numpy().astype(np.float64), "alpha_grad": float(ag[0]),
           "eps": crit.view(ws, "noise").cpu().numpy(),
           "log_pi": crit.view(ws, "log_pi").cpu().numpy(),
           "f": crit.view(ws, "policy_energy").cpu().numpy(),
           "g": crit.unpack_actor(agrads.cpu().numpy()),
           "grads": agrads.cpu().numpy()}
    crit.close()
    return out


def _oracle_actor_step(w, obs, act, phi, psi, actor, log_alpha, step):
    _, x_sa, x_g, x_sg = orelabel.sample_relabel(obs, act, w.batch_size, w.discounting,
                                                 SEED_PHILOX, step, w.goal_lo, w.goal_dim)
    eps = oactor.box_muller_noise(SEED_PHILOX, step, w.batch_size, w.act_dim)
    if w.random_goal_ratio > 0:
        x_sg, x_g, _, _ = oactor.random_goal_mix(x_sg, x_g, w.obs_dim, w.random_goal_ratio,
                                                 SEED_PHILOX, step)
    out = oactor.actor_loss_and_grads(_to64(actor), _to64(phi), _to64(psi), x_sg, x_g,
                                      x_sa[:, :w.obs_dim], eps, log_alpha, w)
    out["eps"] = eps
    return out


CASES = {
    "fp32_dot_ln": SMALL,
    "fp32_l2_relu": SMALL.with_(name="actor_l2_relu", energy_function="l2", activation="relu",
                                batch_size=133),
    # the other energies of the critic on the policy's action
    "fp32_cos_ln": SMALL.with_(name="actor_cos", energy_function="cos"),
    "fp32_l2sq_ln": SMALL.with_(name="actor_l2sq", energy_function="l2sq"),
    "fp32_l1_ln": SMALL.with_(name="actor_l1", energy_function="l1", batch_size=150),
    # 64-deep K steps throughout: the policy's and critic's GEMMs take the
    # direct-to-LDS kernel, with ragged M (first-layer dW) and N (16-wide head)
    "bf16_dot_ln": SMALL.with_(name="actor_bf16", precision="bf16", logits="fused",
                               batch_size=256, hidden=(128, 128), actor_hidden=(128,) * 3),
    "bf16_l2_ln_ragged": SMALL.with_(name="actor_bf16_ragged", precision="bf16", logits="fused",
                                     energy_function="l2", batch_size=264, hidden=(128, 128),
                                     actor_hidden=(96, 96, 96)),
    # random goals (Appendix C): half, and all, of the policy's goals taken
    # from other samples of the batch
    "fp32_dot_ln_random_goals_half": SMALL.with_(name="actor_rg_half", random_goal_ratio=0.5),
    "fp32_l2_relu_random_goals_all": SMALL.with_(name="actor_rg_all", energy_function="l2",
                                                 activation="relu", random_goal_ratio=1.0),
    "bf16_dot_ln_random_goals": SMALL.with_(name="actor_rg_bf16", precision="bf16",
                                            logits="fused", batch_size=256, hidden=(128, 128),
                                            actor_hidden=(128,) * 3, random_goal_ratio=0.3),
    # a wide action: the input gradient over the action columns has N = 70, a
    # 128-wide tile with a ragged tail, and the head 192 columns
    "bf16_dot_ln_wide_action": SMALL.with_(name="actor_wide_action", precision="bf16",
                                           logits="fused", act_dim=70, batch_size=256,
                                           hidden=(128, 128), actor_hidden=(128, 128)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_actor_step_matches_oracle(case):
    w = CASES[case]
    bf16 = w.precision == "bf16"
    obs, act, phi, psi = setup(w, perturb=0.1)
    actor = _actor_layers(w)
    la, step = 0.3, 3
    g = _gpu_actor_step(w, obs, act, phi, psi, actor, la, step)
    o = _oracle_actor_step(w, obs, act, phi, psi, actor, la, step)
    # the noise: same 23-bit uniforms, FP32 log / sqrt / sincospi
    err_eps = np.max(np.abs(g["eps"] - o["eps"]) / np.maximum(1.0, np.abs(o["eps"])))
    log(f"[actor] eps max rel err {err_eps:.2e}")
    assert err_eps < 1e-5
    # log pi sums act_dim terms, each carrying the BF16 rounding of the head's
    # outputs: the BF16 bar grows with the action width beyond 17
    tol_loss = 1e-2 * max(1.0, w.act_dim / 17) if bf16 else 1e-4
    scale = abs(math.exp(la) * o["mean_log_pi"]) + abs(np.mean(o["f"]))
    d_loss = abs(g["loss"][0] - o["loss"])
    d_lp = abs(g["loss"][1] - o["mean_log_pi"])
    d_ag = abs(g["alpha_grad"] - o["d_log_alpha"])
    log(f"[actor] L_pi gpu {g['loss'][0]:.6f} oracle {o['loss']:.6f} (|d| {d_loss:.2e}); "
        f"mean log pi d {d_lp:.2e}; dlog alpha d {d_ag:.2e}")
    assert d_loss <= tol_loss * scale
    assert d_lp <= tol_loss * max(1.0, abs(o["mean_log_pi"]))
    assert d_ag <= tol_loss * max(1.0, abs(o["d_log_alpha"]))
    assert rel_l2(g["log_pi"], o["log_pi"]) < (2 * tol_loss if bf16 else 1e-5)
    assert rel_l2(g["f"], o["f"]) < (2e-2 if bf16 else 1e-5)
    cos_min = 0.999 if bf16 else 0.99999
    for l, (gl, ol) in enumerate(zip(g["g"], o["g_actor"])):
        for k in ol:
            c, r = cosine(gl[k], ol[k]), rel_l2(gl[k], ol[k])
            log(f"[actor]   layer {l} {k:5s} cos {c:.6f} rel_l2 {r:.2e}")
            assert c >= cos_min, (l, k, c)
            if not bf16:
                assert r < 1e-3, (l, k, r)
    # padding of the policy vector (gaps and the output layer's extra columns)
    real = np.zeros(g["grads"].size, bool)
    from paper_2408_11052_amd import Critic
    crit = Critic(w, max_episode_len=obs.shape[1])
    real[np.nonzero(crit.pack_actor([{k: np.ones_like(v) for k, v in L.items()}
                                      for L in actor]))] = True
    crit.close()
    assert np.all(g["grads"][~real] == 0.0)
    assert np.all(np.isfinite(g["grads"]))


def _policy_scale(ref) -> float:
    """Size of the two terms of L_pi = alpha mean(log pi) - mean(f): the loss is
    their difference and can be much smaller than either, so its error is
    measured against them."""
    return abs(ref["alpha"] * ref["mean_log_pi"]) + abs(ref["mean_f"])


def _trajectory(w, steps, tol_c, tol_a, perturb=0.1):
    from paper_2408_11052_amd.update import FullUpdate
    obs, act, phi, psi = setup(w, perturb=perturb)
    actor = _actor_layers(w, perturb=perturb)
    gu = FullUpdate(w, torch.from_numpy(obs).to(DEV), torch.from_numpy(act).to(DEV), phi, psi,
                    actor, seed=SEED_PHILOX)
    ou = OracleUpdate(w, phi, psi, actor, seed=SEED_PHILOX)
    worst_c = worst_a = 0.0
    for n in range(steps):
        gu.enqueue()
        ref = ou.step(obs, act, n)
        torch.cuda.synchronize()
        lc, la = float(gu.loss[0]), float(gu.actor_loss[0])
        lal = float(gu.log_alpha[0])
        ec = abs(lc - ref["critic"]) / abs(ref["critic"])
        ea = abs(la - ref["actor"]) / _policy_scale(ref)
        worst_c, worst_a = max(worst_c, ec), max(worst_a, ea)
        log(f"[full] step {n:2d} critic gpu {lc:.6f} oracle {ref['critic']:.6f} | actor gpu "
            f"{la:.6f} oracle {ref['actor']:.6f} | log alpha gpu {lal:.6f} oracle "
            f"{ref['log_alpha']:.6f}")
        assert ec <= tol_c, (n, lc, ref["critic"])
        assert ea <= tol_a, (n, la, ref["actor"])
        assert abs(lal - ref["log_alpha"]) <= 1e-5 + 2 * (n + 1) * w.alpha_lr * tol_a
    log(f"[full] {steps} steps: worst critic rel err {worst_c:.2e}, actor {worst_a:.2e}")
    gu.close()


def test_full_update_trajectory_fp32():
    """20 full updates at small shapes, FP32 GPU path against the FP64 oracle."""
    _trajectory(SMALL.with_(name="full_small_fp32", batch_size=160), 20, 1e-4, 1e-4)


def test_full_update_trajectory_fp32_random_goals():
    """10 full updates with half of the policy's goals taken from other
    samples (Appendix C), FP32 GPU path against the FP64 oracle."""
    _trajectory(SMALL.with_(name="full_small_fp32_rg", batch_size=160, random_goal_ratio=0.5),
                10, 1e-4, 1e-4)


@pytest.mark.slow
def test_full_update_trajectory_b4096_fp32():
    """Five free-running full updates at the B=4096 full-update shapes (4x1024
    LN+Swish critic, 4x1024 policy) on the FP32 GPU path (FP32 tiles,
    materialised logits) against the FP64 oracle: every step's critic and
    policy losses and log alpha, with no state copied between the two."""
    w = WL.FULL_UPDATE_B4096.with_(name="full_b4096_fp32", precision="fp32",
                                   logits="materialised")
    _trajectory(w, 5, 1e-4, 1e-4, perturb=0.0)


def _oracle_from_gpu(ou, gu):
    """Copy the GPU's whole update state (parameters, Adam moments, log alpha,
    step) into the oracle, in FP64."""
    c = gu.crit
    host = lambda t: t.detach().cpu().numpy()
    ou.phi, ou.psi = (_copy64(x) for x in c.unpack(host(gu.params)))
    ou.mc = [_copy64(x) for x in c.unpack(host(gu.m))]
    ou.vc = [_copy64(x) for x in c.unpack(host(gu.v))]
    ou.actor = _copy64(c.unpack_actor(host(gu.aparams)))
    ou.ma = _copy64(c.unpack_actor(host(gu.am)))
    ou.va = _copy64(c.unpack_actor(host(gu.av)))
    ou.log_alpha = float(gu.log_alpha[0])
    ou.m_alpha, ou.v_alpha = float(gu.m_alpha[0]), float(gu.v_alpha[0])
    ou.t = int(gu.t.item())


def _copy64(layers):
    return [{k: np.array(v, np.float64) for k, v in L.items()} for L in layers]


@pytest.mark.slow
def test_full_update_steps_b4096_bf16():
    """The first 20 full updates of the B=4096 workload (critic: BF16 fused,
    4x1024 LN+Swish encoders; policy 4x1024), step by step against the FP64
    oracle: before each step the oracle takes the GPU's state, so each step's
    critic and policy losses are compared from identical parameters."""
    from paper_2408_11052_amd.update import FullUpdate
    w = WL.FULL_UPDATE_B4096
    obs, act, phi, psi = setup(w, perturb=0.0)
    actor = _actor_layers(w, perturb=0.0)
    gu = FullUpdate(w, torch.from_numpy(obs).to(DEV), torch.from_numpy(act).to(DEV), phi, psi,
                    actor, seed=SEED_PHILOX)
    ou = OracleUpdate(w, phi, psi, actor, seed=SEED_PHILOX)
    worst_c = worst_a = 0.0
    for n in range(20):
        torch.cuda.synchronize()
        _oracle_from_gpu(ou, gu)
        ref = ou.step(obs, act, n)
        gu.enqueue()
        torch.cuda.synchronize()
        lc, la, lal = float(gu.loss[0]), float(gu.actor_loss[0]), float(gu.log_alpha[0])
        ec = abs(lc - ref["critic"]) / abs(ref["critic"])
        ea = abs(la - ref["actor"]) / _policy_scale(ref)
        worst_c, worst_a = max(worst_c, ec), max(worst_a, ea)
        log(f"[full] step {n:2d} critic gpu {lc:.6f} oracle {ref['critic']:.6f} ({ec:.1e}) | "
            f"policy gpu {la:.6f} oracle {ref['actor']:.6f} ({ea:.1e}) | log alpha gpu "
            f"{lal:.6f} oracle {ref['log_alpha']:.6f}")
        assert ec <= 1e-2, (n, lc, ref["critic"])
        assert ea <= 1e-2, (n, la, ref["actor"])
        # from the same state both sides take one Adam step of log alpha; its
        # gradient -(mean log pi + H) agrees to ~1e-2, so the step agrees to a
        # small fraction of lr
        assert abs(lal - ref["log_alpha"]) <= 0.1 * w.alpha_lr + 1e-6
    log(f"[full] 20 steps from the GPU state: worst critic rel err {worst_c:.2e}, "
        f"policy {worst_a:.2e}")
    gu.close()


ADAM_CASES = {
    "fp32": SMALL,
    "bf16_unsplit": CASES["bf16_dot_ln"],
    # B = 2048: the policy's dW launches are split along the batch, so their
    # partials are reduced by the fused Adam reduction
    "bf16_split": CASES["bf16_dot_ln"].with_(name="actor_adam_split", batch_size=2048,
                                             num_envs=64, episode_len=64),
    "bf16_wide_action_random_goals": CASES["bf16_dot_ln_wide_action"].with_(
        name="actor_adam_wide", random_goal_ratio=0.3),
}


@pytest.mark.parametrize("case", list(ADAM_CASES))
def test_actor_step_adam_equals_step_then_adam(case):
    """crl_actor_step_adam against crl_actor_step followed by crl_adam_step on
    the policy vector, on the same batches: policy parameters, BF16 copy, m
    and v bit for bit over three steps; the policy gradient (when kept), dlog
    alpha and the loss terms equal as values."""
    from paper_2408_11052_amd import Critic, crl_adam_step, crl_cast_bf16
    w = ADAM_CASES[case]
    obs, act, phi, psi = setup(w, perturb=0.1)
    actor = _actor_layers(w)
    log(f"[actor_adam] {case}: B={w.batch_size} hidden={w.actor_hidden} prec={w.precision}")
    crit = Critic(w, max_episode_len=obs.shape[1])
    params = torch.from_numpy(crit.pack(phi, psi)).to(DEV)
    pbf = None
    if w.precision == "bf16":
        pbf = torch.empty(crit.nparam, dtype=torch.bfloat16, device=DEV)
        crl_cast_bf16(params, pbf)
    packed = torch.from_numpy(crit.pack_actor(actor)).to(DEV)

    def state():
        s = {"p": packed.clone(), "pb": None, "m": torch.zeros_like(packed),
             "v": torch.zeros_like(packed), "g": torch.full_like(packed, float("nan")),
             "ag": torch.zeros(4, device=DEV), "loss": torch.zeros(4, device=DEV)}
        if w.precision == "bf16":
            s["pb"] = torch.empty(crit.nparam_actor, dtype=torch.bfloat16, device=DEV)
            crl_cast_bf16(s["p"], s["pb"])
        return s

    a, b = state(), state()
    x_sa, x_g, x_sg = crit.inputs(DEV)
    ws = crit.workspace(DEV)
    idx = torch.zeros(w.batch_size, 3, dtype=torch.int32, device=DEV)
    la = torch.tensor([0.3, 0, 0, 0], dtype=torch.float32, device=DEV)
    d_obs, d_act = torch.from_numpy(obs).to(DEV), torch.from_numpy(act).to(DEV)
    t = torch.zeros(1, dtype=torch.int64, device=DEV)
    lr = 6e-4
    bits = lambda x: x.view(torch.int32) if x.dtype == torch.float32 else x.view(torch.int16)
    for step in range(3):
        n = torch.tensor([step], dtype=torch.int64, device=DEV)
        t.fill_(step + 1)
        keep = step != 1
        crit.crl_sample_relabel(d_obs, d_act, SEED_PHILOX, n, idx, x_sa, x_g, x_sg)
        crit.crl_actor_step(params, pbf, a["p"], a["pb"], la, x_sa, x_g, x_sg, SEED_PHILOX, n,
                            ws, a["g"], a["ag"], a["loss"])
        crl_adam_step(a["p"], a["g"], a["m"], a["v"], a["pb"], t, lr)
        crit.crl_sample_relabel(d_obs, d_act, SEED_PHILOX, n, idx, x_sa, x_g, x_sg)
        crit.crl_actor_step_adam(params, pbf, b["p"], b["pb"], la, x_sa, x_g, x_sg, SEED_PHILOX,
                                 n, ws, b["g"] if keep else None, b["ag"], b["loss"], b["m"],
                                 b["v"], t, lr)
        torch.cuda.synchronize()
        if keep:
            assert torch.equal(a["g"], b["g"]), step
        assert torch.equal(a["ag"], b["ag"]) and torch.equal(a["loss"], b["loss"]), step
        for k in ("p", "m", "v", "pb"):
            if a[k] is not None:
                assert torch.equal(bits(a[k]), bits(b[k])), (step, k)
    assert float(a["m"].abs().max()) > 0.0
    crit.close()


@pytest.mark.parametrize("prec", ["bf16", "fp32"])
def test_full_update_graph_replay_equals_eager(prec):
    from paper_2408_11052_amd.update import FullUpdate
    w = SMALL.with_(name=f"full_graph_{prec}", precision=prec,
                    logits="fused" if prec == "bf16" else "materialised")
    obs, act, phi, psi = setup(w, perturb=0.0)
    actor = _actor_layers(w, perturb=0.0)
    d_obs, d_act = torch.from_numpy(obs).to(DEV), torch.from_numpy(act).to(DEV)
    ue = FullUpdate(w, d_obs, d_act, phi, psi, actor, seed=SEED_PHILOX)
    ug = FullUpdate(w, d_obs, d_act, phi, psi, actor, seed=SEED_PHILOX)
    g = ug.capture(2)
    for rep in range(3):
        ue.enqueue()
        ue.enqueue()
        g.replay()
        torch.cuda.synchronize()
        _ = (ue.aparams * 2).sum().item()  # eager work between replays
        for a, b in ((ue.params, ug.params), (ue.aparams, ug.aparams),
                     (ue.log_alpha, ug.log_alpha), (ue.actor_loss, ug.actor_loss),
                     (ue.loss, ug.loss)):
            assert torch.equal(a, b), rep
    assert int(ug.n.item()) == 6 and int(ug.t.item()) == 6
    ue.close()
    ug.close()
