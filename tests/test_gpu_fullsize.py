"""GPU parity at the workloads' full sizes, in the launch configuration that
bench.py times.

The B <= 4096 workloads are compared with the full FP64 oracle, and so are
the D=256 kernels at B=4096 (several column tiles per split) and the D=64
backward past its one-pass range (B=8192).  At B=16384 (D=256) the oracle's
definitions are evaluated in row blocks (tests/blocked_oracle.py) and every
output is compared.  The B=1024 FP32 workload's gradient is also checked
against central differences of the oracle's loss.
"""
import math

import numpy as np
import pytest
import torch

from oracle import critic as ocritic
from oracle import relabel as orelabel
from synthetic import WORKLOADS
from tests.gpu_helpers import compare, gpu_step, log, oracle_step, print_report, setup

pytestmark = pytest.mark.gpu

FULL = ["b256_relu2x256_l2_sym", "b1024_lnswish4x1024_l2_fwd",
        "b4096_lnswish4x1024_dot_sym", "b4096_lnswish4x1024_dot_sym_fp32"]


@pytest.mark.parametrize("name", FULL)
def test_full_size_against_oracle(name):
    w = WORKLOADS[name]
    obs, act, phi, psi = setup(w, perturb=0.0)
    g = gpu_step(w, obs, act, phi, psi, step=0)
    o = oracle_step(w, obs, act, phi, psi, step=0)
    assert np.array_equal(g.idx, o["idx"])
    rep = compare(w, g, o)
    print_report(name, rep)
    if w.precision == "fp32":
        assert rep["loss_total"] <= 1e-5
        assert rep["min_cos"] >= 0.99999
        assert rep["max_rel"] <= 1e-3
    else:
        assert rep["loss_total"] <= 1e-2
        assert rep["min_cos"] >= 0.999


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_b4096_d256_l2_sym_fused_multi_tile():
    """The D=256 kernels with several 64-column tiles per split: the forward
    and both backward passes at B=4096 (16 splits of 256 columns, 4 tiles
    each), L2 energy, symmetric InfoNCE, BF16 tiles, 2 x 1024 encoders,
    against the full FP64 oracle."""
    w = WORKLOADS["b16384_lnswish2x1024_d256_l2_sym"].with_(
        name="b4096_lnswish2x1024_d256_l2_sym", batch_size=4096)
    obs, act, phi, psi = setup(w, perturb=0.0)
    g = gpu_step(w, obs, act, phi, psi, step=1)
    o = oracle_step(w, obs, act, phi, psi, step=1)
    assert np.array_equal(g.idx, o["idx"])
    rep = compare(w, g, o)
    print_report(w.name, rep)
    for k in ("total", "fwd", "bwd", "pen"):
        assert rep["loss_" + k] <= 1e-2, k
    assert rep["r"] <= 1e-2 and rep["c"] <= 1e-2
    assert rep["dphi_cos"] >= 0.999 and rep["dpsi_cos"] >= 0.999
    assert rep["min_cos"] >= 0.999


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_b8192_d64_fused_two_pass_backward():
    """Above 16 row blocks of 256 the D=64 backward leaves the one-pass
    kernel (its partials would grow as B^2) for the row and column passes."""
    w = WORKLOADS["b4096_lnswish4x1024_dot_sym"].with_(
        name="b8192_lnswish2x256_dot_sym", batch_size=8192, hidden=(256, 256), num_envs=1024,
        episode_len=200)
    obs, act, phi, psi = setup(w, perturb=0.0)
    g = gpu_step(w, obs, act, phi, psi, step=2)
    o = oracle_step(w, obs, act, phi, psi, step=2)
    assert np.array_equal(g.idx, o["idx"])
    rep = compare(w, g, o)
    print_report(w.name, rep)
    assert rep["loss_total"] <= 1e-2 and rep["r"] <= 1e-2 and rep["c"] <= 1e-2
    assert rep["min_cos"] >= 0.999


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_b16384_d256_fused_full_size():
    """The B=16384, D=256 workload at full size against the oracle's
    definitions evaluated in row blocks (tests/blocked_oracle.py, pinned
    against the dense oracle): every loss part, r, c and the diagonal,
    dphi / dpsi, and every parameter gradient."""
    from tests.blocked_oracle import infonce_blocked
    w = WORKLOADS["b16384_lnswish2x1024_d256_l2_sym"]
    obs, act, phi, psi = setup(w, perturb=0.0)
    g = gpu_step(w, obs, act, phi, psi, step=0)
    idx, x_sa, x_g, _ = orelabel.sample_relabel(obs, act, w.batch_size, w.discounting, 2, 0,
                                                w.goal_lo, w.goal_dim)
    assert np.array_equal(g.idx, idx)
    ophi, cphi = ocritic.mlp_forward(phi, x_sa, w.activation, w.ln_eps)
    opsi, cpsi = ocritic.mlp_forward(psi, x_g, w.activation, w.ln_eps)
    o = infonce_blocked(ophi, opsi, w.energy_function, w.contrastive_loss_function,
                        w.logsumexp_penalty)
    o["g_phi"], _ = ocritic.mlp_backward(phi, cphi, o["dphi"], w.activation)
    o["g_psi"], _ = ocritic.mlp_backward(psi, cpsi, o["dpsi"], w.activation)
    o["phi"], o["psi"] = ophi, opsi
    rep = compare(w, g, o)
    print_report(w.name, rep)
    for k in ("total", "fwd", "bwd", "pen"):
        assert rep["loss_" + k] <= 1e-2, k
    for k in ("r", "c"):
        assert rep[k] <= 1e-2, k
    assert np.linalg.norm(g.diag - o["diag"]) <= 1e-2 * np.linalg.norm(o["diag"])
    assert rep["phi"] <= 2e-2 and rep["psi"] <= 2e-2
    assert rep["dphi_cos"] >= 0.999 and rep["dpsi_cos"] >= 0.999
    assert rep["min_cos"] >= 0.999
    assert np.all(np.isfinite(g.grads))


@pytest.mark.slow
@pytest.mark.timeout(900)
def test_b1024_fp32_gradient_central_differences():
    """The B=1024, 4 x 1024 LayerNorm + Swish, L2, forward-InfoNCE workload in
    FP32: the hand-written backward against central differences (eps 1e-3)
    of the FP64 oracle's loss on 64 random parameter coordinates."""
    w = WORKLOADS["b1024_lnswish4x1024_l2_fwd"]
    obs, act, phi, psi = setup(w, perturb=0.1)
    g = gpu_step(w, obs, act, phi, psi, step=0)
    _, x_sa, x_g, _ = orelabel.sample_relabel(obs, act, w.batch_size, w.discounting, 2, 0,
                                              w.goal_lo, w.goal_dim)
    p64 = [{k: v.astype(np.float64) for k, v in L.items()} for L in phi]
    q64 = [{k: v.astype(np.float64) for k, v in L.items()} for L in psi]
    rng = np.random.default_rng(11)
    keys = [(side, i, k) for side, layers in (("phi", p64), ("psi", q64))
            for i, L in enumerate(layers) for k in L]
    eps = 1e-3
    worst = 0.0
    for n in range(64):
        side, i, k = keys[rng.integers(len(keys))]
        arr = (p64 if side == "phi" else q64)[i][k]
        j = tuple(int(rng.integers(s)) for s in arr.shape)
        old = arr[j]
        arr[j] = old + eps
        lp = ocritic.loss_only(p64, q64, x_sa, x_g, w)
        arr[j] = old - eps
        lm = ocritic.loss_only(p64, q64, x_sa, x_g, w)
        arr[j] = old
        fd = (lp - lm) / (2 * eps)
        got = float(getattr(g, "g_" + side)[i][k][j])
        err = abs(got - fd) / (abs(fd) + 1e-6)
        worst = max(worst, err)
        assert abs(got - fd) <= 2e-3 * abs(fd) + 2e-6, (side, i, k, j, got, fd)
    log(f"[fd b1024] worst relative deviation over 64 coordinates {worst:.2e}")
