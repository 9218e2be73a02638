"""crl_infonce_fwd_noalloc (the loss on given representations, run on the
library's static scratch array instead of a caller workspace) against
crl_infonce_fwd on the same inputs: the same kernels in the same order, so
loss_out, r, c and the diagonal must agree bit for bit.

Each case makes two calls in a row on one device, the second with a smaller
batch, so the second runs on what the first left in the shared array.  A
context whose loss step needs more than the array holds is rejected on the
host before anything is launched.
"""
import numpy as np
import pytest
import torch

from oracle import critic as ocritic
from oracle import objectives as oobj
from synthetic import workloads as WL
from tests.gpu_helpers import log

pytestmark = pytest.mark.gpu

MAT = WL.LN_FWD_FP32.with_(hidden=(64,), num_envs=8, episode_len=20)
FUSED = WL.DOT_B4096_BF16.with_(hidden=(64,), num_envs=8, episode_len=20)

CASES = [
    pytest.param(MAT, "l2", "symmetric_infonce", 64, (700, 300), id="materialised_fp32_l2_sym"),
    pytest.param(MAT, "cos", "dpo", 32, (520, 130), id="materialised_fp32_cos_dpo"),
    pytest.param(FUSED, "dot", "symmetric_infonce", 64, (1500, 333), id="fused_bf16_dot_sym"),
    pytest.param(FUSED, "l2", "symmetric_infonce", 256, (16384, 4100), id="fused_bf16_l2_d256"),
]


def _inputs(B, D, seed):
    rng = np.random.default_rng(seed)
    phi = rng.standard_normal((B, D)).astype(np.float32) * 0.3
    psi = (phi + 0.2 * rng.standard_normal((B, D))).astype(np.float32)
    return phi, psi


def _both(base, energy, loss, B, D, seed):
    from paper_2408_11052_amd import Critic
    w = base.with_(batch_size=B, repr_dim=D, energy_function=energy,
                   contrastive_loss_function=loss)
    crit = Critic(w)
    dev = torch.device("cuda:0")
    phi, psi = _inputs(B, D, seed)
    tp = torch.from_numpy(phi).to(dev)
    tq = torch.from_numpy(psi).to(dev)
    print(f"[noalloc] {base.logits} {energy} {loss} B={B} D={D}", flush=True)
    # the no-alloc call first, so that it runs on what earlier calls left
    lo_n = torch.full((8,), float("nan"), dtype=torch.float32, device=dev)
    r_n, c_n, d_n = (torch.full((B,), float("nan"), dtype=torch.float32, device=dev)
                     for _ in range(3))
    crit.crl_infonce_fwd_noalloc(tp, tq, lo_n, r_n, c_n, d_n)
    lo_n2 = torch.full((8,), float("nan"), dtype=torch.float32, device=dev)
    crit.crl_infonce_fwd_noalloc(tp, tq, lo_n2)   # the optional outputs left out
    ws = crit.workspace(dev)
    lo_w = torch.full((8,), float("nan"), dtype=torch.float32, device=dev)
    crit.crl_infonce_fwd(tp, tq, ws, lo_w)
    torch.cuda.synchronize()
    got = {"loss": lo_n.cpu().numpy(), "loss2": lo_n2.cpu().numpy(), "r": r_n.cpu().numpy(),
           "c": c_n.cpu().numpy(), "diag": d_n.cpu().numpy()}
    ref = {"loss": lo_w.cpu().numpy(), "r": crit.view(ws, "row_lse").cpu().numpy(),
           "c": crit.view(ws, "col_lse").cpu().numpy(),
           "diag": crit.view(ws, "diag").cpu().numpy()}
    crit.close()
    return phi, psi, got, ref


@pytest.mark.parametrize("base,energy,loss,D,sizes", CASES)
def test_noalloc_matches_the_workspace_entry_point(base, energy, loss, D, sizes):
    for k, B in enumerate(sizes):
        phi, psi, got, ref = _both(base, energy, loss, B, D, seed=10 + k)
        for name in ("r", "c", "diag"):
            assert np.array_equal(got[name], ref[name]), (B, name)
        assert np.array_equal(got["loss"], ref["loss"]), (B, got["loss"], ref["loss"])
        assert np.array_equal(got["loss2"], ref["loss"]), (B, got["loss2"], ref["loss"])
        # and both against the FP64 oracle's loss (small batches only)
        if B <= 2048:
            if base.precision == "bf16":
                phi = torch.from_numpy(phi).bfloat16().float().numpy()
                psi = torch.from_numpy(psi).bfloat16().float().numpy()
            F = ocritic.energy_matrix(phi.astype(np.float64), psi.astype(np.float64), energy)
            o = oobj.contrastive_loss(F, loss, 0.1)
            tol = 1e-4 if base.precision == "fp32" else 1e-3
            log(f"[noalloc] B={B} loss {got['loss'][0]:.7f} oracle {o['total']:.7f}")
            assert abs(got["loss"][0] - o["total"]) <= tol * max(1.0, abs(o["total"]))


def test_noalloc_rejects_a_loss_larger_than_the_array():
    from paper_2408_11052_amd import Critic
    from paper_2408_11052_amd._lib import CRL_EINVAL, lib
    from paper_2408_11052_amd.critic import _ptr, _stream
    B, D = 4096, 64   # materialised FP32: the B x B matrix alone is 64 MiB
    w = MAT.with_(batch_size=B, repr_dim=D, energy_function="l2")
    crit = Critic(w)
    dev = torch.device("cuda:0")
    phi = torch.zeros(B, D, dtype=torch.float32, device=dev)
    lo = torch.full((8,), -7.0, dtype=torch.float32, device=dev)
    rc = lib().crl_infonce_fwd_noalloc(crit.ctx, _ptr(phi), _ptr(phi), _ptr(lo), None, None,
                                       None, _stream())
    msg = lib().crl_last_error().decode()
    torch.cuda.synchronize()
    crit.close()
    assert rc == CRL_EINVAL and "scratch" in msg, (rc, msg)
    assert torch.all(lo == -7.0)   # nothing was launched
