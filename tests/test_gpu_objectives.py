"""GPU parity of every energy and contrastive objective (Appendix A.2) with
the FP64 oracle, through the whole critic step (relabel, encoders, critic
matrix, objective + logsumexp penalty, backward).

* Materialised logits with FP32 tiles: all 5 energies x 9 objectives at a
  ragged batch (B=200) and width (D=48).  Bars: every loss part within
  1e-4 (relative, or absolute against 1 for values near 0: FlatNCE is exactly
  1, Forward-Backward can cross 0), r, c and the diagonal to 1e-4 in relative
  L2, cosine >= 0.99999 for every parameter gradient.
* Fused logits with BF16 tiles: the products (dot, L2, cosine, L2 without the
  root) x the InfoNCE / FlatNCE objectives at B=320 (five 64-row blocks, a
  ragged last column split) and D=64, and the other representation widths
  D=32, 128, 256 on the symmetric InfoNCE.  Bars: loss parts within 1e-2, r
  and c to 1e-2 in relative L2, cosine >= 0.999 per gradient tensor.
"""
import numpy as np
import pytest

from oracle import objectives
from synthetic import workloads as WL
from tests.gpu_helpers import compare, gpu_step, oracle_step, print_report, setup

pytestmark = pytest.mark.gpu

ENERGIES = ["dot", "l2", "cos", "l2sq", "l1"]
BASE_MAT = WL.LN_FWD_FP32.with_(batch_size=200, hidden=(96, 96), repr_dim=48, num_envs=24,
                                episode_len=40)
MAT = [BASE_MAT.with_(name=f"mat_{e}_{l}", energy_function=e, contrastive_loss_function=l)
       for e in ENERGIES for l in objectives.ALL]

FUSED_LOSSES = ["fwd_infonce", "symmetric_infonce", "bwd_infonce", "flatnce_fwd", "flatnce_bwd"]
BASE_FUSED = WL.DOT_B4096_BF16.with_(batch_size=320, hidden=(128, 128), num_envs=32,
                                     episode_len=40)
FUSED = [BASE_FUSED.with_(name=f"fused_{e}_{l}", energy_function=e, contrastive_loss_function=l)
         for e in ("dot", "l2", "cos", "l2sq") for l in FUSED_LOSSES]
FUSED += [BASE_FUSED.with_(name=f"fused_{e}_sym_d{D}", energy_function=e, repr_dim=D)
          for D in (32, 128, 256) for e in ("dot", "l2", "cos")]


def _check(w, g, o, loss_tol, vec_tol, cos_tol):
    assert np.array_equal(g.idx, o["idx"])
    rep = compare(w, g, o)
    print_report(w.name, rep)
    parts = {"total": 0, "fwd": 1, "bwd": 2, "pen": 3, "obj": 7}
    for k, i in parts.items():
        err = abs(g.loss[i] - o[k]) / max(abs(o[k]), 1.0)
        assert err <= loss_tol, (k, g.loss[i], o[k], err)
    assert g.loss[6] == 0.0
    for k in ("r", "c"):
        assert rep[k] <= vec_tol, (k, rep[k])
    dg = np.asarray(o["diag"])
    assert np.linalg.norm(g.diag - dg) <= vec_tol * max(np.linalg.norm(dg), 1.0)
    assert rep["min_cos"] >= cos_tol, rep["min_cos"]
    assert np.all(np.isfinite(g.grads))


@pytest.mark.parametrize("w", MAT, ids=[w.name for w in MAT])
def test_materialised_fp32_all_objectives(w):
    obs, act, phi, psi = setup(w)
    g = gpu_step(w, obs, act, phi, psi, step=5)
    o = oracle_step(w, obs, act, phi, psi, step=5)
    _check(w, g, o, 1e-4, 1e-4, 0.99999)


@pytest.mark.parametrize("w", FUSED, ids=[w.name for w in FUSED])
def test_fused_bf16_products(w):
    obs, act, phi, psi = setup(w)
    g = gpu_step(w, obs, act, phi, psi, step=6)
    o = oracle_step(w, obs, act, phi, psi, step=6)
    _check(w, g, o, 1e-2, 1e-2, 0.999)
