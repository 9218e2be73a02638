"""The contrastive objectives the paper evaluates besides InfoNCE-forward and
InfoNCE-symmetric, in plain FP64 numpy.

What is computed (Appendix A.2, "Energy functions and contrastive
objectives", the list of tested objectives; Section 4.3, "Contrastive
losses"; Section 5.3, the comparison of objectives, where the logsumexp
penalty with coefficient 0.1 is applied to every objective).  F is the B x B
critic matrix F_ij = f(s_i, a_i, g_j), positives on the diagonal.

Readings (the paper writes the objectives inside an expectation over the
batch with sums over i; as for InfoNCE, the sum over positives i is read as a
mean, so that all-zero logits give log B per InfoNCE direction; sums over
negatives j are kept as printed, over the whole batch, j = i included):

* InfoNCE-backward:   L = mean_j (c_j - F_jj), c_j = LSE_i F_ij.
* FlatNCE-forward:    with S_i = sum_j exp(F_ij - F_ii), the printed form is
  -log(S_i / detach(S_i)).  Taken literally its gradient is the negative of
  InfoNCE's, which would push positive pairs apart; the loss is read as the
  FlatNCE estimator it names, S_i / detach(S_i), averaged over i: its value
  is 1 for every row and its gradient is that of mean_i log S_i, i.e.
  (1/B)(P_ij - d_ij) with P_ij = exp(F_ij - r_i).
* FlatNCE-backward:   the same over columns: value 1, gradient
  (1/B)(Pc_ij - d_ij) with Pc_ij = exp(F_ij - c_j).
* Forward-Backward:   L = mean_i [-exp(F_ii) + (1 / (2(B-1))) sum_{j != i}
  exp(F_ij)^2]; for B = 1 the second term (no negatives) is 0.
* DPO:  L = mean_i sum_j -log sigmoid(F_ii - F_ij).
* IPO:  L = mean_i sum_j ((F_ii - F_ij) - 1)^2.
* SPPO: L = mean_i sum_j [(F_ii - 1)^2 + (F_ij + 1)^2].
* every objective gets the penalty beta * mean_i r_i^2, r_i = LSE_j F_ij.

Gradients dL/dF_ij are derived by hand from these definitions.

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import math
from typing import Dict

import numpy as np

from . import critic as C

f64 = np.float64

INFONCE = ("fwd_infonce", "symmetric_infonce")
ALL = ("fwd_infonce", "symmetric_infonce", "bwd_infonce", "flatnce_fwd", "flatnce_bwd",
       "fb", "dpo", "ipo", "sppo")


def _fsum_mean(v) -> float:
    v = np.asarray(v, f64).ravel()
    return math.fsum(v.tolist()) / max(len(v), 1)


def softplus(x):
    return np.logaddexp(0.0, x)


def sigmoid(x):
    return 0.5 * (1.0 + np.tanh(0.5 * x))


def contrastive_loss(F, loss: str, beta: float) -> Dict[str, object]:
    """Loss parts: total, obj (the objective), fwd / bwd (the InfoNCE
    directions mean(r - diag), mean(c - diag)), pen; and r, c, diag."""
    if loss in INFONCE:
        out = C.infonce_loss(F, loss, beta)
        out["obj"] = out["total"] - out["pen"]
        return out
    F = np.asarray(F, f64)
    B = F.shape[0]
    r = C.logsumexp(F, 1)
    c = C.logsumexp(F, 0)
    dg = np.diag(F).copy()
    pen = beta * _fsum_mean(r * r)
    off = ~np.eye(B, dtype=bool)
    if loss == "bwd_infonce":
        obj = _fsum_mean(c - dg)
    elif loss == "flatnce_fwd":
        logS = r - dg                    # log sum_j exp(F_ij - F_ii)
        obj = _fsum_mean(np.exp(logS - logS))
    elif loss == "flatnce_bwd":
        logS = c - dg
        obj = _fsum_mean(np.exp(logS - logS))
    elif loss == "fb":
        neg = np.where(off, np.exp(2.0 * F), 0.0).sum(axis=1)
        scale = 1.0 / (2.0 * (B - 1)) if B > 1 else 0.0
        obj = _fsum_mean(-np.exp(dg) + scale * neg)
    elif loss == "dpo":
        obj = _fsum_mean(softplus(F - dg[:, None]).sum(axis=1))
    elif loss == "ipo":
        obj = _fsum_mean((((dg[:, None] - F) - 1.0) ** 2).sum(axis=1))
    elif loss == "sppo":
        obj = _fsum_mean(B * (dg - 1.0) ** 2 + ((F + 1.0) ** 2).sum(axis=1))
    else:
        raise ValueError(loss)
    # fwd / bwd: the two InfoNCE directions at this F, reported beside any
    # objective
    return {"total": obj + pen, "obj": obj, "fwd": _fsum_mean(r - dg), "bwd": _fsum_mean(c - dg),
            "pen": pen, "r": r, "c": c, "diag": dg}


def contrastive_grad(F, r, c, loss: str, beta: float):
    """dL/dF for the loss of ``contrastive_loss``."""
    if loss in INFONCE:
        return C.infonce_grad(F, r, c, loss, beta)
    F = np.asarray(F, f64)
    B = F.shape[0]
    eye = np.eye(B)
    off = 1.0 - eye
    dg = np.diag(F)
    Pr = np.exp(F - r[:, None])
    G = (2.0 * beta / B) * r[:, None] * Pr            # the penalty
    if loss in ("bwd_infonce", "flatnce_bwd"):
        Pc = np.exp(F - c[None, :])
        G = G + (Pc - eye) / B
    elif loss == "flatnce_fwd":
        G = G + (Pr - eye) / B
    elif loss == "fb":
        scale = 1.0 / (B - 1) if B > 1 else 0.0     # d/dF of exp(2F) / (2(B-1))
        G = G + (-np.exp(dg) * eye + scale * off * np.exp(2.0 * F)) / B
    elif loss == "dpo":
        # d/dF_ij softplus(F_ij - F_ii) = sigmoid(F_ij - F_ii), and minus that
        # on F_ii; the j = i term is constant
        s = off * sigmoid(F - dg[:, None])
        G = G + (s - eye * s.sum(axis=1)[:, None]) / B
    elif loss == "ipo":
        e = off * ((dg[:, None] - F) - 1.0)
        G = G + (-2.0 * e + eye * 2.0 * e.sum(axis=1)[:, None]) / B
    elif loss == "sppo":
        G = G + (2.0 * (F + 1.0) + eye * 2.0 * B * (dg[:, None] - 1.0)) / B
    else:
        raise ValueError(loss)
    return G
