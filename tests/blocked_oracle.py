"""The InfoNCE loss and its gradients at batch sizes whose B x B matrices the
dense oracle cannot hold at once (B = 16384: 2 GiB per FP64 matrix), evaluated
in row blocks from the same definitions as ``oracle.critic`` (Section 3.1
objective; Appendix A.2 energies and InfoNCE variants; the logsumexp
penalty).  Test infrastructure: it is pinned against the dense oracle in
``tests/test_blocked_oracle.py``.

Two passes over row blocks of F (FP64):
  1. r_i = LSE_j F_ij and F_ii per block; column (max, sum) pairs merged over
     the blocks, giving c_j;
  2. G = dL/dF per block from r, c; dphi for the block's rows; dpsi summed
     over blocks (dot: G psi, G^T phi; L2: with H = G / d as in the oracle).
The L2 distances of a block are torch.cdist's direct (non-matmul) evaluation
of ||phi_i - psi_j||, the oracle's definition.
"""
from __future__ import annotations

import math

import numpy as np
import torch


def _energy_block(phi_blk, psi, kind):
    if kind == "dot":
        return phi_blk @ psi.T
    if kind == "l2":
        return -torch.cdist(torch.from_numpy(phi_blk), torch.from_numpy(psi),
                            compute_mode="donot_use_mm_for_euclid_dist").numpy()
    raise ValueError(kind)


def infonce_blocked(phi, psi, kind: str, loss: str, beta: float, block: int = 1024):
    """Loss parts, r, c, diag, dphi, dpsi (FP64) for fwd_infonce / symmetric_infonce."""
    phi = np.asarray(phi, np.float64)
    psi = np.asarray(psi, np.float64)
    B = phi.shape[0]
    sym = loss == "symmetric_infonce"
    if loss not in ("fwd_infonce", "symmetric_infonce"):
        raise ValueError(loss)
    r = np.empty(B)
    dg = np.empty(B)
    cm = np.full(B, -np.inf)
    cs = np.zeros(B)
    for i0 in range(0, B, block):
        F = _energy_block(phi[i0:i0 + block], psi, kind)
        n = F.shape[0]
        m = F.max(axis=1)
        r[i0:i0 + n] = m + np.log(np.exp(F - m[:, None]).sum(axis=1))
        dg[i0:i0 + n] = F[np.arange(n), i0 + np.arange(n)]
        bm = F.max(axis=0)
        nm = np.maximum(cm, bm)
        cs = cs * np.exp(cm - nm) + np.exp(F - nm[None, :]).sum(axis=0)
        cm = nm
    c = cm + np.log(cs)
    l_fwd = math.fsum((r - dg).tolist()) / B
    l_bwd = math.fsum((c - dg).tolist()) / B
    l_pen = beta * math.fsum((r * r).tolist()) / B
    total = l_fwd + (l_bwd if sym else 0.0) + l_pen
    dphi = np.empty_like(phi)
    dpsi = np.zeros_like(psi)
    for i0 in range(0, B, block):
        F = _energy_block(phi[i0:i0 + block], psi, kind)
        n = F.shape[0]
        ri = r[i0:i0 + n, None]
        Pr = np.exp(F - ri)
        G = Pr / B + (2.0 * beta / B) * ri * Pr
        G[np.arange(n), i0 + np.arange(n)] -= 1.0 / B
        if sym:
            G += np.exp(F - c[None, :]) / B
            G[np.arange(n), i0 + np.arange(n)] -= 1.0 / B
        ph = phi[i0:i0 + n]
        if kind == "dot":
            dphi[i0:i0 + n] = G @ psi
            dpsi += G.T @ ph
        else:
            d = -F
            H = np.where(d > 0.0, G / np.where(d > 0.0, d, 1.0), 0.0)
            dphi[i0:i0 + n] = -(H.sum(axis=1)[:, None] * ph - H @ psi)
            dpsi += H.T @ ph - H.sum(axis=0)[:, None] * psi
    return {"total": total, "fwd": l_fwd, "bwd": l_bwd, "pen": l_pen, "r": r, "c": c,
            "diag": dg, "dphi": dphi, "dpsi": dpsi}
