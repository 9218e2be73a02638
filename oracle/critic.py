"""Contrastive critic: encoders, energies, InfoNCE + logsumexp penalty, and
their gradients, in plain FP64 numpy.

What is computed (Section 3.1, "Contrastive Critic Learning"; Appendix A.2,
"Energy functions and contrastive objectives"; Algorithm 1, critic update):

* phi(s, a) and psi(g) are MLPs.  A hidden layer is z = x W + b followed by
  ReLU, or by LayerNorm (over features, biased variance) with affine
  scale/offset and then Swish y * sigmoid(y) (Section 5.4 puts LayerNorm
  before every activation).  The output layer is linear.
* The critic matrix is F_ij = f(s_i, a_i, g_j) over the batch, with one of
  the energies of Appendix A.2 (the sign follows that table): dot
  <phi_i, psi_j>; cosine <phi_i, psi_j> / (||phi_i|| ||psi_j||) (read as 0
  where a norm is 0); L1 -||phi_i - psi_j||_1; L2 -||phi_i - psi_j||_2; and
  L2 without the square root -||phi_i - psi_j||_2^2.
* InfoNCE-forward contrasts each row against its batch, InfoNCE-backward each
  column; the symmetric objective is their sum.  Each is averaged over the
  batch (so all-zero logits give log B per direction).
* The logsumexp penalty, named but not written out in the paper, is read as
  beta * mean_i (LSE_j F_ij)^2 over the row log-sum-exps.

Gradients are derived by hand from these definitions:
  dL/dF_ij = (1/B)[(Pr_ij - d_ij) + s (Pc_ij - d_ij) + 2 beta r_i Pr_ij]
with Pr_ij = exp(F_ij - r_i), Pc_ij = exp(F_ij - c_j), d the Kronecker delta
and s = 1 for the symmetric loss, 0 for the forward one; then through the
energy and, by the chain rule, through the MLPs.

Test infrastructure only (see ``oracle/__init__.py``).
"""
from __future__ import annotations

import math
from typing import Dict, List, Tuple

import numpy as np

f64 = np.float64


def _to64(layers):
    return [{k: np.asarray(v, dtype=f64) for k, v in L.items()} for L in layers]


# --------------------------------------------------------------------------
# encoders
# --------------------------------------------------------------------------
def sigmoid(y):
    return 1.0 / (1.0 + np.exp(-y))


def mlp_forward(layers, x, activation: str, ln_eps: float = 1e-6):
    """Returns (output, caches) of the MLP on x [B, in]."""
    layers = _to64(layers)
    h = np.asarray(x, dtype=f64)
    caches = []
    n = len(layers)
    for i, L in enumerate(layers):
        z = h @ L["W"] + L["b"]
        if i == n - 1:
            caches.append({"x": h})
            return z, caches
        if activation == "relu":
            caches.append({"x": h, "z": z})
            h = np.maximum(z, 0.0)
        elif activation == "ln_swish":
            mu = z.mean(axis=1, keepdims=True)
            var = ((z - mu) ** 2).mean(axis=1, keepdims=True)
            rstd = 1.0 / np.sqrt(var + ln_eps)
            zh = (z - mu) * rstd
            y = L["ln_g"] * zh + L["ln_b"]
            sg = sigmoid(y)
            caches.append({"x": h, "zh": zh, "rstd": rstd, "y": y, "sig": sg,
                           "mu": mu})
            h = y * sg
        else:
            raise ValueError(activation)
    raise AssertionError("empty MLP")


def mlp_backward(layers, caches, dout, activation: str):
    """Gradients of every parameter, and d(loss)/d(input), given dL/d(out)."""
    layers = _to64(layers)
    grads: List[Dict[str, np.ndarray]] = [dict() for _ in layers]
    d = np.asarray(dout, dtype=f64)
    n = len(layers)
    for i in range(n - 1, -1, -1):
        c, L = caches[i], layers[i]
        if i == n - 1:
            dz = d
        elif activation == "relu":
            dz = d * (c["z"] > 0.0)
        else:
            y, sg, zh, rstd = c["y"], c["sig"], c["zh"], c["rstd"]
            dy = d * (sg * (1.0 + y * (1.0 - sg)))       # Swish'(y)
            grads[i]["ln_g"] = (dy * zh).sum(axis=0)
            grads[i]["ln_b"] = dy.sum(axis=0)
            dzh = dy * L["ln_g"]
            dz = rstd * (dzh - dzh.mean(axis=1, keepdims=True)
                         - zh * (dzh * zh).mean(axis=1, keepdims=True))
        grads[i]["W"] = c["x"].T @ dz
        grads[i]["b"] = dz.sum(axis=0)
        d = dz @ L["W"].T
    return grads, d


# --------------------------------------------------------------------------
# energies
# --------------------------------------------------------------------------
def _unit(X):
    n = np.sqrt((X * X).sum(axis=1))
    return X / np.where(n > 0.0, n, 1.0)[:, None] * (n > 0.0)[:, None], n


def energy_matrix(phi, psi, kind: str, block: int = 256):
    """F_ij for all pairs.  The distances are evaluated directly from the
    differences phi_i - psi_j."""
    phi = np.asarray(phi, f64)
    psi = np.asarray(psi, f64)
    if kind == "dot":
        return phi @ psi.T
    if kind == "cos":
        return _unit(phi)[0] @ _unit(psi)[0].T
    if kind in ("l2", "l2sq", "l1"):
        F = np.empty((phi.shape[0], psi.shape[0]), f64)
        for i0 in range(0, phi.shape[0], block):
            diff = phi[i0:i0 + block, None, :] - psi[None, :, :]
            if kind == "l1":
                F[i0:i0 + block] = -np.abs(diff).sum(axis=2)
            elif kind == "l2":
                F[i0:i0 + block] = -np.sqrt((diff * diff).sum(axis=2))
            else:
                F[i0:i0 + block] = -(diff * diff).sum(axis=2)
        return F
    raise ValueError(kind)


def energy_row(phi_i, psi, kind: str):
    """One row F_i. of the critic matrix."""
    phi_i = np.asarray(phi_i, f64)
    psi = np.asarray(psi, f64)
    if kind == "dot":
        return psi @ phi_i
    if kind == "cos":
        return energy_matrix(phi_i[None, :], psi, "cos")[0]
    diff = phi_i[None, :] - psi
    if kind == "l1":
        return -np.abs(diff).sum(axis=1)
    if kind == "l2sq":
        return -(diff * diff).sum(axis=1)
    return -np.sqrt((diff * diff).sum(axis=1))


def pair_energy(phi, psi, kind: str):
    """f_b = energy(phi_b, psi_b) for matching rows b (the critic's diagonal),
    and df_b / dphi_b."""
    phi = np.asarray(phi, f64)
    psi = np.asarray(psi, f64)
    diff = phi - psi
    if kind == "dot":
        return (phi * psi).sum(axis=1), psi.copy()
    if kind == "l2":
        d = np.sqrt((diff * diff).sum(axis=1))
        inv = np.where(d > 0.0, 1.0 / np.where(d > 0.0, d, 1.0), 0.0)
        return -d, -diff * inv[:, None]
    if kind == "l2sq":
        return -(diff * diff).sum(axis=1), -2.0 * diff
    if kind == "l1":
        return -np.abs(diff).sum(axis=1), -np.sign(diff)
    if kind == "cos":
        u, nu = _unit(phi)
        v, _ = _unit(psi)
        f = (u * v).sum(axis=1)
        iu = np.where(nu > 0.0, 1.0 / np.where(nu > 0.0, nu, 1.0), 0.0)
        return f, (v - f[:, None] * u) * iu[:, None]
    raise ValueError(kind)


def energy_backward(phi, psi, F, G, kind: str):
    """Push dL/dF through the energy: returns (dphi, dpsi)."""
    phi = np.asarray(phi, f64)
    psi = np.asarray(psi, f64)
    if kind == "dot":
        return G @ psi, G.T @ phi
    if kind == "l2":
        # dF_ij/dphi_i = -(phi_i - psi_j)/d_ij, dF_ij/dpsi_j = +(phi_i - psi_j)/d_ij
        d = -F
        H = np.where(d > 0.0, G / np.where(d > 0.0, d, 1.0), 0.0)
        dphi = -(H.sum(axis=1)[:, None] * phi - H @ psi)
        dpsi = H.T @ phi - H.sum(axis=0)[:, None] * psi
        return dphi, dpsi
    if kind == "l2sq":
        # dF_ij/dphi_i = -2 (phi_i - psi_j), dF_ij/dpsi_j = +2 (phi_i - psi_j)
        dphi = -2.0 * (G.sum(axis=1)[:, None] * phi - G @ psi)
        dpsi = 2.0 * (G.T @ phi - G.sum(axis=0)[:, None] * psi)
        return dphi, dpsi
    if kind == "cos":
        # with u_i = phi_i / |phi_i|, v_j = psi_j / |psi_j|, F_ij = u_i . v_j:
        # dF_ij/dphi_i = (v_j - F_ij u_i) / |phi_i|, dF_ij/dpsi_j = (u_i - F_ij v_j) / |psi_j|
        u, nu = _unit(phi)
        v, nv = _unit(psi)
        iu = np.where(nu > 0.0, 1.0 / np.where(nu > 0.0, nu, 1.0), 0.0)
        iv = np.where(nv > 0.0, 1.0 / np.where(nv > 0.0, nv, 1.0), 0.0)
        GF = G * F
        dphi = (G @ v - GF.sum(axis=1)[:, None] * u) * iu[:, None]
        dpsi = (G.T @ u - GF.sum(axis=0)[:, None] * v) * iv[:, None]
        return dphi, dpsi
    if kind == "l1":
        # dF_ij/dphi_ik = -sign(phi_ik - psi_jk) (0 where they are equal)
        dphi = np.empty_like(phi)
        dpsi = np.zeros_like(psi)
        for i in range(phi.shape[0]):
            sg = np.sign(phi[i][None, :] - psi)        # [B_psi][D]
            dphi[i] = -(G[i][:, None] * sg).sum(axis=0)
            dpsi += G[i][:, None] * sg
        return dphi, dpsi
    raise ValueError(kind)


# --------------------------------------------------------------------------
# InfoNCE + logsumexp penalty
# --------------------------------------------------------------------------
def logsumexp(x, axis):
    m = x.max(axis=axis, keepdims=True)
    return (m + np.log(np.exp(x - m).sum(axis=axis, keepdims=True))).squeeze(axis)


def infonce_loss(F, loss: str, beta: float) -> Dict[str, object]:
    """Loss parts: total, fwd, bwd, pen; plus r, c (row/col LSE) and diag."""
    F = np.asarray(F, f64)
    B = F.shape[0]
    r = logsumexp(F, 1)
    c = logsumexp(F, 0)
    dg = np.diag(F).copy()
    l_fwd = math.fsum((r - dg).tolist()) / B
    l_bwd = math.fsum((c - dg).tolist()) / B
    l_pen = beta * math.fsum((r * r).tolist()) / B
    if loss == "symmetric_infonce":
        total = l_fwd + l_bwd + l_pen
    elif loss == "fwd_infonce":
        total = l_fwd + l_pen
    else:
        raise ValueError(loss)
    return {"total": total, "fwd": l_fwd, "bwd": l_bwd, "pen": l_pen,
            "r": r, "c": c, "diag": dg}


def infonce_grad(F, r, c, loss: str, beta: float):
    """dL/dF for the loss of ``infonce_loss``."""
    F = np.asarray(F, f64)
    B = F.shape[0]
    eye = np.eye(B)
    Pr = np.exp(F - r[:, None])
    G = (Pr - eye) / B + (2.0 * beta / B) * r[:, None] * Pr
    if loss == "symmetric_infonce":
        Pc = np.exp(F - c[None, :])
        G = G + (Pc - eye) / B
    return G


# --------------------------------------------------------------------------
# whole critic step
# --------------------------------------------------------------------------
def critic_forward(phi_layers, psi_layers, x_sa, x_g, w) -> Dict[str, object]:
    phi, c_phi = mlp_forward(phi_layers, x_sa, w.activation, w.ln_eps)
    psi, c_psi = mlp_forward(psi_layers, x_g, w.activation, w.ln_eps)
    from .objectives import contrastive_loss
    F = energy_matrix(phi, psi, w.energy_function)
    out = contrastive_loss(F, w.contrastive_loss_function, w.logsumexp_penalty)
    out.update(phi=phi, psi=psi, F=F, c_phi=c_phi, c_psi=c_psi)
    return out


def critic_loss_and_grads(phi_layers, psi_layers, x_sa, x_g, w):
    """Forward and backward of the critic loss; grads per layer for phi, psi."""
    fw = critic_forward(phi_layers, psi_layers, x_sa, x_g, w)
    from .objectives import contrastive_grad
    G = contrastive_grad(fw["F"], fw["r"], fw["c"], w.contrastive_loss_function,
                         w.logsumexp_penalty)
    dphi, dpsi = energy_backward(fw["phi"], fw["psi"], fw["F"], G,
                                 w.energy_function)
    g_phi, _ = mlp_backward(phi_layers, fw["c_phi"], dphi, w.activation)
    g_psi, _ = mlp_backward(psi_layers, fw["c_psi"], dpsi, w.activation)
    fw.update(G=G, dphi=dphi, dpsi=dpsi, g_phi=g_phi, g_psi=g_psi)
    return fw


def loss_only(phi_layers, psi_layers, x_sa, x_g, w) -> float:
    return critic_forward(phi_layers, psi_layers, x_sa, x_g, w)["total"]
