"""Python binding of the CRL update library: argument marshalling only.

Every step of the update runs in libcrl.so; this module turns torch tensors
into device pointers and the current HIP stream, and calls the C ABI
(include/crl.h) with the same names.  PyTorch supplies device memory and
streams.
"""
from __future__ import annotations

import ctypes as C
from typing import Dict, List, Tuple

import numpy as np
import torch

from ._lib import (ACT, ENERGY, LOGITS, LOSS, PREC, WS, check, crl_config,
                   crl_layer_info, lib)


def _ptr(t) -> C.c_void_p:
    if t is None:
        return C.c_void_p(None)
    return C.c_void_p(t.data_ptr())


def _stream(stream=None) -> C.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def make_config(w, max_episode_len: int | None = None) -> crl_config:
    """crl_config for a workload record (synthetic.Workload or alike)."""
    hid = tuple(w.hidden)
    if len(set(hid)) != 1:
        raise ValueError("all hidden layers must have the same width")
    c = crl_config()
    c.batch = w.batch_size
    c.obs_dim = w.obs_dim
    c.act_dim = w.act_dim
    c.goal_dim = w.goal_dim
    c.goal_lo = w.goal_lo
    c.n_hidden = len(hid)
    c.hidden = hid[0]
    c.repr_dim = w.repr_dim
    c.activation = ACT[w.activation]
    c.energy = ENERGY[w.energy_function]
    c.loss = LOSS[w.contrastive_loss_function]
    c.precision = PREC[w.precision]
    c.logits = LOGITS[w.logits]
    c.logsumexp_penalty = w.logsumexp_penalty
    c.ln_eps = w.ln_eps
    c.discount = w.discounting
    c.max_episode_len = max_episode_len or w.episode_len
    ahid = tuple(getattr(w, "actor_hidden", ()) or ())
    if ahid:
        if len(set(ahid)) != 1:
            raise ValueError("all policy hidden layers must have the same width")
        c.actor_n_hidden = len(ahid)
        c.actor_hidden = ahid[0]
        c.target_entropy = -float(w.act_dim)
        c.random_goal_ratio = float(getattr(w, "random_goal_ratio", 0.0))
    return c


class Critic:
    """One crl_ctx plus the layouts it defines."""

    def __init__(self, w, max_episode_len: int | None = None):
        self.w = w
        self.cfg = make_config(w, max_episode_len)
        self.ctx = C.c_void_p()
        check(lib().crl_create(C.byref(self.cfg), C.byref(self.ctx)))
        n = C.c_int64()
        check(lib().crl_param_count(self.ctx, C.byref(n)))
        self.nparam = n.value
        ws = C.c_int64()
        check(lib().crl_workspace_size(self.ctx, C.byref(ws)))
        self.ws_bytes = ws.value
        a, b, c, e = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        check(lib().crl_input_layout(self.ctx, C.byref(a), C.byref(b), C.byref(c), C.byref(e)))
        self.ld_sa, self.ld_g, self.ld_sg, self.elem_bytes = a.value, b.value, c.value, e.value
        self.layers: List[List[crl_layer_info]] = []
        for net, depth in ((0, self.cfg.n_hidden), (1, self.cfg.n_hidden),
                           (2, self.cfg.actor_n_hidden)):
            if net == 2 and depth == 0:
                break
            row = []
            for l in range(depth + 1):
                info = crl_layer_info()
                check(lib().crl_layer_layout(self.ctx, net, l, C.byref(info)))
                row.append(info)
            self.layers.append(row)
        check(lib().crl_actor_param_count(self.ctx, C.byref(n)))
        self.nparam_actor = n.value
        self.has_actor = self.nparam_actor > 0

    def close(self):
        if self.ctx:
            lib().crl_destroy(self.ctx)
            self.ctx = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ layouts
    @property
    def act_dtype(self):
        return torch.bfloat16 if self.elem_bytes == 2 else torch.float32

    @staticmethod
    def _pack_into(flat, infos, layers):
        for info, L in zip(infos, layers):
            W = np.asarray(L["W"], np.float32)
            # the policy's output layer may be narrower than its padded width
            assert W.shape[0] == info.fan_in and W.shape[1] <= info.fan_out, (W.shape, info.fan_out)
            full = np.zeros((info.fan_in, info.fan_out), np.float32)
            full[:, :W.shape[1]] = W
            flat[info.w:info.w + full.size] = full.reshape(-1)
            flat[info.b:info.b + W.shape[1]] = L["b"]
            if info.ln_g >= 0:
                flat[info.ln_g:info.ln_g + info.fan_out] = L["ln_g"]
                flat[info.ln_b:info.ln_b + info.fan_out] = L["ln_b"]

    @staticmethod
    def _unpack_from(flat, infos, out_cols=None):
        layers = []
        for i, info in enumerate(infos):
            cols = out_cols if (out_cols is not None and i == len(infos) - 1) else info.fan_out
            L: Dict[str, np.ndarray] = {
                "W": flat[info.w:info.w + info.fan_in * info.fan_out].reshape(
                    info.fan_in, info.fan_out)[:, :cols],
                "b": flat[info.b:info.b + cols]}
            if info.ln_g >= 0:
                L["ln_g"] = flat[info.ln_g:info.ln_g + info.fan_out]
                L["ln_b"] = flat[info.ln_b:info.ln_b + info.fan_out]
            layers.append(L)
        return layers

    def pack(self, phi_layers, psi_layers) -> np.ndarray:
        """Flat FP32 critic vector (zero padding) from per-layer arrays."""
        flat = np.zeros(self.nparam, np.float32)
        self._pack_into(flat, self.layers[0], phi_layers)
        self._pack_into(flat, self.layers[1], psi_layers)
        return flat

    def unpack(self, flat) -> Tuple[list, list]:
        """Per-layer dicts (numpy FP32) from a flat critic vector (params or grads)."""
        flat = np.asarray(flat)
        return self._unpack_from(flat, self.layers[0]), self._unpack_from(flat, self.layers[1])

    def pack_actor(self, layers) -> np.ndarray:
        """Flat FP32 policy vector; the output layer's padding columns are 0."""
        flat = np.zeros(self.nparam_actor, np.float32)
        self._pack_into(flat, self.layers[2], layers)
        return flat

    def unpack_actor(self, flat) -> list:
        """Per-layer dicts of the policy, output layer cut to 2 act_dim columns."""
        return self._unpack_from(np.asarray(flat), self.layers[2], 2 * self.cfg.act_dim)

    def inputs(self, device="cuda"):
        """Empty x_sa, x_g, x_sg in the storage type and strides of this ctx."""
        B = self.cfg.batch
        dt = self.act_dtype
        return (torch.zeros(B, self.ld_sa, dtype=dt, device=device),
                torch.zeros(B, self.ld_g, dtype=dt, device=device),
                torch.zeros(B, self.ld_sg, dtype=dt, device=device))

    def workspace(self, device="cuda"):
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def view(self, ws: torch.Tensor, name: str) -> torch.Tensor:
        off, nb = C.c_int64(), C.c_int64()
        check(lib().crl_workspace_view(self.ctx, WS[name], C.byref(off), C.byref(nb)))
        v = ws[off.value:off.value + nb.value].view(torch.float32)
        B, D = self.cfg.batch, self.cfg.repr_dim
        if name in ("phi", "psi", "dphi", "dpsi"):
            return v.view(B, D)
        if name == "logits":
            ld = (B + 7) // 8 * 8
            return v.view(B, ld)[:, :B]
        A = self.cfg.act_dim
        if name == "policy_out":
            return v.view(B, -1)
        if name == "noise":
            return v.view(B, A)
        if name == "daction":
            return v.view(B, -1)[:, :A]
        return v

    # ------------------------------------------------------------ entry points
    def crl_sample_relabel(self, obs, act, seed: int, step, idx, x_sa, x_g, x_sg=None,
                           stream=None):
        E, T = obs.shape[0], obs.shape[1]
        check(lib().crl_sample_relabel(self.ctx, _ptr(obs), _ptr(act), E, T, seed,
                                       _ptr(step), _ptr(idx), _ptr(x_sa), _ptr(x_g),
                                       _ptr(x_sg), _stream(stream)))

    def crl_ring_sample_relabel(self, obs, act, traj, count, seed: int, step, idx, x_sa, x_g,
                                x_sg=None, stream=None):
        E, Cap = traj.shape[0], traj.shape[1]
        check(lib().crl_ring_sample_relabel(self.ctx, _ptr(obs), _ptr(act), _ptr(traj), E, Cap,
                                            _ptr(count), seed, _ptr(step), _ptr(idx),
                                            _ptr(x_sa), _ptr(x_g), _ptr(x_sg),
                                            _stream(stream)))

    def crl_critic_fwd(self, params, params_bf16, x_sa, x_g, ws, loss_out, advance=None,
                       stream=None):
        """advance: optional int64 device counter incremented by the forward's
        last kernel (in place of a crl_counter_add after the call)."""
        check(lib().crl_critic_fwd(self.ctx, _ptr(params), _ptr(params_bf16), _ptr(x_sa),
                                   _ptr(x_g), _ptr(ws), _ptr(loss_out), _ptr(advance),
                                   _stream(stream)))

    def crl_critic_bwd(self, params, params_bf16, x_sa, x_g, ws, grads, stream=None):
        check(lib().crl_critic_bwd(self.ctx, _ptr(params), _ptr(params_bf16), _ptr(x_sa),
                                   _ptr(x_g), _ptr(ws), _ptr(grads), _stream(stream)))

    def crl_critic_bwd_adam(self, params, params_bf16, x_sa, x_g, ws, grads, m, v, step,
                            lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8,
                            stream=None):
        """The gradient of crl_critic_bwd fed straight into the Adam step
        (params, params_bf16, m, v updated in place; grads may be None)."""
        check(lib().crl_critic_bwd_adam(self.ctx, _ptr(params), _ptr(params_bf16), _ptr(x_sa),
                                        _ptr(x_g), _ptr(ws), _ptr(grads), _ptr(m), _ptr(v),
                                        _ptr(step), lr, b1, b2, eps, _stream(stream)))

    def crl_infonce_fwd(self, phi, psi, ws, loss_out, stream=None):
        check(lib().crl_infonce_fwd(self.ctx, _ptr(phi), _ptr(psi), _ptr(ws), _ptr(loss_out),
                                    _stream(stream)))

    def crl_infonce_bwd(self, phi, psi, ws, dphi, dpsi, stream=None):
        check(lib().crl_infonce_bwd(self.ctx, _ptr(phi), _ptr(psi), _ptr(ws), _ptr(dphi),
                                    _ptr(dpsi), _stream(stream)))

    def crl_infonce_fwd_noalloc(self, phi, psi, loss_out, r_out=None, c_out=None,
                                diag_out=None, stream=None):
        check(lib().crl_infonce_fwd_noalloc(self.ctx, _ptr(phi), _ptr(psi), _ptr(loss_out),
                                            _ptr(r_out), _ptr(c_out), _ptr(diag_out),
                                            _stream(stream)))

    def crl_actor_step(self, params, params_bf16, actor_params, actor_params_bf16, log_alpha,
                       x_sa, x_g, x_sg, seed: int, step, ws, actor_grads, alpha_grad,
                       loss_out, stream=None):
        check(lib().crl_actor_step(self.ctx, _ptr(params), _ptr(params_bf16),
                                   _ptr(actor_params), _ptr(actor_params_bf16),
                                   _ptr(log_alpha), _ptr(x_sa), _ptr(x_g), _ptr(x_sg), seed,
                                   _ptr(step), _ptr(ws), _ptr(actor_grads), _ptr(alpha_grad),
                                   _ptr(loss_out), _stream(stream)))

    def crl_actor_step_adam(self, params, params_bf16, actor_params, actor_params_bf16,
                            log_alpha, x_sa, x_g, x_sg, seed: int, step, ws, actor_grads,
                            alpha_grad, loss_out, actor_m, actor_v, adam_step, lr: float,
                            b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8, stream=None):
        """crl_actor_step with the policy gradient fed straight into its Adam
        step (actor_params, actor_params_bf16, actor_m, actor_v updated in
        place; actor_grads may be None)."""
        check(lib().crl_actor_step_adam(self.ctx, _ptr(params), _ptr(params_bf16),
                                        _ptr(actor_params), _ptr(actor_params_bf16),
                                        _ptr(log_alpha), _ptr(x_sa), _ptr(x_g), _ptr(x_sg), seed,
                                        _ptr(step), _ptr(ws), _ptr(actor_grads),
                                        _ptr(alpha_grad), _ptr(loss_out), _ptr(actor_m),
                                        _ptr(actor_v), _ptr(adam_step), lr, b1, b2, eps,
                                        _stream(stream)))


def crl_replay_insert(obs, act, traj, new_obs, new_act, new_traj, count, stream=None):
    """Append new_* ([U][E][...], time-major) to the ring obs/act/traj ([E][C][...])."""
    E, Cap, d_s = obs.shape
    d_a = act.shape[2] if act is not None else 0
    U = new_obs.shape[0]
    check(lib().crl_replay_insert(_ptr(obs), _ptr(act), _ptr(traj), E, Cap, d_s, d_a,
                                  _ptr(new_obs), _ptr(new_act), _ptr(new_traj), U, _ptr(count),
                                  _stream(stream)))


def crl_adam_step(p, g, m, v, p_bf16, step, lr: float, b1: float = 0.9, b2: float = 0.999,
                  eps: float = 1e-8, stream=None):
    check(lib().crl_adam_step(_ptr(p), _ptr(g), _ptr(m), _ptr(v), _ptr(p_bf16), p.numel(),
                              _ptr(step), lr, b1, b2, eps, _stream(stream)))


def crl_check_finite(loss_out, stream=None) -> int:
    """CRL_OK, or CRL_ENONFINITE when the loss or a row/column term of the
    last forward into ``loss_out`` is not finite (synchronises the stream)."""
    rc = lib().crl_check_finite(_ptr(loss_out), _stream(stream))
    if rc not in (0, -4):
        check(rc)
    return rc


def crl_counter_add(counter, inc: int = 1, stream=None):
    check(lib().crl_counter_add(_ptr(counter), inc, _stream(stream)))


def crl_cast_bf16(src, dst, stream=None):
    check(lib().crl_cast_bf16(_ptr(src), _ptr(dst), src.numel(), _stream(stream)))


def crl_peak_rate(which: str, stream=None) -> float:
    """Measured instructions per second on the current device: "exp"
    (v_exp_f32) or "fma32" (unpacked FP32 FMA).  Synchronises."""
    kind = {"exp": 0, "fma32": 1}[which]
    scratch = torch.empty(8192 * 256, dtype=torch.float32, device="cuda")
    out = C.c_double()
    check(lib().crl_peak_rate(kind, _ptr(scratch), C.byref(out), _stream(stream)))
    return out.value


def crl_timing_enable(enable: bool = True):
    check(lib().crl_timing_enable(1 if enable else 0))


def crl_timing_reset():
    check(lib().crl_timing_reset())


def crl_timing_read() -> list:
    """[(kernel name, launches, ms, algorithmic FLOPs, HBM bytes)] (synchronises)."""
    n = C.c_int32()
    check(lib().crl_timing_count(C.byref(n)))
    out = []
    buf = C.create_string_buffer(256)
    for i in range(n.value):
        la, ms, fl, by = C.c_int64(), C.c_double(), C.c_double(), C.c_double()
        check(lib().crl_timing_read(i, buf, 256, C.byref(la), C.byref(ms), C.byref(fl),
                                    C.byref(by)))
        out.append((buf.value.decode(), la.value, ms.value, fl.value, by.value))
    return out


class CriticLoss(torch.autograd.Function):
    """loss = CriticLoss.apply(params, critic, params_bf16, x_sa, x_g, ws).

    Forward runs crl_critic_fwd; backward runs crl_critic_bwd, which re-uses
    the activations left in ``ws`` and returns d(loss)/d(params) as a flat
    vector (padding entries are zero).
    """

    @staticmethod
    def forward(ctx, params, critic: Critic, params_bf16, x_sa, x_g, ws):
        loss = torch.empty(8, dtype=torch.float32, device=params.device)
        critic.crl_critic_fwd(params, params_bf16, x_sa, x_g, ws, loss)
        ctx.critic = critic
        ctx.save_for_backward(params, params_bf16 if params_bf16 is not None else params,
                              x_sa, x_g, ws)
        ctx.has_bf16 = params_bf16 is not None
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        params, pb, x_sa, x_g, ws = ctx.saved_tensors
        grads = torch.empty_like(params)
        ctx.critic.crl_critic_bwd(params, pb if ctx.has_bf16 else None, x_sa, x_g, ws, grads)
        return grads * grad_out, None, None, None, None, None
