"""ctypes loader for libcrl.so and the C-ABI declarations of include/crl.h.

Loading fails loudly when the library has not been built: there is no
fallback implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcrl.so")

CRL_OK, CRL_EINVAL, CRL_EUNSUPPORTED, CRL_EHIP, CRL_ENONFINITE = 0, -1, -2, -3, -4
ACT = {"relu": 0, "ln_swish": 1}
ENERGY = {"dot": 0, "l2": 1, "cos": 2, "l2sq": 3, "l1": 4}
LOSS = {"fwd_infonce": 0, "symmetric_infonce": 1, "bwd_infonce": 2, "flatnce_fwd": 3,
        "flatnce_bwd": 4, "fb": 5, "dpo": 6, "ipo": 7, "sppo": 8}
PREC = {"fp32": 0, "bf16": 1}
LOGITS = {"materialised": 0, "fused": 1}
WS = {"phi": 0, "psi": 1, "row_lse": 2, "col_lse": 3, "diag": 4, "dphi": 5,
      "dpsi": 6, "logits": 7, "policy_out": 8, "noise": 9, "log_pi": 10,
      "policy_energy": 11, "daction": 12}


class crl_config(C.Structure):
    _fields_ = [
        ("batch", C.c_int32), ("obs_dim", C.c_int32), ("act_dim", C.c_int32),
        ("goal_dim", C.c_int32), ("goal_lo", C.c_int32), ("n_hidden", C.c_int32),
        ("hidden", C.c_int32), ("repr_dim", C.c_int32), ("activation", C.c_int32),
        ("energy", C.c_int32), ("loss", C.c_int32), ("precision", C.c_int32),
        ("logits", C.c_int32), ("logsumexp_penalty", C.c_float),
        ("ln_eps", C.c_float), ("discount", C.c_double),
        ("max_episode_len", C.c_int32), ("actor_n_hidden", C.c_int32),
        ("actor_hidden", C.c_int32), ("target_entropy", C.c_float),
        ("random_goal_ratio", C.c_double), ("reserved", C.c_int32 * 2),
    ]


class crl_layer_info(C.Structure):
    _fields_ = [("w", C.c_int64), ("b", C.c_int64), ("ln_g", C.c_int64),
                ("ln_b", C.c_int64), ("fan_in", C.c_int32), ("fan_out", C.c_int32)]


P = C.c_void_p
I32, I64, U64, F32 = C.c_int32, C.c_int64, C.c_uint64, C.c_float

# name -> (restype, argtypes), exactly the functions declared in include/crl.h
SIGNATURES = {
    "crl_create": (C.c_int, [C.POINTER(crl_config), C.POINTER(P)]),
    "crl_destroy": (C.c_int, [P]),
    "crl_param_count": (C.c_int, [P, C.POINTER(I64)]),
    "crl_actor_param_count": (C.c_int, [P, C.POINTER(I64)]),
    "crl_layer_layout": (C.c_int, [P, I32, I32, C.POINTER(crl_layer_info)]),
    "crl_workspace_size": (C.c_int, [P, C.POINTER(I64)]),
    "crl_input_layout": (C.c_int, [P, C.POINTER(I32), C.POINTER(I32), C.POINTER(I32),
                                   C.POINTER(I32)]),
    "crl_sample_relabel": (C.c_int, [P, P, P, I32, I32, U64, P, P, P, P, P, P]),
    "crl_replay_insert": (C.c_int, [P, P, P, I32, I32, I32, I32, P, P, P, I32, P, P]),
    "crl_ring_sample_relabel": (C.c_int, [P, P, P, P, I32, I32, P, U64, P, P, P, P, P, P]),
    "crl_critic_fwd": (C.c_int, [P, P, P, P, P, P, P, P, P]),
    "crl_critic_bwd": (C.c_int, [P, P, P, P, P, P, P, P]),
    "crl_critic_bwd_adam": (C.c_int, [P, P, P, P, P, P, P, P, P, P, C.c_double, C.c_double,
                                      C.c_double, C.c_double, P]),
    "crl_infonce_fwd": (C.c_int, [P, P, P, P, P, P]),
    "crl_infonce_bwd": (C.c_int, [P, P, P, P, P, P, P]),
    "crl_infonce_fwd_noalloc": (C.c_int, [P, P, P, P, P, P, P, P]),
    "crl_check_finite": (C.c_int, [P, P]),
    "crl_actor_step": (C.c_int, [P, P, P, P, P, P, P, P, P, U64, P, P, P, P, P, P]),
    "crl_actor_step_adam": (C.c_int, [P, P, P, P, P, P, P, P, P, U64, P, P, P, P, P, P, P, P,
                                      C.c_double, C.c_double, C.c_double, C.c_double, P]),
    "crl_adam_step": (C.c_int, [P, P, P, P, P, I64, P, C.c_double, C.c_double, C.c_double,
                                C.c_double, P]),
    "crl_counter_add": (C.c_int, [P, I64, P]),
    "crl_cast_bf16": (C.c_int, [P, P, I64, P]),
    "crl_workspace_view": (C.c_int, [P, I32, C.POINTER(I64), C.POINTER(I64)]),
    "crl_timing_enable": (C.c_int, [I32]),
    "crl_timing_reset": (C.c_int, []),
    "crl_timing_count": (C.c_int, [C.POINTER(I32)]),
    "crl_timing_read": (C.c_int, [I32, C.c_char_p, I32, C.POINTER(I64),
                                  C.POINTER(C.c_double), C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]),
    "crl_peak_rate": (C.c_int, [I32, P, C.POINTER(C.c_double), P]),
    "crl_last_error": (C.c_char_p, []),
}

_lib = None


def lib():
    """The loaded library (raises if libcrl.so is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is not built; run `python -m paper_2408_11052_amd.build`")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class CRLError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"crl error {code}: {msg}")
        self.code = code


def check(rc: int):
    if rc != CRL_OK:
        raise CRLError(rc, lib().crl_last_error().decode(errors="replace"))
    return rc
