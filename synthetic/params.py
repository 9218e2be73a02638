"""Seeded initial parameters for the encoders and the actor.

Every Linear layer gets He-normal weights W ~ N(0, 2/fan_in) stored
``[in][out]`` and zero bias; LayerNorm layers get scale 1 and offset 0.
The values are drawn once on the host in FP32 and handed to both the GPU path
and the FP64 oracle, so both start from the same numbers.

``perturb`` adds small seeded noise to biases and LayerNorm affines so that
tests exercise the gradients of those parameters away from their trivial
initial values.
"""
from __future__ import annotations

from typing import Dict, List, Sequence

import numpy as np

Layer = Dict[str, np.ndarray]


def mlp_layers(rng: np.random.Generator, dims: Sequence[int], layer_norm: bool,
               perturb: float = 0.0) -> List[Layer]:
    """dims = [in, h1, ..., hL, out]; hidden layers get LN params if asked."""
    layers: List[Layer] = []
    n = len(dims) - 1
    for i in range(n):
        fan_in, fan_out = int(dims[i]), int(dims[i + 1])
        W = rng.standard_normal((fan_in, fan_out), dtype=np.float32)
        W *= np.float32(np.sqrt(2.0 / fan_in))
        L: Layer = {"W": W, "b": np.zeros(fan_out, np.float32)}
        hidden = i < n - 1
        if hidden and layer_norm:
            L["ln_g"] = np.ones(fan_out, np.float32)
            L["ln_b"] = np.zeros(fan_out, np.float32)
        if perturb:
            L["b"] += perturb * rng.standard_normal(fan_out, dtype=np.float32)
            if "ln_g" in L:
                L["ln_g"] += perturb * rng.standard_normal(fan_out, dtype=np.float32)
                L["ln_b"] += perturb * rng.standard_normal(fan_out, dtype=np.float32)
        layers.append(L)
    return layers


def critic_params(in_sa: int, in_g: int, hidden: Sequence[int], repr_dim: int,
                  layer_norm: bool, seed: int = 1, perturb: float = 0.0):
    """Return (phi_layers, psi_layers) for phi(s,a) and psi(g)."""
    rng = np.random.default_rng(seed)
    phi = mlp_layers(rng, [in_sa, *hidden, repr_dim], layer_norm, perturb)
    psi = mlp_layers(rng, [in_g, *hidden, repr_dim], layer_norm, perturb)
    return phi, psi


def critic_params_for(w, seed: int = 1, perturb: float = 0.0):
    return critic_params(w.in_sa, w.goal_dim, w.hidden, w.repr_dim,
                         w.activation == "ln_swish", seed=seed, perturb=perturb)


def actor_params(in_sg: int, hidden: Sequence[int], act_dim: int,
                 layer_norm: bool, seed: int = 3, perturb: float = 0.0):
    """Policy MLP [in_sg, hidden..., 2*act_dim] (mean and pre-softplus scale)."""
    rng = np.random.default_rng(seed)
    return mlp_layers(rng, [in_sg, *hidden, 2 * act_dim], layer_norm, perturb)
