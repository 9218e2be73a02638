"""Pin of the row-blocked InfoNCE evaluation (tests/blocked_oracle.py) against
the dense FP64 oracle (no GPU): several blocks with a ragged last one."""
import numpy as np
import pytest

from oracle import critic as C
from tests.blocked_oracle import infonce_blocked


@pytest.mark.parametrize("kind", ["dot", "l2"])
@pytest.mark.parametrize("loss", ["fwd_infonce", "symmetric_infonce"])
@pytest.mark.parametrize("B,block", [(300, 64), (512, 100), (7, 3)])
def test_blocked_matches_dense_oracle(kind, loss, B, block):
    rng = np.random.default_rng(B)
    phi = rng.standard_normal((B, 16)) * 0.8
    psi = rng.standard_normal((B, 16)) * 0.8
    psi[::5] = phi[::5]             # some coincident pairs (L2: d = 0)
    F = C.energy_matrix(phi, psi, kind)
    o = C.infonce_loss(F, loss, 0.1)
    G = C.infonce_grad(F, o["r"], o["c"], loss, 0.1)
    dphi, dpsi = C.energy_backward(phi, psi, F, G, kind)
    b = infonce_blocked(phi, psi, kind, loss, 0.1, block=block)
    for k in ("total", "fwd", "bwd", "pen"):
        assert b[k] == pytest.approx(o[k], rel=1e-13, abs=1e-15), k
    for k in ("r", "c", "diag"):
        assert np.allclose(b[k], o[k], rtol=1e-13, atol=1e-14), k
    assert np.allclose(b["dphi"], dphi, rtol=1e-11, atol=1e-15)
    assert np.allclose(b["dpsi"], dpsi, rtol=1e-11, atol=1e-15)
