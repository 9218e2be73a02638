"""Pins for the oracle's random stream and relabeling (no GPU)."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import philox, relabel
from synthetic import make_buffer

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M64 = (1 << 64) - 1


def _kat():
    rows = []
    with open(os.path.join(GOLDEN, "philox4x64_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            lhs, rhs = line.split("->")
            a = [int(x, 16) for x in lhs.split()]
            b = [int(x, 16) for x in rhs.split()]
            rows.append((a[:4], a[4:], b))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    assert list(philox.philox4x64_10(ctr, key)) == out


def test_philox_matches_numpy_philox():
    # numpy's Philox pre-increments its 256-bit counter before each block,
    # so counter c yields the block for c + 1 (with carry across words).
    rng = np.random.default_rng(123)
    for _ in range(50):
        key = [int(x) for x in rng.integers(0, 2**63, size=2)]
        ctr = [int(x) for x in rng.integers(0, 2**63, size=4)]
        ctr[0] = [0, M64, 12345][int(rng.integers(0, 3))]
        g = np.random.Philox(key=np.array(key, np.uint64),
                             counter=np.array(ctr, np.uint64))
        ref = [int(x) for x in g.random_raw(4)]
        c = sum(v << (64 * i) for i, v in enumerate(ctr)) + 1
        c &= (1 << 256) - 1
        nxt = [(c >> (64 * i)) & M64 for i in range(4)]
        assert list(philox.philox4x64_10(nxt, key)) == ref


def test_mulhi_map_range_and_monotone():
    for n in (1, 2, 7, 1000, 4096):
        assert philox.mulhi64(0, n) == 0
        assert philox.mulhi64(M64, n) == n - 1
        assert philox.mulhi64(1 << 63, n) == n // 2


@pytest.mark.parametrize("gamma", [0.5, 0.9, 0.99, 0.999])
def test_thresholds_track_gamma_powers(gamma):
    thr = relabel.geometric_thresholds(gamma, 600)
    gh = Fraction(gamma)
    # each step floors once and multiplies by G/2^64 < 1: |thr[m]/2^64 - g^m| <= (m+1) 2^-64
    p = Fraction(1)
    for m, t in enumerate(thr, start=1):
        p *= gh
        assert abs(Fraction(t, 1 << 64) - p) <= Fraction(m + 1, 1 << 64)
    assert all(a > b for a, b in zip(thr, thr[1:]) if b > 0)


def test_half_gamma_is_leading_zero_count():
    # gamma = 1/2: thr[m] = 2^(64-m) exactly, so k - 1 is the number of
    # leading zero bits of w2 -- the textbook Geometric(1/2) construction.
    thr = relabel.geometric_thresholds(0.5, 70)
    assert thr[:64] == [1 << (64 - m) for m in range(1, 65)]
    rng = np.random.default_rng(5)
    words = [int(x) for x in rng.integers(0, 2**63, size=200)]
    words += [1 << s for s in range(64)] + [(1 << s) - 1 for s in range(1, 64)]
    for w in words:
        clz = 64 - w.bit_length()
        assert relabel.geometric_offset(w, thr) == 1 + clz


@pytest.mark.parametrize("gamma", [0.5, 0.99])
def test_offset_boundaries(gamma):
    thr = relabel.geometric_thresholds(gamma, 30)
    for m in range(1, 30):
        assert relabel.geometric_offset(thr[m - 1] - 1, thr) == m + 1
        assert relabel.geometric_offset(thr[m - 1], thr) == m
    assert relabel.geometric_offset(M64, thr) == 1
    assert relabel.geometric_offset(0, thr) == 31


@pytest.mark.parametrize("gamma,T", [(0.5, 5), (0.99, 5), (0.99, 40), (0.9, 13)])
def test_goal_pmf_closed_form(gamma, T):
    for t in range(T - 1):
        pmf = relabel.goal_step_pmf(gamma, T, t)
        assert sum(pmf.values()) == 1
        assert min(pmf) == t + 1 and max(pmf) == T - 1
        for j, p in pmf.items():
            k = j - t
            ideal = (1 - gamma) * gamma ** (k - 1) if j < T - 1 else gamma ** (T - 2 - t)
            assert abs(float(p) - ideal) < 1e-15 * T
        mean = sum((j - t) * p for j, p in pmf.items())
        assert abs(float(mean) - (1 - gamma ** (T - 1 - t)) / (1 - gamma)) < 1e-12 * T


def test_relabel_brute_force_tiny_buffer():
    # E=2, T=5: the law of (e, t, t_g) under the stream matches the exact pmf.
    E, T, gamma, n = 2, 5, 0.5, 40000
    idx = relabel.relabel_indices(E, T, n, gamma, seed=9, step=0)
    assert idx[:, 0].min() >= 0 and idx[:, 0].max() < E
    assert idx[:, 1].min() >= 0 and idx[:, 1].max() <= T - 2
    assert np.all(idx[:, 2] > idx[:, 1]) and np.all(idx[:, 2] <= T - 1)
    chi2, dof = 0.0, 0
    for e in range(E):
        for t in range(T - 1):
            pmf = relabel.goal_step_pmf(gamma, T, t)
            for j, p in pmf.items():
                exp = n * float(p) / (E * (T - 1))
                obs = np.sum((idx[:, 0] == e) & (idx[:, 1] == t) & (idx[:, 2] == j))
                chi2 += (obs - exp) ** 2 / exp
                dof += 1
    dof -= 1
    # 5-sigma upper tail of chi2(dof), dof ~ 19
    assert chi2 < dof + 5 * math.sqrt(2 * dof)


def test_relabel_gamma099_mean_offset():
    E, T, gamma, n = 3, 1001, 0.99, 6000
    idx = relabel.relabel_indices(E, T, n, gamma, seed=2, step=7)
    mean_pred = np.mean([(1 - gamma ** (T - 1 - t)) / (1 - gamma) for t in idx[:, 1]])
    off = idx[:, 2] - idx[:, 1]
    # offsets are ~Geom with sd ~ 100: mean of 6000 has sd ~ 1.3
    assert abs(off.mean() - mean_pred) < 6.0


def test_relabel_stream_is_counter_based():
    a = relabel.relabel_indices(10, 50, 64, 0.99, seed=2, step=3)
    b = relabel.relabel_indices(10, 50, 64, 0.99, seed=2, step=3)
    c = relabel.relabel_indices(10, 50, 64, 0.99, seed=2, step=4)
    d = relabel.relabel_indices(10, 50, 128, 0.99, seed=2, step=3)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert np.array_equal(d[:64], a)  # sample b depends on b only


def test_gather_rows():
    obs, act = make_buffer(4, 20, 5, 3, seed=0)
    idx, x_sa, x_g, x_sg = relabel.sample_relabel(obs, act, 16, 0.9, 2, 0, 1, 2)
    for b, (e, t, tg) in enumerate(idx):
        assert np.array_equal(x_sa[b, :5], obs[e, t].astype(np.float64))
        assert np.array_equal(x_sa[b, 5:], act[e, t].astype(np.float64))
        assert np.array_equal(x_g[b], obs[e, tg, 1:3].astype(np.float64))
        assert np.array_equal(x_sg[b], np.concatenate([obs[e, t], obs[e, tg, 1:3]]))
