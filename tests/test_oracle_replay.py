"""Pins for the ring replay buffer and relabeling inside trajectories (no GPU).

The ring's contents are checked against the plain concatenation of the
appended stream; the sampler against the single-episode law it must reduce
to, against the exact clipped-geometric law on tiny buffers (chi-square over
every (e, i, t_g) cell), and against the invariant that a goal never leaves
its trajectory.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import relabel
from oracle.replay import RingBuffer, ring_relabel_indices, ring_sample_relabel, trajectory_end
from synthetic import make_buffer
from synthetic.trajectories import unroll_stream


def _fill(buf, obs, act, traj, chunk):
    for u0 in range(0, obs.shape[0], chunk):
        buf.insert(obs[u0:u0 + chunk], act[u0:u0 + chunk], traj[u0:u0 + chunk])


@pytest.mark.parametrize("n,C,chunk", [(7, 10, 3), (10, 10, 5), (23, 10, 4), (62 * 5, 100, 62),
                                       (31, 8, 8)])
def test_ring_holds_the_last_capacity_steps(n, C, chunk):
    obs, act, traj = unroll_stream(3, n, 4, 2, (2, 6), seed=n)
    buf = RingBuffer(3, C, 4, 2)
    _fill(buf, obs, act, traj, chunk)
    assert buf.count == n and buf.size == min(n, C)
    keep = slice(n - buf.size, n)
    rows = [buf.row_of(i) for i in range(buf.size)]
    assert sorted(rows) == list(range(buf.size)) if n <= C else sorted(rows) == list(range(C))
    for e in range(3):
        assert np.array_equal(buf.obs[e, rows], obs[keep, e])
        assert np.array_equal(buf.act[e, rows], act[keep, e])
        assert np.array_equal(buf.traj[e, rows], traj[keep, e])


def test_ring_rejects_bad_chunks():
    buf = RingBuffer(2, 4, 1, 1)
    with pytest.raises(ValueError):
        buf.insert(np.zeros((5, 2, 1), np.float32), np.zeros((5, 2, 1), np.float32),
                   np.zeros((5, 2), np.int32))
    with pytest.raises(ValueError):
        RingBuffer(1, 1, 1, 1)


def test_trajectory_end_is_the_end_of_the_run():
    obs, act, traj = unroll_stream(4, 57, 2, 1, (1, 7), seed=3)
    buf = RingBuffer(4, 40, 2, 1)
    _fill(buf, obs, act, traj, 9)
    for e in range(4):
        ids = [int(buf.traj[e, buf.row_of(i)]) for i in range(buf.size)]
        pos = 0
        for _, grp in itertools.groupby(ids):
            n = len(list(grp))
            for i in range(pos, pos + n):
                assert trajectory_end(buf.traj[e], buf, i) == pos + n - 1
            pos += n


@pytest.mark.parametrize("wrap", [False, True])
def test_one_trajectory_per_env_reduces_to_the_single_episode_law(wrap):
    # one trajectory per env row: end(i) = size - 1 for every i, so the ring
    # sampler is relabel_indices on the logical view
    E, T, C = 5, 37, 37
    obs, act = make_buffer(E, T + (13 if wrap else 0), 3, 2, seed=4)
    stream_obs = np.ascontiguousarray(obs.transpose(1, 0, 2))
    stream_act = np.ascontiguousarray(act.transpose(1, 0, 2))
    traj = np.zeros(stream_obs.shape[:2], np.int32)
    buf = RingBuffer(E, C, 3, 2)
    _fill(buf, stream_obs, stream_act, traj, 6)
    for step in (0, 3):
        got = ring_relabel_indices(buf, 300, 0.9, T, seed=11, step=step)
        ref = relabel.relabel_indices(E, T, 300, 0.9, seed=11, step=step)
        assert np.array_equal(got[:, 0], ref[:, 0])
        assert np.array_equal(got[:, 1], [buf.row_of(i) for i in ref[:, 1]])
        assert np.array_equal(got[:, 2], [buf.row_of(i) for i in ref[:, 2]])


def _logical(buf, row):
    return (row - (buf.count - buf.size)) % buf.C


def test_goals_stay_inside_their_trajectory():
    obs, act, traj = unroll_stream(6, 300, 3, 2, (1, 40), seed=8)
    buf = RingBuffer(6, 128, 3, 2)
    _fill(buf, obs, act, traj, 62)
    idx = ring_relabel_indices(buf, 4000, 0.9, 1000, seed=5, step=2)
    ends = 0
    for e, r, rg in idx:
        i, j = _logical(buf, r), _logical(buf, rg)
        end = trajectory_end(buf.traj[e], buf, i)
        assert i <= buf.size - 2 and i <= j <= end
        assert buf.traj[e, r] == buf.traj[e, rg]
        assert j > i or end == i
        ends += end == i
    assert ends > 0   # some samples sit on the last step of a trajectory


def _exact_law(buf, e, i, gamma, L):
    """P(t_g = j | e, i) from the closed form (1-g) g^(k-1), the tail on end(i)."""
    end = trajectory_end(buf.traj[e], buf, i)
    if end == i:
        return {i: 1.0}
    law = {i + k: (1 - gamma) * gamma ** (k - 1) for k in range(1, min(end - i, L - 1))}
    law[min(end, i + L - 1)] = 1.0 - sum(law.values())
    return law


@pytest.mark.parametrize("gamma,L", [(0.5, 1000), (0.7, 1000), (0.7, 4)])
def test_brute_force_law_on_a_tiny_ring(gamma, L):
    # E = 2, capacity 9 with three short trajectories per env after a wrap:
    # the counts of every (e, i, t_g) cell follow the exact law (chi-square)
    E, C, n = 2, 9, 60000
    stream_traj = np.array([[0, 0], [0, 0], [0, 1], [1, 1], [1, 1], [1, 1], [1, 2], [2, 2],
                            [3, 2], [3, 2], [3, 3], [3, 4], [4, 4]], np.int32)
    U = stream_traj.shape[0]
    buf = RingBuffer(E, C, 1, 1)
    z = np.zeros((U, E, 1), np.float32)
    _fill(buf, z, z, stream_traj, 5)
    assert buf.size == C and buf.count == U
    idx = ring_relabel_indices(buf, n, gamma, L, seed=21, step=1)
    chi2, dof = 0.0, 0
    for e in range(E):
        for i in range(C - 1):
            law = _exact_law(buf, e, i, gamma, L)
            assert abs(sum(law.values()) - 1.0) < 1e-12
            cell = (idx[:, 0] == e) & (idx[:, 1] == buf.row_of(i))
            for j, p in law.items():
                exp = n * p / (E * (C - 1))
                obs = np.sum(cell & (idx[:, 2] == buf.row_of(j)))
                chi2 += (obs - exp) ** 2 / exp
                dof += 1
            # nothing outside the support
            support = {buf.row_of(j) for j in law}
            assert set(np.unique(idx[cell, 2])) <= support
    dof -= 1
    assert chi2 < dof + 5 * math.sqrt(2 * dof), (chi2, dof)


def test_fewer_than_two_steps_draw_nothing():
    buf = RingBuffer(3, 5, 2, 1)
    assert np.all(ring_relabel_indices(buf, 8, 0.9, 100, 1, 0) == -1)
    buf.insert(np.ones((1, 3, 2), np.float32), np.ones((1, 3, 1), np.float32),
               np.zeros((1, 3), np.int32))
    idx, x_sa, x_g, x_sg = ring_sample_relabel(buf, 8, 0.9, 100, 1, 0, 0, 1)
    assert np.all(idx == -1) and not x_sa.any() and not x_g.any() and not x_sg.any()


def test_ring_gather_rows():
    obs, act, traj = unroll_stream(4, 45, 5, 3, (3, 12), seed=2)
    buf = RingBuffer(4, 30, 5, 3)
    _fill(buf, obs, act, traj, 15)
    idx, x_sa, x_g, x_sg = ring_sample_relabel(buf, 64, 0.9, 50, 2, 0, 1, 2)
    for b, (e, r, rg) in enumerate(idx):
        assert np.array_equal(x_sa[b, :5], buf.obs[e, r].astype(np.float64))
        assert np.array_equal(x_sa[b, 5:], buf.act[e, r].astype(np.float64))
        assert np.array_equal(x_g[b], buf.obs[e, rg, 1:3].astype(np.float64))
        assert np.array_equal(x_sg[b], np.concatenate([buf.obs[e, r], buf.obs[e, rg, 1:3]]))


def test_unroll_stream_episodes():
    obs, act, traj = unroll_stream(3, 2500, 2, 2, 1000, seed=1)
    for e in range(3):
        d = np.diff(traj[:, e])
        assert set(np.unique(d)) <= {0, 1}
        starts = np.flatnonzero(d) + 1
        assert np.all(np.diff(starts) == 1000)   # full episodes after the first
        assert 1 <= starts[0] <= 1000            # staggered first episode
    assert act.min() >= -1 and act.max() <= 1
