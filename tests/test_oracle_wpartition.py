"""Pins of the w-plane partition oracle (CPU): brute force, a hand-derived
example, invariants.  Each checks oracle.wpartition against something other
than its own code path."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import wpartition as P


def _brute_order(w, absolute):
    # P2/P4 restated: numbers ascending by key, NaN last, ties by input index
    def key(i):
        x = abs(w[i]) if absolute else w[i]
        if math.isnan(x):
            return (1, 0.0, i)
        return (0, x + 0.0, i)  # -0.0 + 0.0 == +0.0
    return np.array(sorted(range(len(w)), key=key))


def test_hand_example():
    # |w| sorted: 0.5 (4), 0.5 (5), 1 (1) | 2 (2), 2 (3), 3 (0)
    w = np.array([3.0, -1.0, 2.0, -2.0, 0.5, -0.5])
    order, start, mean = P.partition(w, 2, absolute=True, stat="mean")
    assert order.tolist() == [4, 5, 1, 2, 3, 0]
    assert start.tolist() == [0, 3, 6]
    assert mean[0] == 2.0 / 3.0 and mean[1] == 7.0 / 3.0
    _, _, med = P.partition(w, 2, absolute=True, stat="median")
    assert med.tolist() == [0.5, 2.0]
    # Algorithm 1 (signed): -2 (3), -1 (1), -0.5 (5) | 0.5 (4), 2 (2), 3 (0)
    order, _, mean = P.partition(w, 2, absolute=False, stat="mean")
    assert order.tolist() == [3, 1, 5, 4, 2, 0]
    assert mean[0] == -3.5 / 3.0 and mean[1] == 5.5 / 3.0
    _, _, med = P.partition(w, 3, absolute=False, stat="median")
    assert med.tolist() == [-1.5, 0.0, 2.5]


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("absolute", [True, False])
def test_brute_force_order(seed, absolute):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 40))
    w = rng.choice([-3.0, -1.0, -0.0, 0.0, 1.0, 2.5, 3.0, np.inf, -np.inf, np.nan], n)
    w = np.where(rng.random(n) < 0.5, w, rng.normal(0, 2, n))
    m = int(rng.integers(1, n + 1))
    order, start, _ = P.partition(w, m, absolute=absolute, stat="median")
    assert order.tolist() == _brute_order(w, absolute).tolist()


@pytest.mark.parametrize("n,m", [(1, 1), (7, 7), (8, 7), (505440, 128), (1000, 3), (13, 5)])
def test_plane_sizes(n, m):
    start = P.plane_bounds(n, m)
    sizes = np.diff(start)
    assert start[0] == 0 and start[-1] == n
    assert sizes.min() >= 1 and sizes.max() - sizes.min() <= 1 and sizes.sum() == n


def test_rejects_more_planes_than_records():
    with pytest.raises(ValueError):
        P.plane_bounds(3, 4)
    with pytest.raises(ValueError):
        P.plane_bounds(0, 1)


def test_statistics_on_the_paper_shaped_records():
    w = W.vla_c_74mhz_w()
    assert w.shape == (505440,)
    for stat in ("mean", "median"):
        order, start, wp = P.partition(w, 128, absolute=True, stat=stat)
        key = np.abs(w)[order]
        assert np.all(np.diff(key) >= 0)
        for m in range(128):
            seg = key[start[m]:start[m + 1]]
            assert seg[0] <= wp[m] <= seg[-1]
        assert np.all(np.diff(wp) >= 0)  # planes of a sorted key: monotone statistic
    # each +w/-w pair of records with equal |w| lands in adjacent sorted slots
    w2 = np.concatenate([w[:1000], -w[:1000]])
    order, _, _ = P.partition(w2, 10)
    k = np.abs(w2)[order]
    assert np.all(k[0::2] == k[1::2])


def test_constant_planes_are_exact():
    sizes = [5, 5, 6]  # P1 sizes for n = 16, M = 3
    # dyadic values: the sum of a constant plane is exact, so is its mean
    w = np.repeat(np.array([0.125, 0.75, 3.5]), sizes)
    _, _, mean = P.partition(w, 3, stat="mean")
    assert mean.tolist() == [0.125, 0.75, 3.5]
    w = np.repeat(np.array([0.1, 0.7, 3.3]), sizes)
    _, _, med = P.partition(w, 3, stat="median")
    assert med.tolist() == [0.1, 0.7, 3.3]


def test_mean_is_correctly_rounded():
    # 1e16 + 1 + 1 - 1e16 style cancellation does not arise for |w|; a long
    # plane of values whose naive running sum drifts shows the exact sum
    w = np.full(100001, 0.1)
    _, _, mean = P.partition(w, 1, stat="mean")
    assert mean[0] == 0.1
