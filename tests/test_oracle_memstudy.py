"""Pins of the memory-study statistics (oracle/memstudy.py) against closed forms, hand
examples and a library routine."""
import math

import numpy as np
import pytest

from oracle import memstudy as ms


def test_average_ranks_hand_example():
    assert ms.average_ranks([10, 20, 20, 30]) == [1.0, 2.5, 2.5, 4.0]
    assert ms.average_ranks([3, 1, 2]) == [3.0, 1.0, 2.0]
    assert ms.average_ranks([5, 5, 5]) == [2.0, 2.0, 2.0]


def test_spearman_without_ties_is_the_rank_difference_formula():
    """Without ties rho = 1 - 6 sum d^2 / (n (n^2 - 1)), d the rank differences."""
    rng = np.random.default_rng(61)
    for n in (5, 17, 100):
        x = rng.permutation(n) + 0.5
        y = rng.permutation(n) * 3.0
        rx = np.argsort(np.argsort(x)) + 1
        ry = np.argsort(np.argsort(y)) + 1
        d2 = float(np.sum((rx - ry) ** 2))
        assert ms.spearman(list(x), list(y)) == pytest.approx(1 - 6 * d2 / (n * (n * n - 1)), abs=1e-12)


def test_spearman_monotone_and_with_ties():
    x = list(range(20))
    assert ms.spearman(x, [math.exp(v / 3) for v in x]) == pytest.approx(1.0)
    assert ms.spearman(x, [-v ** 3 for v in x]) == pytest.approx(-1.0)
    scipy_stats = pytest.importorskip("scipy.stats")
    rng = np.random.default_rng(67)
    a = rng.integers(0, 6, 60).astype(float)          # many ties
    b = a + rng.integers(0, 4, 60)
    assert ms.spearman(list(a), list(b)) == pytest.approx(scipy_stats.spearmanr(a, b)[0], abs=1e-12)


def test_slowdown_summary_hand_example():
    s = ms.slowdown_summary([1.0, 1.3, 2.0, 0.9], [1.0, 1.0, 1.0, 1.0])
    assert s["mean"] == pytest.approx((1.0 + 1.3 + 2.0 + 0.9) / 4)
    assert s["over_20"] == 0.5 and s["over_50"] == 0.25
    # exactly 20 % / 50 % slower is not "more than"
    s = ms.slowdown_summary([1.2, 1.5], [1.0, 1.0])
    assert s["over_20"] == pytest.approx(0.5) and s["over_50"] == 0.0


def test_cv_by_group_closed_forms():
    # constant within every group -> 0; the pair (1, 3): sd 1, mean 2 -> 0.5
    assert ms.cv_by_group([4, 4, 7, 7], ["a", "a", "b", "b"]) == 0.0
    assert ms.cv_by_group([1, 3], [0, 0]) == pytest.approx(0.5)
    # median over groups with CVs 0, 0.5 and 1/3 (values 1, 2 around mean 1.5: sd 0.5)
    assert ms.cv_by_group([5, 5, 1, 3, 1, 2], [0, 0, 1, 1, 2, 2]) == pytest.approx(1 / 3)


def test_revisit_drift_of_a_geometric_warm_up():
    """A buffer whose time falls by the factor r at each revisit drifts 1 - r^(v - 1) over v
    visits, whatever the other keys interleaved with it."""
    r, v = 0.9, 8
    times, keys, order = [], [], []
    o = 0
    for visit in range(v):
        for key, base in (("x", 2.0), ("y", 5.0)):
            times.append(base * r ** visit)
            keys.append(key)
            order.append(o)
            o += 1
    assert ms.revisit_drift(times, keys, order) == pytest.approx(1 - r ** (v - 1))
    # listing order does not matter, run order does
    perm = np.random.default_rng(71).permutation(len(times))
    assert ms.revisit_drift([times[i] for i in perm], [keys[i] for i in perm],
                            [order[i] for i in perm]) == pytest.approx(1 - r ** (v - 1))


def test_bandwidth():
    assert ms.bandwidth_gbs(8e9, 1.0) == 8.0
