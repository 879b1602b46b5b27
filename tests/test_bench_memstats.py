"""The memory-study statistics that bench.py reports (vectorised numpy) agree with the oracle's
plain definitions (oracle/memstudy.py) on random data with ties, repeated keys and shuffled
run orders."""
import numpy as np
import pytest

import bench
from oracle import memstudy as ms


def test_ranks_and_spearman_match_oracle():
    rng = np.random.default_rng(81)
    for n in (7, 64, 500):
        x = rng.integers(0, 20, n).astype(float)         # many ties
        y = x * 0.5 + rng.normal(0, 3, n)
        assert np.allclose(bench.avg_ranks(x), ms.average_ranks(list(x)), rtol=0, atol=0)
        assert bench.spearman(x, y) == pytest.approx(ms.spearman(list(x), list(y)), abs=1e-12)


def test_median_cv_and_drift_match_oracle():
    rng = np.random.default_rng(83)
    keys = rng.integers(0, 12, size=(400, 2))            # 2-column keys like (M, K)
    t = rng.uniform(1e-6, 1e-3, 400)
    order = rng.permutation(400)
    tk = [tuple(k) for k in keys]
    assert bench.median_cv(t, keys) == pytest.approx(ms.cv_by_group(list(t), tk), rel=1e-9)
    assert bench.revisit_drift(t, keys, order) == pytest.approx(ms.revisit_drift(list(t), tk, list(order)), rel=1e-12)


def test_slowdown_matches_oracle():
    rng = np.random.default_rng(89)
    iso = rng.uniform(1, 2, 300)
    co = iso * rng.uniform(0.8, 1.9, 300)
    got = bench.slowdown(co, iso)
    want = ms.slowdown_summary(list(co), list(iso))
    for k in ("mean", "over_20", "over_50"):
        assert got[k] == pytest.approx(want[k], rel=1e-12)
