"""Landscape metrics oracle, pinned to the paper's printed ideal-landscape values and to closed forms."""
import json
import os

import numpy as np
import pytest

from oracle import metrics

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_ideal_landscape_matches_paper():
    g = json.load(open(os.path.join(GOLD, "ideal_landscape_arc_b580.json")))
    sizes = list(range(g["grid"]["start"], g["grid"]["stop"] + 1, g["grid"]["step"]))
    L = np.array([[metrics.ideal_tflops(m, n, g["peak_tflops"], g["cores"], g["tile"])
                   for n in sizes] for m in sizes])
    s = metrics.slice_stats(L)
    half = 0.5 * 10 ** -g["printed_decimals"]
    assert abs(s["mean"] - g["paper_mean_tflops"]) <= half          # 97.17 prints as 97.2
    assert abs(s["roughness_n"] - g["paper_roughness_n"]) <= half    # 1.963 prints as 2.0
    assert s["peak"] == g["peak_tflops"]


def test_alignment_worked_example():
    g = json.load(open(os.path.join(GOLD, "alignment_worked_example.json")))
    for N, wgs, util in g["cases"]:
        assert -(-N // g["tile"]) == wgs
        assert metrics.tile_utilisation(N, g["tile"]) == pytest.approx(util, abs=1e-12)
    waste = 1 - metrics.tile_utilisation(896, 256)
    assert waste == pytest.approx(g["printed_gain_896_to_1024"], abs=1e-12)
    gain = metrics.tile_utilisation(1024, 256) / metrics.tile_utilisation(896, 256) - 1
    assert gain == pytest.approx(1.0 / 7.0, abs=1e-12)


def test_tflops_formula():
    assert metrics.tflops(4096, 4096, 4096, 1e-3) == pytest.approx(2 * 4096 ** 3 / 1e9)


def test_roughness_closed_forms():
    assert metrics.roughness([5.0] * 10) == 0.0
    assert metrics.roughness(3.0 + 0.5 * np.arange(32)) == pytest.approx(0.5)
    assert metrics.roughness([0, 2, 0, 2]) == pytest.approx(2.0)
    assert metrics.roughness([1, 4]) == pytest.approx(3.0)
    with pytest.raises(ValueError):
        metrics.roughness([1.0])


def test_roughness_along_axes_and_aggregate():
    m, n, k = np.meshgrid(np.arange(4), np.arange(5), np.arange(6), indexing="ij")
    T = 1.0 * m + 2.0 * n + 3.0 * k
    agg = metrics.aggregate_3d(T)
    assert agg["roughness_m"] == pytest.approx(1.0)
    assert agg["roughness_n"] == pytest.approx(2.0)
    assert agg["roughness_k"] == pytest.approx(3.0)
    assert agg["roughness_3d"] == pytest.approx(2.0)
    assert agg["peak"] == T.max() and agg["mean"] == pytest.approx(T.mean())
