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


def test_wave_quantization_printed_example():
    g = json.load(open(os.path.join(GOLD, "wave_quantization_example.json")))
    import math
    assert math.ceil(g["M"] / g["tile"]) * math.ceil(g["N"] / g["tile"]) == g["workgroups"]
    assert metrics.wave_efficiency(g["M"], g["N"], g["tile"], g["cores"]) == pytest.approx(g["efficiency"])


def test_kol_levels_of_table20():
    g = json.load(open(os.path.join(GOLD, "kol_levels_table20.json")))
    for row in g["rows"]:
        assert metrics.throughput_band(row["tau"]) == row["t_band"], row
        assert metrics.smoothness_band(row["rho"]) == row["s_band"], row
        assert min(row["t_band"], row["s_band"]) == row["level"]


def test_kol_band_edges():
    # Table 19's edges: tau 0.50 / 0.75 / 0.95 open the next band; rho 1.25 / 2 / 3 close one
    assert [metrics.throughput_band(t) for t in (0.49, 0.5, 0.749, 0.75, 0.949, 0.95, 1.0)] == [0, 1, 1, 2, 2, 3, 3]
    assert [metrics.smoothness_band(r) for r in (1.0, 1.25, 1.26, 2.0, 2.01, 3.0, 3.01)] == [3, 3, 2, 2, 1, 1, 0]


MI355X = dict(peak=2516.6, cores=256, bw_gbs=8000.0)


def test_optimal_compute_plateau_is_peak():
    # 4096^3: 256 tiles of 256 fill one wave exactly; 96 MiB of traffic takes 12.6 us against
    # 54.6 us of MFMA time, so the optimal is the peak
    assert metrics.optimal_tflops(4096, 4096, 4096, **MI355X) == pytest.approx(2516.6)


def test_optimal_memory_bound_corner():
    M, N, K = 4096, 4096, 1
    t_mem = (2 * M * K + 2 * K * N + 2 * M * N) / 8000e9
    assert metrics.optimal_tflops(M, N, K, **MI355X) == pytest.approx(2 * M * N * K / t_mem / 1e12)


def test_optimal_picks_the_best_filling_tile():
    # 512 x 512 on 256 cores: tiles 256/128/64 launch 4/16/64 work-groups; the 64 tile fills a
    # quarter of the cores, and memory is far from binding at K = 4096
    got = metrics.optimal_tflops(512, 512, 4096, **MI355X)
    assert got == pytest.approx(2516.6 * 64 / 256)
    only256 = metrics.optimal_tflops(512, 512, 4096, tiles=(256,), **MI355X)
    assert only256 == pytest.approx(2516.6 * 4 / 256)


def test_optimal_single_tile_is_the_ideal_below_one_wave():
    # with one tile, unlimited bandwidth and at most one wave, the optimal is the ideal ceiling;
    # beyond one wave it is at most the ideal (wave quantization)
    for M, N in [(256, 256), (1024, 2048), (4096, 3840), (4096, 4096), (4352, 4096), (8192, 4352)]:
        opt = metrics.optimal_tflops(M, N, 4096, 2516.6, 256, 1e12, tiles=(256,))
        ideal = metrics.ideal_tflops(M, N, 2516.6, 256, 256)
        W = -(-M // 256) * -(-N // 256)
        if W <= 256:
            assert opt == pytest.approx(ideal)
        else:
            assert opt <= ideal + 1e-9


def test_kol_grade_on_hand_landscapes():
    rng = np.random.default_rng(0)
    O = rng.uniform(100, 200, size=(4, 6, 3))
    g = metrics.kol_grade(O, O)
    assert g["tau"] == pytest.approx(1.0) and g["rho"] == pytest.approx(1.0) and g["level"] == 3
    g = metrics.kol_grade(O / 2, O)            # half the throughput, half the roughness
    assert g["tau"] == pytest.approx(0.5) and g["rho"] == pytest.approx(0.5)
    assert (g["t_band"], g["s_band"], g["level"]) == (1, 3, 1)
    A = O.copy()
    A[:, 1::2, :] -= 30.0                       # a sawtooth along N
    g = metrics.kol_grade(A, O)
    assert g["rho"] > 1.0 and g["tau"] < 1.0
