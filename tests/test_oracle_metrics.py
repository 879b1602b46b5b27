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


def test_optimal_memory_bound_corner_counts_the_tensors_bytes():
    # a memory-bound shape (K = 1): the optimal moves every byte of the actual tensors once at
    # the bandwidth; the bytes are counted from arrays of the operand and result types
    for (M, N, K), c_dtype in [((4096, 4096, 1), np.uint16), ((512, 3000, 2), np.float32)]:
        A = np.zeros((M, K), dtype=np.uint16)          # BF16 storage
        B = np.zeros((K, N), dtype=np.uint16)
        C = np.zeros((M, N), dtype=c_dtype)
        nbytes = A.nbytes + B.nbytes + C.nbytes
        got = metrics.optimal_tflops(M, N, K, c_bytes=C.itemsize, **MI355X)
        assert got * 1e12 * (nbytes / 8000e9) == pytest.approx(2.0 * M * N * K, rel=1e-12)


def _channels_touched(L, elem_bytes, channels, interleave, tile_row, rows):
    """Brute force: walk the rows of a tensor with leading dimension L, list every interleave
    block each tile row touches, and count the distinct channels (block number mod channels)."""
    seen = set()
    for r in range(rows):
        start = r * L * elem_bytes
        for byte in range(start, start + tile_row * elem_bytes, interleave):
            seen.add((byte // interleave) % channels)
    return len(seen) / channels


@pytest.mark.parametrize("channels", [6, 8, 12])
@pytest.mark.parametrize("elem_bytes", [2, 4])
def test_channel_utilisation_equals_simulated_striping(channels, elem_bytes):
    for L in range(128, 4097, 128):
        want = _channels_touched(L, elem_bytes, channels, 256, 256, rows=4 * channels)
        assert metrics.channel_utilisation(L, elem_bytes, channels, 256) == pytest.approx(want), (L, elem_bytes)


def test_channel_dip_printed_for_b_at_multiples_of_768():
    # Sec. 9.2: with 6 channels at 256 B, B's utilisation drops to 1/3 whenever N is a multiple
    # of 768 (and only then, for BF16 rows on the 128-step grid)
    for N in range(128, 8193, 128):
        eta = metrics.channel_utilisation(N, 2, 6, 256)
        assert (eta == pytest.approx(1 / 3)) == (N % 768 == 0), N


def test_channel_term_only_lowers_the_memory_roofline():
    # the channel shares are at most 1: adding them never raises the optimal, and it leaves
    # compute-bound shapes (far above the ridge) unchanged
    b580 = dict(peak=108.2, cores=20, bw_gbs=451.0, c_bytes=4)
    for M, N, K in [(128, 768, 128), (256, 1536, 4096), (3840, 3840, 4096), (128, 128, 128)]:
        with_ch = metrics.optimal_tflops(M, N, K, channels=6, **b580)
        without = metrics.optimal_tflops(M, N, K, **b580)
        assert with_ch <= without + 1e-12
    assert metrics.optimal_tflops(3840, 3840, 4096, channels=6, **b580) == pytest.approx(108.2)


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


# ---- Sec. 4 four-surface decomposition ------------------------------------------------------

def test_compute_surface_has_no_texture():
    """The compute surface is the useful FLOP at the dense peak: its throughput is the peak at
    every shape, and along N its time grows by the same amount each step (Fig. 5, smooth)."""
    rng = np.random.default_rng(41)
    for _ in range(50):
        M, N, K = (int(x) for x in rng.integers(1, 9000, 3))
        t = metrics.compute_time(M, N, K, 2516.6)
        assert metrics.tflops(M, N, K, t) == pytest.approx(2516.6, rel=1e-12)
    t_line = [metrics.compute_time(2048, n, 1024, 116.5) for n in range(128, 4097, 128)]
    steps = np.diff(t_line)
    assert np.allclose(steps, 2.0 * 2048 * 128 * 1024 / 116.5e12, rtol=1e-12, atol=0)


def test_overhead_surface_special_cases():
    # a GEMM that takes exactly its compute (or memory) time has no overhead
    assert metrics.overhead_time(3.0, 3.0, 1.0) == 0.0
    assert metrics.overhead_time(3.0, 1.0, 3.0) == 0.0
    # beyond the larger of the two, whichever it is
    assert metrics.overhead_time(5.0, 1.0, 3.0) == 2.0
    assert metrics.overhead_time(5.0, 4.0, 3.0) == 1.0
    # a measured memory time above the GEMM's own gives a negative overhead, kept as is
    assert metrics.overhead_time(2.0, 1.0, 2.5) == -0.5


def test_overhead_share_of_a_constant_fraction():
    """If every GEMM spends the fraction f of its time beyond max(compute, memory) -- the
    paper's constant 32 % floor of Fig. 6 -- the mean share is f."""
    rng = np.random.default_rng(43)
    shapes = [tuple(int(x) for x in rng.integers(128, 4097, 3)) for _ in range(200)]
    t_mem = [float(x) for x in rng.uniform(1e-6, 1e-3, len(shapes))]
    f = 0.32
    t_gemm = [max(metrics.compute_time(*s, 2516.6), tm) / (1.0 - f) for s, tm in zip(shapes, t_mem)]
    d = metrics.decompose(shapes, t_gemm, t_mem, 2516.6, 8000.0)
    assert d["overhead_share"] == pytest.approx(f, abs=1e-12)
    assert all(o > 0 for o in d["t_overhead"])


def test_compute_bound_squares_closed_form():
    """A square n^3 GEMM moves (4 + c) n^2 bytes for 2 n^3 FLOP, so it is compute-bound against
    bandwidth BW exactly when n >= (4 + c) P / (2 BW): on MI355X (2,516.6 TFLOP/s, 8 TB/s) n >= 943.7
    with BF16 output (25 of the 32 step-128 squares) and n >= 1258.3 with FP32 (23 of 32)."""
    sq = [(n, n, n) for n in range(128, 4097, 128)]
    ones = [1.0] * len(sq)
    assert metrics.decompose(sq, ones, ones, 2516.6, 8000.0, c_bytes=2)["cb_bandwidth"] == 25 / 32
    assert metrics.decompose(sq, ones, ones, 2516.6, 8000.0, c_bytes=4)["cb_bandwidth"] == 23 / 32


def test_compute_bound_is_intensity_above_the_ridge():
    """Compute-bound against a bandwidth is the roofline statement: arithmetic intensity
    2MNK / bytes at or above the ridge P / BW."""
    rng = np.random.default_rng(47)
    shapes = [tuple(int(x) for x in rng.integers(1, 8193, 3)) for _ in range(400)]
    for P, BW in ((2516.6, 8000.0), (116.5, 456.0), (100.0, 1e9)):
        ridge = P * 1e12 / (BW * 1e9)
        expect = sum(2.0 * M * N * K / (2.0 * M * K + 2.0 * K * N + 2.0 * M * N) >= ridge * (1 - 1e-12)
                     for M, N, K in shapes) / len(shapes)
        ones = [1.0] * len(shapes)
        assert metrics.decompose(shapes, ones, ones, P, BW)["cb_bandwidth"] == pytest.approx(expect)
    # with unlimited bandwidth every shape is compute-bound
    assert metrics.decompose(shapes, ones, ones, 2516.6, 1e30)["cb_bandwidth"] == 1.0


def test_compute_bound_against_measured_memory_time():
    rng = np.random.default_rng(53)
    shapes = [tuple(int(x) for x in rng.integers(128, 4097, 3)) for _ in range(300)]
    r = rng.uniform(0.5, 2.0, len(shapes))
    t_mem = [metrics.compute_time(*s, 2516.6) * float(x) for s, x in zip(shapes, r)]
    d = metrics.decompose(shapes, [1.0] * len(shapes), t_mem, 2516.6, 8000.0)
    assert d["cb_measured"] == pytest.approx(float(np.mean(r <= 1.0)))
