"""The C-ABI library on the CPU: every declared symbol is exported, and the host-side logic
(dispatch table DP, lookup, save/load, metrics) agrees with the oracle.  No GPU calls."""
import ctypes
import os
import re

import math

import numpy as np
import pytest

import paper_2605_29752_amd as sg
from oracle import dp as odp
from oracle import metrics as om

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = []
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M):
            if not m.group(0).lstrip().startswith(("typedef", "#", "return")):
                names.append(m.group(1))
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(sg.LIB_PATH)
    names = _declared_functions()
    assert len(names) >= 20
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding covers every one of them
    assert sorted(sg.declared_symbols()) == names


def test_variant_family():
    n = sg.num_variants()
    assert n == 39                      # 8 tiles x 4 split-K levels, then stream-K on tiles 0..6
    seen = set()
    for v in range(n):
        info = sg.variant_info(v)
        assert info.lds_bytes <= 160 * 1024
        if v < 32:
            assert info.bk == (128 if v // 4 == 7 else 64) and info.splits == 1 << (v % 4)
        else:
            assert info.bk == 64 and info.splits == 0 and info.name.endswith("_sk")
            plain = sg.variant_info(4 * (v - 32))
            assert (info.bm, info.bn) == (plain.bm, plain.bn)
        seen.add((info.bm, info.bn, info.bk, info.splits))
    assert len(seen) == n
    assert sg.variant_info(28).name == "64x64x128_s1"
    assert sg.variant_info(35).name == "128x128x64_sk"
    with pytest.raises(sg.SGError):
        sg.variant_info(n)


@pytest.mark.parametrize("shape", [(2, 3, 4), (5, 5, 5), (6, 4, 7), (8, 8, 8)])
def test_table_dp_matches_oracle(shape):
    rng = np.random.default_rng(sum(shape))
    nv = 3
    T0 = rng.uniform(1.0, 10.0, size=(nv,) + shape)
    t = sg.Table.from_t0(128, *shape, T0, [0, 3, 6])
    best = T0.min(axis=0)
    T1, T2, act, arg = odp.tables(best)
    assert np.array_equal(t.values(0), best)
    assert np.array_equal(t.values(1), T1)
    assert np.array_equal(t.values(2), T2)
    assert np.array_equal(t.values(3), T0)
    vids = np.array([0, 3, 6])[T0.argmin(axis=0)]
    for cell in np.ndindex(shape):
        M, N, K = [(c + 1) * 128 for c in cell]
        r = t.lookup(M, N, K)
        assert r["action"] == act[cell] and r["arg"] == arg[cell], cell
        if r["action"] == sg.ACT_AS_IS:
            assert r["variant"] == vids[cell]
        if r["action"] == sg.ACT_PAD:
            assert r["variant"] == vids[np.unravel_index(arg[cell], shape)]
        assert t.plan_leaves(M, N, K) == len(odp.plan_leaves(shape, act, arg, cell))


def test_table_lookup_off_grid_and_range():
    T0 = np.random.default_rng(1).uniform(1, 2, size=(1, 4, 4, 4))
    t = sg.Table.from_t0(128, 4, 4, 4, T0, [3])
    assert t.lookup(1, 1, 1)["t0"] == T0[0, 0, 0, 0]
    assert t.lookup(129, 128, 257)["t0"] == T0[0, 1, 0, 2]
    assert t.lookup(512, 512, 512)["t0"] == T0[0, 3, 3, 3]
    with pytest.raises(sg.SGError) as e:
        t.lookup(513, 1, 1)
    assert e.value.code == sg.SG_ERANGE
    with pytest.raises(sg.SGError):
        t.lookup(0, 5, 5)


def test_plan_choice_interpolates_t0_between_cells():
    # T0 multilinear in (M, N, K) is reproduced exactly by trilinear interpolation inside the
    # grid, and clamped to the first / last cell outside it
    g, n = 128, 4
    sizes = (np.arange(n) + 1) * g
    M3, N3, K3 = np.meshgrid(sizes, sizes, sizes, indexing="ij")
    f = lambda m, nn, k: (1.0 + 0.001 * m) * (2.0 + 0.002 * nn) * (0.5 + 0.003 * k)
    T0 = f(M3, N3, K3)[None].astype(np.float64)
    t = sg.Table.from_t0(g, n, n, n, T0, [12])
    for (M, N, K) in [(200, 300, 400), (129, 511, 256), (384, 130, 500), (257, 257, 257)]:
        assert math.isclose(t.plan_choice(M, N, K)["est_best"], f(M, N, K), rel_tol=1e-12)
    assert math.isclose(t.plan_choice(5, 300, 128)["est_best"], f(128, 300, 128), rel_tol=1e-12)


def test_plan_choice_on_grid_always_runs_the_table_plan():
    rng = np.random.default_rng(7)
    T0 = rng.uniform(1.0, 10.0, size=(2, 4, 4, 4))
    t = sg.Table.from_t0(128, 4, 4, 4, T0, [0, 12])
    for cell in np.ndindex(4, 4, 4):
        M, N, K = [(c + 1) * 128 for c in cell]
        ch = t.plan_choice(M, N, K)
        assert ch["use_plan"]
        if t.lookup(M, N, K)["action"] == sg.ACT_AS_IS:
            assert ch["est_plan"] == ch["est_best"] == T0.min(axis=0)[cell]


def test_plan_choice_off_grid_drops_a_split_that_no_longer_pays():
    # one variant along M only: 512 splits into 128 + 384 (2.5 + 3.2 < 7) on the grid
    T0 = np.array([2.5, 3.0, 3.2, 7.0]).reshape(1, 4, 1, 1)
    t = sg.Table.from_t0(128, 4, 1, 1, T0, [12])
    r = t.lookup(512, 128, 128)
    assert r["action"] == sg.ACT_SPLIT_M and r["arg"] == 1 and r["t2"] == 5.7
    assert t.plan_choice(512, 128, 128)["use_plan"]
    # M = 390 (cell 512): pieces 128 + 262 cost 2.5 + 3.009, the variant alone 3.378
    ch = t.plan_choice(390, 128, 128)
    assert math.isclose(ch["est_plan"], 2.5 + 3.0 + 6 / 128 * 0.2, rel_tol=1e-12)
    assert math.isclose(ch["est_best"], 3.2 + 6 / 128 * 3.8, rel_tol=1e-12)
    assert not ch["use_plan"]
    # M = 500: pieces 128 + 372 cost 5.68, the variant alone 6.64: the split still pays
    ch = t.plan_choice(500, 128, 128)
    assert ch["use_plan"] and ch["est_plan"] < 0.95 * ch["est_best"]
    # M = 472: the split is estimated 3 % faster (5.6375 against 5.8125), inside the 5 % margin
    ch = t.plan_choice(472, 128, 128)
    assert math.isclose(ch["est_plan"] / ch["est_best"], 5.6375 / 5.8125, rel_tol=1e-12)
    assert not ch["use_plan"]
    with pytest.raises(sg.SGError) as e:
        t.plan_choice(513, 1, 1)
    assert e.value.code == sg.SG_ERANGE


def test_table_rejects_bad_t0():
    T0 = np.ones((1, 2, 2, 2))
    T0[0, 1, 1, 1] = np.nan
    with pytest.raises(sg.SGError):
        sg.Table.from_t0(128, 2, 2, 2, T0, [0])
    with pytest.raises(sg.SGError):
        sg.Table.from_t0(128, 2, 2, 2, np.ones((1, 2, 2, 2)), [99])
    with pytest.raises(sg.SGError):
        sg.Table.from_t0(0, 2, 2, 2, np.ones((1, 2, 2, 2)), [0])


def test_table_save_load_roundtrip(tmp_path):
    T0 = np.random.default_rng(2).uniform(1, 2, size=(2, 3, 4, 5))
    t = sg.Table.from_t0(64, 3, 4, 5, T0, [1, 2])
    p = str(tmp_path / "t.sgt")
    t.save(p)
    t2 = sg.Table.load(p, force=True)
    for w in range(4):
        assert np.array_equal(t.values(w), t2.values(w))
    assert t2.grid() == (64, 3, 4, 5) and t2.variants() == [1, 2]
    open(p, "r+b").write(b"XXXX")
    with pytest.raises(sg.SGError) as e:
        sg.Table.load(p, force=True)
    assert e.value.code == sg.SG_EIO


def test_metrics_match_oracle():
    rng = np.random.default_rng(3)
    T = rng.uniform(0, 100, size=(5, 6, 7))
    got = sg.landscape_stats(T)
    want = om.aggregate_3d(T)
    for k in ("mean", "peak", "roughness_m", "roughness_n", "roughness_k", "roughness_3d"):
        assert got[k] == pytest.approx(want[k], rel=1e-12), k
    v = rng.uniform(0, 10, size=33)
    assert sg.roughness(v) == pytest.approx(om.roughness(v), rel=1e-12)
    assert np.isnan(sg.roughness([1.0]))
    with pytest.raises(sg.SGError):
        sg.landscape_stats(np.zeros((1, 3, 3)))


def test_ideal_landscape_through_library():
    sizes = list(range(128, 4097, 128))
    L = np.array([[om.ideal_tflops(m, n, 108.2, 20, 256) for n in sizes] for m in sizes])
    # a K axis of two identical slices keeps the per-slice N roughness
    st = sg.landscape_stats(np.stack([L, L], axis=2))
    assert abs(st["mean"] - 97.2) <= 0.05 and abs(st["roughness_n"] - 2.0) <= 0.05


def test_first_principles_landscapes_match_oracle():
    step, nm, nn, nk = 128, 9, 11, 5
    hw = {"peak_tflops": 2516.6, "cores": 256, "bw_gbs": 8000.0}
    ideal = sg.ideal_landscape(step, nm, nn, nk, tile=256, hw=hw)
    opt = sg.optimal_landscape(step, nm, nn, nk, tiles=(256, 128, 64), c_bytes=2, hw=hw)
    for a in range(nm):
        for b in range(nn):
            for c in range(nk):
                M, N, K = (a + 1) * step, (b + 1) * step, (c + 1) * step
                assert ideal[a, b, c] == pytest.approx(om.ideal_tflops(M, N, 2516.6, 256, 256), rel=1e-12)
                assert opt[a, b, c] == pytest.approx(
                    om.optimal_tflops(M, N, K, 2516.6, 256, 8000.0, tiles=(256, 128, 64), c_bytes=2), rel=1e-12)
    # the memory-channel term: the library against the oracle with the paper's Arc B580 constants
    b580hw = {"peak_tflops": 108.2, "cores": 20, "bw_gbs": 451.0}
    och = sg.optimal_landscape(step, nm, nn, nk, tiles=(256, 128, 64), c_bytes=4, hw=b580hw, channels=6)
    for a in range(nm):
        for b in range(nn):
            for c in range(nk):
                M, N, K = (a + 1) * step, (b + 1) * step, (c + 1) * step
                assert och[a, b, c] == pytest.approx(
                    om.optimal_tflops(M, N, K, 108.2, 20, 451.0, tiles=(256, 128, 64), c_bytes=4, channels=6),
                    rel=1e-12)
    # the paper's own ideal through the library: Arc B580 constants (Sec. 9.1)
    b580 = sg.ideal_landscape(128, 32, 32, 2, tile=256, hw={"peak_tflops": 108.2, "cores": 20, "bw_gbs": 451.0})
    st = sg.landscape_stats(b580)
    assert abs(st["mean"] - 97.2) <= 0.05 and abs(st["roughness_n"] - 2.0) <= 0.05
    with pytest.raises(sg.SGError):
        sg.optimal_landscape(128, 2, 2, 2, tiles=(0,), hw=hw)
    with pytest.raises(sg.SGError):
        sg.ideal_landscape(128, 2, 2, 2, hw={"peak_tflops": 0.0, "cores": 256, "bw_gbs": 1.0})


def test_kol_grade_matches_oracle():
    rng = np.random.default_rng(5)
    O = rng.uniform(500, 2500, size=(6, 7, 4))
    for A in (O, 0.3 * O, O + rng.uniform(-200, 200, size=O.shape), np.sort(O, axis=1)):
        got = sg.kol_grade(A, O)
        want = om.kol_grade(A, O)
        for k in ("tau", "rho"):
            assert got[k] == pytest.approx(want[k], rel=1e-12)
        for k in ("t_band", "s_band", "level"):
            assert got[k] == want[k]
    g2 = sg.kol_grade(O[:, :, 0], O[:, :, 0])          # a 2-D slice
    assert g2["level"] == 3
    with pytest.raises(sg.SGError):
        sg.kol_grade(np.ones((2, 1, 1)), np.ones((2, 1, 1)))


def test_decompose_matches_oracle():
    rng = np.random.default_rng(17)
    shapes = [tuple(int(x) for x in rng.integers(1, 8193, 3)) for _ in range(500)]
    t_gemm = rng.uniform(1e-6, 2e-3, len(shapes))
    t_mem = t_gemm * rng.uniform(0.2, 1.3, len(shapes))
    for c_bytes, hw in ((2, sg.MI355X), (4, {"peak_tflops": 116.5, "cores": 20, "bw_gbs": 456.0})):
        got = sg.decompose(shapes, t_gemm, t_mem, c_bytes=c_bytes, hw=hw)
        want = om.decompose(shapes, list(t_gemm), list(t_mem), hw["peak_tflops"], hw["bw_gbs"], c_bytes)
        np.testing.assert_allclose(got["t_compute"], want["t_compute"], rtol=1e-14, atol=0)
        np.testing.assert_allclose(got["t_overhead"], want["t_overhead"], rtol=1e-12, atol=1e-20)
        assert got["overhead_share"] == pytest.approx(want["overhead_share"], rel=1e-12)
        assert got["cb_bandwidth"] == want["cb_bandwidth"]
        assert got["cb_measured"] == want["cb_measured"]
    with pytest.raises(sg.SGError):
        sg.decompose([(0, 5, 5)], [1.0], [1.0])
    with pytest.raises(sg.SGError):
        sg.decompose([(5, 5, 5)], [0.0], [1.0])
    with pytest.raises(sg.SGError):
        sg.decompose([(5, 5, 5)], [1.0], [1.0], c_bytes=0)


def test_synthetic_plans_cover_every_action():
    """The GPU plan-execution tests rely on these synthetic tables producing every action."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    from test_gpu_dp import _random_table
    for seed, shape, variants in [(1, (4, 4, 5), [3, 6, 9, 26]), (2, (5, 5, 5), [3, 6, 10, 25])]:
        t, _ = _random_table(seed, shape, 64, variants)
        acts = {t.lookup(*[(c + 1) * 64 for c in cell])["action"] for cell in np.ndindex(shape)}
        assert acts == {0, 1, 2, 3, 4}


def test_memory_study_host_contract():
    """Block count of the streaming read, and arguments rejected before any device call."""
    L = sg.lib()
    assert L.sg_mem_read_blocks(0) == 1 and L.sg_mem_read_blocks(16) == 1
    assert L.sg_mem_read_blocks(1 << 20) == 64          # 65,536 16-byte chunks / (256 lanes x 4)
    assert L.sg_mem_read_blocks(1 << 30) == 2048        # capped at 8 work-groups per CU
    assert L.sg_mem_read_blocks(-5) == 0
    assert L.sg_mem_read(None, 20, None, None) == sg.SG_EINVAL       # not a multiple of 16
    assert L.sg_mem_read(None, 32, None, None) == sg.SG_EINVAL       # NULL buffer
    assert L.sg_mem_write(None, -16, 0, None) == sg.SG_EINVAL
    assert L.sg_mem_sweep(None, None, 0, 0, 0, 4, 0, 1, None, None) == sg.SG_EINVAL
