"""GPU execution of dispatch-table plans (pad, M/N/K splits, nested) and of the table builder."""
import numpy as np
import pytest

from oracle import dp as odp
from gpu_helpers import check_exact, check_tol, inputs, run_gemm, say

pytestmark = pytest.mark.gpu
sg = pytest.importorskip("paper_2605_29752_amd")
F32, BF16 = 0, 1


@pytest.fixture(scope="module")
def ctx():
    return sg.Context(0)


def _random_table(seed, shape, step, variants):
    """Landscape-like synthetic timings: overhead + volume, per-variant noise, and 30% of the
    cells made 2.5x slower, so that as-is, pad and all three splits occur."""
    rng = np.random.default_rng(seed)
    g = np.meshgrid(*[np.arange(1, n + 1) for n in shape], indexing="ij")
    base = 2.0 + (g[0] * g[1] * g[2]).astype(np.float64)
    noise = rng.uniform(0.7, 1.3, size=(len(variants),) + shape)
    bad = rng.uniform(size=shape) < 0.3
    T0 = base[None] * noise * np.where(bad, 2.5, 1.0)[None]
    return sg.Table.from_t0(step, *shape, T0, variants), T0


def _plans_cover_every_action(T0best_shape, t, shape, step):
    acts = set()
    for cell in np.ndindex(shape):
        acts.add(t.lookup(*[(c + 1) * step for c in cell])["action"])
    return acts


@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_dp_plans_bit_exact_on_grid(ctx, c_dtype):
    step, shape = 64, (4, 4, 5)
    variants = [3, 6, 9, 26]          # 128x128, 64x64, 128x128/s2, 64x64/s4
    t, T0 = _random_table(1, shape, step, variants)
    assert {0, 1, 2, 3, 4} <= _plans_cover_every_action(None, t, shape, step)
    ctx.set_table(t)
    try:
        for cell in np.ndindex(shape):
            M, N, K = [(c + 1) * step for c in cell]
            A, B = inputs(100 + sum(cell), M, N, K, "int")
            out = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_DP)
            check_exact(out, A, B, c_dtype)
    finally:
        ctx.set_table(None)


@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_dp_plans_off_grid_shapes(ctx, c_dtype):
    step, shape = 64, (5, 5, 5)
    t, T0 = _random_table(2, shape, step, [3, 6, 10, 25])
    ctx.set_table(t)
    rng = np.random.default_rng(3)
    try:
        for i in range(25):
            M, N, K = [int(x) for x in rng.integers(1, 5 * step + 1, 3)]
            say("off-grid", (M, N, K), t.lookup(M, N, K))
            A, B = inputs(200 + i, M, N, K, "int")
            out = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_DP)
            check_exact(out, A, B, c_dtype)
            A, B = inputs(300 + i, M, N, K)
            out = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_DP)
            check_tol(out, A, B, c_dtype)
    finally:
        ctx.set_table(None)


def test_dp_bf16_beta_one_with_k_split(ctx):
    # force a K split at every cell with K > 1 step: T0 grows steeply in K
    step, shape = 64, (2, 2, 4)
    g = np.meshgrid(*[np.arange(1, n + 1) for n in shape], indexing="ij")
    T0 = (g[0] * g[1] * g[2] ** 3).astype(np.float64)[None] + 0.01
    t = sg.Table.from_t0(step, *shape, T0, [6])
    assert t.lookup(128, 128, 256)["action"] == sg.ACT_SPLIT_K
    ctx.set_table(t)
    try:
        M, N, K = 128, 128, 256
        A, B = inputs(9, M, N, K)
        import synth
        c0 = synth.f32_to_bf16_bits(synth.uniform_pm1_f32(9, 9, M * N).reshape(M, N))
        out = run_gemm(ctx, A, B, BF16, mode=sg.MODE_DP, beta=1, C0_bits=c0)
        check_tol(out, A, B, BF16, addend=synth.bf16_bits_to_f32(c0).astype(np.float64))
    finally:
        ctx.set_table(None)


def test_best_mode_uses_argmin_variant(ctx):
    step, shape = 128, (2, 2, 2)
    t, T0 = _random_table(4, shape, step, [0, 3, 6])
    ctx.set_table(t)
    try:
        A, B = inputs(5, 200, 250, 256, "int")
        out = run_gemm(ctx, A, B, F32, mode=sg.MODE_BEST)
        check_exact(out, A, B, F32)
    finally:
        ctx.set_table(None)


def test_table_build_on_gpu_and_execute(ctx, tmp_path):
    import torch
    step, nm, nn, nk = 128, 2, 3, 2
    variants = [3, 6, 7]
    pool_a = sg.to_device_bf16(inputs(6, nm * step, 1, nk * step, "int")[0])
    pool_b = sg.to_device_bf16(inputs(6, 1, nn * step, nk * step, "int")[1])
    pool_c = torch.empty(nm * step * nn * step, dtype=torch.bfloat16, device="cuda")
    t = ctx.build_table(step, nm, nn, nk, variants, pool_a, pool_b, pool_c, warmup=2, reps=3,
                        order_seed=7)
    T0 = t.values(3)
    assert T0.shape == (3, nm, nn, nk) and np.all(T0 > 0) and np.all(np.isfinite(T0))
    best = T0.min(axis=0)
    T1, T2, act, arg = odp.tables(best)
    assert np.array_equal(t.values(2), T2)
    p = str(tmp_path / "gpu.sgt")
    t.save(p)
    t2 = sg.Table.load(p)               # same device: fingerprint matches
    assert np.array_equal(t2.values(2), T2)
    ctx.set_table(t2)
    try:
        for cell in np.ndindex((nm, nn, nk)):
            M, N, K = [(c + 1) * step for c in cell]
            A, B = inputs(7, M, N, K, "int")
            out = run_gemm(ctx, A, B, BF16, mode=sg.MODE_DP)
            check_exact(out, A, B, BF16)
    finally:
        ctx.set_table(None)


def test_sweep_driver_and_accounting(ctx):
    import torch
    shapes = [(128, 256, 384), (256, 128, 128), (384, 384, 256)]
    pa = torch.zeros(384 * 384, dtype=torch.bfloat16, device="cuda")
    pb = torch.zeros(384 * 384, dtype=torch.bfloat16, device="cuda")
    pc = torch.zeros(384 * 384, dtype=torch.bfloat16, device="cuda")
    sec = ctx.sweep(shapes, pa, pb, pc, mode=sg.MODE_VARIANT, variant=3, warmup=2, reps=4)
    assert np.all(sec > 0) and np.all(sec < 1.0)
    la, se, fl = ctx.kernel_times()
    assert la[3] == 3 * 4 and la.sum() == 12
    assert fl[3] == pytest.approx(4 * sum(2.0 * m * n * k for m, n, k in shapes))
    # the accounted time is the tile kernel's alone (variant 3 is 256x256 with eight splits: its
    # reduction is left out), so it is at most the runs' time and most of it
    assert 0.5 * 4 * sec.sum() <= se[3] <= 4 * sec.sum() * (1 + 1e-9)


@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_concurrent_split_pieces_bit_identical(ctx, c_dtype):
    """Plans whose M / N pieces run at the same time on the context's streams (each in its own
    workspace slice, split-K variants among them) give the bits of sequential execution, and
    are exact on integer inputs; plans with K pieces keep running sequentially.  Grid and
    off-grid shapes, and a second pass that reuses the streams and events."""
    step, shape = 64, (5, 5, 5)
    t, T0 = _random_table(4, shape, step, [3, 6, 10, 25, 27])
    ctx.set_table(t)
    rng = np.random.default_rng(9)
    shapes = [tuple((c + 1) * step for c in cell) for cell in np.ndindex(shape)][::3]
    shapes += [tuple(int(x) for x in rng.integers(1, 5 * step + 1, 3)) for _ in range(12)]
    try:
        for rnd in range(2):
            for i, (M, N, K) in enumerate(shapes):
                A, B = inputs(800 + i, M, N, K, "int")
                seq = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_DP)
                ctx.set_concurrent_splits(True)
                try:
                    conc = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_DP)
                finally:
                    ctx.set_concurrent_splits(False)
                assert np.array_equal(seq, conc), ((M, N, K), t.lookup(M, N, K))
                if rnd == 0:
                    check_exact(conc, A, B, c_dtype)
    finally:
        ctx.set_table(None)


def test_concurrent_split_sweep_timing(ctx):
    """The sweep times a concurrent plan between two markers on the caller's stream: positive
    and finite for every split cell."""
    import torch
    step, shape = 64, (5, 5, 5)
    t, T0 = _random_table(4, shape, step, [3, 6, 10, 25, 27])
    ctx.set_table(t)
    split = [tuple((c + 1) * step for c in cell) for cell in np.ndindex(shape)
             if t.lookup(*[(c + 1) * step for c in cell])["action"] in (sg.ACT_SPLIT_M, sg.ACT_SPLIT_N)]
    assert split
    pool = torch.zeros(512 * 512, dtype=torch.bfloat16, device="cuda")
    C = torch.zeros(512 * 512, dtype=torch.bfloat16, device="cuda")
    try:
        ctx.set_concurrent_splits(2)
        seq = ctx.sweep(split, pool, pool, C, mode=sg.MODE_DP, warmup=1, reps=3)
        ctx.set_concurrent_splits(1)
        conc = ctx.sweep(split, pool, pool, C, mode=sg.MODE_DP, warmup=1, reps=3)
    finally:
        ctx.set_concurrent_splits(False)
        ctx.set_table(None)
    say("split cells", len(split), "sequential us", seq[:4] * 1e6, "concurrent us", conc[:4] * 1e6)
    assert np.all(conc > 0) and np.all(np.isfinite(conc))
    assert np.all(seq > 0) and np.all(np.isfinite(seq))


def test_sweep_split_variant_on_single_split_k(ctx):
    """A split-K variant whose K extent fits one split runs without a reduction; the sweep must
    time it from the tile kernel alone (regression: it asked for the reduction's event)."""
    import torch
    pool = torch.zeros(256 * 256, dtype=torch.bfloat16, device="cuda")
    C = torch.zeros(256 * 256, dtype=torch.bfloat16, device="cuda")
    for v in (1, 13, 27):                        # 256x256 s2, 128x128 s2, 64x64 s8
        sec = ctx.sweep([(128, 128, 64), (256, 192, 32), (192, 256, 128)], pool, pool, C,
                        mode=sg.MODE_VARIANT, variant=v, warmup=1, reps=2)
        assert np.all(sec > 0) and np.all(np.isfinite(sec))
        la, se, fl = ctx.kernel_times()
        assert la[v] == 6 and se[v] > 0


@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_split_pieces_as_one_grouped_launch(ctx, c_dtype):
    """Concurrent-split mode 3: the M / N pieces of a plan that all run one tile shape (no
    split-K) go out as ONE persistent grouped launch.  The grouped kernel runs the same tile
    body, so the bits equal sequential execution; exact on integer inputs; plans it cannot take
    (split-K pieces, mixed tiles, K pieces) fall back to sequential.  The sweep times it between
    markers."""
    import torch
    step, shape = 64, (5, 5, 5)
    # one tile shape for every variant (128x128 alone) so that every M / N split is groupable,
    # and a second table with a split-K variant so that some are not
    for variants in ([12], [12, 13, 24]):
        t, T0 = _random_table(5, shape, step, variants)
        ctx.set_table(t)
        rng = np.random.default_rng(19)
        shapes = [tuple((c + 1) * step for c in cell) for cell in np.ndindex(shape)][::2]
        shapes += [tuple(int(x) for x in rng.integers(1, 5 * step + 1, 3)) for _ in range(10)]
        try:
            for i, (M, N, K) in enumerate(shapes):
                A, B = inputs(900 + i, M, N, K, "int")
                seq = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_DP)
                ctx.set_concurrent_splits(3)
                try:
                    grp = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_DP)
                finally:
                    ctx.set_concurrent_splits(False)
                assert np.array_equal(seq, grp), ((M, N, K), t.lookup(M, N, K))
                check_exact(grp, A, B, c_dtype)
            split = [s for s in shapes if t.lookup(*s)["action"] in (sg.ACT_SPLIT_M, sg.ACT_SPLIT_N)]
            if split:
                pool = torch.zeros(512 * 512, dtype=torch.bfloat16, device="cuda")
                C = torch.zeros(512 * 512, dtype=torch.bfloat16, device="cuda")
                ctx.set_concurrent_splits(3)
                try:
                    sec = ctx.sweep(split, pool, pool, C, mode=sg.MODE_DP, warmup=1, reps=3)
                finally:
                    ctx.set_concurrent_splits(False)
                assert np.all(sec > 0) and np.all(np.isfinite(sec))
        finally:
            ctx.set_table(None)
