"""Stream-K variants (32 + t): every work-group takes an equal share of the (tile, K stage)
iterations of all tiles; tiles split between work-groups are summed from FP32 partials by a
fix-up kernel in K order.  Parity against the FP64 oracle, bit-exactness on integer inputs,
bit-reproducibility, the addend (beta = 1) both on whole tiles and through the fix-up, packed
(unaligned) operands, and launches with fewer iterations than resident work-groups."""
import numpy as np
import pytest

from gpu_helpers import check_exact, check_tol, inputs, run_gemm, say

pytestmark = pytest.mark.gpu
sg = pytest.importorskip("paper_2605_29752_amd")
F32, BF16 = 0, 1
SK = list(range(32, 39))
# shapes with split tiles (ragged iteration counts), several segments per work-group, a single
# tile with fewer iterations than work-groups, and a tile count that splits evenly
SHAPES = [(520, 392, 712), (1000, 1300, 900), (64, 64, 64), (1, 1, 1), (1024, 1024, 256), (300, 2000, 3000)]


@pytest.fixture(scope="module")
def ctx():
    c = sg.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("variant", SK)
@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_stream_k_integer_exact(ctx, variant, c_dtype):
    for i, (M, N, K) in enumerate(SHAPES):
        say("stream-K", variant, (M, N, K), "dtype", c_dtype)
        A, B = inputs(400 + variant + i, M, N, K, "int")
        out = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_VARIANT, variant=variant)
        check_exact(out, A, B, c_dtype)


@pytest.mark.parametrize("variant", SK)
def test_stream_k_random_within_tolerance_and_reproducible(ctx, variant):
    import torch
    M, N, K = 777, 555, 1333
    A, B = inputs(500 + variant, M, N, K)
    for c_dtype in (F32, BF16):
        out1 = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_VARIANT, variant=variant)
        out2 = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_VARIANT, variant=variant)
        assert np.array_equal(out1, out2), "stream-K result is not reproducible"
        check_tol(out1, A, B, c_dtype)


@pytest.mark.parametrize("variant", [33, 35, 38])
@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_stream_k_beta_one(ctx, variant, c_dtype):
    import synth
    M, N, K = 333, 444, 2222
    A, B = inputs(600 + variant, M, N, K, "int")
    c0 = synth.integer_bf16(601 + variant, 7, M, N)
    c0f = synth.bf16_bits_to_f32(c0).astype(np.float64)
    import oracle
    want = oracle.gemm_f64(A, B, want_d=False) + c0f
    if c_dtype == F32:
        out = run_gemm(ctx, A, B, F32, mode=sg.MODE_VARIANT, variant=variant, beta=1,
                       C0_f32=c0f.astype(np.float32))
        assert np.array_equal(out, want)
    else:
        out = run_gemm(ctx, A, B, BF16, mode=sg.MODE_VARIANT, variant=variant, beta=1, C0_bits=c0)
        assert np.array_equal(out, synth.bf16_bits_to_f32(oracle.f64_to_bf16_rne(want)).astype(np.float64))


@pytest.mark.parametrize("variant", [32, 35, 38])
def test_stream_k_unaligned_operands(ctx, variant):
    for (M, N, K) in [(301, 257, 199), (17, 1031, 1001)]:
        A, B = inputs(700 + variant, M, N, K, "int")
        out = run_gemm(ctx, A, B, BF16, mode=sg.MODE_VARIANT, variant=variant)
        check_exact(out, A, B, BF16)


def test_stream_k_in_dispatch_plans(ctx):
    # a table whose best variant everywhere is a stream-K one, with pads and splits around it
    step, shape = 128, (3, 3, 4)
    rng = np.random.default_rng(8)
    variants = [12, 35, 38]
    T0 = rng.uniform(1.0, 2.0, size=(len(variants),) + shape)
    T0[1] *= 0.5
    t = sg.Table.from_t0(step, *shape, T0, variants)
    ctx.set_table(t)
    try:
        for (M, N, K) in [(384, 384, 512), (200, 300, 450), (129, 257, 385)]:
            A, B = inputs(800 + M, M, N, K, "int")
            for c_dtype in (F32, BF16):
                out = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_DP)
                check_exact(out, A, B, c_dtype)
    finally:
        ctx.set_table(None)
