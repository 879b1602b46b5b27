"""The no-allocation entry point (gemm_bf16_nn_ex_noalloc) against gemm_bf16_nn_ex.

Both calls run the same plan on the same kernels, so every output must be bit-identical; the
oracle bounds both.  Each case runs two calls in a row, the second on a smaller input, so the
second call finds the first call's leftovers in the shared scratch.  Cases that put something
in the scratch: a parallel split-K variant (FP32 partials), operands that need a zero-padded
copy (odd leading dimension), and a dispatch-table plan with a K split and BF16 output (the
FP32 plan accumulator).  A call that needs more scratch than the array holds is refused before
anything is enqueued."""
import numpy as np
import pytest
import torch

from gpu_helpers import check_tol, inputs, say

pytestmark = pytest.mark.gpu
sg = pytest.importorskip("paper_2605_29752_amd")
F32, BF16 = 0, 1


@pytest.fixture(scope="module")
def ctx():
    c = sg.Context(0)
    yield c
    c.set_table(None)
    c.close()


def _run(ctx, A_bits, B_bits, c_dtype, *, mode, variant=0, noalloc, beta=0, C0=None):
    M, K = A_bits.shape
    N = B_bits.shape[1]
    A = sg.to_device_bf16(A_bits)
    B = sg.to_device_bf16(B_bits)
    dt = torch.float32 if c_dtype == F32 else torch.bfloat16
    C = C0.clone() if C0 is not None else torch.full((M, N), float("nan"), dtype=dt, device="cuda")
    ctx.gemm(A, B, C, beta=beta, mode=mode, variant=variant, noalloc=noalloc)
    torch.cuda.synchronize()
    return C


def _bits(C):
    return C.view(torch.int32 if C.dtype == torch.float32 else torch.int16).cpu().numpy()


def _compare(ctx, shapes, c_dtype, mode, variant=0, kind="uniform"):
    for i, (M, N, K) in enumerate(shapes):
        say("noalloc", (M, N, K), "dtype", c_dtype, "mode", mode, "variant", variant)
        A, B = inputs(700 + i, M, N, K, kind)
        ref = _run(ctx, A, B, c_dtype, mode=mode, variant=variant, noalloc=False)
        got = _run(ctx, A, B, c_dtype, mode=mode, variant=variant, noalloc=True)
        assert np.array_equal(_bits(ref), _bits(got)), "no-allocation output differs"
        out = got.float().cpu().numpy().astype(np.float64)
        check_tol(out, A, B, c_dtype)


def test_scratch_size_is_stated():
    assert sg.noalloc_scratch_bytes() == 256 << 20


@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_split_k_partials_in_scratch(ctx, c_dtype):
    # 128x128 with 8 splits (variant 15): partials of S x M x N FP32 in the scratch
    _compare(ctx, [(520, 392, 1712), (136, 264, 520)], c_dtype, sg.MODE_VARIANT, variant=15)


def test_packed_operands_in_scratch(ctx):
    # K and N not multiples of 8: A and B are copied zero-padded into the scratch first
    _compare(ctx, [(301, 257, 199), (77, 65, 33)], BF16, sg.MODE_VARIANT, variant=13)


def test_dp_plan_with_k_split_bf16(ctx):
    # a table whose T0 grows steeply in K makes every cell with K > 1 step split along K; with
    # BF16 output the pieces accumulate in the FP32 plan accumulator in the scratch
    step, shape = 64, (3, 3, 4)
    g = np.meshgrid(*[np.arange(1, n + 1) for n in shape], indexing="ij")
    T0 = (g[0] * g[1] * g[2] ** 3).astype(np.float64)[None] + 0.01
    t = sg.Table.from_t0(step, *shape, T0, [13])
    assert t.lookup(192, 192, 256)["action"] == sg.ACT_SPLIT_K
    ctx.set_table(t)
    try:
        _compare(ctx, [(192, 180, 250), (70, 64, 130)], BF16, sg.MODE_DP)
        _compare(ctx, [(150, 190, 256), (64, 8, 200)], BF16, sg.MODE_DP, kind="int")
    finally:
        ctx.set_table(None)


def test_oversized_call_is_refused_before_launch(ctx):
    # 8 split-K partial slices of 4096 x 4096 FP32 (512 MiB) do not fit the 256 MiB array
    M = N = 4096
    K = 1024
    A = torch.zeros(M, K, dtype=torch.bfloat16, device="cuda")
    B = torch.zeros(K, N, dtype=torch.bfloat16, device="cuda")
    C = torch.full((M, N), 7.0, dtype=torch.bfloat16, device="cuda")
    with pytest.raises(sg.SGError) as e:
        ctx.gemm(A, B, C, mode=sg.MODE_VARIANT, variant=15, noalloc=True)
    assert e.value.code == sg.SG_ERANGE
    torch.cuda.synchronize()
    assert bool((C == 7.0).all()), "a refused call must not write C"
    # the same call through the allocating entry point works
    ctx.gemm(A, B, C, mode=sg.MODE_VARIANT, variant=15)
    torch.cuda.synchronize()
    assert bool((C == 0).all())
