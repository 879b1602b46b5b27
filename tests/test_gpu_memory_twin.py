"""The memory-only twin of each tile kernel (the measured memory surface of the paper's Sec. 4)
through the C ABI: it must move the operands and write C like its GEMM kernel, so what it
writes is exactly beta * C, nothing outside C's M x N window changes, and it runs wherever the
GEMM kernel runs (every variant, split-K, packed operands)."""
import numpy as np
import pytest

import synth
from gpu_helpers import inputs, say

pytestmark = pytest.mark.gpu

sg = pytest.importorskip("paper_2605_29752_amd")
NV = 32          # variants with a memory-only twin (stream-K variants have none)
F32, BF16 = 0, 1


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return sg.Context(0)


def _bits(C, c_dtype):
    """Raw element bits of a device C (uint32 for FP32, uint16 for BF16)."""
    if c_dtype == F32:
        return C.cpu().numpy().view(np.uint32)
    return sg.bf16_tensor_bits(C)


def _run_twin(ctx, M, N, K, variant, c_dtype, ldc_pad, beta, seed, operands="int"):
    import torch
    A, B = inputs(seed, M, N, K, operands)
    dA, dB = sg.to_device_bf16(A), sg.to_device_bf16(B)
    rows, ldc = M + 3, N + ldc_pad
    c0 = synth.uniform_pm1_f32(seed, 9, rows * ldc).reshape(rows, ldc)
    if c_dtype == F32:
        C = torch.from_numpy(c0.copy()).cuda()
    else:
        C = sg.to_device_bf16(synth.f32_to_bf16_bits(c0))
    before = _bits(C, c_dtype).copy()
    ctx.gemm(dA, dB, C, M=M, N=N, K=K, ldc=ldc, beta=beta, mode=sg.MODE_MEMORY, variant=variant)
    torch.cuda.synchronize()
    return before, _bits(C, c_dtype)


@pytest.mark.parametrize("variant", range(NV))
@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_twin_writes_zeros_and_nothing_else(ctx, variant, c_dtype):
    # several tiles of every shape, a ragged tail, K not a multiple of 64; a C row pitch that
    # allows vector stores (N + 8)
    M, N, K = 520, 392, 712
    say("twin variant", variant, "dtype", c_dtype)
    before, after = _run_twin(ctx, M, N, K, variant, c_dtype, 8, 0, 300 + variant)
    assert np.all(after[:M, :N] == 0), int(np.count_nonzero(after[:M, :N]))
    assert np.array_equal(after[M:, :], before[M:, :])
    assert np.array_equal(after[:, N:], before[:, N:])


@pytest.mark.parametrize("variant", [0, 3, 6, 13, 27])
@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_twin_beta_one_leaves_c_unchanged(ctx, variant, c_dtype):
    # beta = 1: the twin reads C as the addend and writes it back (0 + C, exact)
    M, N, K = 264, 328, 520
    before, after = _run_twin(ctx, M, N, K, variant, c_dtype, 8, 1, 400 + variant)
    assert np.array_equal(after, before)


@pytest.mark.parametrize("variant", [0, 4, 8, 12, 16, 20, 24, 27])
@pytest.mark.parametrize("shape", [(264, 331, 1003), (77, 93, 131), (1, 1, 1)])
def test_twin_packed_and_scalar_store_paths(ctx, variant, shape):
    # unaligned K and N (operands packed first) and a C pitch of N + 5 (no vector stores)
    M, N, K = shape
    before, after = _run_twin(ctx, M, N, K, variant, BF16, 5, 0, 500 + variant, "uniform")
    assert np.all(after[:M, :N] == 0)
    assert np.array_equal(after[M:, :], before[M:, :])
    assert np.array_equal(after[:, N:], before[:, N:])


def test_twin_sweep_times(ctx):
    import torch
    shapes = [(128, 128, 128), (1024, 768, 512), (2048, 2048, 2048), (4096, 4096, 128)]
    A = torch.zeros(4096 * 4096, dtype=torch.bfloat16, device="cuda")
    B = torch.zeros(4096 * 4096, dtype=torch.bfloat16, device="cuda")
    C = torch.zeros(4096 * 4096, dtype=torch.bfloat16, device="cuda")
    for v in (0, 12, 24, 25, 28):
        t_mem = ctx.sweep(shapes, A, B, C, mode=sg.MODE_MEMORY, variant=v, warmup=2, reps=5)
        t_gemm = ctx.sweep(shapes, A, B, C, mode=sg.MODE_VARIANT, variant=v, warmup=2, reps=5)
        say("variant", v, "memory", t_mem, "gemm", t_gemm)
        assert np.all(np.isfinite(t_mem)) and np.all(t_mem > 0)
        # on the compute-heavy cube the twin (a subset of its GEMM's work) is never much slower:
        # for the tiles whose load pipeline sets the pace (128x128 and smaller) it runs close to
        # the GEMM's time, for 256x256 (one work-group per CU, loads well covered) clearly below
        # it.  Few-microsecond shapes are left out: single runs there vary by tens of percent.
        assert t_mem[2] < 1.15 * t_gemm[2], (t_mem, t_gemm)
        if v == 0:
            assert t_mem[2] < 0.9 * t_gemm[2]


def test_twin_errors(ctx):
    import torch
    A = torch.zeros(8, 8, dtype=torch.bfloat16, device="cuda")
    C = torch.zeros(8, 8, dtype=torch.float32, device="cuda")
    with pytest.raises(sg.SGError) as e:
        ctx.gemm(A, A, C, mode=sg.MODE_MEMORY, variant=99)
    assert e.value.code == sg.SG_EINVAL
    with pytest.raises(sg.SGError) as e:
        ctx.gemm(A, A, C, mode=6)
    assert e.value.code == sg.SG_EINVAL
