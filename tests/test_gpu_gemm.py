"""GPU parity of the tile family through the C ABI against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from gpu_helpers import TOL, check_exact, check_tol, inputs, run_gemm, say

pytestmark = pytest.mark.gpu

sg = pytest.importorskip("paper_2605_29752_amd")
NV = 39          # every variant: 8 tiles x 4 split-K levels, then stream-K on tiles 0..6
F32, BF16 = 0, 1


@pytest.fixture(scope="module")
def ctx():
    import torch
    assert torch.cuda.is_available()
    return sg.Context(0)


def test_config1_single_256_fp32(ctx):
    # M = N = K = 256, uniform[-1,1] BF16 inputs (seed 1), FP32 output, the plain variant
    say("config1 256^3 plain")
    A, B = inputs(1, 256, 256, 256)
    out = run_gemm(ctx, A, B, F32, mode=sg.MODE_PLAIN)
    err = check_tol(out, A, B, F32)
    say("config1 err %.3e" % err)


def test_paper_form_call(ctx):
    import torch
    A, B = inputs(2, 130, 70, 260)
    C = torch.zeros(130, 70, dtype=torch.float32, device="cuda")
    sg.gemm_bf16_nn(130, 70, 260, sg.to_device_bf16(A), sg.to_device_bf16(B), C)
    torch.cuda.synchronize()
    check_tol(C.cpu().numpy().astype(np.float64), A, B, F32)


@pytest.mark.parametrize("variant", range(NV))
@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_every_variant_ragged(ctx, variant, c_dtype):
    M, N, K = 520, 392, 712          # several tiles of every shape plus a ragged tail; K % 64 != 0
    say("variant", variant, "dtype", c_dtype)
    A, B = inputs(10 + variant, M, N, K)
    out = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_VARIANT, variant=variant)
    check_tol(out, A, B, c_dtype)


@pytest.mark.parametrize("variant", range(NV))
@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_every_variant_integer_exact(ctx, variant, c_dtype):
    M, N, K = 264, 328, 1000          # partial sums stay below 2^24: exact in any order
    A, B = inputs(50 + variant, M, N, K, "int")
    out = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_VARIANT, variant=variant)
    check_exact(out, A, B, c_dtype)


@pytest.mark.parametrize("variant", [0, 3, 6, 13, 27])
@pytest.mark.parametrize("c_dtype", [F32, BF16])
@pytest.mark.parametrize("shape", [(77, 93, 131), (1, 1, 1), (5, 300, 9), (129, 1, 65), (300, 7, 3)])
def test_unaligned_shapes(ctx, variant, c_dtype, shape):
    M, N, K = shape
    A, B = inputs(7, M, N, K)
    out = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_VARIANT, variant=variant)
    check_tol(out, A, B, c_dtype)


@pytest.mark.parametrize("variant", [0, 3, 6, 14, 25])
@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_beta_one_accumulates(ctx, variant, c_dtype):
    M, N, K = 200, 264, 392
    A, B = inputs(3, M, N, K)
    c0 = synth.uniform_pm1_f32(3, 7, M * N).reshape(M, N)
    c0_bits = synth.f32_to_bf16_bits(c0)
    if c_dtype == F32:
        out = run_gemm(ctx, A, B, F32, mode=sg.MODE_VARIANT, variant=variant, beta=1, C0_f32=c0)
        check_tol(out, A, B, F32, addend=c0.astype(np.float64))
    else:
        out = run_gemm(ctx, A, B, BF16, mode=sg.MODE_VARIANT, variant=variant, beta=1, C0_bits=c0_bits)
        check_tol(out, A, B, BF16, addend=synth.bf16_bits_to_f32(c0_bits).astype(np.float64))


@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_identity_returns_b_exactly(ctx, c_dtype):
    K, N = 384, 200
    eye = synth.f32_to_bf16_bits(np.eye(K, dtype=np.float32))
    B = synth.uniform_bf16(4, 1, K, N)
    for v in (0, 3, 6, 11):
        out = run_gemm(ctx, eye, B, c_dtype, mode=sg.MODE_VARIANT, variant=v)
        assert np.array_equal(out, synth.bf16_bits_to_f32(B).astype(np.float64))


def test_permutation_and_rank_one_closed_forms(ctx):
    K, N = 256, 136
    perm = np.random.default_rng(2).permutation(K)
    P = np.zeros((K, K), dtype=np.float32)
    P[np.arange(K), perm] = 1.0
    B = synth.uniform_bf16(5, 1, K, N)
    out = run_gemm(ctx, synth.f32_to_bf16_bits(P), B, F32, mode=sg.MODE_VARIANT, variant=3)
    assert np.array_equal(out, synth.bf16_bits_to_f32(B)[perm].astype(np.float64))
    u = np.array([1.5, -0.75, 2.0, 0.5, -3.0] * 20, dtype=np.float32)
    v = np.array([0.25, -1.25, 1.0, 6.0] * 30, dtype=np.float32)
    A1 = synth.f32_to_bf16_bits(np.repeat(u[:, None], 512, axis=1))
    B1 = synth.f32_to_bf16_bits(np.repeat(v[None, :], 512, axis=0))
    for var in (0, 7, 19):
        out = run_gemm(ctx, A1, B1, F32, mode=sg.MODE_VARIANT, variant=var)
        assert np.array_equal(out, 512.0 * np.outer(u, v).astype(np.float64))


def test_zero_sizes_and_k_zero(ctx):
    import torch
    A = torch.zeros(4, 0, dtype=torch.bfloat16, device="cuda")
    B = torch.zeros(0, 5, dtype=torch.bfloat16, device="cuda")
    C = torch.full((4, 5), 3.0, dtype=torch.float32, device="cuda")
    ctx.gemm(A, B, C, beta=1, mode=sg.MODE_PLAIN)
    torch.cuda.synchronize()
    assert torch.all(C == 3.0)
    ctx.gemm(A, B, C, beta=0, mode=sg.MODE_PLAIN)
    torch.cuda.synchronize()
    assert torch.all(C == 0.0)
    Ce = torch.full((0, 5), 1.0, dtype=torch.float32, device="cuda")
    ctx.gemm(torch.zeros(0, 3, dtype=torch.bfloat16, device="cuda"),
             torch.zeros(3, 5, dtype=torch.bfloat16, device="cuda"), Ce, mode=sg.MODE_PLAIN)


def test_leading_dimensions_views(ctx):
    import torch
    pa = synth.uniform_bf16(8, 0, 300, 520)
    pb = synth.uniform_bf16(8, 1, 400, 600)
    M, N, K = 250, 333, 390
    A = sg.to_device_bf16(pa)
    B = sg.to_device_bf16(pb)
    C = torch.full((260, 400), -7.0, dtype=torch.float32, device="cuda")
    for v in (0, 3, 10):
        ctx.gemm(A, B, C, M=M, N=N, K=K, mode=sg.MODE_VARIANT, variant=v)
        torch.cuda.synchronize()
        out = C.cpu().numpy().astype(np.float64)
        check_tol(out[:M, :N], pa[:M, :K], pb[:K, :N], F32)
        assert np.all(out[M:, :] == -7.0) and np.all(out[:, N:] == -7.0)


@pytest.mark.parametrize("variant", [0, 4, 8, 12, 13, 16, 20, 24, 27])
@pytest.mark.parametrize("case", ["a_only", "b_only", "both", "a_base", "b_ld"])
def test_packed_operands_integer_exact(ctx, variant, case):
    """Operands the direct-to-LDS kernel cannot read in place are copied zero-padded first;
    every combination (A only, B only, both, a misaligned base, a leading dimension that is
    not a multiple of 8) must stay exact on integer inputs, over several tiles and a ragged
    tail."""
    import torch
    M, N, K = {"a_only": (520, 392, 709), "b_only": (520, 389, 712), "both": (264, 331, 1003),
               "a_base": (300, 264, 520), "b_ld": (300, 264, 520)}[case]
    say("variant", variant, "case", case, M, N, K)
    A, B = inputs(90 + variant, M, N, K, "int")
    C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    if case == "a_base":      # A starts one element past a 16-byte boundary
        buf = torch.zeros(M * K + 8, dtype=torch.bfloat16, device="cuda")
        buf[1:1 + M * K] = sg.to_device_bf16(A).reshape(-1)
        dA, dB, lda, ldb = buf[1:1 + M * K].view(M, K), sg.to_device_bf16(B), K, N
    elif case == "b_ld":      # B rows 3 elements apart beyond N
        Bp = np.zeros((K, N + 3), dtype=B.dtype)
        Bp[:, :N] = B
        dA, dB, lda, ldb = sg.to_device_bf16(A), sg.to_device_bf16(Bp), K, N + 3
    else:
        dA, dB, lda, ldb = sg.to_device_bf16(A), sg.to_device_bf16(B), K, N
    ctx.gemm(dA, dB, C, M=M, N=N, K=K, lda=lda, ldb=ldb, mode=sg.MODE_VARIANT, variant=variant)
    torch.cuda.synchronize()
    check_exact(C.cpu().numpy().astype(np.float64), A, B, F32)


def test_errors_are_reported(ctx):
    import torch
    A = torch.zeros(8, 8, dtype=torch.bfloat16, device="cuda")
    C = torch.zeros(8, 8, dtype=torch.float32, device="cuda")
    with pytest.raises(sg.SGError) as e:
        ctx.gemm(A, A, C, mode=sg.MODE_DP)
    assert e.value.code == sg.SG_ENOTABLE
    with pytest.raises(sg.SGError) as e:
        ctx.gemm(A, A, C, M=-1)
    assert e.value.code == sg.SG_EINVAL
    with pytest.raises(sg.SGError):
        ctx.gemm(A, A, C, mode=sg.MODE_VARIANT, variant=99)
    with pytest.raises(sg.SGError):
        ctx.gemm(A, A, C, lda=4)


@pytest.mark.parametrize("kind", [0, 1])
def test_device_generator_matches_host(kind):
    import torch
    n = 1 << 20
    t = torch.empty(n, dtype=torch.bfloat16, device="cuda")
    sg.fill_bf16(t, 123, 4, offset=1000, kind=kind, scale=0.02 if kind else 1.0)
    torch.cuda.synchronize()
    got = sg.bf16_tensor_bits(t)
    if kind == 0:
        want = synth.f32_to_bf16_bits(synth.uniform_pm1_f32(123, 4, n, start=1000))
    else:
        want = synth.f32_to_bf16_bits(synth.normal_f32(123, 4, n, 0.02, start=1000))
    assert np.array_equal(got, want), int(np.count_nonzero(got != want))


@pytest.mark.parametrize("shape,c_dtype,variant", [((4096, 4096, 4096), BF16, 0),
                                                   ((3840, 2048, 4096), BF16, 3),
                                                   ((4096, 4096, 128), BF16, 0),
                                                   ((128, 4096, 4096), BF16, 9),
                                                   ((8192, 8192, 1024), BF16, 0)])
def test_full_size_sampled(ctx, shape, c_dtype, variant):
    """Largest sweep sizes: sampled entries against the oracle computed one by one."""
    import torch
    M, N, K = shape
    say("full size", shape, "variant", variant)
    A, B = inputs(2, M, N, K)
    out = run_gemm(ctx, A, B, c_dtype, mode=sg.MODE_VARIANT, variant=variant)
    rng = np.random.default_rng(0)
    rows = np.concatenate([rng.integers(0, M, 400), [0, M - 1, M - 1, 0]])
    cols = np.concatenate([rng.integers(0, N, 400), [0, N - 1, 0, N - 1]])
    c, d = oracle.gemm_entries(A, B, rows, cols, M=M, N=N, K=K)
    err, where, zv = oracle.scaled_err(out[rows, cols], c, d)
    assert zv == 0 and err <= TOL[c_dtype], err
    assert np.all(np.isfinite(out))
