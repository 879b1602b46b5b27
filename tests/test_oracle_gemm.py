"""The FP64 oracle GEMM, pinned to exact rational arithmetic and to closed forms (CPU only)."""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def _frac_gemm(A, B):
    a = [[Fraction(float(x)) for x in row] for row in synth.bf16_bits_to_f32(A)]
    b = [[Fraction(float(x)) for x in row] for row in synth.bf16_bits_to_f32(B)]
    M, K, N = len(a), len(b), len(b[0])
    C = [[sum(a[i][k] * b[k][j] for k in range(K)) for j in range(N)] for i in range(M)]
    D = [[sum(abs(a[i][k]) * abs(b[k][j]) for k in range(K)) for j in range(N)] for i in range(M)]
    return C, D


@pytest.mark.parametrize("M,N,K", list(itertools.product([1, 2, 3, 5], [1, 2, 4, 6], [1, 3, 4, 6])))
def test_exact_rational_small(M, N, K):
    A = synth.uniform_bf16(M * 100 + N, 0, M, K)
    B = synth.uniform_bf16(M * 100 + N, 1, K, N)
    C, D = oracle.gemm_f64(A, B)
    Cf, Df = _frac_gemm(A, B)
    for i in range(M):
        for j in range(N):
            assert abs(Fraction(C[i, j]) - Cf[i][j]) <= Fraction(1, 10 ** 15) * Df[i][j]
            assert abs(Fraction(D[i, j]) - Df[i][j]) <= Fraction(1, 10 ** 15) * Df[i][j]


def test_exact_rational_random_16():
    rng = np.random.default_rng(1)
    for t in range(6):
        M, N, K = rng.integers(1, 17, 3)
        A = synth.uniform_bf16(t, 0, M, K)
        B = synth.uniform_bf16(t, 1, K, N)
        C, D = oracle.gemm_f64(A, B)
        Cf, Df = _frac_gemm(A, B)
        for i in range(M):
            for j in range(N):
                assert abs(Fraction(C[i, j]) - Cf[i][j]) <= Fraction(1, 10 ** 15) * Df[i][j]


def _bf16(v):
    return synth.f32_to_bf16_bits(np.asarray(v, dtype=np.float32))


def test_identity_gives_b():
    K, N = 37, 29
    B = synth.uniform_bf16(4, 1, K, N)
    C, D = oracle.gemm_f64(_bf16(np.eye(K)), B)
    assert np.array_equal(C, synth.bf16_bits_to_f32(B).astype(np.float64))
    assert np.array_equal(D, np.abs(synth.bf16_bits_to_f32(B)).astype(np.float64))


def test_permutation_permutes_rows():
    K, N = 23, 11
    perm = np.random.default_rng(2).permutation(K)
    P = np.zeros((K, K), dtype=np.float32)
    P[np.arange(K), perm] = 1.0
    B = synth.uniform_bf16(5, 1, K, N)
    C, _ = oracle.gemm_f64(_bf16(P), B)
    assert np.array_equal(C, synth.bf16_bits_to_f32(B)[perm].astype(np.float64))


def test_transpose_is_caught_by_rectangular_permutation():
    # a plausible bug (reading B transposed) would change the result of this non-square case
    A = _bf16(np.arange(6, dtype=np.float32).reshape(2, 3))
    B = _bf16(np.arange(12, dtype=np.float32).reshape(3, 4))
    C, _ = oracle.gemm_f64(A, B)
    expect = np.array([[20, 23, 26, 29], [56, 68, 80, 92]], dtype=np.float64)
    assert np.array_equal(C, expect)


@pytest.mark.parametrize("K", [1, 2, 8, 64, 256])
def test_rank_one_power_of_two(K):
    # u_i v_j with few-bit values, repeated over k: C_ij = K u_i v_j exactly
    u = np.array([1.5, -0.75, 2.0, 0.5, -3.0], dtype=np.float32)
    v = np.array([0.25, -1.25, 1.0, 6.0], dtype=np.float32)
    A = _bf16(np.repeat(u[:, None], K, axis=1))
    B = _bf16(np.repeat(v[None, :], K, axis=0))
    C, D = oracle.gemm_f64(A, B)
    assert np.array_equal(C, K * np.outer(u, v).astype(np.float64))
    assert np.array_equal(D, K * np.abs(np.outer(u, v)).astype(np.float64))


def test_integer_inputs_exact():
    A = synth.integer_bf16(9, 0, 20, 300)
    B = synth.integer_bf16(9, 1, 300, 15)
    C, D = oracle.gemm_f64(A, B)
    a = synth.bf16_bits_to_f32(A).astype(np.int64)
    b = synth.bf16_bits_to_f32(B).astype(np.int64)
    assert np.array_equal(C, (a @ b).astype(np.float64))
    assert np.array_equal(D, (np.abs(a) @ np.abs(b)).astype(np.float64))


def test_leading_dimensions_and_entries():
    pool_a = synth.uniform_bf16(11, 0, 64, 64)
    pool_b = synth.uniform_bf16(11, 1, 64, 64)
    M, N, K = 7, 9, 13
    A = pool_a.ravel()[:M * K].reshape(M, K)      # contiguous view of the pool, lda = K
    B = pool_b.ravel()[:K * N].reshape(K, N)
    C, D = oracle.gemm_f64(A, B)
    rows = np.array([0, 6, 3, 6])
    cols = np.array([0, 8, 4, 0])
    c, d = oracle.gemm_entries(pool_a.ravel(), pool_b.ravel(), rows, cols, M=M, N=N, K=K, lda=K, ldb=N)
    assert np.array_equal(c, C[rows, cols]) and np.array_equal(d, D[rows, cols])


def test_zero_row_gives_zero_normaliser():
    A = synth.uniform_bf16(1, 0, 4, 8)
    A[2] = 0
    B = synth.uniform_bf16(1, 1, 8, 5)
    C, D = oracle.gemm_f64(A, B)
    assert np.all(C[2] == 0) and np.all(D[2] == 0)
    bad = C.copy()
    bad[2, 1] = 1e-30
    e, _, zv = oracle.scaled_err(bad, C, D)
    assert zv == 1 and e == 0.0
    e, _, zv = oracle.scaled_err(C, C, D)
    assert zv == 0 and e == 0.0


def test_scaled_err_detects_error():
    A = synth.uniform_bf16(2, 0, 8, 8)
    B = synth.uniform_bf16(2, 1, 8, 8)
    C, D = oracle.gemm_f64(A, B)
    pert = C.copy()
    pert[3, 4] += 1e-3 * D[3, 4]
    e, am, _ = oracle.scaled_err(pert, C, D)
    assert am == 3 * 8 + 4 and abs(e - 1e-3) < 1e-12


def test_f64_to_bf16_rne_cases():
    one = 1.0
    cases = {one: 0x3F80, one + 2 ** -8: 0x3F80, one + 3 * 2 ** -8: 0x3F82, -2.5: 0xC020,
             0.0: 0x0000, 2 ** -130: None, 3.0e38: 0x7F62, 1 + 2 ** -8 + 2 ** -30: 0x3F81}
    for x, want in cases.items():
        got = int(oracle.f64_to_bf16_rne([x])[0])
        if want is None:       # subnormal: must round-trip to the nearest multiple of 2^-133
            v = float(synth.bf16_bits_to_f32(np.array([got], dtype=np.uint16))[0])
            assert abs(v - x) <= 2 ** -134
        else:
            assert got == want, (x, hex(got))


def test_f64_to_bf16_agrees_with_generator_rounding_on_fp32_values():
    # for FP32-representable values the two independent RNE implementations must agree
    x = synth.uniform_pm1_f32(13, 0, 3000) * np.float32(37.0)
    assert np.array_equal(oracle.f64_to_bf16_rne(x.astype(np.float64)), synth.f32_to_bf16_bits(x))
