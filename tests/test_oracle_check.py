"""Pins of the oracle's fast checks (oracle/check.py) against the plain FP64 loop of oracle.c,
exact arithmetic and planted faults.  CPU only."""
import numpy as np
import pytest

import oracle
import synth
from oracle import check


def _bits(seed, M, N, K, kind="uniform"):
    if kind == "int":
        return synth.integer_bf16(seed, synth.STREAM_A, M, K), synth.integer_bf16(seed, synth.STREAM_B, K, N)
    return synth.uniform_bf16(seed, synth.STREAM_A, M, K), synth.uniform_bf16(seed, synth.STREAM_B, K, N)


def test_bf16_values_match_the_plain_oracle_on_every_pattern():
    bits = np.arange(1 << 16, dtype=np.uint32).astype(np.uint16)
    got = check.bf16_bits_to_f64(bits)
    want = np.array([oracle.bf16_to_f64(int(b)) for b in bits])
    nan = np.isnan(want)
    assert np.array_equal(np.isnan(got), nan)
    assert np.array_equal(got[~nan], want[~nan])


@pytest.mark.parametrize("M,N,K", [(1, 1, 1), (7, 5, 3), (33, 17, 65), (64, 48, 200)])
def test_reference_block_equals_plain_loop_on_integers(M, N, K):
    # integer inputs: every partial sum is an exact integer in FP64, so any summation order
    # gives the plain loop's result bit for bit
    A, B = _bits(M * 7 + N, M, N, K, "int")
    C, D = check.reference_block(check.bf16_bits_to_f64(A), check.bf16_bits_to_f64(B))
    Cp, Dp = oracle.gemm_f64(A, B)
    assert np.array_equal(C, Cp) and np.array_equal(D, Dp)


def test_reference_block_within_summation_bound_on_random_inputs():
    M, N, K = 40, 30, 777
    A, B = _bits(5, M, N, K)
    C, D = check.reference_block(check.bf16_bits_to_f64(A), check.bf16_bits_to_f64(B))
    Cp, Dp = oracle.gemm_f64(A, B)
    assert np.all(np.abs(C - Cp) <= 2 * K * 2.0 ** -53 * Dp)
    assert np.allclose(D, Dp, rtol=2 * K * 2.0 ** -53, atol=0)


def test_reference_block_of_row_and_column_subsets():
    M, N, K = 50, 40, 96
    A, B = _bits(6, M, N, K)
    Af, Bf = check.bf16_bits_to_f64(A), check.bf16_bits_to_f64(B)
    rows = np.array([49, 0, 17, 17, 3])
    cols = np.array([5, 39, 0, 22])
    C, D = check.reference_block(Af[rows], Bf[:, cols])
    Cp, Dp = oracle.gemm_entries(A, B, np.repeat(rows, cols.size), np.tile(cols, rows.size), M=M, N=N, K=K)
    assert np.allclose(C.ravel(), Cp, rtol=0, atol=1e-12)
    assert np.allclose(D.ravel(), Dp, rtol=1e-14, atol=0)


def test_identity_closed_form():
    n = 24
    I = np.eye(n)
    B = check.bf16_bits_to_f64(synth.uniform_bf16(7, synth.STREAM_B, n, 9))
    C, D = check.reference_block(I, B)
    assert np.array_equal(C, B) and np.array_equal(D, np.abs(B))


def test_entries_ratio_recovers_a_planted_error():
    c_ref = np.array([1.0, -2.0, 3.0, 0.0])
    d = np.array([2.0, 4.0, 3.0, 0.0])
    c = c_ref.copy()
    c[1] += 0.01 * 4.0
    err, zv = check.entries_ratio(c, c_ref, d)
    assert err == pytest.approx(0.01) and zv == 0
    c[3] = 1e-30
    assert check.entries_ratio(c, c_ref, d)[1] == 1


def test_sign_vectors():
    X = check.sign_vectors(3, 1000, 2)
    assert X.shape == (1000, 2) and set(np.unique(X)) == {-1.0, 1.0}
    assert np.array_equal(X, check.sign_vectors(3, 1000, 2))
    assert abs(X.mean()) < 0.1


def _freivalds(Cg, Af, Bf, X):
    rhs, bound = check.freivalds_rhs(Af, Bf, X)
    return check.freivalds_ratio(Cg @ X, rhs, bound, Af.shape[1], Bf.shape[1])


def test_freivalds_passes_correct_and_tolerated_results():
    M, N, K = 70, 90, 300
    A, B = _bits(8, M, N, K)
    Af, Bf = check.bf16_bits_to_f64(A), check.bf16_bits_to_f64(B)
    Cp, D = oracle.gemm_f64(A, B)
    X = check.sign_vectors(9, N)
    assert _freivalds(Cp, Af, Bf, X) <= 1e-13
    # an elementwise error of 0.9 tol D, of any signs, stays within tol on every row
    rng = np.random.default_rng(10)
    Ce = Cp + 0.9 * 8e-3 * D * rng.choice([-1.0, 1.0], size=D.shape)
    assert _freivalds(Ce, Af, Bf, X) <= 8e-3


@pytest.mark.parametrize("fault", ["missing_k_piece", "doubled_k_piece", "zero_tile", "transposed_b", "row_shift"])
def test_freivalds_catches_planted_faults(fault):
    n, K = 96, 256
    A, B = _bits(11, n, n, K)
    Af, Bf = check.bf16_bits_to_f64(A), check.bf16_bits_to_f64(B)
    C = oracle.gemm_f64(A, B, want_d=False)
    if fault == "missing_k_piece":
        C = Af[:, 64:] @ Bf[64:, :]
    elif fault == "doubled_k_piece":
        C = C + Af[:, :64] @ Bf[:64, :]
    elif fault == "zero_tile":
        C = C.copy()
        C[32:64, 32:64] = 0.0
    elif fault == "transposed_b":
        Bt = check.bf16_bits_to_f64(synth.uniform_bf16(11, synth.STREAM_B, n, K)).T   # K x n, other layout
        C = Af @ Bt
    elif fault == "row_shift":
        C = np.roll(C, 1, axis=0)
    X = check.sign_vectors(12, n)
    assert _freivalds(C, Af, Bf, X) > 8e-3, fault
