"""Checks of a GEMM result against the FP64 definition at sizes where the plain oracle loop is
too slow to run on every entry -- TEST INFRASTRUCTURE ONLY.

The quantity checked is the paper's problem statement (Sec. 2.2 and Sec. 7.1): C = A B with A
(M x K) and B (K x N) row-major BF16, and the error measure max |C - C_ref| / (|A||B|)
elementwise.  Three forms:

* ``reference_block``: C_ref and D = |A||B| of a block of rows and columns, in FP64, with a
  library matrix product as the one step (BF16 x BF16 products are exact in FP64; only the
  order of the FP64 sum differs from the plain loop of ``oracle.c``, by at most K 2^-53 D);
* ``freivalds_rhs`` / ``freivalds_ratio``: Freivalds' randomized product check (R. Freivalds,
  1977): for random sign vectors x, compare C x with A (B x).  An elementwise error bounded by
  tol D gives |C x - A (B x)| <= tol |A| (|B| |x|) row by row, so a row whose ratio exceeds tol
  holds an error larger than the tolerance allows somewhere; the check costs O(MK + KN) instead
  of O(MNK) and catches gross faults (a missing or doubled K piece, a wrong tile, a transposed
  operand), not single entries just past the tolerance -- the sampled entries cover those;
* ``bf16_bits_to_f64``: the exact value of BF16 bit patterns.
"""
from __future__ import annotations

import numpy as np

# Rounding slack of the FP64 evaluations below, per unit of the bound they are compared with:
# each is a sum of at most K + N + 2 exact products, so its error is at most that many units of
# 2^-53 of the bound (a standard bound for recursive summation).
_U64 = 2.0 ** -53


def bf16_bits_to_f64(bits) -> np.ndarray:
    """BF16 bit patterns (uint16) -> their exact values in FP64."""
    b = np.ascontiguousarray(bits, dtype=np.uint16)
    with np.errstate(invalid="ignore"):          # NaN patterns stay NaN
        return (b.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def reference_block(A: np.ndarray, B: np.ndarray):
    """(C_ref, D) = (A B, |A| |B|) in FP64 for FP64 arrays holding BF16 values: A (r x K),
    B (K x c).  Any rows of A and columns of B may be passed: entry (i, j) of the result is the
    definition's entry for that row and column."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    return A @ B, np.abs(A) @ np.abs(B)


def entries_ratio(c, c_ref, d):
    """(max |c - c_ref| / d over entries with d > 0, count of entries with d == 0 and c != 0);
    the error measure of the problem statement at a set of entries."""
    c = np.asarray(c, dtype=np.float64)
    c_ref = np.asarray(c_ref, dtype=np.float64)
    d = np.asarray(d, dtype=np.float64)
    pos = d > 0
    err = float(np.max(np.abs(c[pos] - c_ref[pos]) / d[pos])) if pos.any() else 0.0
    return err, int(np.count_nonzero((~pos) & (c != 0)))


def sign_vectors(seed: int, n: int, r: int = 2) -> np.ndarray:
    """n x r matrix of independent +-1 entries (seeded)."""
    rng = np.random.default_rng(seed)
    return np.where(rng.integers(0, 2, size=(n, r)) == 1, 1.0, -1.0)


def freivalds_rhs(A: np.ndarray, B: np.ndarray, X: np.ndarray):
    """(A (B X), |A| (|B| |X|)) in FP64: the expected C X and the bound that an elementwise
    error of at most D gives it.  A (M x K), B (K x N), X (N x r)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    return A @ (B @ X), np.abs(A) @ (np.abs(B) @ np.abs(X))


def freivalds_ratio(CX, rhs, bound, K: int, N: int) -> float:
    """Largest |C X - A (B X)| / (|A| (|B| |X|)) over rows and vectors, after taking off the
    rounding slack of the FP64 evaluations ((K + N + 2) units of 2^-53 of the bound for each of
    the two sides).  Rows with a zero bound must match exactly (returns inf otherwise)."""
    CX = np.asarray(CX, dtype=np.float64)
    rhs = np.asarray(rhs, dtype=np.float64)
    bound = np.asarray(bound, dtype=np.float64)
    diff = np.abs(CX - rhs)
    pos = bound > 0
    if np.any(diff[~pos] != 0):
        return float("inf")
    if not pos.any():
        return 0.0
    slack = 2.0 * (K + N + 2) * _U64
    return float(max(0.0, np.max(diff[pos] / bound[pos]) - slack))
