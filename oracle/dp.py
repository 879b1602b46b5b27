"""Padding (T1) and split-plus-padding (T2) tables -- oracle, test infrastructure only.

Follows the paper's Sec. 7.1 ("The T0 -> T1 -> T2 Algorithm") in its own order and notation.
Tables are 3-D arrays over a uniform grid with step g; index i on an axis stands for size
(i + 1) * g.  All arithmetic is on the numbers of T0 alone (no GPU, no timing).

Readings where the text is silent or garbled (listed with the design notes):
* indices in the recurrences are grid-index units; splits happen only at grid multiples;
* each split term shrinks exactly one dimension (the verbatim formula of Step 3);
* no padding beyond the largest grid size (top-edge cells can only split or stay);
* ties: candidates are visited in formula order (as-is, pads in lexicographic (i,j,k), splits
  along M by ascending point, then N, then K) and a candidate replaces the incumbent only when
  strictly smaller.

Plan records use the action codes below; ``arg`` is the pad target (flat cell index) or the
split point in grid units (the first piece has size arg, the second the rest).
"""
from __future__ import annotations

import numpy as np

AS_IS, PAD, SPLIT_M, SPLIT_N, SPLIT_K = 0, 1, 2, 3, 4


def t1_pad(T0: np.ndarray):
    """Step 2: T1[M][N][K] = min over (i,j,k) in {0,1}^3 of T1[M+i][N+j][K+k], visited from the
    largest sizes down ("bottom right to top left"), T1 initialised as T0.

    Returns (T1, target) where target[s] is the flat index of the cell whose T0 realises T1[s]."""
    T0 = np.asarray(T0, dtype=np.float64)
    nM, nN, nK = T0.shape
    T1 = T0.copy()
    target = np.arange(T0.size, dtype=np.int64).reshape(T0.shape)
    for m in range(nM - 1, -1, -1):
        for n in range(nN - 1, -1, -1):
            for k in range(nK - 1, -1, -1):
                best = T1[m, n, k]
                tgt = target[m, n, k]
                for i in (0, 1):
                    for j in (0, 1):
                        for kk in (0, 1):
                            if i == j == kk == 0:
                                continue
                            a, b, c = m + i, n + j, k + kk
                            if a >= nM or b >= nN or c >= nK:
                                continue
                            if T1[a, b, c] < best:
                                best = T1[a, b, c]
                                tgt = target[a, b, c]
                T1[m, n, k] = best
                target[m, n, k] = tgt
    return T1, target


def t2_split_pad(T1: np.ndarray, target: np.ndarray):
    """Step 3: T2 starts as T1 and is visited from the smallest sizes up ("top left to bottom
    right"); each cell may be replaced by the cheapest split into two pieces along one axis:

        T2[M][N][K] = min(T2[M][N][K], T2[M-i][N][K] + T2[i][N][K],
                          T2[M][N-j][K] + T2[M][j][K], T2[M][N][K-k] + T2[M][N][k])

    Returns (T2, action, arg) with the plan record of every cell."""
    T1 = np.asarray(T1, dtype=np.float64)
    nM, nN, nK = T1.shape
    T2 = T1.copy()
    flat = np.arange(T1.size, dtype=np.int64).reshape(T1.shape)
    action = np.where(target == flat, AS_IS, PAD).astype(np.int64)
    arg = np.where(target == flat, 0, target).astype(np.int64)
    for m in range(nM):
        for n in range(nN):
            for k in range(nK):
                best = T2[m, n, k]
                act, ar = action[m, n, k], arg[m, n, k]
                sm, sn, sk = m + 1, n + 1, k + 1          # sizes in grid units
                for i in range(1, sm):                     # pieces of sizes i and sm - i
                    c = T2[sm - i - 1, n, k] + T2[i - 1, n, k]
                    if c < best:
                        best, act, ar = c, SPLIT_M, i
                for j in range(1, sn):
                    c = T2[m, sn - j - 1, k] + T2[m, j - 1, k]
                    if c < best:
                        best, act, ar = c, SPLIT_N, j
                for kk in range(1, sk):
                    c = T2[m, n, sk - kk - 1] + T2[m, n, kk - 1]
                    if c < best:
                        best, act, ar = c, SPLIT_K, kk
                T2[m, n, k] = best
                action[m, n, k] = act
                arg[m, n, k] = ar
    return T2, action, arg


def tables(T0: np.ndarray):
    """T0 -> (T1, T2, action, arg)."""
    T1, target = t1_pad(T0)
    T2, action, arg = t2_split_pad(T1, target)
    return T1, T2, action, arg


def plan_leaves(shape_cells, action, arg, cell):
    """Expand the plan of cell (grid indices) into leaves.

    Each leaf is (m0, n0, k0, m, n, k, run_cell): the sub-problem rows [m0, m0+m), columns
    [n0, n0+n), depth [k0, k0+k) in grid units, executed as the GEMM of grid cell run_cell
    (equal to the sub-problem's own cell unless padded).  Leaves are listed in execution order;
    along K the first leaf of a region writes, later ones accumulate."""
    nM, nN, nK = shape_cells
    out = []

    def rec(m0, n0, k0, m, n, k):
        idx = (m - 1, n - 1, k - 1)
        a = int(action[idx])
        r = int(arg[idx])
        if a == AS_IS:
            out.append((m0, n0, k0, m, n, k, idx))
        elif a == PAD:
            out.append((m0, n0, k0, m, n, k, tuple(int(v) for v in np.unravel_index(r, (nM, nN, nK)))))
        elif a == SPLIT_M:
            rec(m0, n0, k0, r, n, k)
            rec(m0 + r, n0, k0, m - r, n, k)
        elif a == SPLIT_N:
            rec(m0, n0, k0, m, r, k)
            rec(m0, n0 + r, k0, m, n - r, k)
        elif a == SPLIT_K:
            rec(m0, n0, k0, m, n, r)
            rec(m0, n0, k0 + r, m, n, k - r)
        else:
            raise ValueError("bad action %d" % a)

    rec(0, 0, 0, cell[0] + 1, cell[1] + 1, cell[2] + 1)
    return out
