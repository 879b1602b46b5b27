"""Exhaustive optimum over pad/split plan trees -- pins the T1/T2 recurrences (test only).

A plan for a problem of size s (grid units) is a tree: a leaf runs the GEMM of any grid cell
s' >= s (component-wise: padding, paper Sec. 7 "padding-up"), an inner node first pads to some
s' >= s and then cuts s' into two pieces along one axis at a grid point (paper Sec. 7.1, the
three split kinds), each piece solved by a plan of its own.  Cost = sum of leaf times (the
pieces run one after the other).  This module minimises over ALL such trees of depth <= d by
plain recursion, increasing d until the value stops changing.  It shares no step with the
recurrences it checks (it pads anywhere, including before splitting, and splits anywhere).
"""
from __future__ import annotations

import functools
import itertools

import numpy as np


def best_over_trees(T0: np.ndarray, max_depth: int = 64) -> np.ndarray:
    T0 = np.asarray(T0, dtype=np.float64)
    dims = T0.shape

    def cone(s):
        return itertools.product(*[range(s[a], dims[a]) for a in range(3)])

    @functools.lru_cache(maxsize=None)
    def E(s, d):
        best = np.inf
        for sp in cone(s):
            best = min(best, T0[sp])
            if d == 0:
                continue
            for axis in range(3):
                size = sp[axis] + 1
                for first in range(1, size):
                    a = list(sp)
                    b = list(sp)
                    a[axis] = first - 1
                    b[axis] = size - first - 1
                    best = min(best, E(tuple(a), d - 1) + E(tuple(b), d - 1))
        return best

    prev = None
    for d in range(max_depth + 1):
        cur = np.array([E(s, d) for s in itertools.product(*[range(n) for n in dims])]).reshape(dims)
        if prev is not None and np.array_equal(cur, prev):
            return cur
        prev = cur
    return prev


def pad_cone_min(T0: np.ndarray) -> np.ndarray:
    """Closed form of padding alone: min of T0 over every cell s' >= s."""
    T0 = np.asarray(T0, dtype=np.float64)
    out = np.empty_like(T0)
    for s in itertools.product(*[range(n) for n in T0.shape]):
        out[s] = T0[s[0]:, s[1]:, s[2]:].min()
    return out
