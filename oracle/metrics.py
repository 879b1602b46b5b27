"""Landscape metrics -- oracle, test infrastructure only.

Definitions of the paper's Sec. 2.4 (measurement definitions) and Sec. 8.6 (3-D aggregate),
plus the ideal compute landscape of Sec. 9.1.
"""
from __future__ import annotations

import math

import numpy as np


def tflops(M, N, K, seconds):
    """Achieved throughput 2 M N K / (t 1e12)."""
    return 2.0 * np.asarray(M, dtype=np.float64) * N * K / (np.asarray(seconds, dtype=np.float64) * 1e12)


def roughness(values) -> float:
    """Mean absolute step-to-step change along one sweep axis: sum |T_{i+1} - T_i| / (n - 1)."""
    v = [float(x) for x in values]
    n = len(v)
    if n < 2:
        raise ValueError("roughness needs at least two points")
    return sum(abs(v[i + 1] - v[i]) for i in range(n - 1)) / (n - 1)


def roughness_along(T: np.ndarray, axis: int) -> float:
    """Roughness along `axis` of a landscape, averaged over every line parallel to that axis."""
    T = np.moveaxis(np.asarray(T, dtype=np.float64), axis, -1)
    lines = T.reshape(-1, T.shape[-1])
    return sum(roughness(line) for line in lines) / len(lines)


def slice_stats(tf_mn: np.ndarray):
    """Headline statistics of one fixed-K (M x N) slice: mean, peak, N-axis roughness."""
    tf_mn = np.asarray(tf_mn, dtype=np.float64)
    return {"mean": float(tf_mn.mean()), "peak": float(tf_mn.max()),
            "roughness_n": roughness_along(tf_mn, 1)}


def aggregate_3d(tf_mnk: np.ndarray):
    """3-D statistics: mean, peak and the mean of the N-, M- and K-axis roughness over all lines."""
    tf = np.asarray(tf_mnk, dtype=np.float64)
    rM = roughness_along(tf, 0)
    rN = roughness_along(tf, 1)
    rK = roughness_along(tf, 2)
    return {"mean": float(tf.mean()), "peak": float(tf.max()), "roughness_m": rM,
            "roughness_n": rN, "roughness_k": rK, "roughness_3d": (rM + rN + rK) / 3.0}


def ideal_tflops(M: int, N: int, peak: float, cores: int, tile: int) -> float:
    """Ideal compute landscape: peak * min(1, W / C) with W = ceil(M/T) ceil(N/T)."""
    W = math.ceil(M / tile) * math.ceil(N / tile)
    return peak * min(1.0, W / cores)


def tile_utilisation(N: int, tile: int) -> float:
    """Fraction of launched tile columns that hold data: N / (ceil(N/T) T)."""
    return N / (math.ceil(N / tile) * tile)
