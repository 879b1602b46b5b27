"""Landscape metrics -- oracle, test infrastructure only.

Definitions of the paper's Sec. 2 (its closing measurement definitions) and Sec. 8.5, Table 17 (3-D aggregate),
the four-surface decomposition of Sec. 4 (compute, memory, GEMM, overhead; Fig. 6, Table 3),
the ideal compute landscape and the first-principles optimal of Sec. 9, and the attainment /
roughness-ratio grading of Sec. 10 (Kernel Optimality Levels).
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


# Sec. 4: the four surfaces over one grid.  t_memory is measured (a kernel that moves the GEMM's
# operands and result with no matrix work), t_gemm is measured; the other two follow from them.
def compute_time(M: int, N: int, K: int, peak_tflops: float) -> float:
    """Compute surface (Sec. 4.1): the useful FLOP 2MNK at the dense peak; tile-independent."""
    return 2.0 * M * N * K / (peak_tflops * 1e12)


def overhead_time(t_gemm: float, t_compute: float, t_memory: float) -> float:
    """Overhead surface (Sec. 4.1): the GEMM time beyond the larger of compute and memory time."""
    return t_gemm - max(t_compute, t_memory)


def traffic_bytes(M: int, N: int, K: int, c_bytes: int = 2) -> float:
    """Bytes of a GEMM that reads A and B once (BF16) and writes C once (c_bytes per element)."""
    return 2.0 * M * K + 2.0 * K * N + float(c_bytes) * M * N


def decompose(shapes, t_gemm, t_memory, peak_tflops: float, bw_gbs: float, c_bytes: int = 2):
    """Sec. 4 over a list of (M, N, K) shapes with measured GEMM and memory times (seconds).

    Returns per-shape compute and overhead times and the summary:
      overhead_share -- mean over shapes of t_overhead / t_gemm (the stacked view of Fig. 6);
      cb_bandwidth   -- fraction of shapes compute-bound against bandwidth bw_gbs:
                        t_compute >= traffic_bytes / bw (Table 3, a bandwidth row);
      cb_measured    -- fraction with t_compute >= t_memory (against the measured memory time).
    """
    t_comp, t_over = [], []
    share = 0.0
    cb_bw = 0
    cb_meas = 0
    for (M, N, K), tg, tm in zip(shapes, t_gemm, t_memory):
        tc = compute_time(M, N, K, peak_tflops)
        to = overhead_time(tg, tc, tm)
        t_comp.append(tc)
        t_over.append(to)
        share += to / tg
        if tc >= traffic_bytes(M, N, K, c_bytes) / (bw_gbs * 1e9):
            cb_bw += 1
        if tc >= tm:
            cb_meas += 1
    n = len(t_comp)
    return {"t_compute": t_comp, "t_overhead": t_over, "overhead_share": share / n,
            "cb_bandwidth": cb_bw / n, "cb_measured": cb_meas / n}


def ideal_tflops(M: int, N: int, peak: float, cores: int, tile: int) -> float:
    """Ideal compute landscape: peak * min(1, W / C) with W = ceil(M/T) ceil(N/T)."""
    W = math.ceil(M / tile) * math.ceil(N / tile)
    return peak * min(1.0, W / cores)


def tile_utilisation(N: int, tile: int) -> float:
    """Fraction of launched tile columns that hold data: N / (ceil(N/T) T)."""
    return N / (math.ceil(N / tile) * tile)


def wave_efficiency(M: int, N: int, tile: int, cores: int) -> float:
    """Sec. 9.2, compute term: W = ceil(M/T) ceil(N/T) work-groups run in ceil(W/C) waves of C
    cores, so a fraction W / (ceil(W/C) C) of the launched core-slots does work."""
    W = math.ceil(M / tile) * math.ceil(N / tile)
    return W / (math.ceil(W / cores) * cores)


def channel_utilisation(L: int, elem_bytes: int, channels: int, interleave: int = 256,
                        tile_row: int = 256) -> float:
    """Sec. 9.2, memory term: the address space is striped over `channels` channels in blocks of
    `interleave` bytes, and a kernel moves rows of `tile_row` elements of a tensor whose
    leading dimension is L elements.  One such row spans w = min(channels, tile_row e /
    interleave) channels; consecutive rows start s = (L e / interleave) mod channels blocks
    apart, so their starts hit channels / gcd(s, channels) distinct channels; the fraction of
    channels the tensor keeps busy is min(channels, w channels / gcd(s, channels)) / channels."""
    w = min(channels, max(1, (tile_row * elem_bytes) // interleave))
    s = ((L * elem_bytes) // interleave) % channels
    return min(channels, w * channels // math.gcd(s, channels)) / channels


def optimal_tflops(M: int, N: int, K: int, peak: float, cores: int, bw_gbs: float,
                   tiles=(256, 128, 64), c_bytes: int = 2, channels: int = 0,
                   interleave: int = 256) -> float:
    """Sec. 9.2: t_opt = min over tiles T of max(t_compute(T), t_memory), with
    t_compute(T) = 2MNK / (peak wave_efficiency(T)) and t_memory = 2MK / (BW eta_A) +
    2KN / (BW eta_B) + c_bytes MN / (BW eta_D), the channel utilisations eta of A (leading
    dimension K), B and D (leading dimension N) from channel_utilisation; channels = 0 takes
    every eta as 1 (for a memory whose address-to-channel hash is not public).
    Returns 2MNK / t_opt in TFLOP/s (peak in TFLOP/s, BW in GB/s)."""
    flop = 2.0 * M * N * K
    if channels > 0:
        eta_a = channel_utilisation(K, 2, channels, interleave)
        eta_b = channel_utilisation(N, 2, channels, interleave)
        eta_d = channel_utilisation(N, c_bytes, channels, interleave)
    else:
        eta_a = eta_b = eta_d = 1.0
    t_mem = (2.0 * M * K / eta_a + 2.0 * K * N / eta_b + float(c_bytes) * M * N / eta_d) / (bw_gbs * 1e9)
    best = math.inf
    for T in tiles:
        t_comp = flop / (peak * 1e12 * wave_efficiency(M, N, T, cores))
        best = min(best, max(t_comp, t_mem))
    return flop / best / 1e12


# Sec. 10, Table 19: throughput bands by attainment tau, smoothness bands by roughness ratio rho.
def throughput_band(tau: float) -> int:
    if tau >= 0.95:
        return 3
    if tau >= 0.75:
        return 2
    if tau >= 0.50:
        return 1
    return 0


def smoothness_band(rho: float) -> int:
    if rho <= 1.25:
        return 3
    if rho <= 2.0:
        return 2
    if rho <= 3.0:
        return 1
    return 0


def kol_grade(actual: np.ndarray, optimal: np.ndarray):
    """Sec. 10.2-10.3 over a landscape (M x N or M x N x K array, N on axis 1):
    tau = mean(A) / mean(O); rho = R(A) / R(O) with R the N-axis roughness averaged over all
    lines; level = min(throughput band, smoothness band)."""
    A = np.asarray(actual, dtype=np.float64)
    O = np.asarray(optimal, dtype=np.float64)
    tau = float(A.mean() / O.mean())
    rho = float(roughness_along(A, 1) / roughness_along(O, 1))
    t, s_ = throughput_band(tau), smoothness_band(rho)
    return {"tau": tau, "rho": rho, "t_band": t, "s_band": s_, "level": min(t, s_)}
