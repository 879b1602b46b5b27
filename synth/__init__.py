"""Seeded synthetic operand generators (shared by the GPU path's harness and the oracle's tests).

This module holds no GEMM arithmetic.  It turns (seed, stream, element index) into
BF16 bit patterns, so that both sides of every parity check consume the very same bits.

Counter-based generator (SplitMix64, Steele, Lea and Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014; the output function as published by Vigna):

    mix(z)      = z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB; z ^ (z >> 31)
    out(s, i)   = mix(s + i * 0x9E3779B97F4A7C15)          (the i-th output, i >= 1, of SplitMix64 seeded with s)
    word(seed, stream, idx) = out(out(seed, stream + 1), idx + 1)      (all arithmetic mod 2^64)

uniform[-1, 1):  u = word >> 40 (24 bits);  f = (2u + 1 - 2^24) * 2^-24, exact in FP32, never 0 or +-1.
normal(0, std):  Box-Muller in FP64 on two 53-bit uniforms from words 2i and 2i+1, times std,
                 rounded to FP32 (round to nearest even), then to BF16.
BF16:            round-to-nearest-even of the FP32 value (inputs are finite and in range).

Both the host (this module) and the device fill kernel implement this same published definition.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_CHUNK = 1 << 22


def _mix(z: np.ndarray) -> np.ndarray:
    z = z ^ (z >> np.uint64(30))
    z = z * _M1
    z = z ^ (z >> np.uint64(27))
    z = z * _M2
    return z ^ (z >> np.uint64(31))


def stream_key(seed: int, stream: int) -> int:
    """Seed of the per-stream SplitMix64 sequence: output number stream+1 of SplitMix64(seed)."""
    with np.errstate(over="ignore"):
        s = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + np.uint64((stream + 1) & 0xFFFFFFFFFFFFFFFF) * GAMMA
        return int(_mix(np.array([s], dtype=np.uint64))[0])


def words(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """64-bit words number start .. start+count-1 of the stream (uint64 array)."""
    key = np.uint64(stream_key(seed, stream))
    idx = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(key + idx * GAMMA)


def uniform_pm1_f32(seed: int, stream: int, count: int, start: int = 0) -> np.ndarray:
    """FP32 values in (-1, 1), each exactly (2u+1-2^24)/2^24 for a 24-bit u."""
    out = np.empty(count, dtype=np.float32)
    for off in range(0, count, _CHUNK):
        n = min(_CHUNK, count - off)
        u = (words(seed, stream, start + off, n) >> np.uint64(40)).astype(np.int64)
        out[off:off + n] = ((2 * u + 1 - (1 << 24)).astype(np.float64) * 2.0 ** -24).astype(np.float32)
    return out


def normal_f32(seed: int, stream: int, count: int, std: float, start: int = 0) -> np.ndarray:
    """FP32 values std * N(0,1) by Box-Muller (cosine branch) in FP64, one pair of words per value."""
    out = np.empty(count, dtype=np.float32)
    for off in range(0, count, _CHUNK):
        n = min(_CHUNK, count - off)
        w = words(seed, stream, 2 * (start + off), 2 * n)
        u1 = ((w[0::2] >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
        u2 = ((w[1::2] >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0 ** -53
        z = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
        out[off:off + n] = (z * std).astype(np.float32)
    return out


def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    """Round finite FP32 values to BF16 (nearest, ties to even); returns uint16 bit patterns."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    return ((b + np.uint64(0x7FFF) + lsb) >> np.uint64(16)).astype(np.uint16)


def bf16_bits_to_f32(h: np.ndarray) -> np.ndarray:
    """Exact widening of BF16 bit patterns to FP32."""
    return (np.asarray(h, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


def uniform_bf16(seed: int, stream: int, rows: int, cols: int) -> np.ndarray:
    """rows x cols row-major BF16 bit patterns drawn uniform[-1,1] then rounded to BF16."""
    return f32_to_bf16_bits(uniform_pm1_f32(seed, stream, rows * cols)).reshape(rows, cols)


def normal_bf16(seed: int, stream: int, rows: int, cols: int, std: float = 0.02) -> np.ndarray:
    return f32_to_bf16_bits(normal_f32(seed, stream, rows * cols, std)).reshape(rows, cols)


def integer_bf16(seed: int, stream: int, rows: int, cols: int, lo: int = -4, hi: int = 4) -> np.ndarray:
    """Integers uniform in [lo, hi] (exact in BF16), drawn from the same counter generator."""
    w = words(seed, stream, 0, rows * cols)
    span = np.uint64(hi - lo + 1)
    v = (w % span).astype(np.int64) + lo
    return f32_to_bf16_bits(v.astype(np.float32)).reshape(rows, cols)


# Stream numbers used across the workloads: operand A and operand B of a problem.
STREAM_A = 0
STREAM_B = 1
