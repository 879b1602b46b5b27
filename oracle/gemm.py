"""ctypes wrapper around the plain FP64 oracle GEMM in ``oracle.c`` (test infrastructure only).

Definition (paper, Sec. 2.2 and Sec. 7.1): C = A B with A (M x K) and B (K x N) row-major BF16.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i64 = ctypes.c_int64
_p = ctypes.c_void_p


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-ffp-contract=off",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build_oracle(force=True)
        L = ctypes.CDLL(_LIB)
        L.oracle_bf16_to_f64.restype = ctypes.c_double
        L.oracle_bf16_to_f64.argtypes = [ctypes.c_uint16]
        L.oracle_f64_to_bf16_rne.restype = ctypes.c_uint16
        L.oracle_f64_to_bf16_rne.argtypes = [ctypes.c_double]
        L.oracle_gemm_f64.restype = None
        L.oracle_gemm_f64.argtypes = [_i64, _i64, _i64, _p, _i64, _p, _i64, _p, _i64, _p, _i64]
        L.oracle_gemm_entries.restype = None
        L.oracle_gemm_entries.argtypes = [_i64, _i64, _i64, _p, _i64, _p, _i64, _i64, _p, _p, _p, _p]
        L.oracle_scaled_err.restype = ctypes.c_double
        L.oracle_scaled_err.argtypes = [_i64, _p, _p, _p, _p, _p]
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def bf16_to_f64(h: int) -> float:
    return lib().oracle_bf16_to_f64(int(h))


def f64_to_bf16_rne(x) -> np.ndarray:
    """Element-wise FP64 -> BF16 bit patterns (round to nearest even)."""
    x = np.asarray(x, dtype=np.float64)
    f = lib().oracle_f64_to_bf16_rne
    return np.array([f(float(v)) for v in x.ravel()], dtype=np.uint16).reshape(x.shape)


def gemm_f64(A: np.ndarray, B: np.ndarray, want_d: bool = True):
    """Full C_ref (FP64) and normaliser D for row-major BF16 bit arrays A (M x K), B (K x N)."""
    A = np.ascontiguousarray(A, dtype=np.uint16)
    B = np.ascontiguousarray(B, dtype=np.uint16)
    M, K = A.shape
    K2, N = B.shape
    assert K == K2
    C = np.zeros((M, N), dtype=np.float64)
    D = np.zeros((M, N), dtype=np.float64) if want_d else None
    lib().oracle_gemm_f64(M, N, K, _ptr(A), K, _ptr(B), N, _ptr(C), N,
                          _ptr(D) if want_d else None, N)
    return (C, D) if want_d else C


def gemm_entries(A: np.ndarray, B: np.ndarray, rows, cols, M=None, N=None, K=None,
                 lda=None, ldb=None):
    """C_ref and D at the entries (rows[t], cols[t]).  A and B may be larger pools viewed
    with leading dimensions lda/ldb (defaults: the arrays' own widths)."""
    A = np.ascontiguousarray(A, dtype=np.uint16)
    B = np.ascontiguousarray(B, dtype=np.uint16)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int64)
    if K is None:
        K = A.shape[1] if A.ndim == 2 else None
    lda = lda if lda is not None else (A.shape[1] if A.ndim == 2 else K)
    ldb = ldb if ldb is not None else (B.shape[1] if B.ndim == 2 else N)
    n = rows.size
    c = np.zeros(n, dtype=np.float64)
    d = np.zeros(n, dtype=np.float64)
    lib().oracle_gemm_entries(M or 0, N or 0, K, _ptr(A), lda, _ptr(B), ldb, n, _ptr(rows),
                              _ptr(cols), _ptr(c), _ptr(d))
    return c, d


def scaled_err(c_gpu, c_ref, d):
    """(max |C_gpu - C_ref| / D, argmax flat index, count of D == 0 entries where C_gpu != 0)."""
    cg = np.ascontiguousarray(c_gpu, dtype=np.float64).ravel()
    cr = np.ascontiguousarray(c_ref, dtype=np.float64).ravel()
    dd = np.ascontiguousarray(d, dtype=np.float64).ravel()
    am = ctypes.c_int64(0)
    zv = ctypes.c_int64(0)
    e = lib().oracle_scaled_err(cg.size, _ptr(cg), _ptr(cr), _ptr(dd), ctypes.byref(am),
                                ctypes.byref(zv))
    return e, am.value, zv.value
