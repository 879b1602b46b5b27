"""smoothgemm for MI355X: Python binding of the C-ABI library ``libsmoothgemm.so``.

Argument marshalling only: every step of the GEMM path runs in the library's HIP kernels and
host runtime.  PyTorch supplies device memory (tensor storage) and streams.  There is no CPU
fallback: if the library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmoothgemm.so")

SG_OK, SG_EINVAL, SG_ENOMEM, SG_ENOTABLE, SG_EMISMATCH, SG_EHIP, SG_ERANGE, SG_EIO, SG_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
F32, BF16 = 0, 1
MODE_DEFAULT, MODE_PLAIN, MODE_BEST, MODE_DP, MODE_VARIANT = 0, 1, 2, 3, 4
ACT_AS_IS, ACT_PAD, ACT_SPLIT_M, ACT_SPLIT_N, ACT_SPLIT_K = 0, 1, 2, 3, 4

_i64 = ctypes.c_int64
_i32 = ctypes.c_int
_p = ctypes.c_void_p
_d = ctypes.c_double


class SGError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("smoothgemm error %d: %s" % (code, msg))
        self.code = code


class sg_gemm_args(ctypes.Structure):
    _fields_ = [("M", _i64), ("N", _i64), ("K", _i64), ("A", _p), ("lda", _i64), ("B", _p),
                ("ldb", _i64), ("C", _p), ("ldc", _i64), ("c_dtype", _i32), ("beta", _i32),
                ("mode", _i32), ("variant", _i32)]


class sg_variant_info(ctypes.Structure):
    _fields_ = [("id", _i32), ("bm", _i32), ("bn", _i32), ("bk", _i32), ("splits", _i32),
                ("threads", _i32), ("lds_bytes", _i32), ("name", ctypes.c_char * 48)]


class sg_stats(ctypes.Structure):
    _fields_ = [("mean", _d), ("peak", _d), ("rough_m", _d), ("rough_n", _d), ("rough_k", _d),
                ("rough_3d", _d)]


class sg_shape(ctypes.Structure):
    _fields_ = [("M", _i64), ("N", _i64), ("K", _i64)]


class sg_grid(ctypes.Structure):
    _fields_ = [("step", _i32), ("n_m", _i32), ("n_n", _i32), ("n_k", _i32)]


class sg_plan_rec(ctypes.Structure):
    _fields_ = [("action", _i32), ("arg", _i32), ("variant", _i32), ("t0", _d), ("t1", _d), ("t2", _d)]


_SIGS = {
    "sg_last_error": (ctypes.c_char_p, []),
    "sg_version": (ctypes.c_char_p, []),
    "sg_ctx_create": (_i32, [_i32, ctypes.POINTER(_p)]),
    "sg_ctx_destroy": (_i32, [_p]),
    "sg_ctx_set_plain_variant": (_i32, [_p, _i32]),
    "sg_ctx_reserve_workspace": (_i32, [_p, ctypes.c_size_t]),
    "sg_ctx_set_table": (_i32, [_p, _p]),
    "gemm_bf16_nn": (_i32, [_i64, _i64, _i64, _p, _p, _p]),
    "gemm_bf16_nn_ex": (_i32, [_p, ctypes.POINTER(sg_gemm_args), _p]),
    "sg_num_variants": (_i32, []),
    "sg_variant_info_get": (_i32, [_i32, ctypes.POINTER(sg_variant_info)]),
    "sg_roughness": (_d, [_p, _i64]),
    "sg_landscape_stats": (_i32, [_p, _i32, _i32, _i32, ctypes.POINTER(sg_stats)]),
    "sg_sweep": (_i32, [_p, _p, _i64, _i32, _i32, _i32, _i32, _i32, _p, _p, _p, _p, _p]),
    "sg_sweep_kernel_times": (_i32, [_p, _p, _p, _p]),
    "sg_table_from_t0": (_i32, [ctypes.POINTER(sg_grid), _p, _p, _i32, ctypes.POINTER(_p)]),
    "sg_table_build": (_i32, [_p, ctypes.POINTER(sg_grid), _p, _i32, _i32, _i32, _i32,
                              ctypes.c_uint64, _p, _p, _p, _p, ctypes.POINTER(_p)]),
    "sg_table_free": (_i32, [_p]),
    "sg_table_grid": (_i32, [_p, ctypes.POINTER(sg_grid)]),
    "sg_table_lookup": (_i32, [_p, _i64, _i64, _i64, ctypes.POINTER(sg_plan_rec)]),
    "sg_table_values": (_i32, [_p, _i32, _p, _i64]),
    "sg_table_variants": (_i32, [_p, _p, _i32, ctypes.POINTER(_i32)]),
    "sg_table_plan_leaves": (_i32, [_p, _i64, _i64, _i64, ctypes.POINTER(_i32)]),
    "sg_table_save": (_i32, [_p, ctypes.c_char_p]),
    "sg_table_load": (_i32, [ctypes.c_char_p, _i32, ctypes.POINTER(_p)]),
    "sg_fill_bf16": (_i32, [_p, _i64, ctypes.c_uint64, ctypes.c_uint64, _i64, _i32, _d, _p]),
}

_lib = None


def lib():
    """The loaded C library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsmoothgemm.so is not built (run __graft_entry__.build() or "
                              "python -m paper_2605_29752_amd.build); there is no fallback")
        # torch ships its own HIP runtime with the same soname (libamdhip64.so.7); loading torch
        # first makes this library bind to that one instance instead of a second runtime.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def declared_symbols() -> Sequence[str]:
    return list(_SIGS)


def check(rc: int) -> int:
    if rc != SG_OK:
        raise SGError(rc, lib().sg_last_error().decode(errors="replace"))
    return rc


def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _arr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class VariantInfo:
    id: int
    bm: int
    bn: int
    bk: int
    splits: int
    threads: int
    lds_bytes: int
    name: str


def num_variants() -> int:
    return lib().sg_num_variants()


def variant_info(v: int) -> VariantInfo:
    vi = sg_variant_info()
    check(lib().sg_variant_info_get(v, ctypes.byref(vi)))
    return VariantInfo(vi.id, vi.bm, vi.bn, vi.bk, vi.splits, vi.threads, vi.lds_bytes,
                       vi.name.decode())


def roughness(values) -> float:
    a = np.ascontiguousarray(values, dtype=np.float64)
    return lib().sg_roughness(_arr(a), a.size)


def landscape_stats(tflops_mnk: np.ndarray) -> dict:
    t = np.ascontiguousarray(tflops_mnk, dtype=np.float64)
    st = sg_stats()
    check(lib().sg_landscape_stats(_arr(t), t.shape[0], t.shape[1], t.shape[2], ctypes.byref(st)))
    return {"mean": st.mean, "peak": st.peak, "roughness_m": st.rough_m, "roughness_n": st.rough_n,
            "roughness_k": st.rough_k, "roughness_3d": st.rough_3d}


class Table:
    """Dispatch table (owned; freed with the object)."""

    def __init__(self, handle: int):
        self.handle = ctypes.c_void_p(handle)

    def __del__(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            _lib.sg_table_free(self.handle)
            self.handle = ctypes.c_void_p(0)

    @staticmethod
    def from_t0(step: int, n_m: int, n_n: int, n_k: int, T0: np.ndarray, variants) -> "Table":
        g = sg_grid(step, n_m, n_n, n_k)
        t0 = np.ascontiguousarray(T0, dtype=np.float64)
        v = np.ascontiguousarray(variants, dtype=np.int32)
        h = ctypes.c_void_p()
        check(lib().sg_table_from_t0(ctypes.byref(g), _arr(t0), _arr(v), v.size, ctypes.byref(h)))
        return Table(h.value)

    @staticmethod
    def load(path: str, force: bool = False) -> "Table":
        h = ctypes.c_void_p()
        check(lib().sg_table_load(path.encode(), 1 if force else 0, ctypes.byref(h)))
        return Table(h.value)

    def save(self, path: str):
        check(lib().sg_table_save(self.handle, path.encode()))

    def grid(self):
        g = sg_grid()
        check(lib().sg_table_grid(self.handle, ctypes.byref(g)))
        return g.step, g.n_m, g.n_n, g.n_k

    def lookup(self, M: int, N: int, K: int) -> dict:
        r = sg_plan_rec()
        check(lib().sg_table_lookup(self.handle, M, N, K, ctypes.byref(r)))
        return {"action": r.action, "arg": r.arg, "variant": r.variant, "t0": r.t0, "t1": r.t1,
                "t2": r.t2}

    def values(self, which: int) -> np.ndarray:
        step, nm, nn, nk = self.grid()
        cells = nm * nn * nk
        n = cells
        if which == 3:
            nv = len(self.variants())
            out = np.zeros(nv * cells, dtype=np.float64)
            check(lib().sg_table_values(self.handle, 3, _arr(out), out.size))
            return out.reshape(nv, nm, nn, nk)
        out = np.zeros(n, dtype=np.float64)
        check(lib().sg_table_values(self.handle, which, _arr(out), n))
        return out.reshape(nm, nn, nk)

    def variants(self):
        ids = np.zeros(64, dtype=np.int32)
        n = ctypes.c_int()
        check(lib().sg_table_variants(self.handle, _arr(ids), ids.size, ctypes.byref(n)))
        return [int(x) for x in ids[:n.value]]

    def plan_leaves(self, M: int, N: int, K: int) -> int:
        n = ctypes.c_int()
        check(lib().sg_table_plan_leaves(self.handle, M, N, K, ctypes.byref(n)))
        return n.value


class Context:
    """A library context on one device (workspace, timing events, borrowed table)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        check(lib().sg_ctx_create(device, ctypes.byref(h)))
        self.handle = h
        self.device = device
        self._table = None

    def close(self):
        if self.handle and self.handle.value:
            lib().sg_ctx_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_plain_variant(self, v: int):
        check(lib().sg_ctx_set_plain_variant(self.handle, v))

    def reserve_workspace(self, nbytes: int):
        check(lib().sg_ctx_reserve_workspace(self.handle, nbytes))

    def set_table(self, table: Optional[Table]):
        self._table = table
        check(lib().sg_ctx_set_table(self.handle, table.handle if table else None))

    def gemm(self, A, B, C, *, beta: int = 0, mode: int = MODE_DEFAULT, variant: int = 0,
             M=None, N=None, K=None, lda=None, ldb=None, ldc=None, stream=None):
        """C (FP32 or BF16 torch tensor) = A @ B (+ C if beta): A, B BF16 torch CUDA tensors."""
        import torch
        if A.dtype != torch.bfloat16 or B.dtype != torch.bfloat16:
            raise TypeError("A and B must be bfloat16")
        if C.dtype not in (torch.float32, torch.bfloat16):
            raise TypeError("C must be float32 or bfloat16")
        if not (A.is_cuda and B.is_cuda and C.is_cuda):
            raise TypeError("A, B and C must be device tensors")
        M = A.shape[0] if M is None else M
        K = A.shape[1] if K is None else K
        N = B.shape[1] if N is None else N
        a = sg_gemm_args()
        a.M, a.N, a.K = M, N, K
        a.A, a.lda = A.data_ptr(), (A.stride(0) if lda is None else lda)
        a.B, a.ldb = B.data_ptr(), (B.stride(0) if ldb is None else ldb)
        a.C, a.ldc = C.data_ptr(), (C.stride(0) if ldc is None else ldc)
        a.c_dtype = F32 if C.dtype == torch.float32 else BF16
        a.beta, a.mode, a.variant = beta, mode, variant
        check(lib().gemm_bf16_nn_ex(self.handle, ctypes.byref(a), _stream_ptr(stream)))
        return C

    def sweep(self, shapes, A_pool, B_pool, C_pool, *, mode=MODE_PLAIN, variant=0, c_dtype=BF16,
              warmup=5, reps=5, stream=None) -> np.ndarray:
        sh = (sg_shape * len(shapes))(*[sg_shape(int(m), int(n), int(k)) for (m, n, k) in shapes])
        out = np.zeros(len(shapes), dtype=np.float64)
        check(lib().sg_sweep(self.handle, sh, len(shapes), mode, variant, c_dtype, warmup, reps,
                             A_pool.data_ptr(), B_pool.data_ptr(), C_pool.data_ptr(), _arr(out),
                             _stream_ptr(stream)))
        return out

    def kernel_times(self):
        nv = num_variants()
        la = np.zeros(nv, dtype=np.int64)
        se = np.zeros(nv, dtype=np.float64)
        fl = np.zeros(nv, dtype=np.float64)
        check(lib().sg_sweep_kernel_times(self.handle, _arr(la), _arr(se), _arr(fl)))
        return la, se, fl

    def build_table(self, step, n_m, n_n, n_k, variants, A_pool, B_pool, C_pool, *, c_dtype=BF16,
                    warmup=5, reps=5, order_seed=0, stream=None) -> Table:
        g = sg_grid(step, n_m, n_n, n_k)
        v = np.ascontiguousarray(variants, dtype=np.int32)
        h = ctypes.c_void_p()
        check(lib().sg_table_build(self.handle, ctypes.byref(g), _arr(v), v.size, c_dtype, warmup,
                                   reps, order_seed, A_pool.data_ptr(), B_pool.data_ptr(),
                                   C_pool.data_ptr(), _stream_ptr(stream), ctypes.byref(h)))
        return Table(h.value)


def gemm_bf16_nn(M: int, N: int, K: int, A, B, C):
    """Paper-form call on device tensors (C FP32, packed leading dimensions, null stream)."""
    check(lib().gemm_bf16_nn(M, N, K, A.data_ptr(), B.data_ptr(), C.data_ptr()))
    return C


def fill_bf16(dst, seed: int, stream_id: int, *, offset: int = 0, kind: int = 0, scale: float = 1.0,
              stream=None):
    """Fill a BF16 device tensor from the seeded counter generator (kind 0 uniform, 1 normal)."""
    check(lib().sg_fill_bf16(dst.data_ptr(), dst.numel(), seed, stream_id, offset, kind, scale,
                             _stream_ptr(stream)))
    return dst


def to_device_bf16(bits: np.ndarray, device="cuda"):
    """Upload BF16 bit patterns (uint16 numpy) as a bfloat16 device tensor."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(bits).view(np.int16))
    return t.view(torch.bfloat16).to(device)


def bf16_tensor_bits(t) -> np.ndarray:
    """BF16 tensor -> uint16 bit patterns on the host."""
    import torch
    return t.detach().contiguous().view(torch.int16).cpu().numpy().view(np.uint16)
