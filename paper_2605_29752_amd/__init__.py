"""smoothgemm for MI355X: Python binding of the C-ABI library ``libsmoothgemm.so``.

Argument marshalling only: every step of the GEMM path runs in the library's HIP kernels and
host runtime.  PyTorch supplies device memory (tensor storage) and streams.  There is no CPU
fallback: if the library is missing, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os
import sys
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmoothgemm.so")

SG_OK, SG_EINVAL, SG_ENOMEM, SG_ENOTABLE, SG_EMISMATCH, SG_EHIP, SG_ERANGE, SG_EIO, SG_EAGAIN = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
F32, BF16 = 0, 1
MODE_DEFAULT, MODE_PLAIN, MODE_BEST, MODE_DP, MODE_VARIANT, MODE_MEMORY = 0, 1, 2, 3, 4, 5
ACT_AS_IS, ACT_PAD, ACT_SPLIT_M, ACT_SPLIT_N, ACT_SPLIT_K = 0, 1, 2, 3, 4
MEM_READ_A, MEM_READ_B, MEM_WRITE_D, MEM_READ_C = 0, 1, 2, 3
MEM_ISOLATED, MEM_COALLOC = 0, 1

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


class sg_hw(ctypes.Structure):
    _fields_ = [("peak_tflops", _d), ("cores", _i32), ("bw_gbs", _d)]


class sg_kol(ctypes.Structure):
    _fields_ = [("tau", _d), ("rho", _d), ("t_band", _i32), ("s_band", _i32), ("level", _i32)]


class sg_decomp(ctypes.Structure):
    _fields_ = [("overhead_share", _d), ("cb_bandwidth", _d), ("cb_measured", _d)]


class sg_plan_rec(ctypes.Structure):
    _fields_ = [("action", _i32), ("arg", _i32), ("variant", _i32), ("t0", _d), ("t1", _d), ("t2", _d)]


_SIGS = {
    "sg_last_error": (ctypes.c_char_p, []),
    "sg_version": (ctypes.c_char_p, []),
    "sg_ctx_create": (_i32, [_i32, ctypes.POINTER(_p)]),
    "sg_ctx_destroy": (_i32, [_p]),
    "sg_ctx_set_plain_variant": (_i32, [_p, _i32]),
    "sg_ctx_set_progress": (_i32, [_p, _i32]),
    "sg_ctx_reserve_workspace": (_i32, [_p, ctypes.c_size_t]),
    "sg_ctx_set_table": (_i32, [_p, _p]),
    "sg_default_ctx": (_i32, [_i32, ctypes.POINTER(_p)]),
    "sg_set_default_table": (_i32, [_i32, _p]),
    "gemm_bf16_nn": (_i32, [_i64, _i64, _i64, _p, _p, _p]),
    "gemm_bf16_nn_ex": (_i32, [_p, ctypes.POINTER(sg_gemm_args), _p]),
    "gemm_bf16_nn_ex_noalloc": (_i32, [_p, ctypes.POINTER(sg_gemm_args), _p]),
    "sg_noalloc_scratch_bytes": (ctypes.c_size_t, []),
    "sg_num_variants": (_i32, []),
    "sg_variant_info_get": (_i32, [_i32, ctypes.POINTER(sg_variant_info)]),
    "sg_roughness": (_d, [_p, _i64]),
    "sg_landscape_stats": (_i32, [_p, _i32, _i32, _i32, ctypes.POINTER(sg_stats)]),
    "sg_ideal_landscape": (_i32, [ctypes.POINTER(sg_grid), ctypes.POINTER(sg_hw), _i32, _p]),
    "sg_optimal_landscape": (_i32, [ctypes.POINTER(sg_grid), ctypes.POINTER(sg_hw), _p, _i32, _i32, _p]),
    "sg_optimal_landscape_ch": (_i32, [ctypes.POINTER(sg_grid), ctypes.POINTER(sg_hw), _p, _i32, _i32, _i32,
                                       _i32, _p]),
    "sg_kol_grade": (_i32, [_p, _p, _i32, _i32, _i32, ctypes.POINTER(sg_kol)]),
    "sg_decompose": (_i32, [_p, _i64, _p, _p, ctypes.POINTER(sg_hw), _i32, _p, _p, ctypes.POINTER(sg_decomp)]),
    "sg_sweep": (_i32, [_p, _p, _i64, _i32, _i32, _i32, _i32, _i32, _p, _p, _p, _p, _p]),
    "sg_sweep_kernel_times": (_i32, [_p, _p, _p, _p]),
    "sg_ctx_set_interval_timing": (_i32, [_p, _i32]),
    "sg_sweep_interval_times": (_i32, [_p, _p, _i64]),
    "sg_table_from_t0": (_i32, [ctypes.POINTER(sg_grid), _p, _p, _i32, ctypes.POINTER(_p)]),
    "sg_table_build": (_i32, [_p, ctypes.POINTER(sg_grid), _p, _i32, _i32, _i32, _i32,
                              ctypes.c_uint64, _p, _p, _p, _p, ctypes.POINTER(_p)]),
    "sg_table_free": (_i32, [_p]),
    "sg_table_grid": (_i32, [_p, ctypes.POINTER(sg_grid)]),
    "sg_table_lookup": (_i32, [_p, _i64, _i64, _i64, ctypes.POINTER(sg_plan_rec)]),
    "sg_table_values": (_i32, [_p, _i32, _p, _i64]),
    "sg_table_variants": (_i32, [_p, _p, _i32, ctypes.POINTER(_i32)]),
    "sg_table_plan_leaves": (_i32, [_p, _i64, _i64, _i64, ctypes.POINTER(_i32)]),
    "sg_table_plan_choice": (_i32, [_p, _i64, _i64, _i64, ctypes.POINTER(_d), ctypes.POINTER(_d),
                                    ctypes.POINTER(_i32)]),
    "sg_table_group_count": (_i32, [_p, ctypes.POINTER(_i64)]),
    "sg_table_save": (_i32, [_p, ctypes.c_char_p]),
    "sg_table_load": (_i32, [ctypes.c_char_p, _i32, ctypes.POINTER(_p)]),
    "sg_fill_bf16": (_i32, [_p, _i64, ctypes.c_uint64, ctypes.c_uint64, _i64, _i32, _d, _p]),
    "sg_mem_read_blocks": (_i64, [_i64]),
    "sg_ctx_set_concurrent_splits": (_i32, [_p, _i32]),
    "sg_mem_read": (_i32, [_p, _i64, _p, _p]),
    "sg_mem_write": (_i32, [_p, _i64, ctypes.c_uint32, _p]),
    "sg_mem_sweep": (_i32, [_p, _p, _i64, _i32, _i32, _i32, _i32, _i32, _p, _p]),
    "sg_group_plan_create": (_i32, [_p, _i32, _p, _i32, _p, _p, ctypes.POINTER(_p)]),
    "sg_group_plan_launch": (_i32, [_p, _p]),
    "sg_group_plan_update": (_i32, [_p, _p, _p]),
    "sg_group_plan_info": (_i32, [_p, _p, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_d)]),
    "sg_group_plan_destroy": (_i32, [_p]),
    "sg_gemm_grouped": (_i32, [_p, _i32, _p, _i32, _p, _p]),
    "sg_gemm_batch": (_i32, [_p, _i32, _p, _i32, _i32, _i32, _p]),
    "sg_graph_capture_groups": (_i32, [_p, _i32, _p, ctypes.POINTER(_p)]),
    "sg_graph_launch": (_i32, [_p, _p]),
    "sg_graph_destroy": (_i32, [_p]),
    "sg_server_create": (_i32, [_p, _p, ctypes.POINTER(_p)]),
    "sg_server_now": (_i32, [_p, ctypes.POINTER(_d)]),
    "sg_server_submit": (_i32, [_p, _p, _d, ctypes.POINTER(ctypes.c_uint64)]),
    "sg_server_poll": (_i32, [_p, _p, _i32, ctypes.POINTER(_i32)]),
    "sg_server_release": (_i32, [_p, ctypes.c_uint64]),
    "sg_server_drain": (_i32, [_p, _d]),
    "sg_server_stats_get": (_i32, [_p, _p]),
    "sg_server_destroy": (_i32, [_p]),
    "sg_serve_poisson": (_i32, [_p, _d, _d, _d, ctypes.c_uint64, _i64, _p]),
    "sg_serve_closed": (_i32, [_p, _i32, _d, _d, ctypes.c_uint64, _i64, _p]),
}

SERVE_GROUPED, SERVE_PER_REQUEST = 0, 1


class sg_weight(ctypes.Structure):
    _fields_ = [("K", _i64), ("N", _i64), ("B", _p), ("ldb", _i64)]


class sg_server_cfg(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_size_t), ("max_inflight", _i32), ("max_group", _i32),
                ("queue_cap", _i32), ("mode", _i32), ("tile", _i32), ("keep_results", _i32),
                ("n_weights", _i32), ("weights", ctypes.POINTER(sg_weight)), ("max_m", _i64),
                ("seed", ctypes.c_uint64), ("a_scale", _d), ("small_m", _i64), ("small_tile", _i32),
                ("solo_m", _i64), ("tiles_from_table", _i32)]


class sg_request(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("M", _i64), ("weight", _i32)]


class sg_completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("id", ctypes.c_uint64), ("M", _i64), ("N", _i64),
                ("K", _i64), ("weight", _i32), ("status", _i32), ("a_offset", _i64), ("tile", _i32),
                ("group_size", _i32), ("t_arrival", _d), ("t_admit", _d), ("t_launch", _d), ("t_done", _d),
                ("A", _p), ("C", _p)]


class sg_server_stats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("failed", _i64), ("launches", _i64),
                ("pending", _i64), ("flops", _d), ("bytes_in_use", _d), ("peak_bytes", _d)]


class sg_serve_report(ctypes.Structure):
    _fields_ = [("offered", _i64), ("rejected", _i64), ("failed", _i64), ("measured", _i64),
                ("launches", _i64), ("window_s", _d), ("req_per_s", _d), ("tflops", _d),
                ("p50_ms", _d), ("p99_ms", _d), ("mean_ms", _d), ("peak_bytes", _d)]


class sg_problem(ctypes.Structure):
    _fields_ = [("M", _i64), ("N", _i64), ("K", _i64), ("A", _p), ("lda", _i64), ("B", _p),
                ("ldb", _i64), ("C", _p), ("ldc", _i64)]


class sg_group_cfg(ctypes.Structure):
    _fields_ = [("tile", _i32), ("grid_wgs", _i32), ("order", _i32)]

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


def _live() -> bool:
    """Whether library calls from a finaliser are still safe: at interpreter shutdown the HIP
    runtime may already be tearing down, so objects still alive then are left to the process
    exit instead of being destroyed (close() them explicitly to release them earlier)."""
    return _lib is not None and not sys.is_finalizing()


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


MI355X = {"peak_tflops": 2516.6, "cores": 256, "bw_gbs": 8000.0}   # dense BF16 MFMA, CUs, HBM3E


def _hw(hw) -> "sg_hw":
    return sg_hw(float(hw["peak_tflops"]), int(hw["cores"]), float(hw["bw_gbs"]))


def ideal_landscape(step: int, n_m: int, n_n: int, n_k: int, tile: int = 256, hw=MI355X) -> np.ndarray:
    """Ideal ceiling over the grid (paper Sec. 9.1), n_m x n_n x n_k TFLOP/s."""
    out = np.zeros((n_m, n_n, n_k), dtype=np.float64)
    g = sg_grid(step, n_m, n_n, n_k)
    check(lib().sg_ideal_landscape(ctypes.byref(g), ctypes.byref(_hw(hw)), tile, _arr(out)))
    return out


def optimal_landscape(step: int, n_m: int, n_n: int, n_k: int, tiles=(256, 128, 64), c_bytes: int = 2,
                      hw=MI355X, channels: int = 0, interleave: int = 256) -> np.ndarray:
    """First-principles optimal landscape over the grid (paper Sec. 9.2), TFLOP/s; channels > 0
    adds the memory-channel utilisation term (0: every channel share taken as 1)."""
    out = np.zeros((n_m, n_n, n_k), dtype=np.float64)
    g = sg_grid(step, n_m, n_n, n_k)
    t = (ctypes.c_int * len(tiles))(*tiles)
    check(lib().sg_optimal_landscape_ch(ctypes.byref(g), ctypes.byref(_hw(hw)), t, len(tiles), c_bytes,
                                        channels, interleave, _arr(out)))
    return out


def decompose(shapes, t_gemm, t_memory, c_bytes: int = 2, hw=MI355X) -> dict:
    """Four-surface decomposition of measured GEMM and memory times (paper Sec. 4): per-shape
    compute and overhead times (seconds) and the overhead share / compute-bound fractions."""
    n = len(shapes)
    sh = (sg_shape * n)(*[sg_shape(int(m), int(nn), int(k)) for (m, nn, k) in shapes])
    tg = np.ascontiguousarray(t_gemm, dtype=np.float64)
    tm = np.ascontiguousarray(t_memory, dtype=np.float64)
    if tg.size != n or tm.size != n:
        raise ValueError("one GEMM time and one memory time per shape")
    tc = np.zeros(n, dtype=np.float64)
    to = np.zeros(n, dtype=np.float64)
    d = sg_decomp()
    check(lib().sg_decompose(sh, n, _arr(tg), _arr(tm), ctypes.byref(_hw(hw)), c_bytes, _arr(tc),
                             _arr(to), ctypes.byref(d)))
    return {"t_compute": tc, "t_overhead": to, "overhead_share": d.overhead_share,
            "cb_bandwidth": d.cb_bandwidth, "cb_measured": d.cb_measured}


def kol_grade(actual: np.ndarray, optimal: np.ndarray) -> dict:
    """(tau, rho, bands, level) of a landscape against the optimal (paper Sec. 10)."""
    a = np.ascontiguousarray(actual, dtype=np.float64)
    o = np.ascontiguousarray(optimal, dtype=np.float64)
    if a.shape != o.shape:
        raise ValueError("landscapes differ in shape")
    if a.ndim == 2:
        a, o = a[:, :, None], o[:, :, None]
    k = sg_kol()
    check(lib().sg_kol_grade(_arr(np.ascontiguousarray(a)), _arr(np.ascontiguousarray(o)),
                             a.shape[0], a.shape[1], a.shape[2], ctypes.byref(k)))
    return {"tau": k.tau, "rho": k.rho, "t_band": k.t_band, "s_band": k.s_band, "level": k.level}


class Table:
    """Dispatch table (owned; freed with the object)."""

    def __init__(self, handle: int):
        self.handle = ctypes.c_void_p(handle)

    def close(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            h, self.handle = self.handle, ctypes.c_void_p(0)
            check(_lib.sg_table_free(h))

    def __del__(self):
        # at interpreter shutdown the module's globals may already be gone: then the process
        # exit releases the object
        try:
            if _live():
                self.close()
        except (TypeError, NameError, AttributeError):
            pass

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

    def group_schedules(self) -> int:
        """Grouped-launch schedules the grouped autotuner has recorded in this table."""
        n = ctypes.c_int64()
        check(lib().sg_table_group_count(self.handle, ctypes.byref(n)))
        return n.value

    def plan_choice(self, M: int, N: int, K: int) -> dict:
        """Which plan the DP mode runs for (M, N, K): the table plan (always on the grid) or, off
        the grid, the cell's best variant unless the plan is estimated at least 5 % faster."""
        ep, eb, use = ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        check(lib().sg_table_plan_choice(self.handle, M, N, K, ctypes.byref(ep), ctypes.byref(eb),
                                         ctypes.byref(use)))
        return {"est_plan": ep.value, "est_best": eb.value, "use_plan": bool(use.value)}

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
        """Destroy the context (raises with the HIP status if its release reported an error)."""
        if getattr(self, "handle", None) and self.handle.value:
            h, self.handle = self.handle, ctypes.c_void_p(0)
            check(lib().sg_ctx_destroy(h))

    def __del__(self):
        # at interpreter shutdown the module's globals may already be gone: then the process
        # exit releases the object
        try:
            if _live():
                self.close()
        except (TypeError, NameError, AttributeError):
            pass

    def set_plain_variant(self, v: int):
        check(lib().sg_ctx_set_plain_variant(self.handle, v))

    def set_progress(self, every: int):
        check(lib().sg_ctx_set_progress(self.handle, every))

    def set_concurrent_splits(self, mode):
        """Pieces of M / N split plans: 0 / False one after another (kernel-time sum), 1 / True
        at the same time on the context's streams, 2 one after another timed like 1."""
        check(lib().sg_ctx_set_concurrent_splits(self.handle, int(mode)))

    def reserve_workspace(self, nbytes: int):
        check(lib().sg_ctx_reserve_workspace(self.handle, nbytes))

    def set_table(self, table: Optional[Table]):
        self._table = table
        check(lib().sg_ctx_set_table(self.handle, table.handle if table else None))

    def gemm(self, A, B, C, *, beta: int = 0, mode: int = MODE_DEFAULT, variant: int = 0,
             M=None, N=None, K=None, lda=None, ldb=None, ldc=None, stream=None, noalloc=False):
        """C (FP32 or BF16 torch tensor) = A @ B (+ C if beta): A, B BF16 torch CUDA tensors.
        noalloc: use the entry point that takes its scratch from the library's fixed device
        array instead of the context's workspace."""
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
        fn = lib().gemm_bf16_nn_ex_noalloc if noalloc else lib().gemm_bf16_nn_ex
        check(fn(self.handle, ctypes.byref(a), _stream_ptr(stream)))
        return C

    def mem_sweep(self, shapes, op: int, alloc: int, *, elem_bytes: int = 4, warmup: int = 5,
                  reps: int = 5, stream=None) -> np.ndarray:
        """Memory-study sweep (paper Sec. 5): seconds per run of `op` on each shape's buffer."""
        sh = (sg_shape * len(shapes))(*[sg_shape(int(m), int(n), int(k)) for (m, n, k) in shapes])
        out = np.zeros(len(shapes), dtype=np.float64)
        check(lib().sg_mem_sweep(self.handle, sh, len(shapes), op, alloc, elem_bytes, warmup, reps,
                                 _arr(out), _stream_ptr(stream)))
        return out

    def sweep(self, shapes, A_pool, B_pool, C_pool, *, mode=MODE_PLAIN, variant=0, c_dtype=BF16,
              warmup=5, reps=5, stream=None) -> np.ndarray:
        sh = (sg_shape * len(shapes))(*[sg_shape(int(m), int(n), int(k)) for (m, n, k) in shapes])
        out = np.zeros(len(shapes), dtype=np.float64)
        check(lib().sg_sweep(self.handle, sh, len(shapes), mode, variant, c_dtype, warmup, reps,
                             A_pool.data_ptr(), B_pool.data_ptr(), C_pool.data_ptr(), _arr(out),
                             _stream_ptr(stream)))
        return out

    def set_interval_timing(self, on: bool):
        """Also time every sweep run between two stream markers (gaps included)."""
        check(lib().sg_ctx_set_interval_timing(self.handle, 1 if on else 0))

    def interval_times(self, n: int) -> np.ndarray:
        """Per-shape marker-to-marker mean seconds of the most recent sweep (n shapes)."""
        out = np.zeros(n, dtype=np.float64)
        check(lib().sg_sweep_interval_times(self.handle, _arr(out), n))
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


def _problems(probs):
    """[(M, N, K, A_ptr, lda, B_ptr, ldb, C_ptr, ldc), ...] -> ctypes array."""
    arr = (sg_problem * len(probs))()
    for i, p in enumerate(probs):
        arr[i] = sg_problem(*[int(x) for x in p])
    return arr


class GroupPlan:
    """A grouped launch: device-resident descriptors, fixed tile shape and work order."""

    def __init__(self, ctx: "Context", probs, c_dtype: int = BF16, tile: Optional[int] = None,
                 grid_wgs: int = 0, order: int = 0, stream=None):
        self._probs = _problems(probs)
        cfg = None if tile is None else ctypes.byref(sg_group_cfg(tile, grid_wgs, order))
        h = ctypes.c_void_p()
        check(lib().sg_group_plan_create(ctx.handle, len(probs), self._probs, c_dtype, cfg,
                                         _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h

    def launch(self, stream=None):
        check(lib().sg_group_plan_launch(self.handle, _stream_ptr(stream)))

    def update(self, probs, stream=None):
        self._probs = _problems(probs)
        check(lib().sg_group_plan_update(self.handle, self._probs, _stream_ptr(stream)))

    def info(self) -> dict:
        cfg = sg_group_cfg()
        tiles, grid, flops = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        check(lib().sg_group_plan_info(self.handle, ctypes.byref(cfg), ctypes.byref(tiles),
                                       ctypes.byref(grid), ctypes.byref(flops)))
        return {"tile": cfg.tile, "grid_wgs": grid.value, "order": cfg.order,
                "total_tiles": tiles.value, "flops": flops.value}

    def close(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            h, self.handle = self.handle, ctypes.c_void_p(0)
            check(_lib.sg_group_plan_destroy(h))

    def __del__(self):
        # at interpreter shutdown the module's globals may already be gone: then the process
        # exit releases the object
        try:
            if _live():
                self.close()
        except (TypeError, NameError, AttributeError):
            pass


class Graph:
    """hipGraph holding a sequence of grouped launches."""

    def __init__(self, plans, stream):
        arr = (ctypes.c_void_p * len(plans))(*[p.handle.value for p in plans])
        h = ctypes.c_void_p()
        check(lib().sg_graph_capture_groups(arr, len(plans), _stream_ptr(stream), ctypes.byref(h)))
        self.handle = h
        self._plans = list(plans)

    def launch(self, stream=None):
        check(lib().sg_graph_launch(self.handle, _stream_ptr(stream)))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            h, self.handle = self.handle, ctypes.c_void_p(0)
            check(_lib.sg_graph_destroy(h))

    def __del__(self):
        # at interpreter shutdown the module's globals may already be gone: then the process
        # exit releases the object
        try:
            if _live():
                self.close()
        except (TypeError, NameError, AttributeError):
            pass


class Server:
    """Continuous-batching GEMM server (worker thread inside the library)."""

    def __init__(self, ctx: "Context", weights, *, hbm_budget: int, max_inflight: int = 4,
                 max_group: int = 64, queue_cap: int = 1 << 20, mode: int = SERVE_GROUPED,
                 tile: int = 3, keep_results: bool = False, max_m: int = 8192, seed: int = 5,
                 a_scale: float = 0.02, small_m: int = 64, small_tile: int = 6, solo_m: int = 0,
                 tiles_from_table: bool = False):
        """weights: [(K, N, B_ptr, ldb), ...] device-resident BF16 matrices.  Requests with
        M <= small_m run with tile shape small_tile, the others with `tile`, or with
        tiles_from_table the tile of the context table's best variant for their shape; requests
        with M > solo_m (solo_m > 0) are launched on their own, never in a group."""
        self._w = (sg_weight * len(weights))(*[sg_weight(*[int(x) for x in w]) for w in weights])
        cfg = sg_server_cfg(hbm_budget, max_inflight, max_group, queue_cap, mode, tile,
                            1 if keep_results else 0, len(weights), self._w, max_m, seed, a_scale,
                            small_m, small_tile, solo_m, 1 if tiles_from_table else 0)
        h = ctypes.c_void_p()
        check(lib().sg_server_create(ctx.handle, ctypes.byref(cfg), ctypes.byref(h)))
        self.handle = h

    def now(self) -> float:
        t = ctypes.c_double()
        check(lib().sg_server_now(self.handle, ctypes.byref(t)))
        return t.value

    def submit(self, req_id: int, M: int, weight: int, arrival: float = -1.0) -> int:
        r = sg_request(req_id, M, weight)
        tk = ctypes.c_uint64()
        check(lib().sg_server_submit(self.handle, ctypes.byref(r), arrival, ctypes.byref(tk)))
        return tk.value

    def poll(self, max_n: int = 1024):
        buf = (sg_completion * max_n)()
        n = ctypes.c_int()
        check(lib().sg_server_poll(self.handle, buf, max_n, ctypes.byref(n)))
        return [buf[i] for i in range(n.value)]

    def release(self, ticket: int):
        check(lib().sg_server_release(self.handle, ticket))

    def drain(self, timeout: float = 600.0):
        check(lib().sg_server_drain(self.handle, timeout))

    def stats(self) -> dict:
        st = sg_server_stats()
        check(lib().sg_server_stats_get(self.handle, ctypes.byref(st)))
        return {f: getattr(st, f) for f, _ in sg_server_stats._fields_}

    def serve_poisson(self, rate: float, duration: float, warmup: float, seed: int,
                      max_m: int = 8192) -> dict:
        rep = sg_serve_report()
        check(lib().sg_serve_poisson(self.handle, rate, duration, warmup, seed, max_m,
                                     ctypes.byref(rep)))
        return {f: getattr(rep, f) for f, _ in sg_serve_report._fields_}

    def serve_closed(self, outstanding: int, duration: float, warmup: float, seed: int,
                     max_m: int = 8192) -> dict:
        """Closed-loop saturation run: `outstanding` requests kept in the server."""
        rep = sg_serve_report()
        check(lib().sg_serve_closed(self.handle, outstanding, duration, warmup, seed, max_m,
                                    ctypes.byref(rep)))
        return {f: getattr(rep, f) for f, _ in sg_serve_report._fields_}

    def close(self):
        if getattr(self, "handle", None) and self.handle.value and _lib is not None:
            h, self.handle = self.handle, ctypes.c_void_p(0)
            check(_lib.sg_server_destroy(h))

    def __del__(self):
        # at interpreter shutdown the module's globals may already be gone: then the process
        # exit releases the object
        try:
            if _live():
                self.close()
        except (TypeError, NameError, AttributeError):
            pass


def gemm_batch(ctx: "Context", probs, c_dtype: int = BF16, mode: int = MODE_PLAIN, variant: int = 0,
               stream=None, _arr=None):
    """Per-call launches of every problem, issued back to back from the library."""
    arr = _arr if _arr is not None else _problems(probs)
    check(lib().sg_gemm_batch(ctx.handle, len(arr), arr, c_dtype, mode, variant, _stream_ptr(stream)))


def gemm_grouped(ctx: "Context", probs, c_dtype: int = BF16, tile: Optional[int] = 3, stream=None):
    """One-shot grouped launch (plan, launch, wait, free); tile None autotunes the schedule."""
    arr = _problems(probs)
    cfg = None if tile is None else ctypes.byref(sg_group_cfg(tile, 0, 0))
    check(lib().sg_gemm_grouped(ctx.handle, len(probs), arr, c_dtype, cfg, _stream_ptr(stream)))


def set_default_table(device: int, table: Optional["Table"]):
    """Lend `table` to the device's default context: gemm_bf16_nn then runs its DP plans.
    The binding keeps a reference so the table outlives its use (None clears)."""
    _default_tables[device] = table
    check(lib().sg_set_default_table(device, table.handle if table else None))


_default_tables = {}


def noalloc_scratch_bytes() -> int:
    """Size of the fixed device scratch of the no-allocation entry point."""
    return int(lib().sg_noalloc_scratch_bytes())


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


def mem_read_blocks(nbytes: int) -> int:
    return int(lib().sg_mem_read_blocks(int(nbytes)))


def mem_read(buf, sink, nbytes=None, stream=None):
    """Stream-read a device tensor; `sink` (uint32-sized device tensor of at least
    mem_read_blocks(nbytes) words) receives per-block XORs of its 32-bit words."""
    nbytes = buf.numel() * buf.element_size() if nbytes is None else nbytes
    check(lib().sg_mem_read(buf.data_ptr(), nbytes, sink.data_ptr(), _stream_ptr(stream)))


def mem_write(buf, seed: int, nbytes=None, stream=None):
    """Stream-write a device tensor: word i = (i * 0x9E3779B1) ^ seed (mod 2^32)."""
    nbytes = buf.numel() * buf.element_size() if nbytes is None else nbytes
    check(lib().sg_mem_write(buf.data_ptr(), nbytes, seed, _stream_ptr(stream)))


def to_device_bf16(bits: np.ndarray, device="cuda"):
    """Upload BF16 bit patterns (uint16 numpy) as a bfloat16 device tensor."""
    import torch
    t = torch.from_numpy(np.ascontiguousarray(bits).view(np.int16))
    return t.view(torch.bfloat16).to(device)


def bf16_tensor_bits(t) -> np.ndarray:
    """BF16 tensor -> uint16 bit patterns on the host."""
    import torch
    return t.detach().contiguous().view(torch.int16).cpu().numpy().view(np.uint16)
