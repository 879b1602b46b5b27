"""Shared helpers of the GPU parity tests: seeded inputs, the library call, oracle checks."""
import numpy as np

import oracle
import synth

TOL = {0: 1e-5, 1: 8e-3}      # FP32 output, BF16 output: max |C - C_ref| / (|A||B|)


def say(*a):
    print(*a, flush=True)


def inputs(seed, M, N, K, kind="uniform"):
    if kind == "uniform":
        return synth.uniform_bf16(seed, synth.STREAM_A, M, K), synth.uniform_bf16(seed, synth.STREAM_B, K, N)
    if kind == "int":
        return synth.integer_bf16(seed, synth.STREAM_A, M, K), synth.integer_bf16(seed, synth.STREAM_B, K, N)
    raise ValueError(kind)


def run_gemm(ctx, A_bits, B_bits, c_dtype, *, mode, variant=0, beta=0, C0_bits=None, C0_f32=None):
    import torch
    import paper_2605_29752_amd as sg
    M, K = A_bits.shape
    N = B_bits.shape[1]
    A = sg.to_device_bf16(A_bits)
    B = sg.to_device_bf16(B_bits)
    if c_dtype == sg.F32:
        C = torch.from_numpy(C0_f32.copy()).cuda() if C0_f32 is not None else \
            torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    else:
        C = sg.to_device_bf16(C0_bits) if C0_bits is not None else \
            torch.full((M, N), float("nan"), dtype=torch.bfloat16, device="cuda")
    ctx.gemm(A, B, C, beta=beta, mode=mode, variant=variant)
    torch.cuda.synchronize()
    if c_dtype == sg.F32:
        return C.cpu().numpy().astype(np.float64)
    return synth.bf16_bits_to_f32(sg.bf16_tensor_bits(C)).astype(np.float64)


def check_tol(out, A_bits, B_bits, c_dtype, addend=None):
    Cref, D = oracle.gemm_f64(A_bits, B_bits)
    if addend is not None:
        Cref = Cref + addend
        D = D + np.abs(addend)
    err, where, zv = oracle.scaled_err(out, Cref, D)
    assert zv == 0, "non-zero output where the reference is exactly zero"
    assert err <= TOL[c_dtype], "err %.3e at flat %d" % (err, where)
    return err


def check_exact(out, A_bits, B_bits, c_dtype):
    """Integer inputs: FP32 output equals C_ref exactly; BF16 output equals RNE(C_ref)."""
    Cref = oracle.gemm_f64(A_bits, B_bits, want_d=False)
    if c_dtype == 0:
        bad = np.argwhere(out != Cref)
    else:
        want = synth.bf16_bits_to_f32(oracle.f64_to_bf16_rne(Cref)).astype(np.float64)
        bad = np.argwhere(out != want)
    assert bad.size == 0, "first mismatch at %s of %d" % (bad[0], len(bad))


def device_bytes(ptr: int, nbytes: int) -> np.ndarray:
    """Copy nbytes at a raw device address to the host (HIP runtime already loaded by torch)."""
    import ctypes
    import torch  # noqa: F401  (makes torch's HIP runtime the loaded one)
    hip = ctypes.CDLL("libamdhip64.so.7")
    out = np.empty(nbytes, dtype=np.uint8)
    rc = hip.hipMemcpy(out.ctypes.data_as(ctypes.c_void_p), ctypes.c_void_p(ptr),
                       ctypes.c_size_t(nbytes), 2)   # hipMemcpyDeviceToHost
    assert rc == 0, rc
    return out
