"""The landscape verifier's host bookkeeping (tests/pool_verify.py) on the CPU: with outputs
from the plain FP64 oracle it reports no error, and planted faults in one shape's output are
found by the check meant to catch them.  Small grid; no GPU."""
import numpy as np
import pytest

import oracle
import synth
from pool_verify import verify_landscape

torch = pytest.importorskip("torch")


def _run_factory(A_bits, B_bits, fault=None):
    def run(M, N, K):
        A = A_bits[: M * K].reshape(M, K)
        B = B_bits[: K * N].reshape(K, N)
        C = oracle.gemm_f64(A, B, want_d=False)
        bits = oracle.f64_to_bf16_rne(C) if C.size <= 4096 else synth.f32_to_bf16_bits(C.astype(np.float32))
        if fault is not None and (M, N, K) == fault[0]:
            bits = fault[1](bits.copy(), A, B)
        t = torch.from_numpy(bits.view(np.int16).copy()).view(torch.bfloat16)
        return t
    return run


@pytest.fixture(scope="module")
def pools():
    n = 48 * 48
    return synth.uniform_bf16(5, 0, 1, n).ravel(), synth.uniform_bf16(5, 1, 1, n).ravel()


def test_exact_outputs_pass(pools):
    A_bits, B_bits = pools
    sizes = np.array([16, 32, 48])
    rep = verify_landscape(torch, _run_factory(A_bits, B_bits), A_bits, B_bits, sizes, 1, log=lambda *a: None,
                           device="cpu")
    assert rep.outputs == 27 and rep.full_outputs == 27
    assert rep.ok() and rep.frei <= 8e-3 and rep.samp <= 4e-3 and rep.full <= 4e-3


def _zero_block(bits, A, B):
    bits[:8, :8] = 0
    return bits


def _wrong_k(bits, A, B):
    # the result of a missing K piece (the first 16 of K)
    Ah = synth.bf16_bits_to_f32(A[:, 16:]).astype(np.float64)
    Bh = synth.bf16_bits_to_f32(B[16:, :]).astype(np.float64)
    return synth.f32_to_bf16_bits((Ah @ Bh).astype(np.float32))


@pytest.mark.parametrize("fault", [_zero_block, _wrong_k])
def test_planted_faults_are_found(pools, fault):
    A_bits, B_bits = pools
    sizes = np.array([16, 32, 48])
    shape = (32, 48, 32)
    rep = verify_landscape(torch, _run_factory(A_bits, B_bits, (shape, fault)), A_bits, B_bits, sizes, 1,
                           log=lambda *a: None, device="cpu")
    assert not rep.ok()
    assert rep.worst is not None and rep.worst[2] == shape
