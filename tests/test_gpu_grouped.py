"""GPU parity of the persistent grouped kernel, its autotuned plan and hipGraph replays."""
import numpy as np
import pytest

import synth
from gpu_helpers import check_exact, check_tol, inputs, say

pytestmark = pytest.mark.gpu
sg = pytest.importorskip("paper_2605_29752_amd")
F32, BF16 = 0, 1


@pytest.fixture(scope="module")
def ctx():
    return sg.Context(0)


def _group(seed, G, kind, lo=1, hi=700, aligned_only=False):
    """G problems with their own device operands; returns (host bits, device tensors, probs)."""
    import torch
    rng = np.random.default_rng(seed)
    host, dev, probs = [], [], []
    for g in range(G):
        M, N, K = [int(x) for x in rng.integers(lo, hi, 3)]
        if aligned_only:
            M, N, K = [max(8, 8 * (x // 8)) for x in (M, N, K)]
        A, B = inputs(seed * 1000 + g, M, N, K, kind)
        dA, dB = sg.to_device_bf16(A), sg.to_device_bf16(B)
        host.append((A, B))
        dev.append((dA, dB))
        probs.append((M, N, K, dA.data_ptr(), K, dB.data_ptr(), N))
    return host, dev, probs


def _outputs(probs, c_dtype):
    import torch
    dt = torch.float32 if c_dtype == F32 else torch.bfloat16
    return [torch.full((p[0], p[1]), float("nan"), dtype=dt, device="cuda") for p in probs]


def _to_np(C, c_dtype):
    if c_dtype == F32:
        return C.cpu().numpy().astype(np.float64)
    return synth.bf16_bits_to_f32(sg.bf16_tensor_bits(C)).astype(np.float64)


@pytest.mark.parametrize("tile", range(7))
@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_grouped_integer_exact_every_tile(ctx, tile, c_dtype):
    import torch
    say("grouped tile", tile, "dtype", c_dtype)
    host, dev, probs = _group(3 + tile, 24, "int")
    Cs = _outputs(probs, c_dtype)
    full = [p + (C.data_ptr(), p[1]) for p, C in zip(probs, Cs)]
    plan = sg.GroupPlan(ctx, full, c_dtype, tile=tile)
    plan.launch()
    torch.cuda.synchronize()
    for (A, B), C in zip(host, Cs):
        check_exact(_to_np(C, c_dtype), A, B, c_dtype)
    plan.close()


@pytest.mark.parametrize("c_dtype", [F32, BF16])
def test_grouped_equals_alone_bitwise(ctx, c_dtype):
    """Each problem's output in the group equals a per-call launch of the same tile shape."""
    import torch
    host, dev, probs = _group(11, 40, "uniform", hi=900)
    tile = 3
    Cs = _outputs(probs, c_dtype)
    full = [p + (C.data_ptr(), p[1]) for p, C in zip(probs, Cs)]
    plan = sg.GroupPlan(ctx, full, c_dtype, tile=tile)
    plan.launch()
    torch.cuda.synchronize()
    for (A, B), (dA, dB), C, p in zip(host, dev, Cs, probs):
        alone = torch.full_like(C, float("nan"))
        ctx.gemm(dA.view(p[0], p[2]), dB.view(p[2], p[1]), alone, mode=sg.MODE_VARIANT, variant=4 * tile)
        torch.cuda.synchronize()
        assert torch.equal(alone.view(torch.int16 if c_dtype else torch.int32),
                           C.view(torch.int16 if c_dtype else torch.int32))
        check_tol(_to_np(C, c_dtype), A, B, c_dtype)
    plan.close()


def test_grouped_autotune_and_graph_replays(ctx):
    import torch
    host, dev, probs = _group(21, 64, "int", lo=64, hi=520, aligned_only=True)
    Cs = _outputs(probs, BF16)
    full = [p + (C.data_ptr(), p[1]) for p, C in zip(probs, Cs)]
    plan = sg.GroupPlan(ctx, full, BF16)           # autotuned tile shape
    info = plan.info()
    say("autotuned", info)
    assert 0 <= info["tile"] < 7 and info["total_tiles"] > 0
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        graph = sg.Graph([plan], s)
    torch.cuda.synchronize()
    first = None
    for replay in range(3):
        for C in Cs:
            C.fill_(float("nan"))                  # eager work between replays
        torch.cuda.synchronize()
        graph.launch(s)
        s.synchronize()
        outs = [C.clone() for C in Cs]
        if first is None:                          # the oracle checks the first replay ...
            first = outs
            for (A, B), C in zip(host, Cs):
                check_exact(_to_np(C, BF16), A, B, BF16)
        else:                                      # ... and every later one must match it
            assert all(torch.equal(a.view(torch.int16), b.view(torch.int16)) for a, b in zip(first, outs))
    graph.close()
    plan.close()


def test_grouped_plan_update_same_tiles(ctx):
    import torch
    host, dev, probs = _group(31, 8, "int", lo=100, hi=300)
    C1 = _outputs(probs, F32)
    C2 = _outputs(probs, F32)
    plan = sg.GroupPlan(ctx, [p + (C.data_ptr(), p[1]) for p, C in zip(probs, C1)], F32, tile=6)
    plan.update([p + (C.data_ptr(), p[1]) for p, C in zip(probs, C2)])
    plan.launch()
    torch.cuda.synchronize()
    for (A, B), C in zip(host, C2):
        check_exact(_to_np(C, F32), A, B, F32)
    assert all(torch.isnan(C).all() for C in C1)
    plan.close()


def test_grouped_one_shot_and_errors(ctx):
    import torch
    host, dev, probs = _group(41, 5, "int", lo=10, hi=200)
    Cs = _outputs(probs, F32)
    sg.gemm_grouped(ctx, [p + (C.data_ptr(), p[1]) for p, C in zip(probs, Cs)], F32, tile=5)
    for (A, B), C in zip(host, Cs):
        check_exact(_to_np(C, F32), A, B, F32)
    bad = [(0, 5, 5, 1, 5, 1, 5, 1, 5)]
    with pytest.raises(sg.SGError):
        sg.gemm_grouped(ctx, bad, F32)
    with pytest.raises(sg.SGError):
        sg.GroupPlan(ctx, [p + (C.data_ptr(), p[1]) for p, C in zip(probs, Cs)], F32, tile=9)
