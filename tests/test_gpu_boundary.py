"""The boundary calls on the GPU: the paper-form gemm_bf16_nn reaching the dispatch table's
O(1) lookup (paper Sec. 7.1), the one-shot grouped call autotuning its schedule, schedules
recorded in and reused from the table, and plan updates that change the kernel."""
import numpy as np
import pytest

from gpu_helpers import check_exact, check_tol, inputs, say

pytestmark = pytest.mark.gpu
sg = pytest.importorskip("paper_2605_29752_amd")
F32, BF16 = 0, 1


@pytest.fixture(scope="module")
def ctx():
    c = sg.Context(0)
    yield c
    c.set_table(None)
    c.close()


def _split_pad_table():
    """A 64-step table whose plan for (150, 200, 250) splits along K and pads its pieces:
    T0 grows steeply in K (so K splits) and odd cells cost double (so they pad upward)."""
    step, shape = 64, (4, 4, 4)
    g = np.meshgrid(*[np.arange(1, n + 1) for n in shape], indexing="ij")
    base = (g[0] * g[1] * g[2] ** 3).astype(np.float64) + 0.01
    odd = ((g[0] % 2) == 1) | ((g[1] % 2) == 1)
    T0 = (base * np.where(odd, 2.0, 1.0))[None]
    return sg.Table.from_t0(step, *shape, T0, [13])


def test_paper_form_call_runs_the_dp_plan():
    import torch
    t = _split_pad_table()
    M, N, K = 150, 200, 250
    rec = t.lookup(M, N, K)
    assert rec["action"] == sg.ACT_SPLIT_K and t.plan_leaves(M, N, K) >= 2
    # the pieces of the split are padded: their cells are odd-sized along M
    assert t.lookup(M, N, 64)["action"] == sg.ACT_PAD
    sg.set_default_table(0, t)
    try:
        # integer inputs: every plan is bit-exact against the oracle
        A, B = inputs(901, M, N, K, "int")
        C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
        sg.gemm_bf16_nn(M, N, K, sg.to_device_bf16(A), sg.to_device_bf16(B), C)
        torch.cuda.synchronize()
        check_exact(C.cpu().numpy().astype(np.float64), A, B, F32)
        # random inputs: the paper-form call equals the DP plan bit for bit and differs from the
        # plain kernel (the K pieces are summed in another order)
        A, B = inputs(902, M, N, K)
        dA, dB = sg.to_device_bf16(A), sg.to_device_bf16(B)
        C = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
        sg.gemm_bf16_nn(M, N, K, dA, dB, C)
        ref = sg.Context(0)
        ref.set_table(t)
        Cdp = torch.full_like(C, float("nan"))
        ref.gemm(dA, dB, Cdp, mode=sg.MODE_DP)
        Cpl = torch.full_like(C, float("nan"))
        ref.gemm(dA, dB, Cpl, mode=sg.MODE_PLAIN)
        torch.cuda.synchronize()
        ref.set_table(None)
        ref.close()
        assert torch.equal(C.view(torch.int32), Cdp.view(torch.int32))
        assert not torch.equal(C.view(torch.int32), Cpl.view(torch.int32)), "the DP plan did not run"
        check_tol(C.cpu().numpy().astype(np.float64), A, B, F32)
    finally:
        sg.set_default_table(0, None)
    # without a table the paper-form call is the plain kernel again
    C2 = torch.full((M, N), float("nan"), dtype=torch.float32, device="cuda")
    sg.gemm_bf16_nn(M, N, K, dA, dB, C2)
    torch.cuda.synchronize()
    assert torch.equal(C2.view(torch.int32), Cpl.view(torch.int32))


def _group(seed, G, lo, hi):
    rng = np.random.default_rng(seed)
    host, dev, probs = [], [], []
    for g in range(G):
        M, N, K = [8 * int(x) for x in rng.integers(lo // 8, hi // 8, 3)]
        A, B = inputs(seed * 1000 + g, M, N, K, "int")
        dA, dB = sg.to_device_bf16(A), sg.to_device_bf16(B)
        host.append((A, B))
        dev.append((dA, dB))
        probs.append((M, N, K, dA.data_ptr(), K, dB.data_ptr(), N))
    return host, dev, probs


def _f32_outputs(probs):
    import torch
    return [torch.full((p[0], p[1]), float("nan"), dtype=torch.float32, device="cuda") for p in probs]


def test_one_shot_grouped_call_autotunes(ctx):
    host, dev, probs = _group(51, 12, 64, 400)
    Cs = _f32_outputs(probs)
    sg.gemm_grouped(ctx, [p + (C.data_ptr(), p[1]) for p, C in zip(probs, Cs)], F32, tile=None)
    for (A, B), C in zip(host, Cs):
        check_exact(C.cpu().numpy().astype(np.float64), A, B, F32)


def test_schedule_recorded_in_the_table_and_reused(ctx, tmp_path):
    import torch
    t = _split_pad_table()
    ctx.set_table(t)
    try:
        host, dev, probs = _group(61, 16, 64, 600)
        Cs = _f32_outputs(probs)
        full = [p + (C.data_ptr(), p[1]) for p, C in zip(probs, Cs)]
        assert t.group_schedules() == 0
        p1 = sg.GroupPlan(ctx, full, F32)                      # autotuned, recorded
        i1 = p1.info()
        assert t.group_schedules() == 1
        p2 = sg.GroupPlan(ctx, full, F32)                      # taken from the table
        assert t.group_schedules() == 1 and p2.info() == i1
        say("schedule", i1)
        p2.launch()
        torch.cuda.synchronize()
        for (A, B), C in zip(host, Cs):
            check_exact(C.cpu().numpy().astype(np.float64), A, B, F32)
        path = str(tmp_path / "with_sched.sgt")
        t.save(path)
        t2 = sg.Table.load(path, force=True)
        assert t2.group_schedules() == 1
        p1.close()
        p2.close()
    finally:
        ctx.set_table(None)


def test_update_that_changes_the_kernel_asks_for_recapture(ctx):
    import torch
    host, dev, probs = _group(71, 6, 64, 300)
    C1 = _f32_outputs(probs)
    plan = sg.GroupPlan(ctx, [p + (C.data_ptr(), p[1]) for p, C in zip(probs, C1)], F32, tile=3)
    # same M and N (so the same tiles and grid), but problem 0 gets K = 100: no longer aligned
    M0, N0 = probs[0][0], probs[0][1]
    A0, B0 = inputs(7100, M0, N0, 100, "int")
    dA0, dB0 = sg.to_device_bf16(A0), sg.to_device_bf16(B0)
    new = [(M0, N0, 100, dA0.data_ptr(), 100, dB0.data_ptr(), N0)] + probs[1:]
    C2 = _f32_outputs(new)
    with pytest.raises(sg.SGError) as e:
        plan.update([p + (C.data_ptr(), p[1]) for p, C in zip(new, C2)])
    assert e.value.code == sg.SG_EAGAIN
    # the plan itself runs the updated problems with the right kernel
    plan.launch()
    torch.cuda.synchronize()
    for (A, B), C in zip([(A0, B0)] + host[1:], C2):
        check_exact(C.cpu().numpy().astype(np.float64), A, B, F32)
    plan.close()
