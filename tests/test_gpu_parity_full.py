"""Parity at the workloads' full sizes, through the same dispatch machinery the benchmark runs:

* the whole landscape {128..4096}^3 (32,768 shapes) executed through a dispatch table measured
  on this GPU (best-of-N + T1 pad + T2 split, paper Sec. 7.1);
* the 4,096 off-grid shapes M, N, K ~ U{1..8192} (seed 3) through a measured table whose grid
  reaches 8192 (off-grid lookup of the covering cell);
* one sixteenth of the 512 grouped launches of 64 GEMMs (the same seeded shapes and operand
  offsets as the grouped benchmark), autotuned schedule;
* 200 served requests at the serving workload's weight shapes, each equal bit for bit to the
  same GEMM run alone.
Every output is checked against the FP64 oracle: a Freivalds row check, 4,096 sampled
entries, and every entry where M N K <= 2^30 (tests/pool_verify.py).  Operand bits come from
the host generator and are uploaded, so no oracle input comes from the GPU."""
import time

import numpy as np
import pytest

import synth
from oracle import check
from gpu_helpers import say
from pool_verify import FULL_LIMIT, Report, check_one, device_reduce, sample_index, verify_landscape

pytestmark = pytest.mark.gpu
sg = pytest.importorskip("paper_2605_29752_amd")
F32, BF16 = 0, 1
# a small, diverse variant set keeps the table measurement short: 256x256, 128x128 (also with
# two splits), 64x64 (also with four splits), 64x128 with two splits
TABLE_VARIANTS = [0, 12, 13, 21, 24, 26]


@pytest.fixture(scope="module")
def ctx():
    c = sg.Context(0)
    yield c
    c.set_table(None)
    c.close()


def _upload(bits):
    return sg.to_device_bf16(np.ascontiguousarray(bits).ravel())


@pytest.mark.timeout(900)
def test_landscape_through_measured_table(ctx):
    import torch
    n, step = 32, 128
    sizes = np.arange(1, n + 1) * step
    maxd = n * step
    t0 = time.time()
    A_bits = synth.uniform_bf16(2, synth.STREAM_A, 1, maxd * maxd).ravel()
    B_bits = synth.uniform_bf16(2, synth.STREAM_B, 1, maxd * maxd).ravel()
    A, B = _upload(A_bits), _upload(B_bits)
    C = torch.empty(maxd * maxd, dtype=torch.bfloat16, device="cuda")
    table = ctx.build_table(step, n, n, n, TABLE_VARIANTS, A, B, C, c_dtype=BF16, warmup=2, reps=1,
                            order_seed=11)
    acts = {}
    for M in sizes:
        for N in sizes:
            for K in sizes:
                a = table.lookup(int(M), int(N), int(K))["action"]
                acts[a] = acts.get(a, 0) + 1
    say("measured table in %.1f s; actions %s" % (time.time() - t0, acts))
    assert acts.get(sg.ACT_AS_IS, 0) > 0 and len(acts) >= 2
    ctx.set_table(table)

    def run(M, N, K):
        Cv = C[: M * N].view(M, N)
        ctx.gemm(A[: M * K].view(M, K), B[: K * N].view(K, N), Cv, mode=sg.MODE_DP)
        return Cv

    try:
        rep = verify_landscape(torch, run, A_bits, B_bits, sizes, BF16, log=say)
    finally:
        ctx.set_table(None)
    say("landscape: %s (%.1f s)" % (rep, time.time() - t0))
    assert rep.outputs == n ** 3 and rep.full_outputs > 5000
    assert rep.ok(), str(rep)


@pytest.mark.timeout(900)
def test_offgrid_shapes_through_measured_table(ctx):
    import torch
    t0 = time.time()
    maxd = 8192
    A_bits = synth.uniform_bf16(3, synth.STREAM_A, 1, maxd * maxd).ravel()
    B_bits = synth.uniform_bf16(3, synth.STREAM_B, 1, maxd * maxd).ravel()
    A, B = _upload(A_bits), _upload(B_bits)
    C = torch.empty(maxd * maxd, dtype=torch.bfloat16, device="cuda")
    step, n = 1024, 8
    table = ctx.build_table(step, n, n, n, TABLE_VARIANTS, A, B, C, c_dtype=BF16, warmup=2, reps=1,
                            order_seed=13)
    rng = np.random.default_rng(3)
    shapes = [tuple(int(x) for x in s) for s in rng.integers(1, 8193, size=(4096, 3))]
    A64 = check.bf16_bits_to_f64(A_bits)
    B64 = check.bf16_bits_to_f64(B_bits)
    Aa64, Ba64 = np.abs(A64), np.abs(B64)
    X = check.sign_vectors(23, maxd, 2)
    Xg = torch.from_numpy(X).cuda()
    # the Freivalds check needs O(MK + KN) host work per shape with nothing shared between
    # random shapes: a seeded sixteenth of the shapes gets it; every shape gets the sampled entries
    frei = set(np.random.default_rng(5).choice(len(shapes), size=len(shapes) // 16, replace=False).tolist())
    say("off-grid table in %.1f s" % (time.time() - t0))
    ctx.set_table(table)
    rep = Report(BF16)
    leaves = 0
    try:
        for i, (M, N, K) in enumerate(shapes):
            Cv = C[: M * N].view(M, N)
            ctx.gemm(A[: M * K].view(M, K), B[: K * N].view(K, N), Cv, mode=sg.MODE_DP)
            leaves += table.plan_leaves(M, N, K)
            rows = sample_index(31 * i + 1, M)
            cols = sample_index(37 * i + 2, N)
            y, s = device_reduce(torch, Cv, Xg, torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda())
            full = Cv.cpu() if M * N * K <= FULL_LIMIT else None
            Af = A64[: M * K].reshape(M, K)
            Bf = B64[: K * N].reshape(K, N)
            Aa = Aa64[: M * K].reshape(M, K)
            Ba = Ba64[: K * N].reshape(K, N)
            s = s.cpu().numpy()
            if i in frei:
                check_one(torch, rep, Af, Bf, X[:N], y.cpu().numpy(), rows, cols, s, full, (M, N, K), Aa, Ba)
            else:
                # sampled entries (and every entry when small) without the row check
                Cb, Db = Af[rows] @ Bf[:, cols], Aa[rows] @ Ba[:, cols]
                e, zv = check.entries_ratio(s, Cb, Db)
                rep.add("samp", e, (M, N, K))
                rep.zero_viol += zv
                if full is not None:
                    from pool_verify import full_ratio
                    e, zv = full_ratio(torch, full, *check.reference_block(Af, Bf))
                    rep.add("full", e, (M, N, K))
                    rep.zero_viol += zv
                    rep.full_outputs += 1
                rep.outputs += 1
            if (i + 1) % 512 == 0:
                say("off-grid %d / %d: %s" % (i + 1, len(shapes), rep))
    finally:
        ctx.set_table(None)
    say("off-grid: %s; %d plan leaves for %d shapes (%.1f s)" % (rep, leaves, len(shapes), time.time() - t0))
    assert rep.outputs == 4096 and leaves > 4096
    assert rep.ok(), str(rep)


def _config4_groups():
    """The grouped benchmark's problem list: 512 groups x 64 GEMMs, M, N, K log-uniform over
    [64, 4096] rounded to multiples of 8 (seed 4), operands at seeded 8-aligned offsets of two
    2^26-element pools."""
    rng = np.random.default_rng(4)
    pool = 1 << 26

    def dim():
        return int(np.clip(8 * np.round(np.exp(rng.uniform(np.log(64), np.log(4096))) / 8), 64, 4096))

    groups = []
    for g in range(512):
        probs = []
        for j in range(64):
            M, N, K = dim(), dim(), dim()
            oa = int(rng.integers(0, (pool - M * K) // 8 + 1)) * 8
            ob = int(rng.integers(0, (pool - K * N) // 8 + 1)) * 8
            probs.append((M, N, K, oa, ob))
        groups.append(probs)
    return pool, groups


@pytest.mark.timeout(900)
def test_grouped_config4_sixteenth_at_full_size(ctx):
    import torch
    t0 = time.time()
    pool, groups = _config4_groups()
    A_bits = synth.uniform_bf16(4, synth.STREAM_A, 1, pool).ravel()
    B_bits = synth.uniform_bf16(4, synth.STREAM_B, 1, pool).ravel()
    A, B = _upload(A_bits), _upload(B_bits)
    A64, B64 = check.bf16_bits_to_f64(A_bits), check.bf16_bits_to_f64(B_bits)
    X = check.sign_vectors(29, 4096, 2)
    Xg = torch.from_numpy(X).cuda()
    rep = Report(BF16)
    tiles = []
    for gi in range(0, 512, 16):
        probs = groups[gi]
        Cs = [torch.full((M, N), float("nan"), dtype=torch.bfloat16, device="cuda") for (M, N, K, oa, ob) in probs]
        full = [(M, N, K, A.data_ptr() + 2 * oa, K, B.data_ptr() + 2 * ob, N, Cc.data_ptr(), N)
                for (M, N, K, oa, ob), Cc in zip(probs, Cs)]
        plan = sg.GroupPlan(ctx, full, BF16)          # autotuned schedule
        tiles.append(plan.info()["tile"])
        plan.launch()
        torch.cuda.synchronize()
        for j, ((M, N, K, oa, ob), Cc) in enumerate(zip(probs, Cs)):
            rows, cols = sample_index(gi * 64 + j, M), sample_index(gi * 64 + j + 7, N)
            y, s = device_reduce(torch, Cc, Xg, torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda())
            Af = A64[oa: oa + M * K].reshape(M, K)
            Bf = B64[ob: ob + K * N].reshape(K, N)
            check_one(torch, rep, Af, Bf, X[:N], y.cpu().numpy(), rows, cols, s.cpu().numpy(),
                      Cc.cpu() if M * N * K <= FULL_LIMIT else None, (gi, j, M, N, K))
        plan.close()
        del Cs
    say("grouped 1/16 of config 4: %s; tiles %s (%.1f s)" % (rep, np.bincount(tiles, minlength=7).tolist(),
                                                             time.time() - t0))
    assert rep.outputs == 32 * 64
    assert rep.ok(), str(rep)


@pytest.mark.timeout(900)
def test_served_requests_at_serving_weight_shapes(ctx):
    import torch
    from gpu_helpers import device_bytes
    t0 = time.time()
    WSEED, ASEED = 5, 5
    shapes = [(4096, 4096), (4096, 11008), (11008, 4096), (4096, 14336)]     # (K, N)
    host = [synth.normal_bf16(WSEED, 100 + i, K, N, 0.02) for i, (K, N) in enumerate(shapes)]
    ws = [_upload(h) for h in host]
    W64 = [check.bf16_bits_to_f64(h) for h in host]
    X = check.sign_vectors(41, 14336, 2)
    Xg = torch.from_numpy(X).cuda()
    srv = sg.Server(ctx, [(K, N, t.data_ptr(), N) for (K, N), t in zip(shapes, ws)],
                    hbm_budget=24 << 30, max_inflight=4, max_group=64, mode=sg.SERVE_GROUPED,
                    tile=3, keep_results=True, max_m=8192, seed=ASEED)
    rng = np.random.default_rng(43)
    n_req = 200
    reqs = []
    for i in range(n_req):
        M = int(min(8192, max(1, round(float(np.exp(rng.uniform(0, np.log(8192))))))))
        reqs.append((i, M, int(rng.integers(0, 4))))
    for (i, M, w) in reqs:
        srv.submit(i, M, w)
    rep = Report(BF16)
    done, t_end = 0, time.time() + 600
    while done < n_req and time.time() < t_end:
        for c in srv.poll(64):
            assert c.status == 0
            M, N, K, w = c.M, c.N, c.K, c.weight
            A_req = device_bytes(c.A, M * K * 2).view(np.uint16).reshape(M, K)
            want = synth.f32_to_bf16_bits(synth.normal_f32(ASEED, 0, M * K, 0.02, start=c.a_offset)).reshape(M, K)
            assert np.array_equal(A_req, want), "staged activation differs from the seeded pool"
            # the served output, copied off the server's memory before release
            Cs = _upload(device_bytes(c.C, M * N * 2).view(np.uint16)).view(M, N)
            srv.release(c.ticket)
            dA = _upload(want)
            alone = torch.empty(M, N, dtype=torch.bfloat16, device="cuda")
            assert c.tile == (6 if M <= 64 else 3)
            ctx.gemm(dA.view(M, K), ws[w].view(K, N), alone, mode=sg.MODE_VARIANT, variant=4 * c.tile)
            torch.cuda.synchronize()
            assert torch.equal(alone.view(torch.int16), Cs.view(torch.int16)), "served result differs from alone"
            rows, cols = sample_index(1000 + c.id, M), sample_index(2000 + c.id, N)
            y, s = device_reduce(torch, Cs, Xg, torch.from_numpy(rows).cuda(), torch.from_numpy(cols).cuda())
            check_one(torch, rep, check.bf16_bits_to_f64(want), W64[w], X[:N], y.cpu().numpy(), rows, cols,
                      s.cpu().numpy(), Cs.cpu() if M * N * K <= FULL_LIMIT else None, (c.id, M, N, K))
            done += 1
    st = srv.stats()
    srv.close()
    say("served: %s; %d launches for %d requests (%.1f s)" % (rep, st["launches"], n_req, time.time() - t0))
    assert done == n_req and rep.outputs == n_req
    assert st["launches"] < n_req                 # requests arriving together share launches
    assert rep.ok(), str(rep)
