"""GPU tests of the continuous-batching server: results alone vs served, admission, errors."""
import numpy as np
import pytest

import synth
from gpu_helpers import TOL, check_tol, device_bytes, say

pytestmark = pytest.mark.gpu
sg = pytest.importorskip("paper_2605_29752_amd")
BF16 = 1
WSEED, ASEED = 77, 5


@pytest.fixture(scope="module")
def ctx():
    return sg.Context(0)


@pytest.fixture(scope="module")
def weights():
    import torch
    shapes = [(256, 384), (512, 256), (128, 1024)]     # (K, N)
    ws, host = [], []
    for i, (K, N) in enumerate(shapes):
        t = torch.empty(K * N, dtype=torch.bfloat16, device="cuda")
        sg.fill_bf16(t, WSEED, 100 + i, kind=1, scale=0.02)
        ws.append(t)
        host.append(synth.normal_bf16(WSEED, 100 + i, K, N, 0.02))
    torch.cuda.synchronize()
    assert all(np.array_equal(sg.bf16_tensor_bits(t).reshape(h.shape), h) for t, h in zip(ws, host))
    return shapes, ws, host


def _serve_and_check(ctx, weights, mode, budget, n_req=60, max_group=8, solo_m=0,
                     tiles_from_table=False, expect_tile=lambda M: 6 if M <= 64 else 3):
    import torch
    shapes, ws, host = weights
    srv = sg.Server(ctx, [(K, N, t.data_ptr(), N) for (K, N), t in zip(shapes, ws)],
                    hbm_budget=budget, max_inflight=2, max_group=max_group, mode=mode, tile=3,
                    keep_results=True, max_m=600, seed=ASEED, solo_m=solo_m,
                    tiles_from_table=tiles_from_table)
    rng = np.random.default_rng(1)
    for i in range(n_req):
        srv.submit(i, int(rng.integers(1, 601)), int(rng.integers(0, len(shapes))))
    # results stay allocated until released, so the client copies them out as they finish
    import time
    comps, t_end = [], time.time() + 120
    while len(comps) < n_req and time.time() < t_end:
        for c in srv.poll(256):
            A = device_bytes(c.A, c.M * c.K * 2).view(np.uint16).reshape(c.M, c.K)
            Cb = device_bytes(c.C, c.M * c.N * 2).view(np.uint16).reshape(c.M, c.N)
            comps.append((c.M, c.N, c.K, c.weight, c.status, c.a_offset, A, Cb, c.tile, c.group_size))
            srv.release(c.ticket)
    assert len(comps) == n_req and all(c[4] == 0 for c in comps)
    st = srv.stats()
    assert st["peak_bytes"] <= budget and st["completed"] == n_req
    say("mode", mode, "launches", st["launches"], "peak bytes", st["peak_bytes"])
    for (M, N, K, w, status, a_offset, A, Cb, tile, gsize) in comps:
        assert tile == expect_tile(M)
        assert 1 <= gsize <= (max_group if mode == sg.SERVE_GROUPED else 1)
        if solo_m and M > solo_m:
            assert gsize == 1, 'a solo request was grouped'
        want_a = synth.f32_to_bf16_bits(synth.normal_f32(ASEED, 0, M * K, 0.02, start=a_offset)).reshape(M, K)
        assert np.array_equal(A, want_a), "staged activation differs from the seeded pool"
        # alone: the same tile shape through the per-call entry point
        alone = torch.empty(M, N, dtype=torch.bfloat16, device="cuda")
        ctx.gemm(sg.to_device_bf16(A), ws[w].view(K, N), alone, mode=sg.MODE_VARIANT, variant=4 * tile)
        torch.cuda.synchronize()
        assert np.array_equal(sg.bf16_tensor_bits(alone), Cb), "served result differs from alone"
        check_tol(synth.bf16_bits_to_f32(Cb).astype(np.float64), A, host[w], BF16)
    srv.close()
    st["Ms"] = [c[0] for c in comps]
    st["group_sizes"] = [c[9] for c in comps]
    return st


def test_served_equals_alone_grouped_tight_budget(ctx, weights):
    # 3 MiB holds only a few requests at once: admission must wait for completions
    st = _serve_and_check(ctx, weights, sg.SERVE_GROUPED, 3 << 20)
    assert st["launches"] < 60


def test_served_equals_alone_grouped_solo(ctx, weights):
    # requests with M > 300 launch on their own; the rest still share launches
    st = _serve_and_check(ctx, weights, sg.SERVE_GROUPED, 64 << 20, solo_m=300)
    n_solo = sum(1 for m in st["Ms"] if m > 300)
    assert 0 < n_solo < 60 and n_solo < st["launches"] <= 60


def test_served_equals_alone_tiles_from_table(ctx, weights):
    # a host-built dispatch table whose best variant changes with M (64x64 for M <= 128,
    # 128x128 up to 384, 256x128 above): requests take those tile classes, and a served
    # result still equals the same tile alone
    n_m, n_n, n_k = 5, 8, 8
    T0 = np.ones((3, n_m, n_n, n_k))
    best = [0, 1, 1, 2, 2]
    for cm in range(n_m):
        T0[best[cm], cm] = 0.5
    t = sg.Table.from_t0(128, n_m, n_n, n_k, T0, [24, 12, 4])
    tile_of = {0: 6, 1: 3, 2: 1}
    ctx.set_table(t)
    try:
        st = _serve_and_check(ctx, weights, sg.SERVE_GROUPED, 64 << 20, tiles_from_table=True,
                              expect_tile=lambda M: tile_of[best[min(n_m - 1, (M + 127) // 128 - 1)]])
    finally:
        ctx.set_table(None)
        t.close()
    assert st["completed"] == 60
    # without a table on the context the option is refused
    shapes, ws, host = weights
    with pytest.raises(sg.SGError) as e:
        sg.Server(ctx, [(K, N, w.data_ptr(), N) for (K, N), w in zip(shapes, ws)], hbm_budget=8 << 20,
                  max_m=600, seed=ASEED, tiles_from_table=True)
    assert e.value.code == sg.SG_ENOTABLE


def test_served_equals_alone_per_request(ctx, weights):
    st = _serve_and_check(ctx, weights, sg.SERVE_PER_REQUEST, 64 << 20, n_req=30)
    assert st["launches"] == 30


def test_server_rejects_and_errors(ctx, weights):
    shapes, ws, host = weights
    srv = sg.Server(ctx, [(K, N, t.data_ptr(), N) for (K, N), t in zip(shapes, ws)],
                    hbm_budget=2 << 20, queue_cap=2, max_m=600, seed=ASEED)
    with pytest.raises(sg.SGError) as e:
        srv.submit(0, 601, 0)
    assert e.value.code == sg.SG_EINVAL
    with pytest.raises(sg.SGError):
        srv.submit(0, 10, 7)
    codes = []
    for i in range(200):
        try:
            srv.submit(i, 600, 2)
        except sg.SGError as ex:
            codes.append(ex.code)
    assert sg.SG_EAGAIN in codes
    srv.drain(60.0)
    srv.close()


def test_poisson_smoke(ctx, weights):
    shapes, ws, host = weights
    srv = sg.Server(ctx, [(K, N, t.data_ptr(), N) for (K, N), t in zip(shapes, ws)],
                    hbm_budget=256 << 20, max_m=600, seed=ASEED)
    rep = srv.serve_poisson(500.0, 1.0, 0.2, 3, max_m=600)
    say(rep)
    assert rep["failed"] == 0 and rep["measured"] > 100
    assert 0 < rep["p50_ms"] <= rep["p99_ms"]
    srv.close()


def test_closed_loop_saturation_smoke(ctx, weights):
    shapes, ws, host = weights
    for mode in (sg.SERVE_GROUPED, sg.SERVE_PER_REQUEST):
        srv = sg.Server(ctx, [(K, N, t.data_ptr(), N) for (K, N), t in zip(shapes, ws)],
                        hbm_budget=256 << 20, max_m=600, seed=ASEED, mode=mode)
        rep = srv.serve_closed(32, 1.0, 0.2, 3, max_m=600)
        say(mode, rep)
        assert rep["failed"] == 0 and rep["measured"] > 50 and rep["req_per_s"] > 0
        assert 0 < rep["p50_ms"] <= rep["p99_ms"]
        if mode == sg.SERVE_GROUPED:
            assert rep["launches"] < rep["offered"]      # 32 outstanding requests share launches
        srv.close()
