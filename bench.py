#!/usr/bin/env python
"""Landscape benchmark of the smoothed BF16 NN GEMM stack on one MI355X.

Workload: every (M, N, K) in {128, 256, ..., 4096}^3 (32,768 shapes), BF16 inputs drawn
uniform[-1, 1] (seeded), FP32 accumulation, BF16 output.  Operands are views of one resident
4096 x 4096 pool per operand (A is the first M*K elements with lda = K, B the first K*N with
ldb = N).

Set-up (untimed): measure T0 for every variant of the tile family at every shape (randomized
order, warm-ups, one discarded and `reps` timed launches per shape), then build the dispatch
table (best-of-N, T1 pad, T2 split + pad).
Timed step: one run of every one of the 32,768 shapes' plans, executed through the dispatch
table.  The steps are taken in passes over the shapes in the same randomized order, each pass
giving a shape one untimed run and then `reps` consecutive timed runs of its plan (the table's
own protocol), so `steps` = 20 is four passes.

Prints one JSON line: mean TFLOPs over the 32,768 shapes of the executed smoothed stack, with
roughness and the other stacks (plain single tile, best-of-N, DP as predicted by the table)
beside it, the roofline of the dominant kernel and the FP64 oracle's CPU rate.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_BF16_TFLOPS = 2516.6       # MI355X dense BF16 MFMA (256 CUs x 4096 FLOP/clk x 2.4 GHz)
# The measured variant set (best-of-N's N = 16 of the 32): 13 of tiles 0-6 chosen by greedy
# forward selection of best-of-set mean TFLOPs over a seeded sample of 1,024 landscape cells with
# every variant timed (all 28 reached 476.0 there, these 13 475.8), plus the deep-K 64x64 tile
# without split and with 2 and 4 splits, which win shapes with few tiles (1024^3: 264 against
# 213; 1024 x 1024 x 4096: 411 against 381).  256x256 (variant 0) is the paper's default tile,
# reported beside the plain stack.
DEFAULT_VARIANTS = "0,4,8,12,13,14,16,20,21,22,24,26,27,28,29,30"


T_START = time.perf_counter()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def elapsed() -> float:
    """Seconds since the benchmark process started."""
    return time.perf_counter() - T_START


def ramp_texture(tf):
    """Split the roughness of an (M, N, K) TFLOPs landscape into its ramp and its texture, per
    axis and as the 3-D mean.  Along one line T_0 .. T_{n-1}, sum |T_{i+1} - T_i| is at least
    |T_{n-1} - T_0|, with equality exactly when the line is monotone: the ramp part
    |T_{n-1} - T_0| / (n - 1) is the roughness of the smoothest line with those end points (the
    paper's unavoidable wave-fill ramp is of this kind), and the texture -- roughness minus
    ramp -- is what the line's ups and downs add to it, the part tile selection and the DP can
    remove.  Both are averaged over lines like the roughness."""
    tf = np.asarray(tf, dtype=np.float64)
    out = {}
    for name, axis in (("m", 0), ("n", 1), ("k", 2)):
        t = np.moveaxis(tf, axis, -1)
        n = t.shape[-1]
        rough = np.abs(np.diff(t, axis=-1)).sum(axis=-1) / (n - 1)
        ramp = np.abs(t[..., -1] - t[..., 0]) / (n - 1)
        out["ramp_" + name] = float(ramp.mean())
        out["texture_" + name] = float((rough - ramp).mean())
    out["ramp_3d"] = (out["ramp_m"] + out["ramp_n"] + out["ramp_k"]) / 3.0
    out["texture_3d"] = (out["texture_m"] + out["texture_n"] + out["texture_k"]) / 3.0
    return out


def stack_stats(sg, sec, sizes):
    """Per-shape seconds [nM, nN, nK] -> mean/peak/roughness (3-D and the K = max slice)."""
    M = sizes[:, None, None]
    N = sizes[None, :, None]
    K = sizes[None, None, :]
    tf = 2.0 * M * N * K / (sec * 1e12)
    st = sg.landscape_stats(tf)
    sl = tf[:, :, -1]
    slice_rough = float(np.mean([sg.roughness(row) for row in sl]))
    rt = ramp_texture(tf)
    return {"mean_tflops": st["mean"], "peak_tflops": st["peak"],
            "roughness_3d": st["roughness_3d"], "roughness_n": st["roughness_n"],
            "roughness_m": st["roughness_m"], "roughness_k": st["roughness_k"],
            "ramp_3d": rt["ramp_3d"], "texture_3d": rt["texture_3d"],
            "slice_k%d_mean" % int(sizes[-1]): float(sl.mean()),
            "slice_k%d_roughness_n" % int(sizes[-1]): slice_rough,
            "frac_of_peak_mean": st["mean"] / PEAK_BF16_TFLOPS,
            # roughness as a share of the dense peak per grid step (the paper quotes 14.4 % ->
            # 4.3 % of its peak per step on its K = 4096 slice)
            "slice_roughness_frac_of_peak": slice_rough / PEAK_BF16_TFLOPS,
            "roughness_3d_frac_of_peak": st["roughness_3d"] / PEAK_BF16_TFLOPS}


def first_principles(sg, stack_secs, sizes, step, n):
    """The grid's ideal ceiling and first-principles optimal (paper Sec. 9: MI355X datasheet
    integers, tiles {256, 128, 64}, BF16 output) and each stack's Kernel Optimality Level against
    the optimal (Sec. 10), on the K = max slice (the paper's grading) and over the whole grid."""
    M = sizes[:, None, None]
    N = sizes[None, :, None]
    K = sizes[None, None, :]
    ideal = sg.ideal_landscape(step, n, n, n, tile=256)
    opt = sg.optimal_landscape(step, n, n, n, tiles=(256, 128, 64), c_bytes=2)
    out = {"hw": sg.MI355X, "tiles": [256, 128, 64],
           "ideal": {k: v for k, v in sg.landscape_stats(ideal).items() if k in ("mean", "roughness_n", "roughness_3d")},
           "optimal": {k: v for k, v in sg.landscape_stats(opt).items() if k in ("mean", "roughness_n", "roughness_3d")},
           "kol": {}}
    out["ideal"]["slice_mean"] = float(ideal[:, :, -1].mean())
    out["optimal"]["slice_mean"] = float(opt[:, :, -1].mean())
    for name, sec in stack_secs.items():
        tf = 2.0 * M * N * K / (sec * 1e12)
        out["kol"][name] = {"slice": sg.kol_grade(tf[:, :, -1], opt[:, :, -1]), "grid": sg.kol_grade(tf, opt)}
    return out


def kernel_name(sg, v: int) -> str:
    """Name of the direct-to-LDS tile kernel that variant v launches on aligned operands (as a
    profiler lists it)."""
    vi = sg.variant_info(v)
    if vi.bk == 128:
        return "sg_gemm_tile_dma_k128<%d, %d>" % (vi.bm, vi.bn)
    return "sg_gemm_tile_dma<%d, %d>" % (vi.bm, vi.bn)


def kernel_source_hash() -> str:
    """SHA-1 of the tile kernels' source with comments and whitespace removed, so that only a
    change of the code itself retires recorded counter figures."""
    import hashlib
    import re
    h = hashlib.sha1()
    for f in ("tile_body.h", "tile_body_dma.h", "gemm_tile.hip"):
        text = open(os.path.join(ROOT, "paper_2605_29752_amd", "csrc", f)).read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(re.sub(r"\s+", " ", text).strip().encode())
    return h.hexdigest()


def traffic_bytes(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it was taken on
    the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic_landscape_sweep.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("kernel") != kernel or t.get("source_sha1") != kernel_source_hash():
        return None
    return t["hbm_bytes_per_launch"]


def _cpu_worker(job):
    """One worker of the CPU baseline: the FP64 oracle on its shapes until the deadline."""
    import oracle
    import synth
    shapes, seed, deadline = job
    a_pool = synth.uniform_bf16(seed, synth.STREAM_A, 1, 4096 * 4096).ravel()
    b_pool = synth.uniform_bf16(seed, synth.STREAM_B, 1, 4096 * 4096).ravel()
    done = []
    for (m, n, k) in shapes:
        if time.time() > deadline and done:
            break
        t0 = time.perf_counter()
        oracle.gemm_f64(a_pool[:m * k].reshape(m, k), b_pool[:k * n].reshape(k, n), want_d=False)
        done.append((m, n, k, time.perf_counter() - t0))
    return done


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds_budget: float, seed: int):
    """The FP64 oracle, untuned (a plain single-threaded loop), run in one process per host core
    (at most 16) on a bounded seeded sample of the landscape: one process takes the K = 4096,
    M = 4096 slice's smallest shape (4096 x 128 x 4096), the others seeded grid shapes with
    M N K <= 2^25, until the time budget.  value = total FLOP / wall time."""
    import multiprocessing as mp
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    rng = np.random.default_rng(seed)
    sizes = np.arange(128, 4097, 128)
    cand = [(int(m), int(n), int(k)) for m in sizes for n in sizes for k in sizes if m * n * k <= (1 << 25)]
    order = rng.permutation(len(cand))
    lists = [[] for _ in range(cores)]
    lists[0].append((4096, 128, 4096))
    for t, idx in enumerate(order):
        lists[(t % (cores - 1)) + 1 if cores > 1 else 0].append(cand[idx])
    t_start = time.time()
    deadline = t_start + seconds_budget
    with mp.get_context("fork").Pool(cores) as pool:
        parts = pool.map(_cpu_worker, [(l, seed, deadline) for l in lists])
    wall = time.time() - t_start
    done = [d for p in parts for d in p]
    flops = sum(2.0 * m * n * k for m, n, k, _ in done)
    per_shape = [2.0 * m * n * k / t / 1e12 for m, n, k, t in done]
    slice_done = [d for d in parts[0] if d[:3] == (4096, 128, 4096)]
    return {"value": flops / wall / 1e12, "unit": "TFLOPs", "cores": cores, "kind": "oracle",
            "cpu_model": cpu_model(), "os_cpu_count": os.cpu_count(),
            "sample": "%d shapes (4096x128x4096 from the K = 4096, M = 4096 slice, plus seeded grid shapes "
                      "with M*N*K <= 2^25), plain FP64 C loop, one process per core on %d cores, %.1f s wall; "
                      "value = total FLOP / wall time" % (len(done), cores, wall),
            "per_core_mean_tflops": float(np.mean(per_shape)) if per_shape else None,
            "slice_shape_seconds": slice_done[0][3] if slice_done else None}


def percentile(x, q: float) -> float:
    """Nearest-rank percentile (q in (0, 1]) of a sample."""
    v = np.sort(np.asarray(x, dtype=np.float64))
    k = min(max(int(np.ceil(q * v.size)), 1), v.size)
    return float(v[k - 1])


def run_grouped(args, sg, torch, ctx, stream, reps=None):
    """Config 4: 512 groups x 64 GEMMs, log-uniform dims in [64, 4096] rounded to multiples of 8;
    one persistent grouped launch per group with an autotuned schedule (tile, grid, queue
    order), all 512 captured in one hipGraph, against the same problems as 64 separate per-call
    launches per group: best-of-N (the table's per-shape best variant) and the DP plans when the
    context holds a table, else the group's own tile.  Latency per group: each group's launch
    (grouped) or its 64 calls (per call) bracketed by events on the stream."""
    rng = np.random.default_rng(4)
    G, NG = 64, args.groups
    reps = args.steps if reps is None else reps

    def dim():
        return int(np.clip(8 * np.round(np.exp(rng.uniform(np.log(64), np.log(4096))) / 8), 64, 4096))

    pool = 1 << 26
    A = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    B = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    sg.fill_bf16(A, 4, 0)
    sg.fill_bf16(B, 4, 1)
    Cs = [torch.empty(4096 * 4096, dtype=torch.bfloat16, device="cuda") for _ in range(G)]
    groups, flops = [], 0.0
    for g in range(NG):
        probs = []
        for j in range(G):
            M, N, K = dim(), dim(), dim()
            oa = int(rng.integers(0, (pool - M * K) // 8 + 1)) * 8
            ob = int(rng.integers(0, (pool - K * N) // 8 + 1)) * 8
            probs.append((M, N, K, A.data_ptr() + 2 * oa, K, B.data_ptr() + 2 * ob, N, Cs[j].data_ptr(), N))
            flops += 2.0 * M * N * K
        groups.append(probs)
    gflops = np.array([sum(2.0 * p[0] * p[1] * p[2] for p in pr) for pr in groups])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plans = [sg.GroupPlan(ctx, pr, sg.BF16, stream=stream) for pr in groups]
    tune_s = time.perf_counter() - t0
    infos = [p.info() for p in plans]
    tiles = [i["tile"] for i in infos]
    cfgs = {}
    for i in infos:
        key = "%s grid %d order %s" % (sg.variant_info(4 * i["tile"]).name[:-6], i["grid_wgs"],
                                       "lpt" if i["order"] == 0 else "given")
        cfgs[key] = cfgs.get(key, 0) + 1
    res = {"groups": NG, "problems_per_group": G, "flops": flops, "autotune_s": tune_s,
           "tile_histogram": np.bincount(tiles, minlength=7).tolist(), "schedules": cfgs}
    if ctx._table is not None:
        # the schedules were recorded in the table: planning the same groups again is a lookup
        t0 = time.perf_counter()
        again = [sg.GroupPlan(ctx, pr, sg.BF16, stream=stream) for pr in groups]
        res["replan_from_table_s"] = time.perf_counter() - t0
        res["table_group_schedules"] = ctx._table.group_schedules()
        for p in again:
            p.close()
    log("grouped: autotuned %d groups in %.1f s; tiles %s" % (NG, tune_s, res["tile_histogram"]))
    graph = sg.Graph(plans, stream)

    def timed(fn, n):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ts = []
        for _ in range(n):
            e0.record(stream)
            fn()
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) * 1e-3)
        return float(np.mean(ts))

    def per_group(launch):
        """Seconds of each group, launched one after another, each between two events."""
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(NG)]
        for gi in range(NG):
            ev[gi][0].record(stream)
            launch(gi)
            ev[gi][1].record(stream)
        torch.cuda.synchronize()
        return np.array([a.elapsed_time(b) * 1e-3 for a, b in ev])

    arrs = [sg._problems(pr) for pr in groups]
    t_graph = timed(lambda: graph.launch(stream), reps)
    t_plans = timed(lambda: [p.launch(stream) for p in plans], reps)
    lat_g = per_group(lambda gi: plans[gi].launch(stream))
    res.update({"graph_tflops": flops / t_graph / 1e12, "grouped_no_graph_tflops": flops / t_plans / 1e12,
                "graph_s": t_graph,
                "grouped_latency_ms": {"p50": percentile(lat_g, 0.5) * 1e3, "p99": percentile(lat_g, 0.99) * 1e3,
                                       "mean": float(lat_g.mean()) * 1e3}})
    base = [("same_tile", sg.MODE_VARIANT, None)]
    if ctx._table is not None:
        base = [("best_of_n", sg.MODE_BEST, 0), ("dp", sg.MODE_DP, 0)] + base
    for name, mode, var in base:
        vs = [4 * t for t in tiles] if var is None else [var] * NG
        n_rep = max(2, min(reps, 3))
        t_call = timed(lambda: [sg.gemm_batch(ctx, pr, sg.BF16, mode, v, stream, _arr=a)
                                for pr, v, a in zip(groups, vs, arrs)], n_rep)
        lat_c = per_group(lambda gi: sg.gemm_batch(ctx, groups[gi], sg.BF16, mode, vs[gi], stream, _arr=arrs[gi]))
        res["percall_%s_tflops" % name] = flops / t_call / 1e12
        res["percall_%s_latency_ms" % name] = {"p50": percentile(lat_c, 0.5) * 1e3,
                                               "p99": percentile(lat_c, 0.99) * 1e3,
                                               "mean": float(lat_c.mean()) * 1e3}
        res["speedup_vs_percall_%s" % name] = t_call / t_graph
    res["group_gflop"] = {"p50": percentile(gflops, 0.5) / 1e9, "p99": percentile(gflops, 0.99) / 1e9}
    graph.close()
    for p in plans:
        p.close()
    del Cs, A, B
    return res


def sawtooth(tf, Ns, tile_n):
    """Sawtooth of a fine-N TFLOPs line (Sec. 8.3, Table 13).  The line is detrended by a centred
    moving average over one tile width; then
      * period: the shortest lag (a multiple of the N step, 64..512) whose autocorrelation of the
        detrended line is within 90 % of the highest;
      * valley residue: the N mod tile_n whose detrended mean is lowest, and its depth (TFLOP/s
        below the line's mean);
      * valleys: strict interior local minima, their median spacing and the share of them at the
        valley residue."""
    tf = np.asarray(tf, dtype=np.float64)
    step = int(Ns[1] - Ns[0])
    w = max(3, tile_n // step)
    pad = np.pad(tf, (w, w), mode="edge")
    trend = np.convolve(pad, np.ones(2 * w + 1) / (2 * w + 1), mode="same")[w:-w]
    d = tf - trend
    lags = [L for L in range(64, 513, step) if L // step < len(d) - 4]
    ac = [float(np.corrcoef(d[:-(L // step)], d[L // step:])[0, 1]) for L in lags]
    # the fundamental: the shortest lag within 90 % of the best correlation (a multiple of the
    # period correlates as well as the period itself)
    period = min(L for L, c in zip(lags, ac) if c >= 0.9 * max(ac)) if lags else None
    res = (np.asarray(Ns) % tile_n).astype(int)
    prof = {int(r): float(d[res == r].mean()) for r in np.unique(res)}
    vres = min(prof, key=prof.get)
    v = [i for i in range(1, len(tf) - 1) if tf[i] < tf[i - 1] and tf[i] < tf[i + 1]]
    share = (sum(1 for i in v if int(Ns[i]) % tile_n == vres) / len(v)) if v else None
    return {"period": period, "period_autocorr": max(ac) if ac else None,
            "valley_residue": vres, "valley_depth": -prof[vres], "valleys": len(v),
            "valley_spacing_median": float(np.median(np.diff([Ns[i] for i in v]))) if len(v) > 1 else None,
            "valleys_at_residue": share}


def run_finen(args, sg, torch, ctx, stream):
    """Sec. 8.3-8.4 on MI355X: fine-N sweeps (M = K = 4096, N = 32..4096 step 32) of every tile and
    of the best-of-N envelope; sawtooth period and valley position per tile (Table 13); the DP's
    T0 -> T1 (pad) and T2 (split + pad) applied to each line (Table 14)."""
    M = K = 4096
    step, n = 32, 128
    Ns = np.arange(1, n + 1) * step
    pool = 4096 * 4096
    A = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    B = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    C = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    sg.fill_bf16(A, 2, 0)
    sg.fill_bf16(B, 2, 1)
    torch.cuda.synchronize()
    variants = [int(v) for v in args.variants.split(",")]
    order = np.random.default_rng(args.order_seed).permutation(n)
    shapes = [(M, int(Ns[i]), K) for i in order]
    T0 = np.zeros((len(variants), n))
    for r, v in enumerate(variants):
        sec = ctx.sweep(shapes, A, B, C, mode=sg.MODE_VARIANT, variant=v, c_dtype=sg.BF16,
                        warmup=args.shape_warmup, reps=args.reps, stream=stream)
        T0[r, order] = sec
    fl = 2.0 * M * Ns * K

    def line_stats(rows, vids):
        t = sg.Table.from_t0(step, 1, n, 1, rows.reshape(len(vids), 1, n, 1), vids)
        t0, t1, t2 = (t.values(w).reshape(n) for w in (0, 1, 2))
        out = {}
        for name, sec in (("T0", t0), ("T1", t1), ("T2", t2)):
            tf = fl / sec / 1e12
            out[name] = {"mean": float(tf.mean()), "min": float(tf.min()), "roughness": sg.roughness(tf)}
        out["T1_roughness_reduction"] = 1.0 - out["T1"]["roughness"] / out["T0"]["roughness"]
        out["T2_roughness_reduction"] = 1.0 - out["T2"]["roughness"] / out["T0"]["roughness"]
        return out, fl / t0 / 1e12

    res = {"M": M, "K": K, "N": "32..4096 step 32", "tiles": {}}
    seen = set()
    for r, v in enumerate(variants):
        vi = sg.variant_info(v)
        if vi.splits != 1 or (vi.bm, vi.bn, vi.bk) in seen:
            continue
        seen.add((vi.bm, vi.bn, vi.bk))
        st, tf = line_stats(T0[r:r + 1], [v])
        st.update(sawtooth(tf, Ns, vi.bn))
        st["tile"] = "%dx%d" % (vi.bm, vi.bn)
        res["tiles"][vi.name] = st
        log("fine-N %s: mean %.1f, roughness %.2f -> T1 %.2f; period %s, valleys at N mod %d = %s"
            % (vi.name, st["T0"]["mean"], st["T0"]["roughness"], st["T1"]["roughness"], st["period"],
               vi.bn, st["valley_residue"]))
    env, tf = line_stats(T0, variants)
    env.update(sawtooth(tf, Ns, 128))
    res["best_of_%d" % len(variants)] = env
    return res


def stream_bandwidth(torch, mib: int = 1024) -> float:
    """Measured streaming bandwidth (GB/s): a plain device copy of `mib` MiB, best of five,
    counting the bytes read and written."""
    src = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    best = float("inf")
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1) * 1e-3)
    del src, dst
    return 2.0 * (mib << 20) / best / 1e9


def run_decomp(args, sg, torch, ctx, stream):
    """Sec. 4 on MI355X: the four surfaces over the landscape grid for each tile kernel (its
    one-split variant) -- GEMM time (the kernel), memory time (its memory-only twin: the same
    loads, waits and stores with no matrix-core work, at the same occupancy), compute time
    2MNK / peak and overhead = GEMM - max(compute, memory); the stacked view along N at
    M = K = 4096 (Fig. 6); the compute-/memory-bound split against the HBM specification, a
    measured streaming bandwidth and the measured memory time (Table 3)."""
    step, n = args.step, args.n
    sizes = np.arange(1, n + 1) * step
    pool = int(sizes[-1]) ** 2
    A = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    B = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    C = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    sg.fill_bf16(A, args.seed, 0)
    sg.fill_bf16(B, args.seed, 1)
    torch.cuda.synchronize()
    bw_stream = stream_bandwidth(torch)
    log("streaming copy bandwidth %.0f GB/s" % bw_stream)
    grid = [(int(m), int(nn), int(k)) for m in sizes for nn in sizes for k in sizes]   # K fastest
    order = np.random.default_rng(args.order_seed).permutation(len(grid))
    shapes = [grid[i] for i in order]
    Mg, Ng, Kg = (np.array([s[a] for s in grid], dtype=np.float64).reshape(n, n, n) for a in range(3))
    traffic = 2.0 * Mg * Kg + 2.0 * Kg * Ng + 2.0 * Mg * Ng
    variants = [int(v) for v in args.variants.split(",")]
    res = {"grid": "{%d..%d}^3 step %d" % (step, step * n, step), "stream_bw_gbs": bw_stream,
           "spec_bw_gbs": sg.MI355X["bw_gbs"], "peak_tflops": sg.MI355X["peak_tflops"], "tiles": {}}
    seen = set()
    for v in variants:
        vi = sg.variant_info(v)
        if vi.splits != 1 or (vi.bm, vi.bn, vi.bk) in seen:
            continue
        seen.add((vi.bm, vi.bn, vi.bk))
        tg = np.empty(len(grid))
        tm = np.empty(len(grid))
        tg[order] = ctx.sweep(shapes, A, B, C, mode=sg.MODE_VARIANT, variant=v, c_dtype=sg.BF16,
                              warmup=args.shape_warmup, reps=args.reps, stream=stream)
        tm[order] = ctx.sweep(shapes, A, B, C, mode=sg.MODE_MEMORY, variant=v, c_dtype=sg.BF16,
                              warmup=args.shape_warmup, reps=args.reps, stream=stream)
        d = sg.decompose(grid, tg, tm, c_bytes=2)
        d_stream = sg.decompose(grid, tg, tm, c_bytes=2, hw=dict(sg.MI355X, bw_gbs=bw_stream))
        tc = d["t_compute"].reshape(n, n, n)
        to = d["t_overhead"].reshape(n, n, n)
        tg3, tm3 = tg.reshape(n, n, n), tm.reshape(n, n, n)
        surf = {"compute": tc, "memory": tm3, "gemm": tg3, "overhead": to}
        # texture of each time surface: N-axis roughness (us per step) on the K = max slice and
        # over every line of the grid
        rough = {}
        for name, x in surf.items():
            us = x * 1e6
            rough[name] = {"slice_k_max": float(np.mean([sg.roughness(us[m, :, -1]) for m in range(n)])),
                           "grid": sg.landscape_stats(us)["roughness_n"]}
        line_share = to[-1, :, -1] / tg3[-1, :, -1]           # Fig. 6: M = K = max, N varies
        mem_dom = tm3[-1, :, -1] > tc[-1, :, -1]
        tiles_mn = np.ceil(Mg / vi.bm) * np.ceil(Ng / vi.bn)
        loaded = tiles_mn * Kg * (vi.bm + vi.bn) * 2.0          # operand bytes into LDS per run
        st = {
            "mean_us": {k: float(x.mean() * 1e6) for k, x in surf.items()},
            "overhead_share": d["overhead_share"],
            "overhead_share_median": float(np.median(to / tg3)),
            "compute_bound_spec_bw": d["cb_bandwidth"],
            "compute_bound_stream_bw": d_stream["cb_bandwidth"],
            "compute_bound_measured_memory": d["cb_measured"],
            "roughness_us_per_step": rough,
            "fig6_line": {"overhead_share_mean": float(line_share.mean()),
                          "overhead_share_min": float(line_share.min()),
                          "overhead_share_max": float(line_share.max()),
                          "memory_dominant_points": int(mem_dom.sum()),
                          "memory_dominant_up_to_n": int(sizes[mem_dom].max()) if mem_dom.any() else 0},
            "twin_min_traffic_gbs": {"mean": float((traffic / tm3).mean() / 1e9),
                                     "max": float((traffic / tm3).max() / 1e9)},
            "twin_lds_load_tbs": {"mean": float((loaded / tm3).mean() / 1e12),
                                  "max": float((loaded / tm3).max() / 1e12)},
        }
        res["tiles"][vi.name] = st
        log("decomposition %s: mean us gemm %.1f memory %.1f compute %.1f overhead %.1f; overhead share "
            "%.2f; compute-bound %.2f (spec BW) %.2f (stream BW) %.2f (measured memory)"
            % (vi.name, st["mean_us"]["gemm"], st["mean_us"]["memory"], st["mean_us"]["compute"],
               st["mean_us"]["overhead"], st["overhead_share"], st["compute_bound_spec_bw"],
               st["compute_bound_stream_bw"], st["compute_bound_measured_memory"]))
        if args.dump:
            np.savez(args.dump + ".%s.npz" % vi.name, t_gemm=tg3, t_memory=tm3, t_compute=tc, t_overhead=to)
    return res


# ---- statistics of the memory study (Sec. 5): ranks, rank correlation, spread, drift --------
def avg_ranks(x) -> np.ndarray:
    x = np.asarray(x, dtype=np.float64)
    order = np.argsort(x, kind="mergesort")
    pos = np.empty(len(x))
    pos[order] = np.arange(1, len(x) + 1)
    _, inv, cnt = np.unique(x, return_inverse=True, return_counts=True)
    return (np.bincount(inv, weights=pos) / cnt)[inv]        # ties share their mean position


def spearman(x, y) -> float:
    return float(np.corrcoef(avg_ranks(x), avg_ranks(y))[0, 1])


def median_cv(t, keys) -> float:
    """Median over keys of the coefficient of variation (population) of the times per key."""
    _, inv = np.unique(np.asarray(keys), axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    t = np.asarray(t, dtype=np.float64)
    cnt = np.bincount(inv)
    mean = np.bincount(inv, weights=t) / cnt
    var = np.bincount(inv, weights=t * t) / cnt - mean * mean
    return float(np.median(np.sqrt(np.maximum(var, 0.0)) / mean))


def revisit_drift(t, keys, run_order) -> float:
    """Mean over keys seen more than once of 1 - t(last run) / t(first run)."""
    _, inv = np.unique(np.asarray(keys), axis=0, return_inverse=True)
    inv = inv.reshape(-1)
    t = np.asarray(t, dtype=np.float64)
    o = np.asarray(run_order)
    srt = np.lexsort((o, inv))                      # by key, then run order
    k_s = inv[srt]
    first = np.r_[True, k_s[1:] != k_s[:-1]]
    last = np.r_[k_s[1:] != k_s[:-1], True]
    t_first, t_last = t[srt][first], t[srt][last]
    multi = (np.flatnonzero(last) - np.flatnonzero(first)) > 0
    return float(np.mean(1.0 - t_last[multi] / t_first[multi]))


def slowdown(t_co, t_iso) -> dict:
    r = np.asarray(t_co, dtype=np.float64) / np.asarray(t_iso, dtype=np.float64)
    return {"mean": float(r.mean()), "over_20": float((r > 1.2).mean()), "over_50": float((r > 1.5).mean())}


def run_memory(args, sg, torch, ctx, stream):
    """Sec. 5 on MI355X: FP32 buffer reads and writes over the landscape grid -- read A (M x K),
    read B (K x N), read C and write D (M x N) -- each in a buffer allocated alone per measurement
    (isolated) or alongside the other three (co-allocated), in randomized and in sequential
    (nested M, N, K loop) order.  Reports Table 4 (co-allocation slowdown), the load / store
    asymmetry, the warm-up drift and rank correlation with run order, and the spurious
    dependence of read-A time on N (Fig. 9)."""
    step, n = args.step, args.n
    sizes = np.arange(1, n + 1) * step
    grid = [(int(m), int(nn), int(k)) for m in sizes for nn in sizes for k in sizes]   # sequential
    G = np.array(grid, dtype=np.float64)
    order = np.random.default_rng(args.order_seed).permutation(len(grid))
    rnd = [grid[i] for i in order]
    e = 4
    nbytes = {sg.MEM_READ_A: G[:, 0] * G[:, 2] * e, sg.MEM_READ_B: G[:, 2] * G[:, 1] * e,
              sg.MEM_READ_C: G[:, 0] * G[:, 1] * e, sg.MEM_WRITE_D: G[:, 0] * G[:, 1] * e}
    opname = {sg.MEM_READ_A: "read_A", sg.MEM_READ_B: "read_B", sg.MEM_READ_C: "read_C",
              sg.MEM_WRITE_D: "write_D"}
    T = {}
    for op in (sg.MEM_READ_A, sg.MEM_READ_B, sg.MEM_READ_C, sg.MEM_WRITE_D):
        for alloc, an in ((sg.MEM_ISOLATED, "isolated"), (sg.MEM_COALLOC, "coalloc")):
            t = np.empty(len(grid))
            t[order] = ctx.mem_sweep(rnd, op, alloc, elem_bytes=e, warmup=args.shape_warmup,
                                     reps=args.reps, stream=stream)
            T[(opname[op], an, "random")] = t
            log("memory %s %s randomized: mean %.1f us" % (opname[op], an, t.mean() * 1e6))
    for op, alloc, an in ((sg.MEM_READ_A, sg.MEM_ISOLATED, "isolated"), (sg.MEM_READ_A, sg.MEM_COALLOC, "coalloc"),
                          (sg.MEM_READ_C, sg.MEM_ISOLATED, "isolated"), (sg.MEM_WRITE_D, sg.MEM_ISOLATED, "isolated")):
        T[(opname[op], an, "sequential")] = ctx.mem_sweep(grid, op, alloc, elem_bytes=e,
                                                          warmup=args.shape_warmup, reps=args.reps, stream=stream)
        log("memory %s %s sequential done" % (opname[op], an))
    run_rnd = np.empty(len(grid))
    run_rnd[order] = np.arange(len(grid))
    run_seq = np.arange(len(grid))
    MK = G[:, [0, 2]]
    bw = lambda op, key: float(np.mean(nbytes[op] / T[key]) / 1e9)
    res = {"grid": "{%d..%d}^3 step %d" % (step, step * n, step), "elem_bytes": e, "reps": args.reps}
    res["table4_coalloc_slowdown"] = {nm: slowdown(T[(nm, "coalloc", "random")], T[(nm, "isolated", "random")])
                                     for nm in ("read_A", "read_B", "read_C", "write_D")}
    res["load_store"] = {
        "randomized": {"read_C_gbs": bw(sg.MEM_READ_C, ("read_C", "isolated", "random")),
                       "write_D_gbs": bw(sg.MEM_WRITE_D, ("write_D", "isolated", "random"))},
        "sequential": {"read_C_gbs": bw(sg.MEM_READ_C, ("read_C", "isolated", "sequential")),
                       "write_D_gbs": bw(sg.MEM_WRITE_D, ("write_D", "isolated", "sequential"))}}
    for k in ("randomized", "sequential"):
        res["load_store"][k]["write_over_read"] = res["load_store"][k]["write_D_gbs"] / res["load_store"][k]["read_C_gbs"]
    res["warmup"] = {
        "sequential_isolated_read_A": {"spearman_run_order": spearman(T[("read_A", "isolated", "sequential")], run_seq),
                                       "revisit_drift": revisit_drift(T[("read_A", "isolated", "sequential")], MK, run_seq)},
        "randomized_isolated_read_A": {"spearman_run_order": spearman(T[("read_A", "isolated", "random")], run_rnd),
                                       "revisit_drift": revisit_drift(T[("read_A", "isolated", "random")], MK, run_rnd)}}
    res["read_A_vs_N"] = {}
    for label, key in (("coalloc_sequential", ("read_A", "coalloc", "sequential")),
                       ("isolated_sequential", ("read_A", "isolated", "sequential")),
                       ("isolated_randomized", ("read_A", "isolated", "random"))):
        res["read_A_vs_N"][label] = {"spearman_N": spearman(T[key], G[:, 1]), "median_cv_across_N": median_cv(T[key], MK),
                                     "mean_gbs": bw(sg.MEM_READ_A, key)}
    log("memory: co-allocation slowdown read A %.3f, write/read %.2f (randomized), read-A vs N rho %s"
        % (res["table4_coalloc_slowdown"]["read_A"]["mean"], res["load_store"]["randomized"]["write_over_read"],
           {k: round(v["spearman_N"], 3) for k, v in res["read_A_vs_N"].items()}))
    if args.dump:
        np.savez(args.dump + ".memory.npz", shapes=G, **{"_".join(k): v for k, v in T.items()})
    return res


def run_concurrent(args, sg, torch, ctx, stream):
    """Concurrent execution of split plans (the first step towards a concurrent-split cost model):
    on the landscape's dispatch table, every cell whose plan splits along M or N is timed with its
    pieces one after another -- as a sum of kernel times (the DP's cost model) and between two
    stream markers -- and with its pieces at the same time on the context's streams, between the
    same two markers.  The two marker-timed figures compare like for like."""
    step, n = args.step, args.n
    sizes = np.arange(1, n + 1) * step
    pool = int(sizes[-1]) ** 2
    A = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    B = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    C = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    sg.fill_bf16(A, args.seed, 0)
    sg.fill_bf16(B, args.seed, 1)
    torch.cuda.synchronize()
    variants = [int(v) for v in args.variants.split(",")]
    t0 = time.perf_counter()
    if args.table:
        table = sg.Table.load(args.table)
    else:
        table = ctx.build_table(step, n, n, n, variants, A, B, C, c_dtype=sg.BF16, warmup=args.shape_warmup,
                                reps=args.reps, order_seed=args.order_seed, stream=stream)
    table_s = time.perf_counter() - t0
    ctx.set_table(table)
    cells = [(int(m), int(nn), int(k)) for m in sizes for nn in sizes for k in sizes]
    split = [c for c in cells if table.lookup(*c)["action"] in (sg.ACT_SPLIT_M, sg.ACT_SPLIT_N)]
    order = np.random.default_rng(args.order_seed).permutation(len(split))
    shapes = [split[i] for i in order]
    ksum = np.empty(len(split))     # sequential, sum of kernel times (the table's cost model)
    seq = np.empty(len(split))      # sequential, between stream markers
    conc = np.empty(len(split))     # concurrent pieces, between stream markers
    grp = np.empty(len(split))      # pieces as one grouped launch (same-tile plans), markers
    ksum[order] = ctx.sweep(shapes, A, B, C, mode=sg.MODE_DP, c_dtype=sg.BF16, warmup=args.shape_warmup,
                            reps=args.reps, stream=stream)
    try:
        for mode, out in ((2, seq), (1, conc), (3, grp)):
            ctx.set_concurrent_splits(mode)
            out[order] = ctx.sweep(shapes, A, B, C, mode=sg.MODE_DP, c_dtype=sg.BF16,
                                   warmup=args.shape_warmup, reps=args.reps, stream=stream)
    finally:
        ctx.set_concurrent_splits(0)
    fl = np.array([2.0 * m * nn * k for m, nn, k in split])
    tf_seq, tf_conc, tf_grp = fl / seq / 1e12, fl / conc / 1e12, fl / grp / 1e12
    r = seq / conc
    # which split cells the grouped form can take: every piece on one tile shape, no split-K
    def groupable(c):
        recs = []
        stack = [c]
        vs = set()
        while stack:
            m, nn, k = stack.pop()
            rec = table.lookup(m, nn, k)
            if rec["action"] in (sg.ACT_AS_IS, sg.ACT_PAD):
                vs.add(rec["variant"])
            elif rec["action"] == sg.ACT_SPLIT_M:
                p = rec["arg"] * step
                stack += [(p, nn, k), (m - p, nn, k)]
            elif rec["action"] == sg.ACT_SPLIT_N:
                p = rec["arg"] * step
                stack += [(m, p, k), (m, nn - p, k)]
            else:
                return False
        vi = [sg.variant_info(v) for v in vs]
        return len({(x.bm, x.bn, x.bk) for x in vi}) == 1 and all(x.splits == 1 for x in vi) and vi[0].bk == 64
    g_ok = np.array([groupable(c) for c in split])
    rg = seq / grp
    leaves = np.array([table.plan_leaves(*c) for c in split])
    res = {"table_grid": "{%d..%d}^3 step %d" % (step, step * n, step), "table_build_s": table_s,
           "split_cells": len(split), "frac_of_grid": len(split) / len(cells),
           "leaves_mean": float(leaves.mean()),
           "sequential_kernel_sum_mean_tflops": float((fl / ksum / 1e12).mean()),
           "sequential_mean_tflops": float(tf_seq.mean()), "concurrent_mean_tflops": float(tf_conc.mean()),
           "speedup_mean": float(r.mean()), "speedup_median": float(np.median(r)),
           "frac_faster": float((r > 1.0).mean()), "frac_faster_10pct": float((r > 1.1).mean()),
           "frac_slower_10pct": float((r < 1 / 1.1).mean()),
           # marker-timed: the landscape mean would gain this much if each split cell ran the
           # faster of the two executions
           "landscape_mean_gain_tflops": float(np.sum(np.maximum(tf_conc, tf_seq) - tf_seq) / len(cells)),
           # the same pieces as one persistent grouped launch, where every piece runs one tile shape
           "grouped_cells": int(g_ok.sum()),
           "grouped_mean_tflops": float(tf_grp[g_ok].mean()) if g_ok.any() else None,
           "grouped_sequential_mean_tflops": float(tf_seq[g_ok].mean()) if g_ok.any() else None,
           "grouped_speedup_median": float(np.median(rg[g_ok])) if g_ok.any() else None,
           "grouped_frac_faster": float((rg[g_ok] > 1.0).mean()) if g_ok.any() else None,
           "grouped_landscape_mean_gain_tflops": float(np.sum(np.maximum(tf_grp, tf_seq)[g_ok] - tf_seq[g_ok]) / len(cells))}
    log("concurrent splits: %d cells, sequential %.1f -> concurrent %.1f TFLOP/s mean, speed-up median %.3f; "
        "grouped form on %d cells: median speed-up %s"
        % (len(split), res["sequential_mean_tflops"], res["concurrent_mean_tflops"], res["speedup_median"],
           res["grouped_cells"], res["grouped_speedup_median"]))
    return res


def run_vendor(args, sg, torch, ctx, stream):
    """Context, not this library: the vendor GEMM library (torch.matmul on ROCm) over the same
    landscape with the same protocol -- randomized order, `shape_warmup` warm-up calls, then per
    shape one untimed and `reps` timed calls, BF16 in and out.  Each shape's calls are timed
    here by stream events around the back-to-back calls (host launch gaps included); under a
    kernel trace the same run gives dispatch durations comparable to the library's sweep (a
    one-word fill kernel of this library precedes each shape's calls and marks the boundary).
    The shape order is written to --dump (.vendor_order.npy) when given."""
    step, n = args.step, args.n
    sizes = np.arange(1, n + 1) * step
    pool = int(sizes[-1]) ** 2
    A = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    B = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    C = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    sg.fill_bf16(A, args.seed, 0)
    sg.fill_bf16(B, args.seed, 1)
    torch.cuda.synchronize()
    grid = [(int(m), int(nn), int(k)) for m in sizes for nn in sizes for k in sizes]
    order = np.random.default_rng(args.order_seed).permutation(len(grid))
    sec = np.empty(len(grid))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def call(M, N, K):
        torch.matmul(A[:M * K].view(M, K), B[:K * N].view(K, N), out=C[:M * N].view(M, N))

    mark = torch.empty(16, dtype=torch.bfloat16, device="cuda")
    M, N, K = grid[order[0]]
    for _ in range(args.shape_warmup):
        call(M, N, K)
    for done, i in enumerate(order):
        M, N, K = grid[i]
        sg.fill_bf16(mark, 0, 0)          # one tiny kernel of this library: a shape boundary in a trace
        call(M, N, K)
        e0.record()
        for _ in range(args.reps):
            call(M, N, K)
        e1.record()
        e1.synchronize()
        sec[i] = e0.elapsed_time(e1) * 1e-3 / args.reps
        if (done + 1) % 4096 == 0:
            log("vendor %d / %d shapes" % (done + 1, len(grid)))
    st = stack_stats(sg, sec.reshape(n, n, n), sizes)
    if args.dump:
        np.save(args.dump + ".vendor_order.npy", order)
    return {"grid": "{%d..%d}^3 step %d" % (step, step * n, step), "timing": "stream events",
            "stack": st}


EVIDENCE_SHAPES = [(4096, 4096, 4096), (3840, 2048, 4096), (4096, 4096, 128)]
EVIDENCE_VARIANTS = [0, 8, 12, 16, 24]   # 256x256, 128x256, 128x128, 128x64, 64x64 (no split)


def run_shapes(args, sg, torch, ctx, stream):
    """Single-shape evidence: the square 4096^3, the paper's peak shape 3840 x 2048 x 4096 and the
    small-K 4096 x 4096 x 128, each on several tile kernels and on their memory-only twins
    (the launches a counter run attributes per kernel)."""
    pool = 4096 * 4096
    A = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    B = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    C = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    sg.fill_bf16(A, args.seed, 0)
    sg.fill_bf16(B, args.seed, 1)
    torch.cuda.synchronize()
    out = []
    for (M, N, K) in EVIDENCE_SHAPES:
        for v in EVIDENCE_VARIANTS:
            name = sg.variant_info(v).name
            t = ctx.sweep([(M, N, K)], A, B, C, mode=sg.MODE_VARIANT, variant=v, c_dtype=sg.BF16,
                          warmup=args.shape_warmup, reps=args.reps, stream=stream)[0]
            tm = ctx.sweep([(M, N, K)], A, B, C, mode=sg.MODE_MEMORY, variant=v, c_dtype=sg.BF16,
                           warmup=args.shape_warmup, reps=args.reps, stream=stream)[0]
            bytes_min = 2.0 * M * K + 2.0 * K * N + 2.0 * M * N
            row = {"shape": [M, N, K], "variant": name, "gemm_us": t * 1e6, "twin_us": tm * 1e6,
                   "tflops": 2.0 * M * N * K / t / 1e12,
                   "frac_of_peak": 2.0 * M * N * K / t / 1e12 / sg.MI355X["peak_tflops"],
                   "min_traffic_gbs": bytes_min / t / 1e9}
            out.append(row)
            log("%dx%dx%d %s: %.1f us, %.1f TFLOP/s (%.1f %% of peak); twin %.1f us"
                % (M, N, K, name, row["gemm_us"], row["tflops"], 100 * row["frac_of_peak"], row["twin_us"]))
    return out


def run_offgrid(args, sg, torch, ctx, stream):
    """Config 3: 4,096 GEMMs with M, N, K ~ U{1..8192} (seed 3), BF16 out.  The dispatch table is
    measured on the grid {step..8192}^3 (step 256 by default: 32,768 cells, the landscape's
    count; step 128 would be 262,144), then the shapes run (a) naive pad-to-tile: the plain
    256 x 256 kernel predicated over the ragged edges, (b) best-of-N, (c) DP pad/split
    dispatch."""
    step = args.offgrid_step
    n = 8192 // step
    pool = 8192 * 8192
    A = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    B = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    C = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    sg.fill_bf16(A, 3, 0)
    sg.fill_bf16(B, 3, 1)
    torch.cuda.synchronize()
    variants = [int(v) for v in (args.offgrid_variants or args.variants).split(",")]
    t0 = time.perf_counter()
    table = ctx.build_table(step, n, n, n, variants, A, B, C, c_dtype=sg.BF16,
                            warmup=args.shape_warmup, reps=args.offgrid_reps or args.reps, order_seed=13,
                            stream=stream)
    table_s = time.perf_counter() - t0
    ctx.set_table(table)
    rng = np.random.default_rng(3)
    shapes = [tuple(int(x) for x in s) for s in rng.integers(1, 8193, size=(4096, 3))]
    fl = np.array([2.0 * m * nn * k for m, nn, k in shapes])
    out = {"table_grid": "{%d..%d}^3 step %d" % (step, step * n, step), "table_build_s": table_s}
    secs = {}
    for name, mode in (("naive_pad_to_tile", sg.MODE_PLAIN), ("best_of_n", sg.MODE_BEST),
                       ("dp_split_pad", sg.MODE_DP)):
        log("off-grid: %s" % name)
        sec = ctx.sweep(shapes, A, B, C, mode=mode, c_dtype=sg.BF16, warmup=args.shape_warmup,
                        reps=args.reps, stream=stream)
        secs[name] = sec
        tf = fl / sec / 1e12
        out[name] = {"mean_tflops": float(tf.mean()), "aggregate_tflops": float(fl.sum() / sec.sum() / 1e12),
                     "total_s": float(sec.sum())}
    r = secs["naive_pad_to_tile"] / secs["dp_split_pad"]
    out["dp_vs_naive"] = {"mean_speedup": float(r.mean()), "median_speedup": float(np.median(r)),
                          "frac_faster": float(np.mean(r > 1.0)), "frac_faster_10pct": float(np.mean(r > 1.1))}
    r = secs["best_of_n"] / secs["dp_split_pad"]
    out["dp_vs_best_of_n"] = {"mean_speedup": float(r.mean()), "median_speedup": float(np.median(r)),
                              "frac_faster": float(np.mean(r > 1.0)), "frac_faster_5pct": float(np.mean(r > 1.05)),
                              "frac_slower_5pct": float(np.mean(r < 1 / 1.05))}
    out["variants"] = [sg.variant_info(v).name for v in variants]
    acts = np.array([table.lookup(m, nn, k)["action"] for m, nn, k in shapes])
    out["dp_vs_best_of_n_by_action"] = {
        name: {"shapes": int(np.sum(acts == a)), "mean_speedup": float(r[acts == a].mean())}
        for a, name in ((sg.ACT_AS_IS, "as_is"), (sg.ACT_PAD, "pad"), (sg.ACT_SPLIT_M, "split_m"),
                        (sg.ACT_SPLIT_N, "split_n"), (sg.ACT_SPLIT_K, "split_k")) if np.any(acts == a)}
    choice = [table.plan_choice(m, nn, k) for m, nn, k in shapes]
    use = np.array([c["use_plan"] for c in choice])
    out["dp_runs_table_plan"] = float(use.mean())
    if args.dump:
        np.savez(args.dump, shapes=np.array(shapes), actions=acts, use_plan=use,
                 est_plan=np.array([c["est_plan"] for c in choice]),
                 est_best=np.array([c["est_best"] for c in choice]), **{k: v for k, v in secs.items()})
    ctx.set_table(None)
    return out


def run_serve(args, sg, torch, ctx, table=None):
    """Config 5: Poisson requests over four transformer-layer weights (the full duration), grouped
    continuous batching versus per-request dispatch on the same four stream slots, same arrivals
    and tile classes (the dispatch table's best variant per request shape when a table is at
    hand, else M <= 64 on the small tile and the rest on the main tile).  Then saturation,
    closed loop with a fixed number of requests outstanding: grouped, per-request on four slots,
    per-call dispatch on one stream (each request launched alone, in order, as a caller looping
    over gemm calls would), and the same grouped / per-request pair on a skinny mix (M <= 64,
    where launches rather than matrix work bound the throughput)."""
    shapes = [(4096, 4096), (4096, 11008), (11008, 4096), (4096, 14336)]     # (K, N)
    ws = []
    for i, (K, N) in enumerate(shapes):
        t = torch.empty(K * N, dtype=torch.bfloat16, device="cuda")
        sg.fill_bf16(t, 5, 100 + i, kind=1, scale=0.02)
        ws.append(t)
    torch.cuda.synchronize()
    out = {"rate_req_s": args.serve_rate, "duration_s": args.serve_seconds,
           "warmup_s": args.serve_warmup, "tile": sg.variant_info(4 * args.serve_tile).name[:-6],
           "small_m": args.serve_small_m, "small_tile": sg.variant_info(4 * args.serve_small_tile).name[:-6],
           "solo_m": args.serve_solo_m}
    # tile classes from the dispatch table's best variant per request shape when a table is at
    # hand (the sweep's, or --table), else the fixed classes (M <= small_m on the small tile)
    use_table = table is not None and not args.serve_fixed_tiles
    out["tiles_from_table"] = use_table
    if use_table:
        ctx.set_table(table)       # read once, when each server is created

    def server(mode, slots):
        return sg.Server(ctx, [(K, N, t.data_ptr(), N) for (K, N), t in zip(shapes, ws)],
                         hbm_budget=args.serve_budget_gb << 30, max_inflight=slots, max_group=64,
                         mode=mode, tile=args.serve_tile, max_m=8192, seed=5,
                         small_m=args.serve_small_m, small_tile=args.serve_small_tile,
                         solo_m=args.serve_solo_m if mode == sg.SERVE_GROUPED else 0,
                         tiles_from_table=use_table)

    sat = args.serve_saturate
    for name, mode in (("grouped", sg.SERVE_GROUPED), ("per_request", sg.SERVE_PER_REQUEST)):
        srv = server(mode, 4)
        try:
            log("serving (%s) %.0f req/s for %.0f s" % (name, args.serve_rate, args.serve_seconds))
            rep = srv.serve_poisson(args.serve_rate, args.serve_seconds, args.serve_warmup, 5, 8192)
            out[name] = rep
            log("  p50 %.2f ms p99 %.2f ms, %.1f req/s, %.1f TFLOP/s, %d launches"
                % (rep["p50_ms"], rep["p99_ms"], rep["req_per_s"], rep["tflops"], rep["launches"]))
            if sat > 0:
                for tag, max_m in (("saturated", 8192), ("saturated_skinny", 64)):
                    r = srv.serve_closed(args.serve_outstanding, sat, min(2.0, sat / 4), 7, max_m)
                    out[name + "_" + tag] = r
                    log("  %s (%d outstanding, M <= %d): %.1f req/s, %.1f TFLOP/s, p50 %.2f ms p99 %.2f ms, "
                        "%d launches" % (tag, args.serve_outstanding, max_m, r["req_per_s"], r["tflops"],
                                         r["p50_ms"], r["p99_ms"], r["launches"]))
        finally:
            srv.close()
    if sat > 0:
        srv = server(sg.SERVE_PER_REQUEST, 1)
        try:
            r = srv.serve_closed(args.serve_outstanding, sat, min(2.0, sat / 4), 7, 8192)
            out["per_call_one_stream_saturated"] = r
            log("  per-call, one stream (%d outstanding): %.1f req/s, %.1f TFLOP/s, p50 %.2f ms p99 %.2f ms"
                % (args.serve_outstanding, r["req_per_s"], r["tflops"], r["p50_ms"], r["p99_ms"]))
        finally:
            srv.close()

        def ratio(a, b):
            return {"throughput_ratio": a["req_per_s"] / b["req_per_s"] if b["req_per_s"] else None,
                    "p99_ratio": a["p99_ms"] / b["p99_ms"] if b["p99_ms"] else None}
        g = out["grouped_saturated"]
        out["saturation"] = {"outstanding": args.serve_outstanding, "seconds": sat,
                             "grouped_vs_per_request_4_slots": ratio(g, out["per_request_saturated"]),
                             "grouped_vs_per_call_one_stream": ratio(g, out["per_call_one_stream_saturated"]),
                             "skinny_grouped_vs_per_request_4_slots": ratio(out["grouped_saturated_skinny"],
                                                                            out["per_request_saturated_skinny"])}
    if use_table:
        ctx.set_table(None)
    del ws
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps: timed runs of every shape's plan, taken `reps` at a time")
    ap.add_argument("--warmup", type=int, default=2, help="untimed passes before timing")
    ap.add_argument("--reps", type=int, default=5,
                    help="timed runs per shape in the table measurement (one more is discarded), and "
                         "the least number of timed runs per shape over all timed passes")
    ap.add_argument("--reps-per-pass", type=int, default=0,
                    help="timed runs per shape in each timed pass (0: reps); the timed steps are "
                         "taken in passes of this many consecutive runs per shape")
    ap.add_argument("--budget", type=float, default=560.0,
                    help="wall-clock seconds the default run aims to finish in: the grouped and "
                         "serving legs are skipped (and named in the output) when they would not fit")
    ap.add_argument("--no-grouped", action="store_true", help="skip the grouped leg of the sweep")
    ap.add_argument("--shape-warmup", type=int, default=5, help="warm-up runs before a pass")
    ap.add_argument("--step", type=int, default=128, help="grid step")
    ap.add_argument("--n", type=int, default=32, help="grid points per axis")
    ap.add_argument("--variants", default=DEFAULT_VARIANTS)
    ap.add_argument("--plain-variant", type=int, default=0)
    ap.add_argument("--table", default=None, help="load this table instead of measuring one")
    ap.add_argument("--save-table", default=None)
    ap.add_argument("--seed", type=int, default=2)
    ap.add_argument("--order-seed", type=int, default=11)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--dump", default=None, help="write per-shape arrays (.npz) here")
    ap.add_argument("--workload", choices=["sweep", "grouped", "serve", "offgrid", "fineN", "decomp", "shapes", "memory", "concurrent", "vendor"], default="sweep",
                    help="sweep: the landscape (headline) plus a serving leg; grouped: config 4; "
                         "serve: config 5 at its full duration; offgrid: config 3; fineN: the "
                         "fine-N cross-tile sweep; decomp: the four-surface decomposition of "
                         "every tile kernel with its memory-only twin; shapes: 4096^3, 3840x2048x4096 "
                         "and 4096x4096x128 on several tile kernels (counter evidence); memory: the "
                         "buffer read/write study (co-allocation, load/store, warm-up, order); "
                         "concurrent: the DP's M/N split plans with their pieces run at the same time; "
                         "vendor: the vendor GEMM library over the landscape, for context")
    ap.add_argument("--groups", type=int, default=512)
    ap.add_argument("--offgrid-step", type=int, default=256, help="grid step of the off-grid table")
    ap.add_argument("--offgrid-variants", default=None, help="variant set of the off-grid table")
    ap.add_argument("--offgrid-reps", type=int, default=0, help="timed runs per cell of the off-grid table")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="duration of each serving run (the serving workload's 60 s)")
    ap.add_argument("--serve-warmup", type=float, default=5.0)
    ap.add_argument("--serve-tile", type=int, default=3)
    ap.add_argument("--serve-small-m", type=int, default=64)
    ap.add_argument("--serve-small-tile", type=int, default=6)
    ap.add_argument("--serve-fixed-tiles", action="store_true",
                    help="serve with the fixed tile classes even when a dispatch table is at hand")
    ap.add_argument("--serve-solo-m", type=int, default=256,
                    help="grouped serving launches requests with M above this on their own (0: never)")
    ap.add_argument("--serve-saturate", type=float, default=8.0,
                    help="seconds of closed-loop saturation per serving mode (0: skip)")
    ap.add_argument("--serve-outstanding", type=int, default=64)
    ap.add_argument("--serve-budget-gb", type=int, default=64)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg of the sweep")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="before the sweep, copy MIB MiB three times with a plain copy kernel (a "
                         "known-size reference for hardware byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU: the landscape sweep, its dispatch table and every kernel "
              "run on a single MI355X; runs on %d GPUs are not part of this build" % max(args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    # the CPU baseline runs first, in worker processes forked before anything touches the GPU
    cpu = None
    if args.workload == "sweep" and not args.no_cpu_baseline:
        log("cpu baseline")
        cpu = cpu_baseline(args.cpu_seconds, args.seed)
        log("cpu baseline done (%.0f s since start): %.4f TFLOP/s on %d cores"
            % (elapsed(), cpu["value"], cpu["cores"]))

    import torch
    import paper_2605_29752_amd as sg

    assert torch.cuda.is_available(), "bench.py needs the GPU"
    dev = torch.cuda.current_device()
    props = torch.cuda.get_device_properties(dev)
    ctx = sg.Context(dev)
    ctx.set_plain_variant(args.plain_variant)
    ctx.set_progress(2048)
    stream = torch.cuda.current_stream()
    common = {"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "scaling": "weak",
              "vs_baseline": None, "dtype": "bf16", "data": "synthetic", "device": props.name}

    if args.workload == "serve":
        res = run_serve(args, sg, torch, ctx, sg.Table.load(args.table) if args.table else None)
        g, p = res["grouped"], res["per_request"]
        print(json.dumps(dict(
            metric="served p99 latency, continuous batching (Poisson %.0f req/s)" % args.serve_rate,
            value=g["p99_ms"], unit="ms", higher_is_better=False,
            ms_per_step=args.serve_seconds * 1e3,
            config={"workload": "GEMM serving: Poisson %.0f req/s for %.0f s, M log-uniform 1..8192, "
                                "(N,K) in {(4096,4096),(11008,4096),(4096,11008),(14336,4096)}, "
                                "N(0,0.02) BF16, BF16 out, HBM budget %d GiB"
                                % (args.serve_rate, args.serve_seconds, args.serve_budget_gb)},
            serving=res, **common)), flush=True)
        return
    if args.workload == "fineN":
        res = run_finen(args, sg, torch, ctx, stream)
        env = res["best_of_%d" % len(args.variants.split(","))]
        print(json.dumps(dict(
            metric="fine-N best-of-N envelope roughness after DP padding (T1)",
            value=env["T1"]["roughness"], unit="TFLOPs/step", higher_is_better=False,
            ms_per_step=None,
            config={"workload": "fine-N sweep: M = K = 4096, N = 32..4096 step 32, BF16 NN, BF16 out, "
                                "every tile of the variant set and their best-of envelope"},
            fine_n=res, **common)), flush=True)
        return
    if args.workload == "vendor":
        res = run_vendor(args, sg, torch, ctx, stream)
        print(json.dumps(dict(
            metric="context: vendor GEMM library (torch.matmul) mean BF16 TFLOPs over the landscape",
            value=res["stack"]["mean_tflops"], unit="TFLOPs", higher_is_better=True, ms_per_step=None,
            config={"workload": "BF16 NN GEMM landscape {%d..%d}^3 step %d through torch.matmul, BF16 out"
                                % (args.step, args.step * args.n, args.step)},
            vendor=res, **common)), flush=True)
        return
    if args.workload == "concurrent":
        res = run_concurrent(args, sg, torch, ctx, stream)
        print(json.dumps(dict(
            metric="split plans: median speed-up of concurrent over sequential pieces",
            value=res["speedup_median"], unit="ratio", higher_is_better=True, ms_per_step=None,
            config={"workload": "every M/N-split cell of the {%d..%d}^3 step %d dispatch table, BF16 NN, "
                                "BF16 out" % (args.step, args.step * args.n, args.step)},
            concurrent=res, **common)), flush=True)
        return
    if args.workload == "memory":
        res = run_memory(args, sg, torch, ctx, stream)
        print(json.dumps(dict(
            metric="memory study: mean co-allocation slowdown of read A (randomized order)",
            value=res["table4_coalloc_slowdown"]["read_A"]["mean"], unit="ratio", higher_is_better=False,
            ms_per_step=None,
            config={"workload": "FP32 buffer reads (A M x K, B K x N, C M x N) and writes (D M x N) over "
                                "{%d..%d}^3 step %d, isolated vs co-allocated, randomized vs sequential"
                                % (args.step, args.step * args.n, args.step)},
            memory=res, **common)), flush=True)
        return
    if args.workload == "shapes":
        if args.calibrate_copy > 0:
            src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device="cuda")
            dst = torch.empty_like(src)
            for _ in range(3):
                dst.copy_(src)
            torch.cuda.synchronize()
            del src, dst
        res = run_shapes(args, sg, torch, ctx, stream)
        best = max(r["tflops"] for r in res if r["shape"] == [4096, 4096, 4096])
        print(json.dumps(dict(
            metric="BF16 TFLOP/s at 4096^3, best tile kernel", value=best, unit="TFLOP/s",
            higher_is_better=True, ms_per_step=None,
            config={"workload": "single shapes 4096^3, 3840x2048x4096, 4096x4096x128, BF16 NN, BF16 out, "
                                "tile kernels and their memory-only twins"},
            shapes=res, **common)), flush=True)
        return
    if args.workload == "decomp":
        res = run_decomp(args, sg, torch, ctx, stream)
        plain = sg.variant_info(args.plain_variant).name
        print(json.dumps(dict(
            metric="four-surface decomposition: mean overhead share of the plain kernel's GEMM time",
            value=res["tiles"][plain]["overhead_share"] if plain in res["tiles"] else None,
            unit="fraction", higher_is_better=False, ms_per_step=None,
            config={"workload": "landscape {%d..%d}^3 step %d, BF16 NN, BF16 out: every tile kernel "
                                "and its memory-only twin" % (args.step, args.step * args.n, args.step)},
            decomposition=res, **common)), flush=True)
        return
    if args.workload == "offgrid":
        res = run_offgrid(args, sg, torch, ctx, stream)
        print(json.dumps(dict(
            metric="off-grid mean BF16 TFLOPs: DP pad/split dispatch vs naive pad-to-tile",
            value=res["dp_split_pad"]["mean_tflops"], unit="TFLOPs", higher_is_better=True,
            ms_per_step=res["dp_split_pad"]["total_s"] * 1e3,
            config={"workload": "4096 BF16 NN GEMMs, M,N,K ~ U{1..8192} (seed 3), uniform[-1,1] "
                                "BF16 inputs, FP32 accumulate, BF16 out"},
            offgrid=res, **common)), flush=True)
        return
    if args.workload == "grouped":
        if args.table:
            ctx.set_table(sg.Table.load(args.table))
        # a stream of its own: graph capture needs a non-null stream (default priority)
        res = run_grouped(args, sg, torch, ctx, torch.cuda.Stream())
        print(json.dumps(dict(
            metric="grouped BF16 GEMM throughput (hipGraph of persistent grouped launches)",
            value=res["graph_tflops"], unit="TFLOP/s", higher_is_better=True,
            ms_per_step=res["graph_s"] * 1e3,
            config={"workload": "%d groups x 64 BF16 NN GEMMs, M,N,K log-uniform [64,4096] rounded "
                                "to multiples of 8, BF16 out" % args.groups},
            grouped=res, **common)), flush=True)
        return

    n, step = args.n, args.step
    sizes = np.arange(1, n + 1, dtype=np.float64) * step
    maxdim = n * step
    pool = maxdim * maxdim
    A = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    B = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    C = torch.empty(pool, dtype=torch.bfloat16, device="cuda")
    sg.fill_bf16(A, args.seed, 0)           # same bits as the host generator (tested)
    sg.fill_bf16(B, args.seed, 1)
    torch.cuda.synchronize()

    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy << 18, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    variants = [int(v) for v in args.variants.split(",")]
    t_tab = time.perf_counter()
    if args.table:
        table = sg.Table.load(args.table)
        variants = table.variants()
    else:
        log("measuring T0: %d variants x %d shapes" % (len(variants), n ** 3))
        table = ctx.build_table(step, n, n, n, variants, A, B, C, c_dtype=sg.BF16,
                                warmup=args.shape_warmup, reps=args.reps,
                                order_seed=args.order_seed, stream=stream)
        if args.save_table:
            table.save(args.save_table)
    table_s = time.perf_counter() - t_tab
    log("table ready in %.1f s (%.0f s since start)" % (table_s, elapsed()))
    ctx.set_table(table)

    T0all = table.values(3)
    T0best, T1, T2 = table.values(0), table.values(1), table.values(2)
    # the plain stack: one tile shape with no split for every shape -- the measured variant
    # fastest at the grid's largest cell (the single-kernel choice a user tuning on the big cube
    # would make); the paper's default 256 x 256 tile is reported beside it
    no_split = [r for r, v in enumerate(variants) if sg.variant_info(v).splits == 1]
    plain_row = min(no_split, key=lambda r: T0all[r][-1, -1, -1])
    plain_variant = variants[plain_row]
    default_row = variants.index(0) if 0 in variants else None

    rng = np.random.default_rng(args.order_seed)
    cells = rng.permutation(n ** 3)
    idx = np.array(np.unravel_index(cells, (n, n, n))).T
    shapes = [(int((i + 1) * step), int((j + 1) * step), int((k + 1) * step)) for i, j, k in idx]
    # A step is one timed run of every shape's plan.  The steps are taken in passes of
    # `reps_pass` consecutive runs per shape, each pass after one untimed run of the shape --
    # the table's own protocol (one discarded launch, then `reps` timed ones), so executed and
    # tabulated times are measured alike (a lone timed launch after the discarded one reads
    # 13-17 % slower on small shapes than the mean of five).
    reps_pass = max(1, min(args.reps_per_pass or args.reps, args.steps))
    pass_reps = [reps_pass] * (args.steps // reps_pass) + ([args.steps % reps_pass] if args.steps % reps_pass else [])

    def one_pass(mode=sg.MODE_DP, variant=0, reps=reps_pass, interval=False):
        ctx.set_interval_timing(interval)
        sec = ctx.sweep(shapes, A, B, C, mode=mode, variant=variant, c_dtype=sg.BF16,
                        warmup=args.shape_warmup, reps=reps, stream=stream)
        return sec, (ctx.interval_times(len(shapes)) if interval else None)

    def to_grid(v):
        out = np.zeros(n ** 3)
        out[cells] = v
        return out.reshape(n, n, n)

    for w in range(args.warmup):
        log("warm-up pass %d" % w)
        one_pass(reps=1)
    torch.cuda.synchronize()
    passes = []
    launches = np.zeros(sg.num_variants(), dtype=np.int64)
    ksec = np.zeros(sg.num_variants())
    kflops = np.zeros(sg.num_variants())
    t0 = time.perf_counter()
    for s_, r_ in enumerate(pass_reps):
        sec, _ = one_pass(reps=r_)
        la, se, fl = ctx.kernel_times()
        launches += la
        ksec += se
        kflops += fl
        passes.append(to_grid(sec))
        log("timed pass %d (%d runs per shape) done (%.0f s since start)" % (s_, r_, elapsed()))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / args.steps * 1e3
    exec_sec = np.average(passes, axis=0, weights=pass_reps)
    # gap-included executions: every run of the DP plans and of the plain variant timed as a
    # whole between two stream markers (one pass each, `reps` marker-timed runs per shape)
    log("interval-timed passes (DP plans, plain %s)" % sg.variant_info(plain_variant).name)
    _, iv = one_pass(reps=args.reps, interval=True)
    exec_iv = to_grid(iv)
    _, p_iv = one_pass(sg.MODE_VARIANT, plain_variant, args.reps, interval=True)
    plain_exec_iv = to_grid(p_iv)

    M3 = sizes[:, None, None]
    N3 = sizes[None, :, None]
    K3 = sizes[None, None, :]
    W3 = 2.0 * M3 * N3 * K3
    pname = "plain_%s" % sg.variant_info(plain_variant).name
    stack_secs = {
        pname: T0all[plain_row],
        "best_of_%d" % len(variants): T0best,
        "dp_pad_table": T1,
        "dp_split_pad_table": T2,
        "dp_split_pad_executed": exec_sec,
    }
    if default_row is not None and default_row != plain_row:
        stack_secs["paper_default_256x256x64_s1"] = T0all[default_row]
    stacks = {name: stack_stats(sg, sec, sizes) for name, sec in stack_secs.items()}
    # best single variant by mean over the sweep
    means = [stack_stats(sg, T0all[r], sizes)["mean_tflops"] for r in range(len(variants))]
    best_single = variants[int(np.argmax(means))]
    stacks["best_single_%s" % sg.variant_info(best_single).name] = \
        stack_stats(sg, T0all[variants.index(best_single)], sizes)
    # the DP on one fixed tile (Table 10's "DP pad / split+pad (fixed tile)" rows), as the tables
    # predict them: the same recurrence over the single variant's own T0
    for row in sorted({plain_row, variants.index(best_single)}):
        ft = sg.Table.from_t0(step, n, n, n, T0all[row][None], [variants[row]])
        vname = sg.variant_info(variants[row]).name
        stacks["dp_pad_fixed_%s_table" % vname] = stack_stats(sg, ft.values(1), sizes)
        stacks["dp_split_pad_fixed_%s_table" % vname] = stack_stats(sg, ft.values(2), sizes)
        ft.close()
    # gap-included (marker-interval) executions of the DP and plain stacks
    stacks["dp_split_pad_executed_interval"] = stack_stats(sg, exec_iv, sizes)
    stacks[pname + "_executed_interval"] = stack_stats(sg, plain_exec_iv, sizes)
    for st in stacks.values():
        st["relative_roughness_3d"] = st["roughness_3d"] / st["mean_tflops"]

    # noise floor: the roughness that measurement noise alone puts into one pass (from the
    # difference of consecutive passes, scaled by 1/sqrt 2), and what is left of it in the
    # mean of all passes (1/sqrt(passes) of that)
    noise = {}
    full = [p for p, r_ in zip(passes, pass_reps) if r_ == reps_pass]
    if len(full) >= 2:
        tfp = [W3 / p / 1e12 for p in full]
        single = [sg.landscape_stats((tfp[i] - tfp[i + 1]) / np.sqrt(2.0)) for i in range(len(tfp) - 1)]
        r1 = float(np.mean([x["roughness_3d"] for x in single]))
        sl1 = float(np.mean([np.mean([sg.roughness(row) for row in ((tfp[i] - tfp[i + 1]) / np.sqrt(2.0))[:, :, -1]])
                             for i in range(len(tfp) - 1)]))
        cv = float(np.median(np.std(np.array(full), axis=0) / np.mean(full, axis=0)))
        # (a shorter remainder pass, if any, is left out of these estimates)
        noise = {"single_pass_roughness_3d": r1, "single_pass_roughness_slice": sl1,
                 "mean_of_passes_roughness_3d": r1 / np.sqrt(len(full)),
                 "mean_of_passes_roughness_slice": sl1 / np.sqrt(len(full)),
                 "median_cv_across_passes": cv, "passes": len(full), "timed_runs_per_shape_per_pass": reps_pass}

    # dominant kernel: the tile kernel with the most execution time, over every variant that
    # launches it (the split-K variants of a tile run the same kernel; their accounted time is
    # the tile kernel's own, the reduction excluded)
    tile_keys = sorted({(sg.variant_info(v).bm, sg.variant_info(v).bn, sg.variant_info(v).bk)
                        for v in range(sg.num_variants())})
    tile_of = np.array([tile_keys.index((sg.variant_info(v).bm, sg.variant_info(v).bn, sg.variant_info(v).bk))
                        for v in range(sg.num_variants())])
    ntiles = len(tile_keys)
    t_sec = np.array([ksec[tile_of == t].sum() for t in range(ntiles)])
    t_launch = np.array([launches[tile_of == t].sum() for t in range(ntiles)])
    t_flops = np.array([kflops[tile_of == t].sum() for t in range(ntiles)])
    dom_tile = int(np.argmax(t_sec))
    vi = sg.variant_info(int(np.flatnonzero(tile_of == dom_tile)[0]))
    dom_kernel = kernel_name(sg, vi.id)
    achieved = t_flops[dom_tile] / t_sec[dom_tile] / 1e12
    dom_variants = [sg.variant_info(v).name for v in np.flatnonzero((tile_of == dom_tile) & (launches > 0))]
    ex = stacks["dp_split_pad_executed"]
    plain = stacks[pname]
    bestn = stacks["best_of_%d" % len(variants)]

    actions = {}
    for c in range(n ** 3):
        i, j, k = np.unravel_index(c, (n, n, n))
        a = table.lookup(int((i + 1) * step), int((j + 1) * step), int((k + 1) * step))["action"]
        actions[a] = actions.get(a, 0) + 1
    names = {0: "as_is", 1: "pad", 2: "split_m", 3: "split_n", 4: "split_k"}

    def gain(a, b):
        return {"mean": a["mean_tflops"] / b["mean_tflops"] - 1.0,
                "roughness_3d": a["roughness_3d"] / b["roughness_3d"] - 1.0,
                "texture_3d": a["texture_3d"] / b["texture_3d"] - 1.0,
                "roughness_slice": a["slice_k%d_roughness_n" % maxdim] / b["slice_k%d_roughness_n" % maxdim] - 1.0,
                "relative_roughness_3d": a["relative_roughness_3d"] / b["relative_roughness_3d"] - 1.0}

    result = {
        "metric": "mean BF16 TFLOPs + roughness over 32,768-shape sweep; served p50/p99 latency",
        "value": ex["mean_tflops"],
        "unit": "TFLOPs",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic",
        "config": {"workload": "BF16 NN GEMM landscape sweep, (M,N,K) in {%d..%d}^3 step %d "
                               "(%d shapes), uniform[-1,1] BF16 inputs, FP32 accumulate, BF16 "
                               "output, executed through best-of-N + DP pad/split dispatch table"
                               % (step, maxdim, step, n ** 3),
                   "shapes": n ** 3, "variants": [sg.variant_info(v).name for v in variants],
                   "table_reps_per_shape": args.reps, "timed_runs_per_shape_per_pass": reps_pass,
                   "order": "randomized (seed %d)" % args.order_seed},
        "roughness_3d": ex["roughness_3d"],
        "roughness_slice_k%d" % maxdim: ex["slice_k%d_roughness_n" % maxdim],
        "relative_roughness_3d": ex["relative_roughness_3d"],
        "peak_tflops": ex["peak_tflops"],
        "frac_of_bf16_peak_mean": ex["mean_tflops"] / PEAK_BF16_TFLOPS,
        "executed_interval_mean_tflops": stacks["dp_split_pad_executed_interval"]["mean_tflops"],
        "plain_variant": sg.variant_info(plain_variant).name,
        "gain_vs_plain": gain(ex, plain),
        "gain_vs_best_of_n": gain(ex, bestn),
        "best_single_variant": sg.variant_info(best_single).name,
        "gain_vs_best_single": gain(ex, stacks["best_single_%s" % sg.variant_info(best_single).name]),
        "noise_floor": noise,
        "stacks": stacks,
        "first_principles": first_principles(sg, stack_secs, sizes, args.step, n),
        "dp_actions": {names[a]: c / n ** 3 for a, c in sorted(actions.items())},
        # shapes where the DP's plan beats best-of-N: in the table (T2 below the best single
        # variant's T0) and as executed (re-measured plan time below that T0)
        "dp_beats_best_of_n": {"table": float(np.mean(T2 < T0best * (1 - 1e-9))),
                               "executed": float(np.mean(exec_sec < T0best)),
                               "executed_by_5pct": float(np.mean(exec_sec < 0.95 * T0best))},
        "table_build_s": table_s,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_BF16_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_BF16_TFLOPS,
                     "traffic": traffic_bytes(dom_kernel),
                     "kernel": dom_kernel, "variants": dom_variants,
                     "launches": int(t_launch[dom_tile]),
                     "avg_launch_us": t_sec[dom_tile] / max(t_launch[dom_tile], 1) * 1e6,
                     "flop_per_launch": t_flops[dom_tile] / max(t_launch[dom_tile], 1)},
        "device": props.name,
    }
    if cpu is not None:
        result["cpu_baseline"] = cpu
    skipped = []
    # grouped batching (config 4) with the table set: per-call best-of-N / DP baselines
    if not args.no_grouped:
        if elapsed() + 60 < args.budget:
            g = run_grouped(args, sg, torch, ctx, torch.cuda.Stream(), reps=min(args.steps, 5))
            result["grouped"] = g
            log("grouped done (%.0f s since start)" % elapsed())
        else:
            skipped.append("grouped")
    ctx.set_table(None)
    if not args.no_serve:
        need = 2 * (args.serve_seconds + 2 * args.serve_saturate + 10) + args.serve_saturate + 5
        if elapsed() + need < args.budget:
            srv = run_serve(args, sg, torch, ctx, table)
            result["served_p50_ms"] = srv["grouped"]["p50_ms"]
            result["served_p99_ms"] = srv["grouped"]["p99_ms"]
            result["serving"] = srv
            log("serving done (%.0f s since start)" % elapsed())
        else:
            skipped.append("serving")
    if skipped:
        result["skipped_for_time_budget"] = skipped
    result["wall_s"] = elapsed()
    if args.dump:
        np.savez_compressed(args.dump, sizes=sizes, T0=T0all, T0best=T0best, T1=T1, T2=T2,
                            executed=exec_sec, executed_interval=exec_iv, passes=np.array(passes),
                            variants=np.array(variants), plain_interval=plain_exec_iv)
    # release everything before the interpreter shuts down (HIP status checked on each)
    table.close()
    ctx.close()
    del A, B, C
    torch.cuda.synchronize()
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
