// Persistent grouped BF16 NN GEMM: many independent problems of uneven shape in one launch.
//
// The grid holds as many work-groups as the device keeps resident at once.  Each work-group
// takes the next tile from a global work queue (an atomic counter), finds its problem by binary
// search over the per-problem tile prefix sums, and runs the same tile body as the per-call
// kernel, so every output element is computed exactly as a per-call launch of the same tile
// shape computes it.  Problems are ordered longest-K first (largest tile cost first), so the
// greedy queue behaves like longest-processing-time scheduling.  The last work-group to finish
// returns the counters to zero, so one launch can be replayed (hipGraph) without a reset node.
#include <hip/hip_ext.h>

#include <algorithm>
#include <cmath>
#include <numeric>

#include "sg_internal.h"
#include "sg_table.h"
#include "tile_body.h"
#include "tile_body_dma.h"

namespace sg {


// ALL_ALIGNED: every problem of the launch takes the aligned fast path, so the kernel does not
// carry the element-wise fallback body (fewer registers, more resident work-groups).
// Waves of a grouped kernel: the per-call kernels' count when every problem is aligned (so the
// tile body is the same), four when the element-wise body (written for four waves) may run.
template <int BM, int BN, bool ALL_ALIGNED>
constexpr int grouped_waves() { return ALL_ALIGNED ? call_waves<BM, BN>() : 4; }

template <int BM, int BN, bool ALL_ALIGNED>
__global__ __launch_bounds__((64 * grouped_waves<BM, BN, ALL_ALIGNED>())) void sg_gemm_grouped(
        const GroupProblem* __restrict__ probs, int G, int total_tiles, int out_bf16, int* __restrict__ counters) {
    constexpr int NW = grouped_waves<BM, BN, ALL_ALIGNED>();
    // the aligned body's ring, or the larger of it and the element-wise body's stages
    constexpr int kSmem = (ALL_ALIGNED || dma_smem_bytes<BM, BN, false, NW>() / 2 > smem_elems<BM, BN>())
                              ? dma_smem_bytes<BM, BN, false, NW>() / 2 : smem_elems<BM, BN>();
    __shared__ __attribute__((aligned(1024))) uint16_t smem[kSmem];
    __shared__ int s_tile;
    for (;;) {
        __syncthreads();                       // previous tile done with the LDS and s_tile
        if (threadIdx.x == 0) s_tile = atomicAdd(&counters[0], 1);
        __syncthreads();
        const int t = s_tile;
        if (t >= total_tiles) break;           // every work-group leaves once the queue is empty
        int lo = 0, hi = G - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (probs[mid].tile_begin <= t) lo = mid;
            else hi = mid - 1;
        }
        const GroupProblem& q = probs[lo];
        const int local = t - q.tile_begin;
        const int tm = local % q.tiles_m;      // M fastest: consecutive tiles share a B panel
        const int tn = local / q.tiles_m;
        KArgs a{};
        a.A = q.A; a.B = q.B; a.C = q.C; a.add = nullptr;
        a.lda = q.lda; a.ldb = q.ldb; a.ldc = q.ldc; a.ldadd = 0; a.ws_slice = 0;
        a.M = q.M; a.N = q.N; a.K = q.K; a.Kl = q.K; a.k_chunk = ((q.K + kBK - 1) / kBK) * kBK;
        a.tiles_m = q.tiles_m; a.tiles_n = q.tiles_n;
        a.out_bf16 = out_bf16; a.add_kind = ADD_NONE;
        a.vec_ok = q.vec_ok;
        a.a_bytes = q.a_bytes; a.b_bytes = q.b_bytes;
        if (ALL_ALIGNED || q.aligned) {
            // (no cross-stage fragment prefetch for 256 x 256 here: its registers would spill)
            tile_body_dma<BM, BN, false, false, NW, !(BM == 256 && BN == 256)>(a, tm * BM, tn * BN, 0, smem);
        } else {
            if constexpr (!ALL_ALIGNED) tile_body<BM, BN>(a, tm * BM, tn * BN, 0, smem);
        }
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const int done = atomicAdd(&counters[1], 1);
        if (done == (int)gridDim.x - 1) {      // last one out: reset for the next launch
            atomicExch(&counters[0], 0);
            atomicExch(&counters[1], 0);
        }
    }
}

typedef void (*GroupedKernel)(const GroupProblem*, int, int, int, int*);

template <bool AA>
static GroupedKernel grouped_kernel_t(int tile) {
    switch (tile) {
        case 0: return sg_gemm_grouped<256, 256, AA>;
        case 1: return sg_gemm_grouped<256, 128, AA>;
        case 2: return sg_gemm_grouped<128, 256, AA>;
        case 3: return sg_gemm_grouped<128, 128, AA>;
        case 4: return sg_gemm_grouped<128, 64, AA>;
        case 5: return sg_gemm_grouped<64, 128, AA>;
        default: return sg_gemm_grouped<64, 64, AA>;
    }
}

static GroupedKernel grouped_kernel(int tile, bool all_aligned) {
    return all_aligned ? grouped_kernel_t<true>(tile) : grouped_kernel_t<false>(tile);
}

static int grouped_threads(int tile, bool all_aligned) {
    if (!all_aligned) return 256;
    switch (tile) {
        case 0: return 64 * call_waves<256, 256>();
        case 1: return 64 * call_waves<256, 128>();
        case 2: return 64 * call_waves<128, 256>();
        case 3: return 64 * call_waves<128, 128>();
        case 4: return 64 * call_waves<128, 64>();
        case 5: return 64 * call_waves<64, 128>();
        default: return 64 * call_waves<64, 64>();
    }
}

int grouped_fill(const sg_problem* probs, int G, int tile, int c_dtype, bool lpt, GroupProblem* out,
                 int* order, int* total_tiles, double* flops, bool* all_aligned) {
    const TileShape ts = kTiles[tile];
    std::iota(order, order + G, 0);
    if (lpt) std::stable_sort(order, order + G, [&](int a, int b) { return probs[a].K > probs[b].K; });
    int64_t tiles = 0;
    double fl = 0.0;
    bool aa = true;
    const size_t esz = c_dtype == SG_BF16 ? 2 : 4;
    for (int i = 0; i < G; ++i) {
        const sg_problem& q = probs[order[i]];
        GroupProblem& g = out[i];
        g.A = (const uint16_t*)q.A; g.B = (const uint16_t*)q.B; g.C = q.C;
        g.lda = q.lda; g.ldb = q.ldb; g.ldc = q.ldc;
        g.M = (int)q.M; g.N = (int)q.N; g.K = (int)q.K;
        g.tiles_m = (int)((q.M + ts.bm - 1) / ts.bm);
        g.tiles_n = (int)((q.N + ts.bn - 1) / ts.bn);
        g.tile_begin = (int)tiles;
        const int64_t ab = ((q.M - 1) * q.lda + q.K) * 2, bb = ((q.K - 1) * q.ldb + q.N) * 2;
        const bool al = q.lda % 8 == 0 && q.ldb % 8 == 0 && q.K % 8 == 0 && q.N % 8 == 0 &&
                        (uintptr_t)q.A % 16 == 0 && (uintptr_t)q.B % 16 == 0 && ab < 0x7FFFFFFF &&
                        bb < 0x7FFFFFFF;
        g.aligned = al ? 1 : 0;
        aa = aa && al;
        g.a_bytes = al ? (int)ab : 0;
        g.b_bytes = al ? (int)bb : 0;
        g.vec_ok = (q.ldc % 4 == 0 && (uintptr_t)q.C % (4 * esz) == 0) ? 1 : 0;
        tiles += (int64_t)g.tiles_m * g.tiles_n;
        fl += 2.0 * (double)q.M * (double)q.N * (double)q.K;
        if (tiles > 0x7FFFFFFF) return fail(SG_EINVAL, "grouped: too many tiles");
    }
    *total_tiles = (int)tiles;
    *flops = fl;
    *all_aligned = aa;
    return SG_OK;
}

int grouped_grid(int tile, bool all_aligned, int device, int total_tiles, int grid_wgs, int* grid) {
    int per_cu = 1, cus = 0;
    SG_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, grouped_kernel(tile, all_aligned),
                                                        grouped_threads(tile, all_aligned), 0));
    SG_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device));
    int g = std::max(1, per_cu) * cus;
    if (grid_wgs > 0) g = grid_wgs;
    *grid = std::min(g, std::max(1, total_tiles));
    return SG_OK;
}

int grouped_enqueue(int tile, bool all_aligned, const GroupProblem* d_probs, int G, int total_tiles,
                    int grid, int c_dtype, int* d_counters, hipStream_t s, hipEvent_t start,
                    hipEvent_t stop) {
    hipExtLaunchKernelGGL(grouped_kernel(tile, all_aligned), dim3(grid), dim3(grouped_threads(tile, all_aligned)), 0, s,
                          start, stop, 0, d_probs, G,
                          total_tiles, c_dtype == SG_BF16 ? 1 : 0, d_counters);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

}  // namespace sg

using namespace sg;

struct sg_group_plan {
    int device = 0;
    int G = 0;
    int c_dtype = SG_BF16;
    sg_group_cfg cfg{};
    int total_tiles = 0;
    int grid = 0;
    bool all_aligned = false;
    double flops = 0.0;
    std::vector<sg_problem> probs;    // host copy, in queue order
    GroupProblem* d_probs = nullptr;
    int* d_counters = nullptr;
};

struct sg_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

namespace {

int validate_problems(int G, const sg_problem* p) {
    if (G <= 0 || !p) return fail(SG_EINVAL, "grouped: empty problem list");
    for (int i = 0; i < G; ++i) {
        const sg_problem& q = p[i];
        if (q.M <= 0 || q.N <= 0 || q.K <= 0) return fail(SG_EINVAL, "grouped: every problem needs M, N, K > 0");
        if (!q.A || !q.B || !q.C) return fail(SG_EINVAL, "grouped: NULL operand");
        if (q.lda < q.K || q.ldb < q.N || q.ldc < q.N) return fail(SG_EINVAL, "grouped: leading dimension too small");
        if (q.M > 0x7FFFFFFF || q.N > 0x7FFFFFFF || q.K > 0x7FFFFFFF) return fail(SG_EINVAL, "grouped: dimension too large");
    }
    return SG_OK;
}

// Build descriptors for the tile shape, in longest-tile-first order, and upload them.
int plan_upload(sg_group_plan* pl, const sg_problem* probs, hipStream_t s) {
    const int G = pl->G;
    std::vector<GroupProblem> h(G);
    std::vector<int> order(G);
    int rc = grouped_fill(probs, G, pl->cfg.tile, pl->c_dtype, pl->cfg.order == 0, h.data(),
                          order.data(), &pl->total_tiles, &pl->flops, &pl->all_aligned);
    if (rc) return rc;
    pl->probs.resize(G);
    for (int i = 0; i < G; ++i) pl->probs[i] = probs[order[i]];
    if (!pl->d_probs) SG_HIP(hipMalloc(&pl->d_probs, sizeof(GroupProblem) * G));
    SG_HIP(hipMemcpyAsync(pl->d_probs, h.data(), sizeof(GroupProblem) * G, hipMemcpyHostToDevice, s));
    SG_HIP(hipStreamSynchronize(s));
    return grouped_grid(pl->cfg.tile, pl->all_aligned, pl->device, pl->total_tiles, pl->cfg.grid_wgs,
                        &pl->grid);
}

int plan_enqueue(sg_group_plan* pl, hipStream_t s, hipEvent_t start = nullptr, hipEvent_t stop = nullptr) {
    return grouped_enqueue(pl->cfg.tile, pl->all_aligned, pl->d_probs, pl->G, pl->total_tiles, pl->grid,
                           pl->c_dtype, pl->d_counters, s, start, stop);
}

// Key of a group's schedule in the table: the problem list in the caller's order (dimensions,
// and the alignment classes that choose the kernel body and the store width) and c_dtype.
uint64_t group_key(const sg_problem* probs, int G, int c_dtype) {
    uint64_t h = 0xcbf29ce484222325ull;
    auto mix = [&](uint64_t v) {
        h ^= v + 0x9E3779B97F4A7C15ull + (h << 6) + (h >> 2);
        h *= 0x100000001b3ull;
    };
    mix((uint64_t)G);
    mix((uint64_t)c_dtype);
    for (int i = 0; i < G; ++i) {
        const sg_problem& q = probs[i];
        mix((uint64_t)q.M);
        mix((uint64_t)q.N);
        mix((uint64_t)q.K);
        const uint64_t cls = (uint64_t)(q.lda % 8 == 0) | ((uint64_t)(q.ldb % 8 == 0) << 1) |
                             ((uint64_t)((uintptr_t)q.A % 16 == 0) << 2) |
                             ((uint64_t)((uintptr_t)q.B % 16 == 0) << 3) | ((uint64_t)(q.ldc % 4 == 0) << 4) |
                             ((uint64_t)((uintptr_t)q.C % 16 == 0) << 5);
        mix(cls);
    }
    return h;
}

// Time one configuration: upload its descriptors, one warm-up launch, best of three.
int time_config(sg_group_plan* pl, const sg_problem* probs, const sg_group_cfg& c, hipStream_t s,
                hipEvent_t e0, hipEvent_t e1, double* sec) {
    pl->cfg = c;
    int rc = plan_upload(pl, probs, s);
    if (rc) return rc;
    rc = plan_enqueue(pl, s);
    if (rc) return rc;
    double best = INFINITY;
    for (int r = 0; r < 3; ++r) {
        rc = plan_enqueue(pl, s, e0, e1);
        if (rc) return rc;
        SG_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        SG_HIP(hipEventElapsedTime(&ms, e0, e1));
        best = std::min(best, (double)ms * 1e-3);
    }
    *sec = best;
    return SG_OK;
}

// Autotune a group's schedule: every tile shape at full residency with the longest-K-first
// queue, then, for the two fastest tiles, the queue in the caller's order and smaller grids
// (one work-group per CU, and half the resident count), so that fewer, fuller work-groups can
// win where the tail of the queue is short.  The winner is left in pl->cfg (descriptors
// uploaded); *sec receives its time.
int autotune(sg_group_plan* pl, const sg_problem* probs, hipStream_t s, double* sec) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    SG_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(SG_EHIP, "grouped: event creation failed");
    }
    int cus = 0;
    int rc = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, pl->device) == hipSuccess
                 ? SG_OK : fail(SG_EHIP, "grouped: device query failed");
    std::vector<std::pair<double, sg_group_cfg>> tried;
    for (int t = 0; t < kNumGroupTiles && rc == SG_OK; ++t) {
        double x = 0;
        const sg_group_cfg c{t, 0, 0};
        rc = time_config(pl, probs, c, s, e0, e1, &x);
        if (rc == SG_OK) tried.emplace_back(x, c);
    }
    if (rc == SG_OK) {
        std::sort(tried.begin(), tried.end(), [](const auto& a, const auto& b) { return a.first < b.first; });
        const size_t top = std::min<size_t>(2, tried.size());
        for (size_t i = 0; i < top && rc == SG_OK; ++i) {
            const int t = tried[i].second.tile;
            int full = 0;
            rc = grouped_grid(t, pl->all_aligned, pl->device, INT32_MAX, 0, &full);
            if (rc) break;
            std::vector<sg_group_cfg> more{{t, 0, 1}};
            if (full > cus) more.push_back({t, cus, 0});
            if (full > 2 * cus) more.push_back({t, (full / cus / 2) * cus, 0});
            for (const sg_group_cfg& c : more) {
                double x = 0;
                rc = time_config(pl, probs, c, s, e0, e1, &x);
                if (rc) break;
                tried.emplace_back(x, c);
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    const auto best = *std::min_element(tried.begin(), tried.end(),
                                        [](const auto& a, const auto& b) { return a.first < b.first; });
    pl->cfg = best.second;
    *sec = best.first;
    return plan_upload(pl, probs, s);
}

}  // namespace

extern "C" {

int sg_group_plan_create(sg_ctx* ctx, int G, const sg_problem* probs, int c_dtype,
                         const sg_group_cfg* cfg, void* stream, sg_group_plan** out) {
    if (!ctx || !out) return fail(SG_EINVAL, "NULL argument");
    *out = nullptr;
    int rc = validate_problems(G, probs);
    if (rc) return rc;
    if (c_dtype != SG_F32 && c_dtype != SG_BF16) return fail(SG_EINVAL, "bad c_dtype");
    if (cfg && (cfg->tile < 0 || cfg->tile >= kNumGroupTiles || (cfg->order != 0 && cfg->order != 1) || cfg->grid_wgs < 0))
        return fail(SG_EINVAL, "bad group configuration");
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    hipStream_t s = (hipStream_t)stream;
    sg_group_plan* pl = new (std::nothrow) sg_group_plan();
    if (!pl) return fail(SG_ENOMEM, "plan allocation failed");
    pl->device = dev;
    pl->G = G;
    pl->c_dtype = c_dtype;
    if (hipMalloc(&pl->d_counters, 2 * sizeof(int)) != hipSuccess) {
        delete pl;
        return fail(SG_ENOMEM, "grouped: counter allocation failed");
    }
    // counters start at zero once; every launch returns them to zero itself
    if (hipMemset(pl->d_counters, 0, 2 * sizeof(int)) != hipSuccess) {
        sg_group_plan_destroy(pl);
        return fail(SG_EHIP, "grouped: counter reset failed");
    }
    if (cfg) {
        pl->cfg = *cfg;
        rc = plan_upload(pl, probs, s);
    } else {
        // a schedule recorded in the context's table for this very group is taken by lookup;
        // otherwise the autotuner times candidates and records its winner there
        const sg_table* tab = ctx_table(ctx);
        const uint64_t key = group_key(probs, G, c_dtype);
        bool hit = false;
        if (tab) {
            std::lock_guard<std::mutex> lk(tab->group_mu);
            auto it = tab->group_sched.find(key);
            if (it != tab->group_sched.end()) {
                pl->cfg = sg_group_cfg{it->second.tile, it->second.grid_wgs, it->second.order};
                hit = true;
            }
        }
        if (hit) {
            rc = plan_upload(pl, probs, s);
        } else {
            double sec = 0.0;
            rc = autotune(pl, probs, s, &sec);
            if (rc == SG_OK && tab) {
                std::lock_guard<std::mutex> lk(tab->group_mu);
                tab->group_sched[key] = sg_table::GroupSched{pl->cfg.tile, pl->cfg.grid_wgs, pl->cfg.order, sec};
            }
        }
    }
    if (rc) {
        sg_group_plan_destroy(pl);
        return rc;
    }
    *out = pl;
    return SG_OK;
}

int sg_group_plan_launch(sg_group_plan* pl, void* stream) {
    if (!pl) return fail(SG_EINVAL, "NULL plan");
    return plan_enqueue(pl, (hipStream_t)stream);
}

int sg_group_plan_update(sg_group_plan* pl, const sg_problem* probs, void* stream) {
    if (!pl) return fail(SG_EINVAL, "NULL plan");
    int rc = validate_problems(pl->G, probs);
    if (rc) return rc;
    const int old_tiles = pl->total_tiles, old_grid = pl->grid;
    const bool old_aligned = pl->all_aligned;
    rc = plan_upload(pl, probs, (hipStream_t)stream);
    if (rc) return rc;
    if (pl->total_tiles != old_tiles || pl->grid != old_grid || pl->all_aligned != old_aligned) {
        // a captured graph bakes in the launch arguments and the kernel (the all-aligned one
        // carries no element-wise body): signal that it must be recaptured
        return fail(SG_EAGAIN, "grouped: tile count, grid or kernel changed; recapture graphs that hold this plan");
    }
    return SG_OK;
}

int sg_group_plan_info(const sg_group_plan* pl, sg_group_cfg* cfg, int* total_tiles, int* grid, double* flops) {
    if (!pl) return fail(SG_EINVAL, "NULL plan");
    if (cfg) *cfg = pl->cfg;
    if (total_tiles) *total_tiles = pl->total_tiles;
    if (grid) *grid = pl->grid;
    if (flops) *flops = pl->flops;
    return SG_OK;
}

int sg_group_plan_destroy(sg_group_plan* pl) {
    if (!pl) return SG_OK;
    // every resource is released even after a failure; the first HIP error is reported
    hipError_t first = hipDeviceSynchronize();
    const char* what = "hipDeviceSynchronize";
    if (pl->d_probs) {
        const hipError_t e = hipFree(pl->d_probs);
        if (first == hipSuccess && e != hipSuccess) { first = e; what = "hipFree"; }
    }
    if (pl->d_counters) {
        const hipError_t e = hipFree(pl->d_counters);
        if (first == hipSuccess && e != hipSuccess) { first = e; what = "hipFree"; }
    }
    delete pl;
    return first == hipSuccess ? SG_OK : hip_fail(first, what);
}

int sg_gemm_grouped(sg_ctx* ctx, int G, const sg_problem* probs, int c_dtype, const sg_group_cfg* cfg,
                    void* stream) {
    sg_group_plan* pl = nullptr;
    int rc = sg_group_plan_create(ctx, G, probs, c_dtype, cfg, stream, &pl);
    if (rc) return rc;
    rc = plan_enqueue(pl, (hipStream_t)stream);
    if (rc == SG_OK && hipStreamSynchronize((hipStream_t)stream) != hipSuccess) rc = fail(SG_EHIP, "grouped: sync failed");
    sg_group_plan_destroy(pl);
    return rc;
}

int sg_graph_capture_groups(sg_group_plan* const* plans, int n, void* stream, sg_graph** out) {
    if (!plans || n <= 0 || !out) return fail(SG_EINVAL, "bad arguments");
    *out = nullptr;
    hipStream_t s = (hipStream_t)stream;
    if (!s) return fail(SG_EINVAL, "graph capture needs a non-null stream");
    sg_graph* g = new (std::nothrow) sg_graph();
    if (!g) return fail(SG_ENOMEM, "graph allocation failed");
    SG_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = SG_OK;
    for (int i = 0; i < n && rc == SG_OK; ++i) {
        if (!plans[i]) { rc = fail(SG_EINVAL, "NULL plan"); break; }
        rc = plan_enqueue(plans[i], s);
    }
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc == SG_OK && e != hipSuccess) rc = hip_fail(e, "hipStreamEndCapture");
    if (rc == SG_OK) {
        e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
        if (e != hipSuccess) rc = hip_fail(e, "hipGraphInstantiate");
    }
    g->graph = graph;
    if (rc) {
        sg_graph_destroy(g);
        return rc;
    }
    *out = g;
    return SG_OK;
}

int sg_graph_launch(sg_graph* g, void* stream) {
    if (!g || !g->exec) return fail(SG_EINVAL, "NULL graph");
    SG_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
    return SG_OK;
}

int sg_graph_destroy(sg_graph* g) {
    if (!g) return SG_OK;
    hipError_t first = hipSuccess;
    if (g->exec) first = hipGraphExecDestroy(g->exec);
    if (g->graph) {
        const hipError_t e = hipGraphDestroy(g->graph);
        if (first == hipSuccess) first = e;
    }
    delete g;
    return first == hipSuccess ? SG_OK : hip_fail(first, "graph destroy");
}

}  // extern "C"
