// smoothgemm host runtime: contexts, the per-call GEMM entry points, plan execution, the sweep
// driver, the memory-study sweep and the landscape metrics.  The dispatch-table construction
// lives in table.cpp.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "sg_internal.h"
#include "sg_table.h"

namespace sg {

static thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return SG_EHIP;
}

}  // namespace sg

using namespace sg;

struct sg_ctx {
    int device = 0;
    int num_cus = 0;
    int plain_variant = 0;
    int progress_every = 0;           // >0: a stderr line every this many shapes
    void* ws = nullptr;
    size_t ws_bytes = 0;
    const sg_table* table = nullptr;
    std::vector<hipEvent_t> events;   // stamped by kernel dispatches only
    std::vector<hipEvent_t> marks;    // recorded on streams only (forks, joins, interval ends):
                                      // an event is never used both ways
    // concurrent execution of split plans: the pieces of a plan without K pieces go to these
    // streams (default priority), forked from and joined back into the caller's stream
    int concurrent_splits = 0;    // 0 off, 1 concurrent streams, 2 sequential timed like 1,
                                  // 3 one persistent grouped launch of the pieces
    std::vector<hipStream_t> aux;
    // mode 3: the pieces' descriptors (host copy, device copy) and the queue counters
    std::vector<GroupProblem> gp_host;
    GroupProblem* gp_dev = nullptr;
    int gp_cap = 0;
    int* gp_counters = nullptr;
    // accounting of the most recent sweep (timed runs only)
    std::vector<int64_t> acct_launches;
    std::vector<double> acct_seconds;
    std::vector<double> acct_flops;
    // interval timing: sweeps also time each run between two markers on the caller's stream
    // (launch and inter-kernel gaps included); per-shape means of the most recent sweep
    int interval_timing = 0;
    std::vector<double> interval_sec;
};

namespace {

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

int ensure_events(sg_ctx* ctx, size_t n) {
    while (ctx->events.size() < n) {
        hipEvent_t e;
        SG_HIP(hipEventCreate(&e));
        ctx->events.push_back(e);
    }
    return SG_OK;
}

int ensure_marks(sg_ctx* ctx, size_t n) {
    while (ctx->marks.size() < n) {
        hipEvent_t e;
        SG_HIP(hipEventCreate(&e));
        ctx->marks.push_back(e);
    }
    return SG_OK;
}

int ensure_ws(sg_ctx* ctx, size_t bytes) {
    if (bytes <= ctx->ws_bytes) return SG_OK;
    size_t want = std::max(bytes, ctx->ws_bytes * 2);
    want = (want + 0xFFFFF) & ~size_t(0xFFFFF);
    void* p = nullptr;
    if (ctx->ws) {
        // the old buffer may still be read by queued work: wait for the device first
        SG_HIP(hipDeviceSynchronize());
        SG_HIP(hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
    }
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SG_ENOMEM, "workspace allocation of " + std::to_string(want) + " bytes failed");
    }
    ctx->ws = p;
    ctx->ws_bytes = want;
    return SG_OK;
}

// One leaf of an execution plan: a sub-problem run by one variant.
struct Leaf {
    int64_t m0, n0, k0, m, n, k;  // data region (elements)
    int64_t Ml, Nl, Kl;           // launch extent (>= data; padding)
    int variant;
    bool first, last;             // first / last piece along K of its output region
};

// Expand the table plan of a problem of actual size (m, n, k) at offset (m0, n0, k0).
// `cell` is the grid cell whose record applies (sizes in steps).  A split point at or beyond
// the actual extent drops the empty piece and runs the covering piece's plan on the whole
// region (its cell still covers it).
void expand_plan(const sg_table* t, int64_t m0, int64_t n0, int64_t k0, int64_t m, int64_t n,
                 int64_t k, int cm, int cn, int ck, bool first, bool last, std::vector<Leaf>& out) {
    const int g = t->grid.step;
    const int64_t c = t->cell_index(cm, cn, ck);
    const int act = t->action[c];
    const int arg = t->arg[c];
    if (act == SG_ACT_AS_IS || act == SG_ACT_PAD) {
        Leaf L;
        L.m0 = m0; L.n0 = n0; L.k0 = k0; L.m = m; L.n = n; L.k = k;
        int64_t run = (act == SG_ACT_AS_IS) ? c : arg;
        int rm, rn, rk;
        t->cell_coords(run, &rm, &rn, &rk);
        if (act == SG_ACT_PAD) {
            // the target's variant over the target's M and N extent (tiles wholly outside the
            // data exit at once) and over the region's own depth: depth beyond K would only add
            // products of zeros -- more MFMA work, the same tile grid and the same result
            (void)rk;
            L.Ml = std::max<int64_t>(m, (int64_t)(rm + 1) * g);
            L.Nl = std::max<int64_t>(n, (int64_t)(rn + 1) * g);
            L.Kl = k;
        } else {
            L.Ml = m; L.Nl = n; L.Kl = k;
        }
        L.variant = t->best_var[run];
        L.first = first;
        L.last = last;
        out.push_back(L);
        return;
    }
    const int64_t p = (int64_t)arg * g;  // split point in elements
    if (act == SG_ACT_SPLIT_M) {
        if (p >= m) { expand_plan(t, m0, n0, k0, m, n, k, arg - 1, cn, ck, first, last, out); return; }
        expand_plan(t, m0, n0, k0, p, n, k, arg - 1, cn, ck, first, last, out);
        expand_plan(t, m0 + p, n0, k0, m - p, n, k, cm - arg, cn, ck, first, last, out);
    } else if (act == SG_ACT_SPLIT_N) {
        if (p >= n) { expand_plan(t, m0, n0, k0, m, n, k, cm, arg - 1, ck, first, last, out); return; }
        expand_plan(t, m0, n0, k0, m, p, k, cm, arg - 1, ck, first, last, out);
        expand_plan(t, m0, n0 + p, k0, m, n - p, k, cm, cn - arg, ck, first, last, out);
    } else {
        if (p >= k) { expand_plan(t, m0, n0, k0, m, n, k, cm, cn, arg - 1, first, last, out); return; }
        expand_plan(t, m0, n0, k0, m, n, p, cm, cn, arg - 1, first, false, out);
        expand_plan(t, m0, n0, k0 + p, m, n, k - p, cm, cn, ck - arg, false, last, out);
    }
}

// Off-grid plan choice.  A cell's plan was made for the cell's own sizes.  On a shape inside
// the cell but off the grid, a split's pieces lose the alignment the split was chosen for while
// still paying their extra launches, and a pad target may fit the shape worse than the cell's
// own best variant.  So off the grid the plan is kept only when its leaves, each costed by its
// variant's T0 interpolated at the leaf's launch extent, are estimated at least kOffGridMargin
// faster than the cell's best-of-N variant on the whole shape; on the grid the table's plan
// always runs.  The margin is measured: over 4,096 shapes U{1..8192}^3 on a step-256 table,
// split plans estimated 0-5 % faster ran 5.4 % slower than the best variant alone, 5-10 %
// faster broke even, and more than 10 % faster ran 7-18 % faster; pads estimated up to 10 %
// faster ran 0-1 % slower (the interpolation sees neither a piece's own launch and tail nor
// the tile quantization between grid points).
constexpr double kOffGridMargin = 0.05;
void plan_estimates(const sg_table* t, const std::vector<Leaf>& leaves, int64_t M, int64_t N,
                    int64_t K, int best_variant, double* est_plan, double* est_best) {
    double e = 0.0;
    for (const Leaf& L : leaves) {
        const int r = variant_row(t, L.variant);
        e += r >= 0 ? t0_interp(t, r, L.Ml, L.Nl, L.Kl) : HUGE_VAL;
    }
    *est_plan = e;
    const int rb = variant_row(t, best_variant);
    *est_best = rb >= 0 ? t0_interp(t, rb, M, N, K) : HUGE_VAL;
}

// The table's plan for (M, N, K), or off the grid the cell's best variant alone when that is
// estimated faster (above).  *use_plan (optional) says which.
void table_plan(const sg_table* t, int64_t M, int64_t N, int64_t K, int cm, int cn, int ck,
                std::vector<Leaf>& leaves, double* est_plan, double* est_best, int* use_plan) {
    leaves.clear();
    expand_plan(t, 0, 0, 0, M, N, K, cm, cn, ck, true, true, leaves);
    const bool on_grid = t->on_grid(M, N, K);
    if (on_grid && !est_plan && !est_best && !use_plan) return;     // the lookup alone
    const int vb = t->best_var[t->cell_index(cm, cn, ck)];
    double ep = 0.0, eb = 0.0;
    plan_estimates(t, leaves, M, N, K, vb, &ep, &eb);
    const bool keep = on_grid || ep <= (1.0 - kOffGridMargin) * eb;
    if (!keep) leaves.assign(1, Leaf{0, 0, 0, M, N, K, M, N, K, vb, true, true});
    if (est_plan) *est_plan = ep;
    if (est_best) *est_best = eb;
    if (use_plan) *use_plan = keep ? 1 : 0;
}

struct Problem {
    int64_t M, N, K;
    const uint16_t* A; int64_t lda;
    const uint16_t* B; int64_t ldb;
    void* C; int64_t ldc;
    int c_bf16;
    int beta;
    int mem_only;   // SG_MODE_MEMORY: every leaf runs its variant's memory-only twin
};

// Plan of one call as a list of leaves (single leaf for PLAIN / VARIANT / BEST).
int make_plan(const sg_ctx* ctx, const Problem& pr, int mode, int variant, std::vector<Leaf>& leaves) {
    leaves.clear();
    if (mode == SG_MODE_DEFAULT) mode = ctx->table ? SG_MODE_DP : SG_MODE_PLAIN;
    if (mode == SG_MODE_PLAIN || mode == SG_MODE_VARIANT || mode == SG_MODE_MEMORY) {
        const int v = (mode == SG_MODE_PLAIN) ? ctx->plain_variant : variant;
        if (v < 0 || v >= kNumVariants) return fail(SG_EINVAL, "variant out of range");
        leaves.push_back(Leaf{0, 0, 0, pr.M, pr.N, pr.K, pr.M, pr.N, pr.K, v, true, true});
        return SG_OK;
    }
    if (mode != SG_MODE_BEST && mode != SG_MODE_DP) return fail(SG_EINVAL, "unknown mode");
    const sg_table* t = ctx->table;
    if (!t) return fail(SG_ENOTABLE, "table-driven mode requested but no dispatch table is set");
    int cm, cn, ck;
    if (!t->covering_cell(pr.M, pr.N, pr.K, &cm, &cn, &ck))
        return fail(SG_ERANGE, "shape outside the dispatch table's grid");
    if (mode == SG_MODE_BEST) {
        const int v = t->best_var[t->cell_index(cm, cn, ck)];
        leaves.push_back(Leaf{0, 0, 0, pr.M, pr.N, pr.K, pr.M, pr.N, pr.K, v, true, true});
        return SG_OK;
    }
    table_plan(t, pr.M, pr.N, pr.K, cm, cn, ck, leaves, nullptr, nullptr, nullptr);
    return SG_OK;
}

// Workspace layout: [plan accumulator M*N FP32 (only for BF16 output with a K split)]
//                   [split-K partials of the largest leaf].
size_t plan_workspace(const Problem& pr, const std::vector<Leaf>& leaves, size_t* acc_bytes) {
    bool ksplit = false;
    size_t part = 0;
    for (const Leaf& L : leaves) {
        if (!(L.first && L.last)) ksplit = true;
        LaunchDesc d{};
        d.M = L.m; d.N = L.n; d.K = L.k; d.Ml = L.Ml; d.Nl = L.Nl; d.Kl = L.Kl;
        d.A = pr.A + L.m0 * pr.lda + L.k0; d.lda = pr.lda;   // operand views, as run_leaf
        d.B = pr.B + L.k0 * pr.ldb + L.n0; d.ldb = pr.ldb;
        part = std::max(part, launch_workspace_bytes(L.variant, d));
    }
    size_t acc = (ksplit && pr.c_bf16) ? (size_t)pr.M * (size_t)pr.N * sizeof(float) : 0;
    acc = (acc + 255) & ~size_t(255);
    *acc_bytes = acc;
    return acc + part;
}

// A plan whose leaves may run at the same time: two or more leaves, none of them a K piece
// (K pieces accumulate into one output region; M and N pieces write disjoint regions).
bool plan_is_concurrent(const std::vector<Leaf>& leaves) {
    if (leaves.size() < 2) return false;
    for (const Leaf& L : leaves)
        if (!(L.first && L.last)) return false;
    return true;
}

// Workspace of a concurrent plan: one slice per leaf (split-K partials, packed operands), so
// leaves in flight together never share scratch.  offs[i] = byte offset of leaf i's slice.
size_t plan_workspace_concurrent(const Problem& pr, const std::vector<Leaf>& leaves, std::vector<size_t>& offs) {
    size_t total = 0;
    offs.clear();
    for (const Leaf& L : leaves) {
        LaunchDesc d{};
        d.M = L.m; d.N = L.n; d.K = L.k; d.Ml = L.Ml; d.Nl = L.Nl; d.Kl = L.Kl;
        d.A = pr.A + L.m0 * pr.lda + L.k0; d.lda = pr.lda;
        d.B = pr.B + L.k0 * pr.ldb + L.n0; d.ldb = pr.ldb;
        offs.push_back(total);
        total += (launch_workspace_bytes(L.variant, d) + 255) & ~size_t(255);
    }
    return total;
}

// Launch description of one leaf.  Output routing (C FP32: accumulate in place; C BF16 with a
// K split: accumulate in the FP32 plan accumulator W and round once in the last piece).
LaunchDesc leaf_desc(const Problem& pr, const Leaf& L, void* ws) {
    LaunchDesc d{};
    d.mem_only = pr.mem_only;
    d.M = L.m; d.N = L.n; d.K = L.k; d.Ml = L.Ml; d.Nl = L.Nl; d.Kl = L.Kl;
    d.A = pr.A + L.m0 * pr.lda + L.k0; d.lda = pr.lda;
    d.B = pr.B + L.k0 * pr.ldb + L.n0; d.ldb = pr.ldb;
    const int64_t coff = L.m0 * pr.ldc + L.n0;
    float* W = (float*)ws;
    const int64_t woff = L.m0 * pr.N + L.n0;
    if (!pr.c_bf16) {
        d.C = (float*)pr.C + coff; d.ldc = pr.ldc; d.out_bf16 = 0;
        const bool accumulate = !L.first || pr.beta;
        d.add = accumulate ? d.C : nullptr; d.ldadd = pr.ldc; d.add_kind = accumulate ? ADD_F32 : ADD_NONE;
    } else if (L.first && L.last) {
        d.C = (uint16_t*)pr.C + coff; d.ldc = pr.ldc; d.out_bf16 = 1;
        d.add = pr.beta ? d.C : nullptr; d.ldadd = pr.ldc; d.add_kind = pr.beta ? ADD_BF16 : ADD_NONE;
    } else if (!L.last) {
        d.C = W + woff; d.ldc = pr.N; d.out_bf16 = 0;
        if (L.first) {
            d.add = pr.beta ? (const void*)((uint16_t*)pr.C + coff) : nullptr;
            d.ldadd = pr.ldc; d.add_kind = pr.beta ? ADD_BF16 : ADD_NONE;
        } else {
            d.add = W + woff; d.ldadd = pr.N; d.add_kind = ADD_F32;
        }
    } else {  // last piece of a K split, BF16 output: round (W + acc) once
        d.C = (uint16_t*)pr.C + coff; d.ldc = pr.ldc; d.out_bf16 = 1;
        d.add = W + woff; d.ldadd = pr.N; d.add_kind = ADD_F32;
    }
    return d;
}

// Enqueue one leaf; the events (may be null) are stamped as LaunchDesc describes.
int run_leaf(const Problem& pr, const Leaf& L, void* ws, size_t acc_bytes, hipStream_t s,
             hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr, hipEvent_t ev_mid = nullptr) {
    LaunchDesc d = leaf_desc(pr, L, ws);
    d.ev_start = ev_start;
    d.ev_mid = ev_mid;
    d.ev_stop = ev_stop;
    return launch_variant(L.variant, d, (char*)ws + acc_bytes, s);
}

__global__ void sg_scale_zero_f32(float* C, int64_t ldc, int64_t M, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M * N;
         i += (int64_t)gridDim.x * blockDim.x)
        C[(i / N) * ldc + i % N] = 0.0f;
}
__global__ void sg_scale_zero_bf16(uint16_t* C, int64_t ldc, int64_t M, int64_t N) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < M * N;
         i += (int64_t)gridDim.x * blockDim.x)
        C[(i / N) * ldc + i % N] = 0;
}

int validate(const sg_gemm_args* a) {
    if (!a) return fail(SG_EINVAL, "NULL args");
    if (a->M < 0 || a->N < 0 || a->K < 0) return fail(SG_EINVAL, "negative dimension");
    if (a->c_dtype != SG_F32 && a->c_dtype != SG_BF16) return fail(SG_EINVAL, "bad c_dtype");
    if (a->beta != 0 && a->beta != 1) return fail(SG_EINVAL, "beta must be 0 or 1");
    if (a->mode < SG_MODE_DEFAULT || a->mode > SG_MODE_MEMORY) return fail(SG_EINVAL, "bad mode");
    if (a->M == 0 || a->N == 0) return SG_OK;
    if (!a->C) return fail(SG_EINVAL, "NULL C with non-zero size");
    if (a->ldc < a->N) return fail(SG_EINVAL, "ldc < N");
    if (a->K > 0) {
        if (!a->A || !a->B) return fail(SG_EINVAL, "NULL A or B with non-zero size");
        if (a->lda < a->K || a->ldb < a->N) return fail(SG_EINVAL, "leading dimension too small");
    }
    if (a->M > 0x7FFFFFFF || a->N > 0x7FFFFFFF || a->K > 0x7FFFFFFF)
        return fail(SG_EINVAL, "dimension exceeds 2^31 - 1");
    return SG_OK;
}

constexpr size_t kMaxAux = 4;   // streams for the pieces of one concurrent plan

int ensure_aux(sg_ctx* ctx, size_t n) {
    while (ctx->aux.size() < n) {
        hipStream_t st;
        SG_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));   // default priority
        ctx->aux.push_back(st);
    }
    return SG_OK;
}

// Enqueue a concurrent plan: `fork` is recorded on s and every auxiliary stream waits for it;
// leaf i runs on stream i % n in its own workspace slice offs[i]; each stream then records
// joins[j] and s waits for all of them.
int run_concurrent(sg_ctx* ctx, const Problem& pr, const std::vector<Leaf>& leaves,
                   const std::vector<size_t>& offs, hipStream_t s, hipEvent_t fork, const hipEvent_t* joins) {
    const size_t ns = std::min(leaves.size(), kMaxAux);
    int rc = ensure_aux(ctx, ns);
    if (rc) return rc;
    SG_HIP(hipEventRecord(fork, s));
    for (size_t j = 0; j < ns; ++j) SG_HIP(hipStreamWaitEvent(ctx->aux[j], fork, 0));
    for (size_t i = 0; i < leaves.size(); ++i) {
        rc = run_leaf(pr, leaves[i], ctx->ws, offs[i], ctx->aux[i % ns]);
        if (rc) return rc;
    }
    for (size_t j = 0; j < ns; ++j) {
        SG_HIP(hipEventRecord(joins[j], ctx->aux[j]));
        SG_HIP(hipStreamWaitEvent(s, joins[j], 0));
    }
    return SG_OK;
}

// Mode 3: the tile shape shared by every piece of a concurrent plan when they can all run in
// one grouped launch (no split-K or stream-K piece, no addend, a tile the grouped kernel
// carries), else -1.
int grouped_pieces_tile(const Problem& pr, const std::vector<Leaf>& leaves) {
    if (pr.beta || pr.mem_only || !plan_is_concurrent(leaves)) return -1;
    const int t = variant_tile(leaves[0].variant);
    for (const Leaf& L : leaves)
        if (variant_is_sk(L.variant) || variant_splits(L.variant) != 1 || variant_tile(L.variant) != t)
            return -1;
    return t < kNumGroupTiles ? t : -1;
}

// Mode 3: enqueue the pieces as one persistent grouped launch of tile t: descriptors built on
// the host and copied (from pageable memory, so the host copy is free again when the call
// returns) to a device buffer the context keeps, then the grouped kernel.
int run_grouped_pieces(sg_ctx* ctx, const Problem& pr, const std::vector<Leaf>& leaves, int t, hipStream_t s) {
    const int G = (int)leaves.size();
    if (G > ctx->gp_cap) {
        if (ctx->gp_dev) {
            SG_HIP(hipDeviceSynchronize());         // queued launches may still read the old buffer
            SG_HIP(hipFree(ctx->gp_dev));
            ctx->gp_dev = nullptr;
            ctx->gp_cap = 0;
        }
        SG_HIP(hipMalloc(&ctx->gp_dev, sizeof(GroupProblem) * (size_t)G));
        ctx->gp_cap = G;
    }
    if (!ctx->gp_counters) {
        SG_HIP(hipMalloc(&ctx->gp_counters, 2 * sizeof(int)));
        SG_HIP(hipMemset(ctx->gp_counters, 0, 2 * sizeof(int)));   // every launch returns them to zero
    }
    const size_t esz = pr.c_bf16 ? 2 : 4;
    std::vector<sg_problem> probs(G);
    for (int i = 0; i < G; ++i) {
        const Leaf& L = leaves[i];
        probs[i] = sg_problem{L.m, L.n, L.k, pr.A + L.m0 * pr.lda + L.k0, pr.lda, pr.B + L.k0 * pr.ldb + L.n0,
                              pr.ldb, (char*)pr.C + (L.m0 * pr.ldc + L.n0) * esz, pr.ldc};
    }
    ctx->gp_host.resize(G);
    std::vector<int> order(G);
    int total = 0, grid = 0;
    double fl = 0.0;
    bool aa = false;
    int rc = grouped_fill(probs.data(), G, t, pr.c_bf16 ? SG_BF16 : SG_F32, true, ctx->gp_host.data(), order.data(),
                          &total, &fl, &aa);
    if (rc) return rc;
    rc = grouped_grid(t, aa, ctx->device, total, 0, &grid);
    if (rc) return rc;
    SG_HIP(hipMemcpyAsync(ctx->gp_dev, ctx->gp_host.data(), sizeof(GroupProblem) * (size_t)G, hipMemcpyHostToDevice, s));
    return grouped_enqueue(t, aa, ctx->gp_dev, G, total, grid, pr.c_bf16 ? SG_BF16 : SG_F32, ctx->gp_counters, s,
                           nullptr, nullptr);
}

// One call.  fixed_ws != nullptr: run in that caller-provided scratch of fixed_cap bytes
// instead of the context's workspace (no allocation, pieces always one after another); a plan
// that needs more gives SG_ERANGE before anything is enqueued.
int gemm_impl(sg_ctx* ctx, const sg_gemm_args* a, hipStream_t s, std::vector<Leaf>* keep = nullptr,
              void* fixed_ws = nullptr, size_t fixed_cap = 0) {
    int rc = validate(a);
    if (rc) return rc;
    if (a->M == 0 || a->N == 0) return SG_OK;
    if (a->K == 0) {
        if (a->beta) return SG_OK;
        int64_t blocks = std::min<int64_t>((a->M * a->N + 255) / 256, 65536);
        if (a->c_dtype == SG_F32)
            hipLaunchKernelGGL(sg_scale_zero_f32, dim3((unsigned)blocks), dim3(256), 0, s,
                               (float*)a->C, a->ldc, a->M, a->N);
        else
            hipLaunchKernelGGL(sg_scale_zero_bf16, dim3((unsigned)blocks), dim3(256), 0, s,
                               (uint16_t*)a->C, a->ldc, a->M, a->N);
        SG_HIP(hipGetLastError());
        return SG_OK;
    }
    Problem pr{a->M, a->N, a->K, (const uint16_t*)a->A, a->lda, (const uint16_t*)a->B, a->ldb,
               a->C, a->ldc, a->c_dtype == SG_BF16, a->beta, a->mode == SG_MODE_MEMORY};
    std::vector<Leaf> local;
    std::vector<Leaf>& leaves = keep ? *keep : local;
    rc = make_plan(ctx, pr, a->mode, a->variant, leaves);
    if (rc) return rc;
    if (fixed_ws) {
        size_t acc_bytes = 0;
        const size_t need = plan_workspace(pr, leaves, &acc_bytes);
        if (need > fixed_cap)
            return fail(SG_ERANGE, "this call needs " + std::to_string(need) + " bytes of scratch; the "
                        "no-allocation entry point has " + std::to_string(fixed_cap));
        for (const Leaf& L : leaves) {
            rc = run_leaf(pr, L, fixed_ws, acc_bytes, s);
            if (rc) return rc;
        }
        return SG_OK;
    }
    if (ctx->concurrent_splits == 3) {
        const int t = grouped_pieces_tile(pr, leaves);
        if (t >= 0) return run_grouped_pieces(ctx, pr, leaves, t, s);
    }
    if (ctx->concurrent_splits == 1 && plan_is_concurrent(leaves)) {
        std::vector<size_t> offs;
        rc = ensure_ws(ctx, plan_workspace_concurrent(pr, leaves, offs));
        if (rc) return rc;
        rc = ensure_marks(ctx, 1 + kMaxAux);
        if (rc) return rc;
        return run_concurrent(ctx, pr, leaves, offs, s, ctx->marks[0], &ctx->marks[1]);
    }
    size_t acc_bytes = 0;
    size_t need = plan_workspace(pr, leaves, &acc_bytes);
    rc = ensure_ws(ctx, need);
    if (rc) return rc;
    for (const Leaf& L : leaves) {
        rc = run_leaf(pr, L, ctx->ws, acc_bytes, s);
        if (rc) return rc;
    }
    return SG_OK;
}

std::mutex g_default_mu;
sg_ctx* g_default[64] = {nullptr};

// ---- fixed device scratch for gemm_bf16_nn_ex_noalloc ----------------------------------------
// Split-K partials, zero-padded operand copies and the FP32 accumulator of BF16 K-split plans
// of the no-allocation entry point live here.  Every call writes each byte it later reads (the
// partial slices, the packed copies and the accumulator's first piece are written whole), so
// nothing needs clearing between calls.  In host code `scratch` only names the symbol: the
// device address of each GPU's copy comes from hipGetSymbolAddress, taken once per device when
// a context is created on it, and only that address is handed to kernels.
constexpr size_t kScratchBytes = (size_t)256 << 20;
__device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {nullptr};

// With `device` current: look up this device's copy of the scratch array (once per device).
int scratch_init(int device) {
    if (device < 0 || device >= 64) return fail(SG_EINVAL, "device ordinal too large");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return SG_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!p) return fail(SG_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = p;
    return SG_OK;
}

void* scratch_of(int device) {
    if (device < 0 || device >= 64) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}

}  // namespace

namespace sg {
const sg_table* ctx_table(const sg_ctx* ctx) { return ctx ? ctx->table : nullptr; }
}  // namespace sg

extern "C" {

const char* sg_last_error(void) { return g_err.c_str(); }
const char* sg_version(void) { return "smoothgemm 0.1 (gfx950)"; }

int sg_ctx_create(int device, sg_ctx** out) {
    if (!out) return fail(SG_EINVAL, "NULL out");
    *out = nullptr;
    int n = 0;
    SG_HIP(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(SG_EINVAL, "no such device");
    DeviceGuard guard(device);
    hipDeviceProp_t prop;
    SG_HIP(hipGetDeviceProperties(&prop, device));
    sg_ctx* c = new (std::nothrow) sg_ctx();
    if (!c) return fail(SG_ENOMEM, "context allocation failed");
    c->device = device;
    c->num_cus = prop.multiProcessorCount;
    c->acct_launches.assign(kNumVariants, 0);
    c->acct_seconds.assign(kNumVariants, 0.0);
    c->acct_flops.assign(kNumVariants, 0.0);
    const int rc = scratch_init(device);     // the device's scratch address, for the no-allocation call
    if (rc) {
        delete c;
        return rc;
    }
    *out = c;
    return SG_OK;
}

int sg_ctx_destroy(sg_ctx* ctx) {
    if (!ctx) return SG_OK;
    {
        std::lock_guard<std::mutex> lk(g_default_mu);
        for (sg_ctx*& d : g_default)
            if (d == ctx) d = nullptr;              // a destroyed default context is recreated on use
    }
    DeviceGuard guard(ctx->device);
    // every resource is released even after a failure; the first HIP error is reported
    hipError_t first = hipSuccess;
    const char* what = nullptr;
    auto note = [&](hipError_t e, const char* w) {
        if (e != hipSuccess && first == hipSuccess) { first = e; what = w; }
    };
    for (hipStream_t st : ctx->aux) {
        note(hipStreamSynchronize(st), "hipStreamSynchronize");
        note(hipStreamDestroy(st), "hipStreamDestroy");
    }
    if (ctx->gp_dev || ctx->gp_counters) note(hipDeviceSynchronize(), "hipDeviceSynchronize");
    if (ctx->gp_dev) note(hipFree(ctx->gp_dev), "hipFree");
    if (ctx->gp_counters) note(hipFree(ctx->gp_counters), "hipFree");
    for (hipEvent_t e : ctx->events) note(hipEventDestroy(e), "hipEventDestroy");
    for (hipEvent_t e : ctx->marks) note(hipEventDestroy(e), "hipEventDestroy");
    if (ctx->ws) {
        note(hipDeviceSynchronize(), "hipDeviceSynchronize");
        note(hipFree(ctx->ws), "hipFree");
    }
    delete ctx;
    if (first != hipSuccess) return hip_fail(first, what);
    return SG_OK;
}

int sg_ctx_set_plain_variant(sg_ctx* ctx, int variant) {
    if (!ctx) return fail(SG_EINVAL, "NULL ctx");
    if (variant < 0 || variant >= kNumVariants) return fail(SG_EINVAL, "variant out of range");
    ctx->plain_variant = variant;
    return SG_OK;
}

int sg_ctx_set_concurrent_splits(sg_ctx* ctx, int on) {
    if (!ctx || on < 0 || on > 3) return fail(SG_EINVAL, "bad argument");
    ctx->concurrent_splits = on;
    return SG_OK;
}

int sg_ctx_set_progress(sg_ctx* ctx, int every) {
    if (!ctx || every < 0) return fail(SG_EINVAL, "bad argument");
    ctx->progress_every = every;
    return SG_OK;
}

int sg_ctx_reserve_workspace(sg_ctx* ctx, size_t bytes) {
    if (!ctx) return fail(SG_EINVAL, "NULL ctx");
    DeviceGuard guard(ctx->device);
    return ensure_ws(ctx, bytes);
}

int sg_ctx_set_table(sg_ctx* ctx, const sg_table* t) {
    if (!ctx) return fail(SG_EINVAL, "NULL ctx");
    ctx->table = t;
    return SG_OK;
}

// The per-device default context of the paper-form call, created on first use.  Called with
// g_default_mu held.
static int default_ctx_locked(int dev, sg_ctx** out) {
    if (dev < 0 || dev >= 64) return fail(SG_EINVAL, "device ordinal out of range");
    if (!g_default[dev]) {
        int n = 0;
        SG_HIP(hipGetDeviceCount(&n));
        if (dev >= n) return fail(SG_EINVAL, "no such device");
        const int rc = sg_ctx_create(dev, &g_default[dev]);
        if (rc) return rc;
    }
    *out = g_default[dev];
    return SG_OK;
}

int sg_default_ctx(int device, sg_ctx** out) {
    if (!out) return fail(SG_EINVAL, "NULL out");
    std::lock_guard<std::mutex> lk(g_default_mu);
    return default_ctx_locked(device, out);
}

int sg_set_default_table(int device, const sg_table* t) {
    std::lock_guard<std::mutex> lk(g_default_mu);
    sg_ctx* ctx = nullptr;
    const int rc = default_ctx_locked(device, &ctx);
    if (rc) return rc;
    ctx->table = t;
    return SG_OK;
}

int gemm_bf16_nn(int64_t M, int64_t N, int64_t K, const void* A, const void* B, void* C) {
    int dev = 0;
    SG_HIP(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_default_mu);
    sg_ctx* ctx = nullptr;
    int rc = default_ctx_locked(dev, &ctx);
    if (rc) return rc;
    DeviceGuard guard(ctx->device);
    sg_gemm_args a{};
    a.M = M; a.N = N; a.K = K;
    a.A = A; a.lda = K; a.B = B; a.ldb = N; a.C = C; a.ldc = N;
    a.c_dtype = SG_F32; a.beta = 0; a.mode = SG_MODE_DEFAULT; a.variant = 0;
    return gemm_impl(ctx, &a, nullptr);
}

int gemm_bf16_nn_ex(sg_ctx* ctx, const sg_gemm_args* args, void* stream) {
    if (!ctx) return fail(SG_EINVAL, "NULL ctx");
    DeviceGuard guard(ctx->device);
    return gemm_impl(ctx, args, (hipStream_t)stream);
}

int gemm_bf16_nn_ex_noalloc(sg_ctx* ctx, const sg_gemm_args* args, void* stream) {
    if (!ctx) return fail(SG_EINVAL, "NULL ctx");
    DeviceGuard guard(ctx->device);
    void* ws = scratch_of(ctx->device);
    if (!ws) return fail(SG_EINVAL, "no scratch address for this device (create the context first)");
    // host-side leaf list kept per thread: it grows only for a plan longer than any before
    static thread_local std::vector<Leaf> leaves;
    if (leaves.capacity() < 256) leaves.reserve(256);
    return gemm_impl(ctx, args, (hipStream_t)stream, &leaves, ws, kScratchBytes);
}

size_t sg_noalloc_scratch_bytes(void) { return kScratchBytes; }

int sg_gemm_batch(sg_ctx* ctx, int G, const sg_problem* probs, int c_dtype, int mode, int variant,
                  void* stream) {
    if (!ctx || G < 0 || (G > 0 && !probs)) return fail(SG_EINVAL, "bad arguments");
    DeviceGuard guard(ctx->device);
    for (int i = 0; i < G; ++i) {
        const sg_problem& q = probs[i];
        sg_gemm_args a{};
        a.M = q.M; a.N = q.N; a.K = q.K;
        a.A = q.A; a.lda = q.lda; a.B = q.B; a.ldb = q.ldb; a.C = q.C; a.ldc = q.ldc;
        a.c_dtype = c_dtype; a.beta = 0; a.mode = mode; a.variant = variant;
        const int rc = gemm_impl(ctx, &a, (hipStream_t)stream);
        if (rc) return rc;
    }
    return SG_OK;
}

int sg_num_variants(void) { return kNumVariants; }

int sg_variant_info_get(int v, sg_variant_info* out) {
    if (!out || v < 0 || v >= kNumVariants) return fail(SG_EINVAL, "bad variant or NULL out");
    const TileShape& t = kTiles[variant_tile(v)];
    out->id = v;
    out->bm = t.bm;
    out->bn = t.bn;
    out->bk = tile_split_granule(variant_tile(v));
    out->splits = variant_splits(v);
    out->threads = 256;
    out->lds_bytes = lds_bytes_of_tile(variant_tile(v));
    if (variant_is_sk(v)) {
        out->splits = 0;
        std::snprintf(out->name, sizeof out->name, "%dx%dx%d_sk", t.bm, t.bn, out->bk);
    } else {
        std::snprintf(out->name, sizeof out->name, "%dx%dx%d_s%d", t.bm, t.bn, out->bk, out->splits);
    }
    return SG_OK;
}

double sg_roughness(const double* T, int64_t n) {
    if (!T || n < 2) return NAN;
    double s = 0.0;
    for (int64_t i = 0; i + 1 < n; ++i) s += std::fabs(T[i + 1] - T[i]);
    return s / (double)(n - 1);
}

int sg_landscape_stats(const double* tf, int nM, int nN, int nK, sg_stats* out) {
    if (!tf || !out || nM < 2 || nN < 2 || nK < 2) return fail(SG_EINVAL, "stats need every axis >= 2");
    auto at = [&](int m, int n, int k) { return tf[((int64_t)m * nN + n) * nK + k]; };
    double sum = 0.0, peak = -INFINITY;
    const int64_t total = (int64_t)nM * nN * nK;
    for (int64_t i = 0; i < total; ++i) {
        sum += tf[i];
        peak = std::max(peak, tf[i]);
    }
    std::vector<double> line;
    double rm = 0.0, rn = 0.0, rk = 0.0;
    line.resize(nM);
    for (int n = 0; n < nN; ++n)
        for (int k = 0; k < nK; ++k) {
            for (int m = 0; m < nM; ++m) line[m] = at(m, n, k);
            rm += sg_roughness(line.data(), nM);
        }
    line.resize(nN);
    for (int m = 0; m < nM; ++m)
        for (int k = 0; k < nK; ++k) {
            for (int n = 0; n < nN; ++n) line[n] = at(m, n, k);
            rn += sg_roughness(line.data(), nN);
        }
    line.resize(nK);
    for (int m = 0; m < nM; ++m)
        for (int n = 0; n < nN; ++n) {
            for (int k = 0; k < nK; ++k) line[k] = at(m, n, k);
            rk += sg_roughness(line.data(), nK);
        }
    out->mean = sum / (double)total;
    out->peak = peak;
    out->rough_m = rm / ((double)nN * nK);
    out->rough_n = rn / ((double)nM * nK);
    out->rough_k = rk / ((double)nM * nN);
    out->rough_3d = (out->rough_m + out->rough_n + out->rough_k) / 3.0;
    return SG_OK;
}

int sg_fill_bf16(void* dst, int64_t n, uint64_t seed, uint64_t stream, int64_t offset, int kind,
                 double scale, void* stream_handle) {
    return launch_fill((uint16_t*)dst, n, seed, stream, offset, kind, scale, (hipStream_t)stream_handle);
}

}  // extern "C"

// ---- sweep driver ----------------------------------------------------------------------------
namespace sg {

// Whether a leaf's launch runs a second kernel after its tile kernel (a split-K reduction over
// the splits that are not empty on the leaf's K extent, or a stream-K fix-up) and so stamps its
// mid event.
bool stamps_mid(const Problem& pr, const Leaf& L, void* ws) {
    return launch_has_second_kernel(L.variant, leaf_desc(pr, L, ws));
}

// Time `reps` runs of the plan `leaves` (after one untimed run).  Every kernel launch carries
// start/stop events stamped by its own dispatch packet, so a run's time is the sum of its
// kernels' execution times (host launch gaps excluded).  Returns mean seconds per run; adds
// per-variant tile-kernel time (a split-K reduction excluded: a third event ends at the tile
// kernel), launch counts and algorithmic FLOP to the context's accounting.
int time_plan_concurrent(sg_ctx* ctx, const Problem& pr, const std::vector<Leaf>& leaves, int reps,
                         hipStream_t s, double* sec, bool account);

// interval != nullptr: `reps` further runs follow, each bracketed by two markers recorded on s
// (from an event pool of their own) and carrying no per-dispatch timing events, and *interval
// receives their mean marker-to-marker time (kernels plus the gaps between them).
int time_plan(sg_ctx* ctx, const Problem& pr, const std::vector<Leaf>& leaves, int reps,
              hipStream_t s, double* sec, bool account, double* interval = nullptr) {
    if (ctx->concurrent_splits != 0 && plan_is_concurrent(leaves)) {
        const int rc = time_plan_concurrent(ctx, pr, leaves, reps, s, sec, account);
        if (rc == SG_OK && interval) *interval = *sec;      // already a marker interval
        return rc;
    }
    size_t acc_bytes = 0;
    int rc = ensure_ws(ctx, plan_workspace(pr, leaves, &acc_bytes));
    if (rc) return rc;
    for (const Leaf& L : leaves) {
        rc = run_leaf(pr, L, ctx->ws, acc_bytes, s);
        if (rc) return rc;
    }
    const size_t nl = leaves.size();
    const size_t ne = 3 * (size_t)reps * nl;       // start, stop, end of the tile kernel
    rc = ensure_events(ctx, ne);
    if (rc) return rc;
    size_t e = 0;
    for (int r = 0; r < reps; ++r) {
        for (const Leaf& L : leaves) {
            const bool split = stamps_mid(pr, L, ctx->ws);
            rc = run_leaf(pr, L, ctx->ws, acc_bytes, s, ctx->events[e], ctx->events[e + 1],
                          split ? ctx->events[e + 2] : nullptr);
            if (rc) return rc;
            e += 3;
        }
    }
    if (interval) {
        // `reps` more runs, each between two markers and with no timing events of its own
        // inside, so the interval holds the plan's kernels and the gaps between them only
        rc = ensure_marks(ctx, 2 * (size_t)reps);
        if (rc) return rc;
        for (int r = 0; r < reps; ++r) {
            SG_HIP(hipEventRecord(ctx->marks[2 * r], s));
            for (const Leaf& L : leaves) {
                rc = run_leaf(pr, L, ctx->ws, acc_bytes, s);
                if (rc) return rc;
            }
            SG_HIP(hipEventRecord(ctx->marks[2 * r + 1], s));
        }
    }
    SG_HIP(hipEventSynchronize(ctx->events[ne - 2]));
    if (interval) {
        SG_HIP(hipEventSynchronize(ctx->marks[2 * reps - 1]));
        double t = 0.0;
        for (int r = 0; r < reps; ++r) {
            float ms = 0.f;
            SG_HIP(hipEventElapsedTime(&ms, ctx->marks[2 * r], ctx->marks[2 * r + 1]));
            t += (double)ms * 1e-3;
        }
        *interval = t / reps;
    }
    double total = 0.0;
    e = 0;
    for (int r = 0; r < reps; ++r)
        for (const Leaf& L : leaves) {
            const bool split = stamps_mid(pr, L, ctx->ws);
            float ms = 0.f, ms_kernel = 0.f;
            SG_HIP(hipEventElapsedTime(&ms, ctx->events[e], ctx->events[e + 1]));
            if (split) SG_HIP(hipEventElapsedTime(&ms_kernel, ctx->events[e], ctx->events[e + 2]));
            else ms_kernel = ms;
            e += 3;
            total += (double)ms * 1e-3;
            if (account) {
                ctx->acct_launches[L.variant] += 1;
                ctx->acct_seconds[L.variant] += (double)ms_kernel * 1e-3;
                ctx->acct_flops[L.variant] += 2.0 * (double)L.m * (double)L.n * (double)L.k;
            }
        }
    *sec = total / reps;
    return SG_OK;
}

// The same for a plan whose leaves may run together: a run's time is the interval between two
// markers on the caller's stream, one before the leaves (the fork) and one after them (after
// the joins), so it includes the launch and fork / join latency that a sum of kernel times does
// not.  Mode 1 runs the leaves on the auxiliary streams; mode 2 runs them one after another on
// s, timed the same way, as the like-for-like reference.  These runs are not added to the
// per-variant kernel accounting.
int time_plan_concurrent(sg_ctx* ctx, const Problem& pr, const std::vector<Leaf>& leaves, int reps,
                         hipStream_t s, double* sec, bool /*account*/) {
    std::vector<size_t> offs;
    int rc = ensure_ws(ctx, plan_workspace_concurrent(pr, leaves, offs));
    if (rc) return rc;
    const size_t ns = std::min(leaves.size(), kMaxAux);
    const size_t per = 2 + ns;                     // fork, joins, end marker
    rc = ensure_marks(ctx, per * (size_t)reps);
    if (rc) return rc;
    const int gt = ctx->concurrent_splits == 3 ? grouped_pieces_tile(pr, leaves) : -1;
    auto run = [&](size_t b) -> int {
        if (ctx->concurrent_splits == 1) return run_concurrent(ctx, pr, leaves, offs, s, ctx->marks[b], &ctx->marks[b + 1]);
        SG_HIP(hipEventRecord(ctx->marks[b], s));
        if (gt >= 0) return run_grouped_pieces(ctx, pr, leaves, gt, s);
        for (size_t i = 0; i < leaves.size(); ++i) {
            int e = run_leaf(pr, leaves[i], ctx->ws, offs[i], s);
            if (e) return e;
        }
        return SG_OK;
    };
    rc = run(0);                                   // untimed
    if (rc) return rc;
    SG_HIP(hipStreamSynchronize(s));
    for (int r = 0; r < reps; ++r) {
        const size_t b = per * r;
        rc = run(b);
        if (rc) return rc;
        SG_HIP(hipEventRecord(ctx->marks[b + 1 + ns], s));
    }
    SG_HIP(hipStreamSynchronize(s));
    double total = 0.0;
    for (int r = 0; r < reps; ++r) {
        const size_t b = per * r;
        float ms = 0.f;
        SG_HIP(hipEventElapsedTime(&ms, ctx->marks[b], ctx->marks[b + 1 + ns]));
        total += (double)ms * 1e-3;
    }
    *sec = total / reps;
    return SG_OK;
}

}  // namespace sg

extern "C" int sg_table_plan_choice(const sg_table* t, int64_t M, int64_t N, int64_t K,
                                    double* est_plan, double* est_best, int* use_plan) {
    if (!t || !est_plan || !est_best || !use_plan) return fail(SG_EINVAL, "NULL argument");
    if (M <= 0 || N <= 0 || K <= 0) return fail(SG_EINVAL, "plan choice needs positive dims");
    int cm, cn, ck;
    if (!t->covering_cell(M, N, K, &cm, &cn, &ck)) return fail(SG_ERANGE, "shape outside the table grid");
    std::vector<Leaf> leaves;
    table_plan(t, M, N, K, cm, cn, ck, leaves, est_plan, est_best, use_plan);
    return SG_OK;
}

extern "C" int sg_sweep(sg_ctx* ctx, const sg_shape* shapes, int64_t n, int mode, int variant,
                        int c_dtype, int warmup, int reps, const void* A_pool, const void* B_pool,
                        void* C_pool, double* out_sec, void* stream) {
    if (!ctx || (n > 0 && (!shapes || !out_sec || !A_pool || !B_pool || !C_pool)))
        return fail(SG_EINVAL, "sg_sweep: NULL argument");
    if (n < 0 || warmup < 0 || reps < 1) return fail(SG_EINVAL, "sg_sweep: bad counts");
    if (c_dtype != SG_F32 && c_dtype != SG_BF16) return fail(SG_EINVAL, "bad c_dtype");
    DeviceGuard guard(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    std::fill(ctx->acct_launches.begin(), ctx->acct_launches.end(), 0);
    std::fill(ctx->acct_seconds.begin(), ctx->acct_seconds.end(), 0.0);
    std::fill(ctx->acct_flops.begin(), ctx->acct_flops.end(), 0.0);
    ctx->interval_sec.assign(ctx->interval_timing ? (size_t)n : 0, 0.0);
    std::vector<Leaf> leaves;
    for (int64_t i = 0; i < n; ++i) {
        const sg_shape& sh = shapes[i];
        if (sh.M <= 0 || sh.N <= 0 || sh.K <= 0) return fail(SG_EINVAL, "sg_sweep: empty shape");
        Problem pr{sh.M, sh.N, sh.K, (const uint16_t*)A_pool, sh.K, (const uint16_t*)B_pool, sh.N,
                   C_pool, sh.N, c_dtype == SG_BF16, 0, mode == SG_MODE_MEMORY};
        int rc = make_plan(ctx, pr, mode, variant, leaves);
        if (rc) return rc;
        if (i == 0) {
            size_t acc_bytes = 0;
            rc = ensure_ws(ctx, plan_workspace(pr, leaves, &acc_bytes));
            if (rc) return rc;
            for (int w = 0; w < warmup; ++w)
                for (const Leaf& L : leaves) {
                    rc = run_leaf(pr, L, ctx->ws, acc_bytes, s);
                    if (rc) return rc;
                }
        }
        rc = time_plan(ctx, pr, leaves, reps, s, &out_sec[i], true,
                       ctx->interval_timing ? &ctx->interval_sec[i] : nullptr);
        if (rc) return rc;
        if (ctx->progress_every > 0 && (i + 1) % ctx->progress_every == 0)
            std::fprintf(stderr, "[smoothgemm] sweep %lld / %lld shapes\n", (long long)(i + 1), (long long)n);
    }
    return SG_OK;
}

extern "C" int sg_mem_sweep(sg_ctx* ctx, const sg_shape* shapes, int64_t n, int op, int alloc,
                            int elem_bytes, int warmup, int reps, double* out_sec, void* stream) {
    if (!ctx || (n > 0 && (!shapes || !out_sec))) return fail(SG_EINVAL, "sg_mem_sweep: NULL argument");
    if (n < 0 || warmup < 0 || reps < 1) return fail(SG_EINVAL, "sg_mem_sweep: bad counts");
    if (op != SG_MEM_READ_A && op != SG_MEM_READ_B && op != SG_MEM_READ_C && op != SG_MEM_WRITE_D)
        return fail(SG_EINVAL, "sg_mem_sweep: bad op");
    if (alloc != SG_MEM_ISOLATED && alloc != SG_MEM_COALLOC) return fail(SG_EINVAL, "sg_mem_sweep: bad alloc");
    if (elem_bytes != 2 && elem_bytes != 4) return fail(SG_EINVAL, "sg_mem_sweep: elem_bytes must be 2 or 4");
    for (int64_t i = 0; i < n; ++i)
        if (shapes[i].M <= 0 || shapes[i].N <= 0 || shapes[i].K <= 0)
            return fail(SG_EINVAL, "sg_mem_sweep: empty shape");
    DeviceGuard guard(ctx->device);
    hipStream_t s = (hipStream_t)stream;
    int rc = ensure_events(ctx, 2 * (size_t)reps);
    if (rc) return rc;
    uint32_t* sink = nullptr;
    if (hipMalloc((void**)&sink, 2048 * sizeof(uint32_t)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(SG_ENOMEM, "sg_mem_sweep: sink allocation failed");
    }
    // Buffers of one shape: A (M x K), B (K x N), C and D (M x N); lengths rounded up to 16 bytes.
    void* buf[4] = {nullptr, nullptr, nullptr, nullptr};
    auto release = [&]() {
        for (void*& b : buf)
            if (b) { (void)hipFree(b); b = nullptr; }
    };
    auto run = [&](void* target, int64_t bytes, hipEvent_t e0, hipEvent_t e1) {
        return op == SG_MEM_WRITE_D ? launch_mem_write(target, bytes, 0x5eedu, s, e0, e1)
                                    : launch_mem_read(target, bytes, sink, s, e0, e1);
    };
    const int target_idx = op == SG_MEM_READ_A ? 0 : op == SG_MEM_READ_B ? 1 : op == SG_MEM_READ_C ? 2 : 3;
    for (int64_t i = 0; i < n && rc == SG_OK; ++i) {
        const sg_shape& sh = shapes[i];
        int64_t len[4] = {sh.M * sh.K, sh.K * sh.N, sh.M * sh.N, sh.M * sh.N};
        for (int64_t& l : len) l = (l * elem_bytes + 15) / 16 * 16;
        // isolated: the measured buffer alone; co-allocated: A, B, C, D in that order
        for (int b = 0; b < 4 && rc == SG_OK; ++b) {
            if (alloc == SG_MEM_ISOLATED && b != target_idx) continue;
            if (hipMalloc(&buf[b], (size_t)len[b]) != hipSuccess) {
                (void)hipGetLastError();
                buf[b] = nullptr;
                rc = fail(SG_ENOMEM, "sg_mem_sweep: buffer allocation failed");
            }
        }
        void* target = buf[target_idx];
        const int64_t bytes = len[target_idx];
        for (int w = 0; w < (i == 0 ? warmup : 0) + 1 && rc == SG_OK; ++w) rc = run(target, bytes, nullptr, nullptr);
        for (int r = 0; r < reps && rc == SG_OK; ++r)
            rc = run(target, bytes, ctx->events[2 * r], ctx->events[2 * r + 1]);
        if (rc == SG_OK) {
            hipError_t e = hipEventSynchronize(ctx->events[2 * reps - 1]);
            double total = 0.0;
            for (int r = 0; r < reps && e == hipSuccess; ++r) {
                float ms = 0.f;
                e = hipEventElapsedTime(&ms, ctx->events[2 * r], ctx->events[2 * r + 1]);
                total += (double)ms * 1e-3;
            }
            if (e != hipSuccess) rc = hip_fail(e, "sg_mem_sweep timing");
            else out_sec[i] = total / reps;
        }
        release();
        if (rc == SG_OK && ctx->progress_every > 0 && (i + 1) % ctx->progress_every == 0)
            std::fprintf(stderr, "[smoothgemm] memory sweep %lld / %lld shapes\n", (long long)(i + 1), (long long)n);
    }
    release();
    (void)hipFree(sink);
    return rc;
}

extern "C" int sg_ctx_set_interval_timing(sg_ctx* ctx, int on) {
    if (!ctx || (on != 0 && on != 1)) return fail(SG_EINVAL, "bad argument");
    ctx->interval_timing = on;
    return SG_OK;
}

extern "C" int sg_sweep_interval_times(const sg_ctx* ctx, double* out_sec, int64_t n) {
    if (!ctx || (n > 0 && !out_sec)) return fail(SG_EINVAL, "NULL argument");
    if ((size_t)n != ctx->interval_sec.size())
        return fail(SG_EINVAL, "the most recent sweep did not record " + std::to_string(n) + " interval times");
    std::copy(ctx->interval_sec.begin(), ctx->interval_sec.end(), out_sec);
    return SG_OK;
}

extern "C" int sg_sweep_kernel_times(const sg_ctx* ctx, int64_t* launches, double* seconds,
                                     double* flops) {
    if (!ctx) return fail(SG_EINVAL, "NULL ctx");
    for (int v = 0; v < kNumVariants; ++v) {
        if (launches) launches[v] = ctx->acct_launches[v];
        if (seconds) seconds[v] = ctx->acct_seconds[v];
        if (flops) flops[v] = ctx->acct_flops[v];
    }
    return SG_OK;
}

// ---- table measurement (used by table.cpp) ----------------------------------------------------
namespace sg {

int measure_t0(sg_ctx* ctx, const std::vector<sg_shape>& order, const std::vector<int64_t>& cells,
               const int* variants, int nvar, int c_dtype, int warmup, int reps,
               const void* A_pool, const void* B_pool, void* C_pool, hipStream_t s,
               std::vector<double>& T0, int64_t ncells) {
    DeviceGuard guard(ctx->device);
    std::vector<Leaf> leaves(1);
    for (size_t i = 0; i < order.size(); ++i) {
        const sg_shape& sh = order[i];
        Problem pr{sh.M, sh.N, sh.K, (const uint16_t*)A_pool, sh.K, (const uint16_t*)B_pool, sh.N,
                   C_pool, sh.N, c_dtype == SG_BF16, 0, 0};
        for (int v = 0; v < nvar; ++v) {
            leaves[0] = Leaf{0, 0, 0, sh.M, sh.N, sh.K, sh.M, sh.N, sh.K, variants[v], true, true};
            if (i == 0 && v == 0) {
                size_t acc_bytes = 0;
                int rc = ensure_ws(ctx, plan_workspace(pr, leaves, &acc_bytes));
                if (rc) return rc;
                for (int w = 0; w < warmup; ++w) {
                    rc = run_leaf(pr, leaves[0], ctx->ws, acc_bytes, s);
                    if (rc) return rc;
                }
            }
            double sec = 0.0;
            int rc = time_plan(ctx, pr, leaves, reps, s, &sec, false);
            if (rc) return rc;
            T0[(size_t)v * ncells + cells[i]] = sec;
        }
        if (ctx->progress_every > 0 && (i + 1) % ctx->progress_every == 0)
            std::fprintf(stderr, "[smoothgemm] T0 %zu / %zu shapes x %d variants\n", i + 1, order.size(), nvar);
    }
    return SG_OK;
}

}  // namespace sg
