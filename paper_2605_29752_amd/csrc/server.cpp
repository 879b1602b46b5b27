// Continuous-batching GEMM server.
//
// Requests C_i = A_i * B_w arrive at any time (B_w one of a few shared, device-resident weight
// matrices).  A scheduler thread runs three steps in a loop:
//   1. completion: query the event of every busy stream slot; finished requests get their
//      completion time, their device memory goes back to the pool;
//   2. admission: pending requests, oldest first, are admitted while their A and C fit in the
//      HBM budget (one device allocation carved by a first-fit pool);
//   3. launch: while a slot is free, the admitted requests (up to max_group, oldest first) are
//      staged (A copied in from the resident activation pool) and launched as ONE persistent
//      grouped kernel on that slot's stream, so work admitted while earlier groups run overlaps
//      them on the device.  Per-request mode launches each request on its own instead.
// A request's tile shape (its class) comes from M (a small tile for skinny requests) or, given a
// dispatch table at creation, from the table's best variant for the request's shape; a launch
// runs one class.  Every request's output is computed by the same tile body whatever group it
// lands in, so a result is bit-identical alone and in the mix (for the same tile shape).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <deque>
#include <map>
#include <mutex>
#include <random>
#include <thread>
#include <unordered_map>
#include <vector>

#include "sg_internal.h"
#include "sg_table.h"

using namespace sg;

namespace {

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

// First-fit allocator over [0, size) with 256-byte granules; host-side bookkeeping only.
class Pool {
  public:
    explicit Pool(size_t size) { free_[0] = size; }
    bool alloc(size_t bytes, size_t* off) {
        bytes = (bytes + 255) & ~size_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                *off = it->first;
                const size_t rest = it->second - bytes;
                const size_t noff = it->first + bytes;
                free_.erase(it);
                if (rest) free_[noff] = rest;
                used_ += bytes;
                peak_ = std::max(peak_, used_);
                return true;
            }
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~size_t(255);
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t used() const { return used_; }
    size_t peak() const { return peak_; }

  private:
    size_t used_ = 0, peak_ = 0;
    std::map<size_t, size_t> free_;
};

struct Req {
    uint64_t ticket = 0, id = 0;
    int64_t M = 0;
    int w = 0;
    int tile = 0;             // tile shape this request runs with (its class)
    bool solo = false;        // launched on its own even in grouped mode
    int group = 0;            // requests in the launch that ran it
    int64_t a_offset = 0;     // element offset of A in the activation pool
    size_t offA = 0, offC = 0, bytesA = 0, bytesC = 0;
    double t_arr = 0, t_adm = 0, t_launch = 0, t_done = 0;
    int status = 0;
    bool has_mem = false;
};

struct Slot {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    std::vector<uint64_t> tickets;
    GroupProblem* h_desc = nullptr;   // pinned staging, reused only when the slot is idle
    GroupProblem* d_desc = nullptr;
    int* d_counters = nullptr;
};

uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

}  // namespace

struct sg_server {
    sg_server_cfg cfg{};
    std::vector<sg_weight> weights;
    int device = 0;
    char* arena = nullptr;            // hbm_budget bytes for request A and C
    uint16_t* act_pool = nullptr;     // resident activation pool (N(0, a_scale) BF16)
    int64_t act_elems = 0;
    Pool* pool = nullptr;
    std::vector<Slot> slots;
    std::chrono::steady_clock::time_point t0;
    // tiles_from_table: tile class of a request of weight w whose M falls in table row-cell c
    int table_step = 0;
    std::vector<std::vector<int>> table_tile;   // [weight][M cell]

    std::mutex mu;                    // guards everything below
    std::deque<uint64_t> pending;     // submitted, not admitted
    std::deque<uint64_t> admitted;    // admitted, not launched
    std::unordered_map<uint64_t, Req> reqs;
    std::deque<sg_completion> done;
    uint64_t next_ticket = 1;
    int64_t n_submitted = 0, n_completed = 0, n_failed = 0, n_launches = 0;
    double flops_done = 0.0;
    std::string worker_error;

    std::atomic<bool> stop{false};
    std::thread worker;
};

namespace {

void fill_completion(const sg_server* sv, const Req& r, sg_completion* c) {
    const sg_weight& w = sv->weights[r.w];
    c->ticket = r.ticket;
    c->id = r.id;
    c->M = r.M;
    c->N = w.N;
    c->K = w.K;
    c->weight = r.w;
    c->status = r.status;
    c->a_offset = r.a_offset;
    c->tile = r.tile;
    c->group_size = r.group;
    c->t_arrival = r.t_arr;
    c->t_admit = r.t_adm;
    c->t_launch = r.t_launch;
    c->t_done = r.t_done;
    c->A = r.has_mem ? sv->arena + r.offA : nullptr;
    c->C = r.has_mem ? sv->arena + r.offC : nullptr;
}

// Worker: one pass of completion -> admission -> launch.  Returns true if anything happened.
bool worker_pass(sg_server* sv) {
    bool progress = false;
    // 1. completions
    for (Slot& sl : sv->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.ev);
        if (q == hipErrorNotReady) continue;
        const double t = now_s(sv->t0);
        std::lock_guard<std::mutex> lk(sv->mu);
        for (uint64_t tk : sl.tickets) {
            Req& r = sv->reqs[tk];
            r.t_done = t;
            r.status = (q == hipSuccess) ? 0 : SG_EHIP;
            if (q == hipSuccess) {
                const sg_weight& w = sv->weights[r.w];
                sv->flops_done += 2.0 * (double)r.M * (double)w.N * (double)w.K;
                ++sv->n_completed;
            } else {
                ++sv->n_failed;
            }
            if (!sv->cfg.keep_results) {       // kept results hold A and C until release
                sv->pool->release(r.offA, r.bytesA);
                sv->pool->release(r.offC, r.bytesC);
                r.has_mem = false;
            }
            sg_completion c{};
            fill_completion(sv, r, &c);
            sv->done.push_back(c);
            if (!sv->cfg.keep_results) sv->reqs.erase(tk);
        }
        if (q != hipSuccess) sv->worker_error = hipGetErrorString(q);
        sl.tickets.clear();
        sl.busy = false;
        progress = true;
    }
    // 2. admission (oldest first; a request that does not fit blocks the ones behind it)
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        while (!sv->pending.empty()) {
            Req& r = sv->reqs[sv->pending.front()];
            const sg_weight& w = sv->weights[r.w];
            r.bytesA = (size_t)r.M * (size_t)w.K * 2;
            r.bytesC = (size_t)r.M * (size_t)w.N * 2;
            size_t oa, oc;
            if (!sv->pool->alloc(r.bytesA, &oa)) break;
            if (!sv->pool->alloc(r.bytesC, &oc)) {
                sv->pool->release(oa, r.bytesA);
                break;
            }
            r.offA = oa;
            r.offC = oc;
            r.has_mem = true;
            r.t_adm = now_s(sv->t0);
            sv->admitted.push_back(r.ticket);
            sv->pending.pop_front();
            progress = true;
        }
    }
    // 3. launch onto free slots: a group is the oldest admitted request and the admitted
    //    requests after it of the same tile class (every launch runs one tile shape), oldest
    //    first, at most an equal share of the admitted requests per free slot, so that work
    //    admitted together spreads over the free slots and runs side by side.  A solo request
    //    is a group of its own and is never added to another request's group.
    int free_slots = 0;
    for (const Slot& sl : sv->slots) free_slots += sl.busy ? 0 : 1;
    for (Slot& sl : sv->slots) {
        if (sl.busy) continue;
        std::vector<Req*> group;
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            const int share = (int)((sv->admitted.size() + free_slots - 1) / std::max(free_slots, 1));
            const int cap = sv->cfg.mode == SG_SERVE_GROUPED ? std::max(1, std::min(sv->cfg.max_group, share)) : 1;
            --free_slots;
            if (!sv->admitted.empty()) {
                const Req& first = sv->reqs[sv->admitted.front()];
                const int cls = first.tile;
                const int lim = first.solo ? 1 : cap;
                for (auto it = sv->admitted.begin(); it != sv->admitted.end() && (int)group.size() < lim;) {
                    Req& r = sv->reqs[*it];
                    if (r.tile == cls && (group.empty() || !r.solo)) {
                        group.push_back(&r);
                        it = sv->admitted.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
        }
        if (group.empty()) break;
        const int tile = group[0]->tile;
        const double t = now_s(sv->t0);
        std::vector<sg_problem> probs(group.size());
        for (size_t i = 0; i < group.size(); ++i) {
            Req& r = *group[i];
            const sg_weight& w = sv->weights[r.w];
            // the activation arrives: copy it into the request's own buffer
            (void)hipMemcpyAsync(sv->arena + r.offA, sv->act_pool + r.a_offset, r.bytesA,
                                 hipMemcpyDeviceToDevice, sl.s);
            probs[i] = sg_problem{r.M, w.N, w.K, sv->arena + r.offA, w.K, w.B, w.ldb,
                                  sv->arena + r.offC, w.N};
            r.t_launch = t;
            r.group = (int)group.size();
            sl.tickets.push_back(r.ticket);
        }
        int rc = SG_OK;
        if (probs.size() > 1) {
            int total = 0, grid = 0;
            double fl = 0;
            bool aa = false;
            std::vector<int> order(group.size());
            rc = grouped_fill(probs.data(), (int)probs.size(), tile, SG_BF16, true, sl.h_desc,
                              order.data(), &total, &fl, &aa);
            if (rc == SG_OK) rc = grouped_grid(tile, aa, sv->device, total, 0, &grid);
            if (rc == SG_OK && hipMemcpyAsync(sl.d_desc, sl.h_desc, sizeof(GroupProblem) * probs.size(),
                                              hipMemcpyHostToDevice, sl.s) != hipSuccess)
                rc = SG_EHIP;
            if (rc == SG_OK)
                rc = grouped_enqueue(tile, aa, sl.d_desc, (int)probs.size(), total, grid, SG_BF16,
                                     sl.d_counters, sl.s, nullptr, nullptr);
        } else {
            // a single request (per-request mode, or a group of one) runs the tile kernel
            // directly: no descriptors to stage, no work queue; the same tile body, so the
            // result is the one the grouped kernel would give it
            const sg_problem& q = probs[0];
            LaunchDesc d{};
            d.M = q.M; d.N = q.N; d.K = q.K; d.Ml = q.M; d.Nl = q.N; d.Kl = q.K;
            d.A = (const uint16_t*)q.A; d.lda = q.lda; d.B = (const uint16_t*)q.B; d.ldb = q.ldb;
            d.C = q.C; d.ldc = q.ldc; d.out_bf16 = 1; d.add = nullptr; d.ldadd = 0; d.add_kind = ADD_NONE;
            rc = launch_variant(tile * kSplitLevels, d, nullptr, sl.s);
        }
        if (rc == SG_OK && hipEventRecord(sl.ev, sl.s) != hipSuccess) rc = SG_EHIP;
        if (rc != SG_OK) {
            // the launch never happened: fail these requests now
            std::lock_guard<std::mutex> lk(sv->mu);
            for (uint64_t tk : sl.tickets) {
                Req& r = sv->reqs[tk];
                r.status = rc;
                r.t_done = now_s(sv->t0);
                ++sv->n_failed;
                sv->pool->release(r.offA, r.bytesA);
                sv->pool->release(r.offC, r.bytesC);
                r.has_mem = false;
                sg_completion c{};
                fill_completion(sv, r, &c);
                sv->done.push_back(c);
            }
            sv->worker_error = "launch failed";
            sl.tickets.clear();
            continue;
        }
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            ++sv->n_launches;
        }
        sl.busy = true;
        progress = true;
    }
    return progress;
}

void worker_main(sg_server* sv) {
    (void)hipSetDevice(sv->device);
    while (!sv->stop.load(std::memory_order_relaxed)) {
        if (!worker_pass(sv)) std::this_thread::yield();
    }
}

}  // namespace

extern "C" {

int sg_server_create(sg_ctx* ctx, const sg_server_cfg* cfg, sg_server** out) {
    if (!cfg || !out) return fail(SG_EINVAL, "NULL argument");
    *out = nullptr;
    if (cfg->hbm_budget < (1u << 20) || cfg->max_inflight < 1 || cfg->max_inflight > 16 ||
        cfg->max_group < 1 || cfg->max_group > 4096 || cfg->queue_cap < 1 || cfg->n_weights < 1 ||
        !cfg->weights || cfg->tile < 0 || cfg->tile >= kNumGroupTiles || cfg->max_m < 1 ||
        cfg->small_m < 0 || cfg->small_tile < 0 || cfg->small_tile >= kNumGroupTiles || cfg->solo_m < 0 ||
        (cfg->mode != SG_SERVE_GROUPED && cfg->mode != SG_SERVE_PER_REQUEST))
        return fail(SG_EINVAL, "bad server configuration");
    int64_t maxK = 0;
    for (int i = 0; i < cfg->n_weights; ++i) {
        const sg_weight& w = cfg->weights[i];
        if (w.K <= 0 || w.N <= 0 || !w.B || w.ldb < w.N) return fail(SG_EINVAL, "bad weight");
        maxK = std::max(maxK, w.K);
    }
    if (cfg->tiles_from_table != 0 && cfg->tiles_from_table != 1) return fail(SG_EINVAL, "bad server configuration");
    const sg_table* tab = cfg->tiles_from_table ? (ctx ? ctx_table(ctx) : nullptr) : nullptr;
    if (cfg->tiles_from_table && !tab)
        return fail(SG_ENOTABLE, "tiles_from_table needs a dispatch table on the context");
    sg_server* sv = new (std::nothrow) sg_server();
    if (!sv) return fail(SG_ENOMEM, "server allocation failed");
    if (tab) {
        // per weight and M cell, the tile of the table's best variant at (M cell, N, K), each
        // axis clamped to the grid (a shape beyond it takes the largest cell's choice); a
        // split-K or stream-K variant gives its tile, the deep-K 64 x 64 the 64 x 64 tile
        const sg_grid& g = tab->grid;
        auto cell_of = [&](int64_t d, int n) { return (int)std::min<int64_t>(n - 1, std::max<int64_t>(0, (d + g.step - 1) / g.step - 1)); };
        sv->table_step = g.step;
        sv->table_tile.resize(cfg->n_weights);
        for (int i = 0; i < cfg->n_weights; ++i) {
            const int cn = cell_of(cfg->weights[i].N, g.n_n), ck = cell_of(cfg->weights[i].K, g.n_k);
            for (int cm = 0; cm < g.n_m; ++cm) {
                int t = variant_tile(tab->best_var[tab->cell_index(cm, cn, ck)]);
                if (t >= kNumGroupTiles) t = kNumGroupTiles - 1;
                sv->table_tile[i].push_back(t);
            }
        }
    }
    sv->cfg = *cfg;
    sv->weights.assign(cfg->weights, cfg->weights + cfg->n_weights);
    sv->cfg.weights = sv->weights.data();
    SG_HIP(hipGetDevice(&sv->device));
    auto cleanup = [&](int rc, const char* msg) {
        sg_server_destroy(sv);
        return fail(rc, msg);
    };
    if (hipMalloc(&sv->arena, cfg->hbm_budget) != hipSuccess) return cleanup(SG_ENOMEM, "HBM budget allocation failed");
    sv->pool = new Pool(cfg->hbm_budget);
    // resident activation pool: one maximal A plus slack for per-request offsets
    sv->act_elems = (int64_t)cfg->max_m * maxK + (1 << 20);
    if (hipMalloc(&sv->act_pool, (size_t)sv->act_elems * 2) != hipSuccess)
        return cleanup(SG_ENOMEM, "activation pool allocation failed");
    if (launch_fill(sv->act_pool, sv->act_elems, cfg->seed, 0, 0, 1, cfg->a_scale, nullptr) != SG_OK)
        return cleanup(SG_EHIP, "activation pool fill failed");
    if (hipDeviceSynchronize() != hipSuccess) return cleanup(SG_EHIP, "activation pool fill failed");
    sv->slots.resize(cfg->max_inflight);
    for (Slot& sl : sv->slots) {
        if (hipStreamCreateWithFlags(&sl.s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void**)&sl.h_desc, sizeof(GroupProblem) * cfg->max_group, hipHostMallocDefault) != hipSuccess ||
            hipMalloc(&sl.d_desc, sizeof(GroupProblem) * cfg->max_group) != hipSuccess ||
            hipMalloc(&sl.d_counters, 2 * sizeof(int)) != hipSuccess ||
            hipMemset(sl.d_counters, 0, 2 * sizeof(int)) != hipSuccess)
            return cleanup(SG_EHIP, "slot set-up failed");
    }
    if (hipDeviceSynchronize() != hipSuccess) return cleanup(SG_EHIP, "slot set-up failed");
    sv->t0 = std::chrono::steady_clock::now();
    sv->worker = std::thread(worker_main, sv);
    *out = sv;
    return SG_OK;
}

int sg_server_now(sg_server* sv, double* t) {
    if (!sv || !t) return fail(SG_EINVAL, "NULL argument");
    *t = now_s(sv->t0);
    return SG_OK;
}

int sg_server_submit(sg_server* sv, const sg_request* req, double arrival_s, uint64_t* ticket) {
    if (!sv || !req) return fail(SG_EINVAL, "NULL argument");
    if (req->M < 1 || req->M > sv->cfg.max_m || req->weight < 0 || req->weight >= (int)sv->weights.size())
        return fail(SG_EINVAL, "request M or weight out of range");
    const sg_weight& w = sv->weights[req->weight];
    const size_t need = (size_t)req->M * (size_t)(w.K + w.N) * 2 + 512;
    if (need > sv->cfg.hbm_budget) return fail(SG_EINVAL, "request can never fit the HBM budget");
    std::lock_guard<std::mutex> lk(sv->mu);
    if ((int)sv->pending.size() >= sv->cfg.queue_cap) return fail(SG_EAGAIN, "server queue is full");
    Req r;
    r.ticket = sv->next_ticket++;
    r.id = req->id;
    r.M = req->M;
    r.w = req->weight;
    if (!sv->table_tile.empty()) {
        const std::vector<int>& tt = sv->table_tile[req->weight];
        const int64_t cm = std::min<int64_t>((int64_t)tt.size() - 1, (req->M + sv->table_step - 1) / sv->table_step - 1);
        r.tile = tt[(size_t)std::max<int64_t>(0, cm)];
    } else {
        r.tile = req->M <= sv->cfg.small_m ? sv->cfg.small_tile : sv->cfg.tile;
    }
    r.solo = sv->cfg.solo_m > 0 && req->M > sv->cfg.solo_m;
    const int64_t span = sv->act_elems - req->M * w.K;
    r.a_offset = (int64_t)(mix64(sv->cfg.seed ^ mix64(req->id + 1)) % (uint64_t)(span / 8 + 1)) * 8;
    r.t_arr = arrival_s >= 0 ? arrival_s : now_s(sv->t0);
    sv->reqs[r.ticket] = r;
    sv->pending.push_back(r.ticket);
    ++sv->n_submitted;
    if (ticket) *ticket = r.ticket;
    return SG_OK;
}

int sg_server_poll(sg_server* sv, sg_completion* out, int max, int* n) {
    if (!sv || !n || (max > 0 && !out)) return fail(SG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    int k = 0;
    while (k < max && !sv->done.empty()) {
        out[k++] = sv->done.front();
        sv->done.pop_front();
    }
    *n = k;
    return SG_OK;
}

int sg_server_release(sg_server* sv, uint64_t ticket) {
    if (!sv) return fail(SG_EINVAL, "NULL server");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->reqs.find(ticket);
    if (it == sv->reqs.end() || it->second.t_done == 0.0) return fail(SG_EINVAL, "unknown or unfinished ticket");
    if (it->second.has_mem) {
        sv->pool->release(it->second.offA, it->second.bytesA);
        sv->pool->release(it->second.offC, it->second.bytesC);
    }
    sv->reqs.erase(it);
    return SG_OK;
}

int sg_server_drain(sg_server* sv, double timeout_s) {
    if (!sv) return fail(SG_EINVAL, "NULL server");
    const double end = now_s(sv->t0) + timeout_s;
    for (;;) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            if (sv->n_completed + sv->n_failed >= sv->n_submitted) return SG_OK;
        }
        if (now_s(sv->t0) > end) return fail(SG_EAGAIN, "drain timed out");
        std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
}

int sg_server_stats_get(sg_server* sv, sg_server_stats* st) {
    if (!sv || !st) return fail(SG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(sv->mu);
    *st = sg_server_stats{};
    st->submitted = sv->n_submitted;
    st->completed = sv->n_completed;
    st->failed = sv->n_failed;
    st->launches = sv->n_launches;
    st->flops = sv->flops_done;
    st->pending = (int64_t)sv->pending.size();
    st->bytes_in_use = (double)sv->pool->used();
    st->peak_bytes = (double)sv->pool->peak();
    return SG_OK;
}

int sg_server_destroy(sg_server* sv) {
    if (!sv) return SG_OK;
    sv->stop.store(true);
    if (sv->worker.joinable()) sv->worker.join();
    // every resource is released even after a failure; the first HIP error is reported
    hipError_t first = hipDeviceSynchronize();
    auto note = [&](hipError_t e) {
        if (first == hipSuccess) first = e;
    };
    for (Slot& sl : sv->slots) {
        if (sl.s) note(hipStreamDestroy(sl.s));
        if (sl.ev) note(hipEventDestroy(sl.ev));
        if (sl.h_desc) note(hipHostFree(sl.h_desc));
        if (sl.d_desc) note(hipFree(sl.d_desc));
        if (sl.d_counters) note(hipFree(sl.d_counters));
    }
    if (sv->arena) note(hipFree(sv->arena));
    if (sv->act_pool) note(hipFree(sv->act_pool));
    delete sv->pool;
    delete sv;
    return first == hipSuccess ? SG_OK : hip_fail(first, "server teardown");
}

int sg_serve_poisson(sg_server* sv, double rate, double duration_s, double warmup_s, uint64_t seed,
                     int64_t max_m, sg_serve_report* rep) {
    if (!sv || !rep || rate <= 0 || duration_s <= 0 || warmup_s < 0 || warmup_s >= duration_s || max_m < 1)
        return fail(SG_EINVAL, "bad arguments");
    *rep = sg_serve_report{};
    std::mt19937_64 rng(seed);
    std::exponential_distribution<double> gap(rate);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    std::uniform_int_distribution<int> wsel(0, (int)sv->weights.size() - 1);
    double t_start = 0;
    sg_server_now(sv, &t_start);
    double t = 0;
    uint64_t id = 0;
    int64_t rejected = 0;
    std::vector<std::pair<uint64_t, double>> tickets;   // ticket, scheduled arrival
    const double lnmax = std::log((double)max_m);
    for (;;) {
        t += gap(rng);
        if (t >= duration_s) break;
        sg_request r;
        r.id = id++;
        r.M = std::min<int64_t>(max_m, std::max<int64_t>(1, std::llround(std::exp(u01(rng) * lnmax))));
        r.weight = wsel(rng);
        const double at = t_start + t;
        for (;;) {                                   // open loop: wait for the arrival time
            double nw;
            sg_server_now(sv, &nw);
            if (nw >= at) break;
            if (at - nw > 2e-4) std::this_thread::sleep_for(std::chrono::microseconds(100));
        }
        uint64_t tk = 0;
        const int rc = sg_server_submit(sv, &r, at, &tk);
        if (rc == SG_EAGAIN) { ++rejected; continue; }
        if (rc) return rc;
        tickets.emplace_back(tk, t);
    }
    int rc = sg_server_drain(sv, 600.0);
    if (rc) return rc;
    std::vector<sg_completion> comp(4096);
    std::vector<double> lat;
    double flops = 0, first = INFINITY, last = 0;
    int64_t measured = 0, failed = 0;
    for (;;) {
        int n = 0;
        sg_server_poll(sv, comp.data(), (int)comp.size(), &n);
        if (n == 0) break;
        for (int i = 0; i < n; ++i) {
            const sg_completion& c = comp[i];
            if (c.status != 0) { ++failed; continue; }
            if (c.t_arrival - t_start < warmup_s) continue;
            lat.push_back(c.t_done - c.t_arrival);
            flops += 2.0 * (double)c.M * (double)c.N * (double)c.K;
            first = std::min(first, c.t_arrival);
            last = std::max(last, c.t_done);
            ++measured;
        }
    }
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
        if (lat.empty()) return (double)NAN;
        size_t k = (size_t)std::ceil(p * lat.size());   // nearest rank
        k = std::min(std::max<size_t>(k, 1), lat.size());
        return lat[k - 1];
    };
    sg_server_stats st{};
    sg_server_stats_get(sv, &st);
    rep->offered = (int64_t)id;
    rep->rejected = rejected;
    rep->failed = failed;
    rep->measured = measured;
    rep->window_s = (measured > 0) ? last - first : 0.0;
    rep->req_per_s = rep->window_s > 0 ? measured / rep->window_s : 0.0;
    rep->tflops = rep->window_s > 0 ? flops / rep->window_s / 1e12 : 0.0;
    rep->p50_ms = pct(0.50) * 1e3;
    rep->p99_ms = pct(0.99) * 1e3;
    double s = 0;
    for (double x : lat) s += x;
    rep->mean_ms = lat.empty() ? NAN : s / lat.size() * 1e3;
    rep->launches = st.launches;
    rep->peak_bytes = st.peak_bytes;
    return SG_OK;
}

int sg_serve_closed(sg_server* sv, int outstanding, double duration_s, double warmup_s, uint64_t seed,
                    int64_t max_m, sg_serve_report* rep) {
    if (!sv || !rep || outstanding < 1 || duration_s <= 0 || warmup_s < 0 || warmup_s >= duration_s ||
        max_m < 1 || max_m > sv->cfg.max_m)
        return fail(SG_EINVAL, "bad arguments");
    *rep = sg_serve_report{};
    sg_server_stats st0{};
    sg_server_stats_get(sv, &st0);
    std::mt19937_64 rng(seed);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    std::uniform_int_distribution<int> wsel(0, (int)sv->weights.size() - 1);
    const double lnmax = std::log((double)max_m);
    double t_start = 0;
    sg_server_now(sv, &t_start);
    const double t_stop = t_start + duration_s;
    uint64_t id = 0;
    int in_flight = 0;
    auto submit_one = [&]() -> int {
        sg_request r;
        r.id = id++;
        r.M = std::min<int64_t>(max_m, std::max<int64_t>(1, std::llround(std::exp(u01(rng) * lnmax))));
        r.weight = wsel(rng);
        uint64_t tk = 0;
        const int rc = sg_server_submit(sv, &r, -1.0, &tk);
        if (rc == SG_OK) ++in_flight;
        return rc;
    };
    std::vector<sg_completion> comp(1024);
    std::vector<double> lat;
    double flops = 0, first = INFINITY, last = 0;
    int64_t measured = 0, failed = 0;
    auto collect = [&](bool count) {
        int n = 0;
        sg_server_poll(sv, comp.data(), (int)comp.size(), &n);
        for (int i = 0; i < n; ++i) {
            const sg_completion& c = comp[i];
            --in_flight;
            if (c.status != 0) { ++failed; continue; }
            if (!count || c.t_arrival - t_start < warmup_s || c.t_arrival >= t_stop) continue;
            lat.push_back(c.t_done - c.t_arrival);
            flops += 2.0 * (double)c.M * (double)c.N * (double)c.K;
            first = std::min(first, c.t_arrival);
            last = std::max(last, c.t_done);
            ++measured;
        }
        return n;
    };
    for (;;) {                       // keep `outstanding` requests in the server until the end
        double now = 0;
        sg_server_now(sv, &now);
        if (now >= t_stop) break;
        while (in_flight < outstanding) {
            const int rc = submit_one();
            if (rc == SG_EAGAIN) break;
            if (rc) return rc;
        }
        if (collect(true) == 0) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    int rc = sg_server_drain(sv, 600.0);
    if (rc) return rc;
    collect(true);
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double p) {
        if (lat.empty()) return (double)NAN;
        size_t k = (size_t)std::ceil(p * lat.size());   // nearest rank
        k = std::min(std::max<size_t>(k, 1), lat.size());
        return lat[k - 1];
    };
    sg_server_stats st{};
    sg_server_stats_get(sv, &st);
    rep->offered = (int64_t)id;
    rep->failed = failed;
    rep->measured = measured;
    rep->window_s = (measured > 0) ? last - first : 0.0;
    rep->req_per_s = rep->window_s > 0 ? measured / rep->window_s : 0.0;
    rep->tflops = rep->window_s > 0 ? flops / rep->window_s / 1e12 : 0.0;
    rep->p50_ms = pct(0.50) * 1e3;
    rep->p99_ms = pct(0.99) * 1e3;
    double sum = 0;
    for (double x : lat) sum += x;
    rep->mean_ms = lat.empty() ? NAN : sum / lat.size() * 1e3;
    rep->launches = st.launches - st0.launches;
    rep->peak_bytes = st.peak_bytes;
    return SG_OK;
}

}  // extern "C"
