// Dispatch-table construction (paper Sec. 7.1, "The T0 -> T1 -> T2 Algorithm"), O(1) lookup and
// (de)serialisation with a device fingerprint.
//
// Cell (i_m, i_n, i_k) stands for the GEMM of size ((i_m+1) g, (i_n+1) g, (i_k+1) g).
//  Step 1  T0: measured seconds per variant; best-of-N keeps the per-cell minimum and its variant.
//  Step 2  T1: initialised as T0, visited from the largest cell down; each cell takes the least
//          of itself and its seven neighbours one step larger along any subset of axes (padding).
//          No padding beyond the largest grid size.
//  Step 3  T2: initialised as T1, visited from the smallest cell up; each cell may be replaced by
//          the cheapest cut into two pieces along exactly one axis at a grid point (the pieces
//          run one after the other, so their times add).
// Ties keep the earlier candidate: as-is, pads in lexicographic (i,j,k) order, cuts along M by
// ascending first-piece size, then N, then K; a candidate wins only when strictly cheaper.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <random>

#include "sg_internal.h"
#include "sg_table.h"

namespace sg {

int build_dp(sg_table* t) {
    const int nM = t->grid.n_m, nN = t->grid.n_n, nK = t->grid.n_k;
    const int64_t C = t->cells();
    t->T0best.assign(C, INFINITY);
    t->best_var.assign(C, -1);
    for (int v = 0; v < t->nvar; ++v)
        for (int64_t c = 0; c < C; ++c) {
            const double x = t->T0[(size_t)v * C + c];
            if (x < t->T0best[c]) {
                t->T0best[c] = x;
                t->best_var[c] = t->variants[v];
            }
        }
    for (int64_t c = 0; c < C; ++c)
        if (t->best_var[c] < 0 || !(t->T0best[c] > 0.0) || !std::isfinite(t->T0best[c]))
            return fail(SG_EINVAL, "T0 must be finite and positive in every cell");

    // Step 2: padding.
    t->T1 = t->T0best;
    std::vector<int64_t> target(C);
    std::iota(target.begin(), target.end(), (int64_t)0);
    for (int m = nM - 1; m >= 0; --m)
        for (int n = nN - 1; n >= 0; --n)
            for (int k = nK - 1; k >= 0; --k) {
                const int64_t c = t->cell_index(m, n, k);
                double best = t->T1[c];
                int64_t tg = target[c];
                for (int d = 1; d < 8; ++d) {
                    const int i = (d >> 2) & 1, j = (d >> 1) & 1, kk = d & 1;
                    if (m + i >= nM || n + j >= nN || k + kk >= nK) continue;
                    const int64_t o = t->cell_index(m + i, n + j, k + kk);
                    if (t->T1[o] < best) {
                        best = t->T1[o];
                        tg = target[o];
                    }
                }
                t->T1[c] = best;
                target[c] = tg;
            }

    // Step 3: splitting.
    t->T2 = t->T1;
    t->action.assign(C, SG_ACT_AS_IS);
    t->arg.assign(C, 0);
    for (int64_t c = 0; c < C; ++c)
        if (target[c] != c) {
            t->action[c] = SG_ACT_PAD;
            t->arg[c] = (int32_t)target[c];
        }
    for (int m = 0; m < nM; ++m)
        for (int n = 0; n < nN; ++n)
            for (int k = 0; k < nK; ++k) {
                const int64_t c = t->cell_index(m, n, k);
                double best = t->T2[c];
                int act = t->action[c];
                int32_t ar = t->arg[c];
                const int sm = m + 1, sn = n + 1, sk = k + 1;   // sizes in steps
                for (int i = 1; i < sm; ++i) {
                    const double x = t->T2[t->cell_index(i - 1, n, k)] + t->T2[t->cell_index(sm - i - 1, n, k)];
                    if (x < best) { best = x; act = SG_ACT_SPLIT_M; ar = i; }
                }
                for (int j = 1; j < sn; ++j) {
                    const double x = t->T2[t->cell_index(m, j - 1, k)] + t->T2[t->cell_index(m, sn - j - 1, k)];
                    if (x < best) { best = x; act = SG_ACT_SPLIT_N; ar = j; }
                }
                for (int kk = 1; kk < sk; ++kk) {
                    const double x = t->T2[t->cell_index(m, n, kk - 1)] + t->T2[t->cell_index(m, n, sk - kk - 1)];
                    if (x < best) { best = x; act = SG_ACT_SPLIT_K; ar = kk; }
                }
                t->T2[c] = best;
                t->action[c] = (uint8_t)act;
                t->arg[c] = ar;
            }
    return SG_OK;
}

static int check_grid(const sg_grid* g) {
    if (!g || g->step <= 0 || g->n_m <= 0 || g->n_n <= 0 || g->n_k <= 0)
        return fail(SG_EINVAL, "bad grid");
    if ((int64_t)g->n_m * g->n_n * g->n_k > (1 << 24)) return fail(SG_EINVAL, "grid too large");
    if ((int64_t)g->step * std::max(g->n_m, std::max(g->n_n, g->n_k)) > 0x7FFFFFFF)
        return fail(SG_EINVAL, "grid sizes exceed 2^31 - 1");
    return SG_OK;
}

static std::string device_fingerprint(int* cus, int* rt) {
    int dev = 0;
    *cus = 0;
    *rt = 0;
    if (hipGetDevice(&dev) != hipSuccess) return "unknown";
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, dev) != hipSuccess) return "unknown";
    *cus = p.multiProcessorCount;
    (void)hipRuntimeGetVersion(rt);
    return std::string(p.gcnArchName);   // the marketing name is not stable (profilers blank it)
}

// T0 of row `row` at extents (M, N, K): trilinear interpolation between the grid cells that
// bracket each extent (cell c holds size (c + 1) g), clamped to the first and last cells.  At a
// grid point it is the measured value itself.
double t0_interp(const sg_table* t, int row, int64_t M, int64_t N, int64_t K) {
    const double g = (double)t->grid.step;
    auto axis = [g](int64_t d, int n, int* lo, int* hi, double* f) {
        const double x = (double)d / g;             // cell lo holds (lo + 1) g
        if (x <= 1.0) { *lo = *hi = 0; *f = 0.0; return; }
        if (x >= (double)n) { *lo = *hi = n - 1; *f = 0.0; return; }
        const int c = (int)std::floor(x) - 1;
        *lo = c;
        *hi = c + 1;
        *f = x - (double)(c + 1);
    };
    int m0, m1, n0, n1, k0, k1;
    double fm, fn, fk;
    axis(M, t->grid.n_m, &m0, &m1, &fm);
    axis(N, t->grid.n_n, &n0, &n1, &fn);
    axis(K, t->grid.n_k, &k0, &k1, &fk);
    const double* T = t->T0.data() + (size_t)row * (size_t)t->cells();
    auto at = [&](int a, int b, int c) { return T[t->cell_index(a, b, c)]; };
    double v = 0.0;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b)
            for (int c = 0; c < 2; ++c) {
                const double w = (a ? fm : 1.0 - fm) * (b ? fn : 1.0 - fn) * (c ? fk : 1.0 - fk);
                if (w != 0.0) v += w * at(a ? m1 : m0, b ? n1 : n0, c ? k1 : k0);
            }
    return v;
}

int variant_row(const sg_table* t, int variant) {
    for (int r = 0; r < t->nvar; ++r)
        if (t->variants[r] == variant) return r;
    return -1;
}

}  // namespace sg

using namespace sg;

extern "C" {

int sg_table_from_t0(const sg_grid* grid, const double* T0, const int* variant_ids, int nvar,
                     sg_table** out) {
    if (!out) return fail(SG_EINVAL, "NULL out");
    *out = nullptr;
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!T0 || !variant_ids || nvar <= 0) return fail(SG_EINVAL, "bad T0 / variants");
    for (int v = 0; v < nvar; ++v)
        if (variant_ids[v] < 0 || variant_ids[v] >= kNumVariants) return fail(SG_EINVAL, "bad variant id");
    sg_table* t = new (std::nothrow) sg_table();
    if (!t) return fail(SG_ENOMEM, "table allocation failed");
    t->grid = *grid;
    t->nvar = nvar;
    t->variants.assign(variant_ids, variant_ids + nvar);
    t->T0.assign(T0, T0 + (size_t)nvar * t->cells());
    t->device = "host";
    rc = build_dp(t);
    if (rc) {
        delete t;
        return rc;
    }
    *out = t;
    return SG_OK;
}

int sg_table_build(sg_ctx* ctx, const sg_grid* grid, const int* variant_ids, int nvar, int c_dtype,
                   int warmup, int reps, uint64_t order_seed, const void* A_pool,
                   const void* B_pool, void* C_pool, void* stream, sg_table** out) {
    if (!out || !ctx) return fail(SG_EINVAL, "NULL argument");
    *out = nullptr;
    int rc = check_grid(grid);
    if (rc) return rc;
    if (!variant_ids || nvar <= 0 || !A_pool || !B_pool || !C_pool || reps < 1 || warmup < 0)
        return fail(SG_EINVAL, "bad arguments");
    if (c_dtype != SG_F32 && c_dtype != SG_BF16) return fail(SG_EINVAL, "bad c_dtype");
    for (int v = 0; v < nvar; ++v)
        if (variant_ids[v] < 0 || variant_ids[v] >= kNumVariants) return fail(SG_EINVAL, "bad variant id");
    sg_table* t = new (std::nothrow) sg_table();
    if (!t) return fail(SG_ENOMEM, "table allocation failed");
    t->grid = *grid;
    t->nvar = nvar;
    t->variants.assign(variant_ids, variant_ids + nvar);
    const int64_t C = t->cells();
    t->T0.assign((size_t)nvar * C, 0.0);
    // randomized measurement order (seeded Fisher-Yates via mt19937_64)
    std::vector<int64_t> cells(C);
    std::iota(cells.begin(), cells.end(), (int64_t)0);
    std::mt19937_64 rng(order_seed);
    for (int64_t i = C - 1; i > 0; --i) {
        std::uniform_int_distribution<int64_t> d(0, i);
        std::swap(cells[i], cells[d(rng)]);
    }
    std::vector<sg_shape> order(C);
    for (int64_t i = 0; i < C; ++i) {
        int m, n, k;
        t->cell_coords(cells[i], &m, &n, &k);
        order[i] = sg_shape{(int64_t)(m + 1) * grid->step, (int64_t)(n + 1) * grid->step,
                            (int64_t)(k + 1) * grid->step};
    }
    rc = measure_t0(ctx, order, cells, variant_ids, nvar, c_dtype, warmup, reps, A_pool, B_pool,
                    C_pool, (hipStream_t)stream, t->T0, C);
    if (rc == SG_OK) rc = build_dp(t);
    if (rc) {
        delete t;
        return rc;
    }
    t->device = device_fingerprint(&t->cus, &t->hip_runtime);
    t->c_dtype = c_dtype;
    *out = t;
    return SG_OK;
}

int sg_table_free(sg_table* t) {
    delete t;
    return SG_OK;
}

int sg_table_grid(const sg_table* t, sg_grid* out) {
    if (!t || !out) return fail(SG_EINVAL, "NULL argument");
    *out = t->grid;
    return SG_OK;
}

int sg_table_lookup(const sg_table* t, int64_t M, int64_t N, int64_t K, sg_plan_rec* out) {
    if (!t || !out) return fail(SG_EINVAL, "NULL argument");
    if (M <= 0 || N <= 0 || K <= 0) return fail(SG_EINVAL, "lookup needs positive dims");
    int m, n, k;
    if (!t->covering_cell(M, N, K, &m, &n, &k)) return fail(SG_ERANGE, "shape outside the table grid");
    const int64_t c = t->cell_index(m, n, k);
    out->action = t->action[c];
    out->arg = t->arg[c];
    if (out->action == SG_ACT_AS_IS) out->variant = t->best_var[c];
    else if (out->action == SG_ACT_PAD) out->variant = t->best_var[out->arg];
    else out->variant = -1;
    out->t0 = t->T0best[c];
    out->t1 = t->T1[c];
    out->t2 = t->T2[c];
    return SG_OK;
}

int sg_table_values(const sg_table* t, int which, double* out, int64_t n) {
    if (!t || !out) return fail(SG_EINVAL, "NULL argument");
    const std::vector<double>* src = nullptr;
    switch (which) {
        case 0: src = &t->T0best; break;
        case 1: src = &t->T1; break;
        case 2: src = &t->T2; break;
        case 3: src = &t->T0; break;
        default: return fail(SG_EINVAL, "bad table selector");
    }
    if (n < (int64_t)src->size()) return fail(SG_EINVAL, "output array too small");
    std::memcpy(out, src->data(), src->size() * sizeof(double));
    return SG_OK;
}

int sg_table_variants(const sg_table* t, int* ids, int cap, int* nvar) {
    if (!t || !nvar || (cap > 0 && !ids)) return fail(SG_EINVAL, "NULL argument");
    *nvar = t->nvar;
    for (int i = 0; i < t->nvar && i < cap; ++i) ids[i] = t->variants[i];
    return SG_OK;
}

int sg_table_plan_leaves(const sg_table* t, int64_t M, int64_t N, int64_t K, int* out_leaves) {
    if (!t || !out_leaves) return fail(SG_EINVAL, "NULL argument");
    int m, n, k;
    if (!t->covering_cell(M, N, K, &m, &n, &k)) return fail(SG_ERANGE, "shape outside the table grid");
    // count leaves of the cell plan (off-grid shapes may drop empty pieces: upper bound)
    std::vector<int64_t> stack{t->cell_index(m, n, k)};
    int leaves = 0;
    while (!stack.empty()) {
        const int64_t c = stack.back();
        stack.pop_back();
        const int a = t->action[c];
        if (a == SG_ACT_AS_IS || a == SG_ACT_PAD) { ++leaves; continue; }
        int cm, cn, ck;
        t->cell_coords(c, &cm, &cn, &ck);
        const int p = t->arg[c];
        if (a == SG_ACT_SPLIT_M) { stack.push_back(t->cell_index(p - 1, cn, ck)); stack.push_back(t->cell_index(cm - p, cn, ck)); }
        if (a == SG_ACT_SPLIT_N) { stack.push_back(t->cell_index(cm, p - 1, ck)); stack.push_back(t->cell_index(cm, cn - p, ck)); }
        if (a == SG_ACT_SPLIT_K) { stack.push_back(t->cell_index(cm, cn, p - 1)); stack.push_back(t->cell_index(cm, cn, ck - p)); }
    }
    *out_leaves = leaves;
    return SG_OK;
}

int sg_table_group_count(const sg_table* t, int64_t* n) {
    if (!t || !n) return fail(SG_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(t->group_mu);
    *n = (int64_t)t->group_sched.size();
    return SG_OK;
}

static const char kMagic[8] = {'S', 'G', 'T', 'B', 'L', '0', '0', '1'};

int sg_table_save(const sg_table* t, const char* path) {
    if (!t || !path) return fail(SG_EINVAL, "NULL argument");
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(SG_EIO, std::string("cannot open ") + path);
    bool ok = true;
    auto w = [&](const void* p, size_t n) { ok = ok && std::fwrite(p, 1, n, f) == n; };
    w(kMagic, 8);
    uint32_t dl = (uint32_t)t->device.size();
    w(&dl, 4);
    w(t->device.data(), dl);
    w(&t->cus, 4);
    w(&t->hip_runtime, 4);
    w(&t->c_dtype, 4);
    w(&t->grid, sizeof(sg_grid));
    w(&t->nvar, 4);
    w(t->variants.data(), sizeof(int) * t->nvar);
    w(t->T0.data(), sizeof(double) * t->T0.size());
    {   // grouped-launch schedules (a trailing section; files without it load with none)
        std::lock_guard<std::mutex> lk(t->group_mu);
        const uint32_t ns = (uint32_t)t->group_sched.size();
        w(&ns, 4);
        for (const auto& kv : t->group_sched) {
            const int32_t v[3] = {kv.second.tile, kv.second.grid_wgs, kv.second.order};
            w(&kv.first, 8);
            w(v, sizeof v);
            w(&kv.second.seconds, 8);
        }
    }
    ok = (std::fclose(f) == 0) && ok;
    return ok ? SG_OK : fail(SG_EIO, std::string("write failed: ") + path);
}

int sg_table_load(const char* path, int force, sg_table** out) {
    if (!path || !out) return fail(SG_EINVAL, "NULL argument");
    *out = nullptr;
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(SG_EIO, std::string("cannot open ") + path);
    sg_table* t = new (std::nothrow) sg_table();
    if (!t) {
        std::fclose(f);
        return fail(SG_ENOMEM, "table allocation failed");
    }
    bool ok = true;
    auto r = [&](void* p, size_t n) { ok = ok && std::fread(p, 1, n, f) == n; };
    char magic[8];
    r(magic, 8);
    ok = ok && std::memcmp(magic, kMagic, 8) == 0;
    uint32_t dl = 0;
    r(&dl, 4);
    ok = ok && dl < 4096;
    if (ok) {
        t->device.resize(dl);
        r(&t->device[0], dl);
    }
    r(&t->cus, 4);
    r(&t->hip_runtime, 4);
    r(&t->c_dtype, 4);
    r(&t->grid, sizeof(sg_grid));
    r(&t->nvar, 4);
    ok = ok && t->nvar > 0 && t->nvar <= kNumVariants && check_grid(&t->grid) == SG_OK;
    if (ok) {
        t->variants.resize(t->nvar);
        r(t->variants.data(), sizeof(int) * t->nvar);
        t->T0.resize((size_t)t->nvar * t->cells());
        r(t->T0.data(), sizeof(double) * t->T0.size());
    }
    if (ok) {
        uint32_t ns = 0;
        if (std::fread(&ns, 1, 4, f) == 4) {           // optional trailing section
            ok = ns <= (1u << 24);
            for (uint32_t i = 0; i < ns && ok; ++i) {
                uint64_t key = 0;
                int32_t v[3] = {0, 0, 0};
                double sec = 0.0;
                r(&key, 8);
                r(v, sizeof v);
                r(&sec, 8);
                ok = ok && v[0] >= 0 && v[0] < kNumGroupTiles && v[1] >= 0 && (v[2] == 0 || v[2] == 1);
                if (ok) t->group_sched[key] = sg_table::GroupSched{v[0], v[1], v[2], sec};
            }
        }
    }
    std::fclose(f);
    if (!ok) {
        delete t;
        return fail(SG_EIO, std::string("malformed table file: ") + path);
    }
    for (int v : t->variants)
        if (v < 0 || v >= kNumVariants) {
            delete t;
            return fail(SG_EMISMATCH, "table names variants this library does not have");
        }
    if (!force) {
        int cus = 0, rt = 0;
        std::string dev = device_fingerprint(&cus, &rt);
        if (dev != t->device || cus != t->cus || rt != t->hip_runtime) {
            std::string msg = "table fingerprint " + t->device + " (" + std::to_string(t->cus) +
                              " CUs, runtime " + std::to_string(t->hip_runtime) + ") does not match this device " +
                              dev + " (" + std::to_string(cus) + " CUs, runtime " + std::to_string(rt) + ")";
            delete t;
            return fail(SG_EMISMATCH, msg);
        }
    }
    int rc = build_dp(t);
    if (rc) {
        delete t;
        return rc;
    }
    *out = t;
    return SG_OK;
}

}  // extern "C"
