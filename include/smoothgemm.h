/*
 * smoothgemm -- BF16 NN GEMM over the (M, N, K) shape landscape, with best-of-N tile
 * selection and the dynamic-programming pad-and-split dispatch table, for AMD MI355X (gfx950).
 *
 * The operation (paper Sec. 2.2 and Sec. 7.1): C = A * B, A is M x K, B is K x N, no
 * transposes ("NN").  A and B hold BF16 values; products are accumulated in FP32; C is FP32
 * or BF16 (rounded to nearest even from the FP32 accumulator, once).
 *
 * Conventions for every call below:
 *  - Matrices are row-major.  lda >= K, ldb >= N, ldc >= N are in elements.
 *  - "device pointer" means memory the GPU can address (hipMalloc, torch CUDA tensors); host
 *    pointers are plain host memory.  The caller owns every buffer it passes in.
 *  - Work is enqueued asynchronously on `stream` (a hipStream_t; NULL = the null stream);
 *    results are ready once the caller synchronises that stream or an event recorded on it.
 *  - Every call returns SG_OK (0) or a negative SG_E* code and never aborts; no C++ exception
 *    crosses this interface.  sg_last_error() returns a message for the calling thread's most
 *    recent failure (valid until that thread's next call).
 *  - A context is not thread-safe: use one per host thread or lock around it.
 */
#ifndef SMOOTHGEMM_H
#define SMOOTHGEMM_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------------- */
#define SG_OK          0
#define SG_EINVAL     -1   /* bad argument: negative size, NULL pointer with non-zero size, bad enum */
#define SG_ENOMEM     -2   /* device or host allocation failed                                       */
#define SG_ENOTABLE   -3   /* a table-driven mode was requested but no dispatch table is set        */
#define SG_EMISMATCH  -4   /* a saved table does not match this device / grid / variant set         */
#define SG_EHIP       -5   /* the HIP runtime reported an error (message has the HIP error string)  */
#define SG_ERANGE     -6   /* shape outside the range covered by the dispatch table                 */
#define SG_EIO        -7   /* file could not be read or written                                     */
#define SG_EAGAIN     -8   /* resource temporarily full (server queue); retry later                 */

/* ---- enums ------------------------------------------------------------------------------ */
#define SG_F32   0         /* C element type: FP32 */
#define SG_BF16  1         /* C element type: BF16 (round to nearest even)  */

#define SG_MODE_DEFAULT  0 /* DP plan if the context holds a table, else the plain variant        */
#define SG_MODE_PLAIN    1 /* the context's fixed "plain" variant (one tile shape, no split)      */
#define SG_MODE_BEST     2 /* best-of-N: per shape the variant with the least measured time        */
#define SG_MODE_DP       3 /* dispatch-table plan: pad and/or split, each leaf on its best variant */
#define SG_MODE_VARIANT  4 /* the variant given in sg_gemm_args.variant                            */

/* ---- errors / version ------------------------------------------------------------------- */
const char* sg_last_error(void);
const char* sg_version(void);

/* ---- context ------------------------------------------------------------------------------
 * Owns the split-K / plan workspace (device memory, grown on demand), the events used for
 * timing and a borrowed pointer to the dispatch table.  `device` is a HIP device ordinal. */
typedef struct sg_ctx sg_ctx;
int sg_ctx_create(int device, sg_ctx** out);
int sg_ctx_destroy(sg_ctx* ctx);
/* Fixed variant used by SG_MODE_PLAIN (default: variant 0, the 256 x 256 tile, no split). */
int sg_ctx_set_plain_variant(sg_ctx* ctx, int variant);
/* Reserve at least `bytes` of workspace now, so later calls do not allocate. */
int sg_ctx_reserve_workspace(sg_ctx* ctx, size_t bytes);

/* ---- GEMM ----------------------------------------------------------------------------------
 * Paper-form call (Sec. 7.1 problem statement): C (FP32, ldc = N) = A (lda = K) * B (ldb = N).
 * Device pointers; uses a per-device default context and the null stream, SG_MODE_DEFAULT.
 * M == 0 or N == 0: no-op.  K == 0: C is set to zero. */
int gemm_bf16_nn(int64_t M, int64_t N, int64_t K, const void* A, const void* B, void* C);

typedef struct sg_gemm_args {
    int64_t M, N, K;
    const void* A; int64_t lda;   /* device, BF16, M x K row-major          */
    const void* B; int64_t ldb;   /* device, BF16, K x N row-major          */
    void* C;       int64_t ldc;   /* device, c_dtype, M x N row-major       */
    int c_dtype;                  /* SG_F32 or SG_BF16                      */
    int beta;                     /* 0: C = A B;  1: C = A B + C (accumulate into C's old value) */
    int mode;                     /* SG_MODE_*                              */
    int variant;                  /* used when mode == SG_MODE_VARIANT      */
} sg_gemm_args;

/* Extended call.  K == 0 gives C = beta * C.  SG_MODE_BEST / SG_MODE_DP without a table:
 * SG_ENOTABLE (no silent fallback).  Shapes beyond the table's largest cell: SG_ERANGE.
 * A K split with BF16 output accumulates in an FP32 workspace and rounds once. */
int gemm_bf16_nn_ex(sg_ctx* ctx, const sg_gemm_args* args, void* stream);

/* ---- kernel variants (the tile family) ----------------------------------------------------
 * Variant v: tile BM x BN (64-deep K step, 256 threads, MFMA 16x16x32 BF16) and a parallel
 * split-K factor S (S > 1: FP32 partials in the workspace, then a fixed-order reduction). */
typedef struct sg_variant_info {
    int id, bm, bn, bk, splits, threads;
    int lds_bytes;
    char name[48];
} sg_variant_info;
int sg_num_variants(void);
int sg_variant_info_get(int variant, sg_variant_info* out);

/* ---- landscape metrics (paper Sec. 2.4, Sec. 8.6) -------------------------------------------
 * sg_roughness: sum_i |T[i+1] - T[i]| / (n - 1); n < 2 returns NaN.
 * sg_landscape_stats: tflops is an nM x nN x nK array (K fastest) of throughputs; fills
 * mean, peak, roughness along M, N and K (each averaged over every line along that axis) and
 * their mean (the 3-D aggregate).  Any axis of length < 2 gives SG_EINVAL. */
double sg_roughness(const double* T, int64_t n);
typedef struct sg_stats {
    double mean, peak, rough_m, rough_n, rough_k, rough_3d;
} sg_stats;
int sg_landscape_stats(const double* tflops, int nM, int nN, int nK, sg_stats* out);

/* ---- sweep driver (paper Sec. 3 timing protocol, Sec. 4.5 randomized order) -----------------
 * Runs the n shapes in the order given (shuffle them for the randomized protocol) with
 * `warmup` untimed runs of the first shape up front, then per shape one untimed run and `reps`
 * timed runs; out_sec[i] = mean seconds of one run of shape i.  Each run is one complete
 * execution in `mode` (a DP run may be several kernel launches).  Each shape views the pools as
 * A = first M*K elements (lda = K), B = first K*N (ldb = N), C = first M*N (ldc = N): pools must
 * hold at least max(M*K), max(K*N), max(M*N) elements.  out_launch_sec / out_launches, if not
 * NULL, receive per-shape summed kernel-launch seconds of the dominant variant (see
 * sg_sweep_kernel_times). */
typedef struct sg_shape { int64_t M, N, K; } sg_shape;
int sg_sweep(sg_ctx* ctx, const sg_shape* shapes, int64_t n, int mode, int variant, int c_dtype,
             int warmup, int reps, const void* A_pool, const void* B_pool, void* C_pool,
             double* out_sec, void* stream);
/* Per-variant launch accounting of the most recent sg_sweep on this context: for variant v,
 * launches[v] kernel launches took seconds[v] in total (event to event, timed runs only) and
 * did flops[v] algorithmic FLOP (2 M N K of the data shape of each launch). Arrays hold
 * sg_num_variants() entries. */
int sg_sweep_kernel_times(const sg_ctx* ctx, int64_t* launches, double* seconds, double* flops);

/* ---- dispatch table (paper Sec. 7.1) ---------------------------------------------------------
 * Grid: sizes (i + 1) * step for i < n_m (M axis), n_n (N axis), n_k (K axis).  T0 holds, per
 * variant and cell, measured seconds; best-of-N takes the per-cell minimum; T1 pads
 * (min over the 8 neighbours {0,1}^3 ahead, visited from the largest cell down); T2 splits
 * (min over cuts along one axis of T2[a] + T2[b], visited from the smallest cell up).
 * The table is owned by the library; free it with sg_table_free. */
typedef struct sg_grid { int step, n_m, n_n, n_k; } sg_grid;
typedef struct sg_table sg_table;

#define SG_ACT_AS_IS    0
#define SG_ACT_PAD      1
#define SG_ACT_SPLIT_M  2
#define SG_ACT_SPLIT_N  3
#define SG_ACT_SPLIT_K  4
typedef struct sg_plan_rec {
    int action;     /* SG_ACT_*                                                          */
    int arg;        /* PAD: flat index of the target cell; SPLIT_*: first piece size in steps */
    int variant;    /* variant that runs this cell (AS_IS) or the pad target (PAD); -1 for splits */
    double t0, t1, t2;   /* best-of-N T0, T1 and T2 of the cell, seconds                   */
} sg_plan_rec;

/* Pure host computation from given timings: T0 is nvar x cells (cell index
 * (i_m * n_n + i_n) * n_k + i_k), variant_ids[v] names the variant of row v. */
int sg_table_from_t0(const sg_grid* grid, const double* T0, const int* variant_ids, int nvar,
                     sg_table** out);
/* Measure T0 on the GPU (sg_sweep protocol over all cells, shapes in an order shuffled by
 * order_seed, all variants per shape), then build the table as sg_table_from_t0.  Pools as in
 * sg_sweep; c_dtype is the output type measured. */
int sg_table_build(sg_ctx* ctx, const sg_grid* grid, const int* variant_ids, int nvar, int c_dtype,
                   int warmup, int reps, uint64_t order_seed, const void* A_pool,
                   const void* B_pool, void* C_pool, void* stream, sg_table** out);
int sg_table_free(sg_table* t);
int sg_table_grid(const sg_table* t, sg_grid* out);
/* O(1) lookup: the record of the cell covering (M, N, K): index ceil(dim / step) - 1 per axis. */
int sg_table_lookup(const sg_table* t, int64_t M, int64_t N, int64_t K, sg_plan_rec* out);
/* Copy out tables: which = 0: best-of-N T0, 1: T1, 2: T2 (cells doubles), 3: the full
 * per-variant T0 (nvar x cells doubles). */
int sg_table_values(const sg_table* t, int which, double* out, int64_t n);
/* Variant ids of the table's T0 rows: writes min(cap, nvar) ids, *nvar = the row count. */
int sg_table_variants(const sg_table* t, int* ids, int cap, int* nvar);
/* Number of leaves (kernel launches, split-K reductions not counted) the plan of (M,N,K) runs. */
int sg_table_plan_leaves(const sg_table* t, int64_t M, int64_t N, int64_t K, int* out_leaves);
/* Binary file with a fingerprint (device name, compute-unit count, HIP runtime version, grid,
 * variant set, output type); load refuses a mismatch with SG_EMISMATCH unless `force` != 0.
 * Loading requires the current HIP device only when force == 0. */
int sg_table_save(const sg_table* t, const char* path);
int sg_table_load(const char* path, int force, sg_table** out);
/* Borrow the table for SG_MODE_DEFAULT / BEST / DP calls (NULL clears). */
int sg_ctx_set_table(sg_ctx* ctx, const sg_table* t);

/* ---- device operand generator (the seeded counter generator, on the GPU) ---------------------
 * Element idx of stream `stream` under `seed`: SplitMix64 word
 * out(out(seed, stream + 1), idx + 1 + offset); kind 0: uniform[-1,1) as (2u+1-2^24)/2^24 with u
 * the top 24 bits; kind 1: `scale` * N(0,1) by Box-Muller in FP64 on words 2i, 2i+1.  Rounded to
 * FP32 then BF16 (nearest even).  Writes n BF16 values to device memory `dst`. */
int sg_fill_bf16(void* dst, int64_t n, uint64_t seed, uint64_t stream, int64_t offset, int kind,
                 double scale, void* stream_handle);

#ifdef __cplusplus
}
#endif
#endif /* SMOOTHGEMM_H */
