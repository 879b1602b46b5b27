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
/* Memory-only twin of sg_gemm_args.variant (the memory surface of Sec. 4): the same operand
 * loads into LDS (with the same packing of unaligned operands), the same waits and barriers and
 * the same stores of C as that variant's kernel, with the fragment reads and the matrix-core
 * products left out.  C receives beta * C (zeros for beta = 0).  A measuring instrument, not a
 * GEMM.  Operands that the direct-to-LDS path cannot load give SG_EINVAL. */
#define SG_MODE_MEMORY   5

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
/* every > 0: sweeps and table measurements print one progress line to stderr every `every`
 * shapes; 0 (default) keeps them silent. */
int sg_ctx_set_progress(sg_ctx* ctx, int every);
/* Concurrent split plans: on = 1 runs the pieces of a dispatch-table plan that has no K pieces
 * (its M and N pieces write disjoint parts of C) at the same time, on up to four streams the
 * context owns (default priority), forked from and joined back into the caller's stream, each
 * piece in its own slice of the workspace; sg_sweep then times such a run between two markers
 * on the caller's stream (the fork and a marker after the joins, so fork / join latency is
 * included) and leaves it out of the per-variant kernel accounting.  Plans with K pieces stay
 * sequential.  on = 2 runs such plans one after another on the caller's stream but times them
 * between the same two markers (the like-for-like reference for on = 1).  on = 3 runs the
 * pieces of such a plan as ONE persistent grouped launch (the grouped kernel below, its
 * descriptors copied to a buffer the context keeps) when every piece runs the same tile shape
 * without split-K or stream-K and beta = 0, else one after another; timed between the same
 * markers.
 * Default 0: pieces run one after another on the caller's stream, as the paper executes them,
 * and a run's time is the sum of its kernels' times. */
int sg_ctx_set_concurrent_splits(sg_ctx* ctx, int on);
/* Reserve at least `bytes` of workspace now, so later calls do not allocate. */
int sg_ctx_reserve_workspace(sg_ctx* ctx, size_t bytes);

/* ---- GEMM ----------------------------------------------------------------------------------
 * Paper-form call (Sec. 7.1 problem statement): C (FP32, ldc = N) = A (lda = K) * B (ldb = N).
 * Device pointers; runs on the current device's default context (sg_default_ctx) and the null
 * stream in SG_MODE_DEFAULT: the DP plan when a table was lent with sg_set_default_table, else
 * the plain variant.  M == 0 or N == 0: no-op.  K == 0: C is set to zero. */
int gemm_bf16_nn(int64_t M, int64_t N, int64_t K, const void* A, const void* B, void* C);

typedef struct sg_gemm_args {
    int64_t M, N, K;
    const void* A; int64_t lda;   /* device, BF16, M x K row-major          */
    const void* B; int64_t ldb;   /* device, BF16, K x N row-major          */
    void* C;       int64_t ldc;   /* device, c_dtype, M x N row-major       */
    int c_dtype;                  /* SG_F32 or SG_BF16                      */
    int beta;                     /* 0: C = A B;  1: C = A B + C (accumulate into C's old value) */
    int mode;                     /* SG_MODE_*                              */
    int variant;                  /* used when mode == SG_MODE_VARIANT or SG_MODE_MEMORY */
} sg_gemm_args;

/* Extended call.  K == 0 gives C = beta * C.  SG_MODE_BEST / SG_MODE_DP without a table:
 * SG_ENOTABLE (no silent fallback).  Shapes beyond the table's largest cell: SG_ERANGE.
 * A K split with BF16 output accumulates in an FP32 workspace and rounds once. */
int gemm_bf16_nn_ex(sg_ctx* ctx, const sg_gemm_args* args, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gemm_bf16_nn_ex with the same arguments, modes and
 * results (the same plan and kernels, so bit-identical output), but whatever scratch the call
 * needs (split-K partials, zero-padded copies of unaligned operands, the FP32 accumulator of a
 * BF16 K-split plan) comes from a fixed device array of sg_noalloc_scratch_bytes() bytes
 * (256 MiB) that the library holds on each GPU it runs on until the process ends.  The call
 * makes no hipMalloc / hipFree and no other allocating library call; the context must have been
 * created beforehand (creation looks up the array's address on its device).  A call whose plan
 * needs more scratch than that returns SG_ERANGE before enqueueing anything.  Pieces of a plan
 * always run one after another on `stream` (the context's concurrent-split setting is ignored).
 * Every call on a GPU shares that GPU's array and leaves its contents behind: calls that may
 * overlap on one GPU (other streams, other threads, other contexts) race and must be ordered
 * by the caller.  Nothing in the array needs to start at zero. */
int gemm_bf16_nn_ex_noalloc(sg_ctx* ctx, const sg_gemm_args* args, void* stream);
size_t sg_noalloc_scratch_bytes(void);

/* ---- kernel variants (the tile family) ----------------------------------------------------
 * Variant v = 4 t + log2(S), v < 32: tile t (BM x BN, 256 threads, MFMA 16x16x32 BF16) and a
 * parallel split-K factor S in {1, 2, 4, 8} (S > 1: FP32 partials in the workspace, then a
 * fixed-order reduction).  Tiles 0..7: 256x256, 256x128, 128x256, 128x128, 128x64, 64x128,
 * 64x64, and 64x64 with 128-deep K stages (for shapes with few tiles; per-call only, not in
 * grouped launches).
 * Variant 32 + t, t = 0..6: stream-K on tile t -- exactly as many work-groups as the GPU keeps
 * resident, each taking an equal share of the (tile, K stage) iterations of all tiles; a tile
 * split between work-groups is summed from FP32 partials (workspace) by a fix-up kernel in K
 * order, so results are bit-reproducible.  splits = 0 marks these variants.  Needs a workspace
 * (like S > 1); there is no memory-only twin.
 * bk is the K granularity of a split (64; 128 for tile 7), lds_bytes the LDS of the aligned
 * kernel (its ring of K stages). */
typedef struct sg_variant_info {
    int id, bm, bn, bk, splits, threads;
    int lds_bytes;
    char name[48];
} sg_variant_info;
int sg_num_variants(void);
int sg_variant_info_get(int variant, sg_variant_info* out);

/* ---- landscape metrics (paper Sec. 2 definitions, Sec. 8.5 Table 17) -------------------------------------------
 * sg_roughness: sum_i |T[i+1] - T[i]| / (n - 1); n < 2 returns NaN.
 * sg_landscape_stats: tflops is an nM x nN x nK array (K fastest) of throughputs; fills
 * mean, peak, roughness along M, N and K (each averaged over every line along that axis) and
 * their mean (the 3-D aggregate).  Any axis of length < 2 gives SG_EINVAL. */
double sg_roughness(const double* T, int64_t n);
typedef struct sg_stats {
    double mean, peak, rough_m, rough_n, rough_k, rough_3d;
} sg_stats;
int sg_landscape_stats(const double* tflops, int nM, int nN, int nK, sg_stats* out);

/* ---- first-principles landscape and Kernel Optimality Levels (paper Sec. 9, Sec. 10) --------
 * Computed from datasheet integers alone, no kernel run.  hw: peak (TFLOP/s, dense), cores (the
 * work-group slots of one wave: compute units), bandwidth (GB/s).  Landscapes are over the grid
 * cells (M, N, K) = ((i+1) step, (j+1) step, (k+1) step), written as an n_m x n_n x n_k array,
 * K fastest (the layout of sg_landscape_stats).
 * sg_ideal_landscape (Sec. 9.1): peak * min(1, W / C), W = ceil(M/T) ceil(N/T) for the tile T.
 * sg_optimal_landscape (Sec. 9.2): 2MNK / t_opt, t_opt = min over the ntiles square tile edges T
 *   of max(2MNK / (peak * eta(T)), t_mem), eta(T) = W_T / (ceil(W_T / C) C) the fraction of the
 *   launched core-slots that work (wave quantization), t_mem = (2MK + 2KN + c_bytes MN) / BW
 *   (per-channel utilisation taken as 1: the HBM address hash is not public; the paper's GDDR6
 *   channel term is sg_optimal_landscape_ch).
 * sg_kol_grade (Sec. 10.2-10.3): attainment tau = mean(actual) / mean(optimal); roughness ratio
 *   rho = R(actual) / R(optimal), R the N-axis roughness averaged over every line along N;
 *   bands of Table 19 (tau: < 0.5, < 0.75, < 0.95, else; rho: > 3, > 2, > 1.25, else) and level
 *   = min(t_band, s_band), 0 (L0) to 3 (L3).  Arrays are n_m x n_n x n_k (K fastest), n_n >= 2.
 * NULL pointers, non-positive sizes or hardware values give SG_EINVAL. */
typedef struct sg_hw { double peak_tflops; int cores; double bw_gbs; } sg_hw;
typedef struct sg_kol { double tau, rho; int t_band, s_band, level; } sg_kol;
struct sg_grid;
int sg_ideal_landscape(const struct sg_grid* grid, const sg_hw* hw, int tile, double* out);
int sg_optimal_landscape(const struct sg_grid* grid, const sg_hw* hw, const int* tiles, int ntiles,
                         int c_bytes, double* out);
/* The same with the paper's memory-channel term (Sec. 9.2): t_mem = 2MK / (BW eta_A) +
 * 2KN / (BW eta_B) + c_bytes MN / (BW eta_D), where a tensor with leading dimension L (K for A,
 * N for B and D) moved in rows of 256 elements of e bytes over `channels` channels striped in
 * `interleave`-byte blocks keeps eta = min(channels, w channels / gcd(s, channels)) / channels
 * of them busy, w = min(channels, 256 e / interleave), s = (L e / interleave) mod channels.
 * channels = 0 takes every eta as 1 (sg_optimal_landscape). */
int sg_optimal_landscape_ch(const struct sg_grid* grid, const sg_hw* hw, const int* tiles, int ntiles,
                            int c_bytes, int channels, int interleave, double* out);
int sg_kol_grade(const double* actual, const double* optimal, int n_m, int n_n, int n_k, sg_kol* out);

/* ---- four-surface decomposition (paper Sec. 4) ------------------------------------------------
 * For n shapes with a measured GEMM time t_gemm[i] and a measured memory time t_memory[i]
 * (seconds; e.g. sg_sweep of one variant in SG_MODE_VARIANT and in SG_MODE_MEMORY):
 *   compute surface   t_compute[i]  = 2 M N K / (peak_tflops 1e12)  (useful FLOP at the dense
 *                     peak, tile-independent, Sec. 4.1);
 *   overhead surface  t_overhead[i] = t_gemm[i] - max(t_compute[i], t_memory[i]) (negative where
 *                     the memory time exceeds the GEMM's own time);
 * and out: overhead_share = mean over shapes of t_overhead / t_gemm (the stacked view of Fig. 6);
 * cb_bandwidth = fraction of shapes with t_compute >= (2 M K + 2 K N + c_bytes M N) / bw_gbs
 * (compute-bound against that bandwidth, Table 3); cb_measured = fraction with t_compute >=
 * t_memory.  t_compute and t_overhead may be NULL.  Only hw->peak_tflops and hw->bw_gbs are
 * read.  NULL inputs, n <= 0, an empty shape, a non-positive GEMM time or hardware value, or
 * c_bytes <= 0 give SG_EINVAL. */
typedef struct sg_decomp { double overhead_share, cb_bandwidth, cb_measured; } sg_decomp;
struct sg_shape;
int sg_decompose(const struct sg_shape* shapes, int64_t n, const double* t_gemm,
                 const double* t_memory, const sg_hw* hw, int c_bytes, double* t_compute,
                 double* t_overhead, sg_decomp* out);

/* ---- sweep driver (paper Sec. 3 timing protocol, Sec. 5.4 randomized order) -----------------
 * Runs the n shapes in the order given (shuffle them for the randomized protocol) with
 * `warmup` untimed runs of the first shape up front, then per shape one untimed run and `reps`
 * timed runs; out_sec[i] = mean seconds of one run of shape i.  Each run is one complete
 * execution in `mode` (a DP run may be several kernel launches).  A run's time is the sum of
 * its kernels' execution times, each taken from the start/end timestamps of its own dispatch
 * (the kernel time a profiler reports; host launch gaps are excluded).  Each shape views the
 * pools as A = first M*K elements (lda = K), B = first K*N (ldb = N), C = first M*N (ldc = N):
 * pools must hold at least max(M*K), max(K*N), max(M*N) elements.  Per-variant totals of the
 * timed runs are kept in the context (sg_sweep_kernel_times). */
typedef struct sg_shape { int64_t M, N, K; } sg_shape;
int sg_sweep(sg_ctx* ctx, const sg_shape* shapes, int64_t n, int mode, int variant, int c_dtype,
             int warmup, int reps, const void* A_pool, const void* B_pool, void* C_pool,
             double* out_sec, void* stream);
/* Per-variant launch accounting of the most recent sg_sweep on this context: for variant v,
 * launches[v] tile-kernel launches took seconds[v] of tile-kernel execution in total (timed runs
 * only; for split-K variants the reduction kernel that follows is not included) and did
 * flops[v] algorithmic FLOP (2 M N K of the data shape of each launch). Arrays hold
 * sg_num_variants() entries. */
int sg_sweep_kernel_times(const sg_ctx* ctx, int64_t* launches, double* seconds, double* flops);
/* Interval timing (on = 1; default 0): after a shape's timed runs, sg_sweep runs it `reps`
 * more times, each run between two markers recorded on the stream and with no timing events
 * of its own inside, so that each run is timed as a whole -- the kernels, the device-side gaps
 * between them and any host launch gap (for a multi-kernel plan, the time a caller actually
 * waits).  sg_sweep's own out_sec keeps the kernel-time sum; the interval means of the most
 * recent sweep (n = its shape count) are read with sg_sweep_interval_times (SG_EINVAL if that
 * sweep ran without interval timing or had another shape count). */
int sg_ctx_set_interval_timing(sg_ctx* ctx, int on);
int sg_sweep_interval_times(const sg_ctx* ctx, double* out_sec, int64_t n);

/* ---- memory-subsystem study (paper Sec. 5) -----------------------------------------------------
 * Bandwidth microbenchmarks over the GEMM's buffers: read A (M x K), read B (K x N), read C and
 * write D (M x N, the identical buffers of the load / store comparison), elem_bytes per element
 * (the paper uses FP32 buffers: 4).
 * sg_mem_read: streams `bytes` of the device buffer `buf` with 16-byte loads and folds every
 *   32-bit word into an XOR; writes sg_mem_read_blocks(bytes) (at most 2048) partial XORs to
 *   the device array `sink`, whose XOR is the XOR of all the buffer's words.
 * sg_mem_write: stores 32-bit word i of the buffer (counting from its start) as
 *   (i * 0x9E3779B1) ^ seed, modulo 2^32.
 *   Both: `bytes` a non-negative multiple of 16, `buf` 16-byte aligned, else SG_EINVAL; async on
 *   the stream.
 * sg_mem_sweep: per shape, in the order given (sequential or shuffled, Sec. 5.4), allocates the
 *   buffers -- the measured one alone (SG_MEM_ISOLATED, one allocation per measurement) or A, B,
 *   C (M x N) and D in that order (SG_MEM_COALLOC, as the GEMM's operands sit together) --, runs
 *   `op` once untimed (plus `warmup` untimed runs before the first shape) and `reps` times timed,
 *   frees the buffers, and writes the mean seconds of a timed run to out_sec[i] (each run timed
 *   by its own dispatch's timestamps).  Lengths are rounded up to 16 bytes.  Allocation failure:
 *   SG_ENOMEM.  Synchronous (it waits for each shape's timing events). */
#define SG_MEM_READ_A   0
#define SG_MEM_READ_B   1
#define SG_MEM_WRITE_D  2
#define SG_MEM_READ_C   3
#define SG_MEM_ISOLATED 0
#define SG_MEM_COALLOC  1
int64_t sg_mem_read_blocks(int64_t bytes);
int sg_mem_read(const void* buf, int64_t bytes, uint32_t* sink, void* stream);
int sg_mem_write(void* buf, int64_t bytes, uint32_t seed, void* stream);
int sg_mem_sweep(sg_ctx* ctx, const sg_shape* shapes, int64_t n, int op, int alloc, int elem_bytes,
                 int warmup, int reps, double* out_sec, void* stream);

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
/* Number of leaves (kernel launches, split-K reductions not counted) of the table plan of the
 * cell covering (M,N,K).  Off the grid the runtime may run the cell's best variant instead
 * (sg_table_plan_choice). */
int sg_table_plan_leaves(const sg_table* t, int64_t M, int64_t N, int64_t K, int* out_leaves);
/* Which plan SG_MODE_DP runs for (M,N,K).  A shape on the grid (every dimension a multiple of
 * the step) runs the table plan of its cell (Sec. 7.1's O(1) lookup).  Off the grid the cell's
 * plan, made for the cell's own sizes, is applied to the shape (splits at the same points, a
 * pad to the target's M and N extent), and it runs only if its leaves -- each costed by its
 * variant's T0 interpolated trilinearly between the grid cells that bracket the leaf's launch
 * extent, clamped at the grid's ends -- are estimated at least 5 % faster than the cell's best
 * variant on the whole shape; else that variant runs alone.  est_plan and est_best receive the two
 * estimates (seconds), *use_plan 1 when the table plan runs.  Host only; errors: SG_EINVAL
 * (NULL, non-positive dims), SG_ERANGE (beyond the grid). */
int sg_table_plan_choice(const sg_table* t, int64_t M, int64_t N, int64_t K, double* est_plan,
                         double* est_best, int* use_plan);
/* Binary file with a fingerprint (GPU architecture, compute-unit count, HIP runtime version, grid,
 * variant set, output type); load refuses a mismatch with SG_EMISMATCH unless `force` != 0.
 * Loading requires the current HIP device only when force == 0. */
/* Number of grouped-launch schedules recorded in the table (see sg_group_plan_create). */
int sg_table_group_count(const sg_table* t, int64_t* n);
int sg_table_save(const sg_table* t, const char* path);
int sg_table_load(const char* path, int force, sg_table** out);
/* Borrow the table for SG_MODE_DEFAULT / BEST / DP calls (NULL clears). */
int sg_ctx_set_table(sg_ctx* ctx, const sg_table* t);
/* The per-device default context that gemm_bf16_nn uses (created on first use; the library owns
 * it, and a caller that destroys it gets a fresh one on next use).  sg_set_default_table lends
 * it a table, so that the paper-form call runs the DP plan of Sec. 7.1 by O(1) lookup (NULL
 * clears: the plain variant again).  The table must outlive its use. */
int sg_default_ctx(int device, sg_ctx** out);
int sg_set_default_table(int device, const sg_table* t);

/* ---- grouped batching: many independent GEMMs in one persistent launch -------------------
 * One problem per entry: device pointers, row-major, the same conventions as sg_gemm_args
 * (beta = 0; all problems share c_dtype).  A plan uploads the descriptors once (device-resident,
 * owned by the plan) and fixes the tile shape and work order; sg_group_plan_launch enqueues one
 * persistent kernel that drains a queue of every problem's tiles.  Launches of one plan must
 * not overlap each other (they share the plan's queue counters); launches of different plans
 * may.  The caller owns A, B, C of every problem and keeps them alive while launches are
 * queued. */
typedef struct sg_problem {
    int64_t M, N, K;
    const void* A; int64_t lda;
    const void* B; int64_t ldb;
    void* C;       int64_t ldc;
} sg_problem;
typedef struct sg_group_cfg {
    int tile;       /* tile shape index 0..6: 256x256, 256x128, 128x256, 128x128, 128x64, 64x128, 64x64
                       (tile 7, the deep-K 64x64, is per-call only) */
    int grid_wgs;   /* resident work-groups; 0 = as many as the occupancy allows on every CU */
    int order;      /* 0: longest K first (greedy longest-processing-time), 1: as given */
} sg_group_cfg;
typedef struct sg_group_plan sg_group_plan;
/* cfg == NULL autotunes the schedule (tile shape, resident grid, queue order): every tile shape
 * is timed on this group at full residency with the longest-K-first queue (one warm-up, best of
 * three), then the two fastest tiles also with the queue in the given order and with smaller
 * grids (one work-group per CU, half the resident count), and the fastest configuration kept.
 * When ctx holds a dispatch table, the winner is recorded in the table under a key of the
 * problem list (shapes, alignment classes, c_dtype), and a later cfg == NULL plan of the same
 * problem list takes it from there without timing anything (O(1) lookup); saved tables carry
 * these schedules.  Synchronises `stream`. */
int sg_group_plan_create(sg_ctx* ctx, int G, const sg_problem* probs, int c_dtype,
                         const sg_group_cfg* cfg, void* stream, sg_group_plan** out);
int sg_group_plan_launch(sg_group_plan* plan, void* stream);
/* Replace the problems (same count).  Returns SG_EAGAIN when the tile count, the grid or the
 * kernel (all problems aligned or not) changed: graphs that captured this plan must then be
 * captured again (they would replay the old launch). */
int sg_group_plan_update(sg_group_plan* plan, const sg_problem* probs, void* stream);
int sg_group_plan_info(const sg_group_plan* plan, sg_group_cfg* cfg, int* total_tiles, int* grid,
                       double* flops);
int sg_group_plan_destroy(sg_group_plan* plan);
/* One-shot form: plan (cfg NULL = autotune, as sg_group_plan_create), launch, wait, free. */
int sg_gemm_grouped(sg_ctx* ctx, int G, const sg_problem* probs, int c_dtype,
                    const sg_group_cfg* cfg, void* stream);

/* Per-call form of the same work: every problem is one ordinary gemm_bf16_nn_ex call (beta 0,
 * the given mode / variant), issued back to back on `stream` from the library — the baseline a
 * grouped launch is compared with.  Stops at the first failing problem. */
int sg_gemm_batch(sg_ctx* ctx, int G, const sg_problem* probs, int c_dtype, int mode, int variant,
                  void* stream);

/* hipGraph of n grouped launches in sequence (captured on `stream`, which must not be NULL).
 * Replays reuse the plans' device descriptors: update them with sg_group_plan_update. */
typedef struct sg_graph sg_graph;
int sg_graph_capture_groups(sg_group_plan* const* plans, int n, void* stream, sg_graph** out);
int sg_graph_launch(sg_graph* graph, void* stream);
int sg_graph_destroy(sg_graph* graph);

/* ---- serving: continuous batching of GEMM requests ---------------------------------------
 * Requests C = A * B_w (B_w one of n_weights shared, device-resident weights; BF16 output) are
 * submitted at any time from any thread.  A worker thread admits pending requests, oldest
 * first, while their A (M x K) and C (M x N) fit in an HBM budget carved from one device
 * allocation; stages each admitted request's A (copied from a resident pool of N(0, a_scale)
 * activations at a per-request offset derived from (seed, id)); and launches admitted requests
 * as one grouped kernel on any free stream slot, so new work overlaps running work.  Every
 * request belongs to a tile class (small_tile for M <= small_m, else tile; or, with
 * tiles_from_table, the tile of the dispatch table's best variant for its shape); a launch takes the
 * oldest admitted request and up to max_group - 1 admitted requests after it of its class.  A
 * request with M > solo_m (solo_m > 0) is launched on its own even in grouped mode: it fills the
 * device by itself, and in a group it would only wait for the group's other members.  A
 * launch of one request runs the tile kernel directly (no descriptors, no work queue).
 * SG_SERVE_PER_REQUEST launches every request on its own (the per-call baseline), with the same
 * tile classes.  Times are
 * seconds on the server's clock (sg_server_now).  The caller owns the weights and keeps them
 * alive for the server's lifetime; the server owns request memory. */
#define SG_SERVE_GROUPED      0
#define SG_SERVE_PER_REQUEST  1
typedef struct sg_weight { int64_t K, N; const void* B; int64_t ldb; } sg_weight;
typedef struct sg_server_cfg {
    size_t hbm_budget;          /* device bytes for request A and C (>= 1 MiB)                  */
    int max_inflight;           /* stream slots, 1..16                                           */
    int max_group;              /* requests per grouped launch, 1..4096                          */
    int queue_cap;              /* pending requests before submit returns SG_EAGAIN              */
    int mode;                   /* SG_SERVE_GROUPED or SG_SERVE_PER_REQUEST                      */
    int tile;                   /* tile shape index 0..6 of requests with M > small_m (S = 1)      */
    int keep_results;           /* 1: C stays allocated until sg_server_release                  */
    int n_weights;
    const sg_weight* weights;   /* copied at creation                                            */
    int64_t max_m;              /* largest request M                                             */
    uint64_t seed;              /* activation pool and per-request offsets                       */
    double a_scale;             /* activation standard deviation                                 */
    int64_t small_m;            /* requests with M <= small_m run with small_tile (0: none)      */
    int small_tile;             /* tile shape index 0..6 for those skinny requests               */
    int64_t solo_m;             /* requests with M > solo_m launch alone (0: every request groups) */
    int tiles_from_table;       /* 1: a request's tile class is the tile of the best variant of the
                                   context's dispatch table (held at creation) for its (M, N, K),
                                   each axis clamped to the grid; split-K and stream-K variants give
                                   their tile, the deep-K 64 x 64 the 64 x 64 tile; small_m,
                                   small_tile and tile are then unused.  SG_ENOTABLE without a
                                   table.  0: the small_m rule                                      */
} sg_server_cfg;
typedef struct sg_request { uint64_t id; int64_t M; int weight; } sg_request;
typedef struct sg_completion {
    uint64_t ticket, id;
    int64_t M, N, K;
    int weight;
    int status;                 /* SG_OK or the failure code                                     */
    int64_t a_offset;           /* element offset of A in the activation pool                    */
    int tile;                   /* tile shape the request ran with                               */
    int group_size;             /* requests in the launch that ran it (1: launched alone)        */
    double t_arrival, t_admit, t_launch, t_done;
    const void* A;              /* device; valid until release when keep_results, else NULL      */
    const void* C;
} sg_completion;
typedef struct sg_server_stats {
    int64_t submitted, completed, failed, launches, pending;
    double flops, bytes_in_use, peak_bytes;
} sg_server_stats;
typedef struct sg_server sg_server;
int sg_server_create(sg_ctx* ctx, const sg_server_cfg* cfg, sg_server** out);
int sg_server_now(sg_server* server, double* t);
/* Non-blocking.  arrival_s < 0 stamps the current time.  SG_EAGAIN when the queue is full;
 * SG_EINVAL for an M or weight out of range or a request that can never fit the budget. */
int sg_server_submit(sg_server* server, const sg_request* req, double arrival_s, uint64_t* ticket);
/* Move up to max finished requests (oldest first) into out; *n receives the count. */
int sg_server_poll(sg_server* server, sg_completion* out, int max, int* n);
int sg_server_release(sg_server* server, uint64_t ticket);
/* Wait until every submitted request has finished (SG_EAGAIN after timeout_s). */
int sg_server_drain(sg_server* server, double timeout_s);
int sg_server_stats_get(sg_server* server, sg_server_stats* st);
int sg_server_destroy(sg_server* server);

/* Open-loop load: Poisson arrivals at `rate` per second for duration_s, M = clamp(round(
 * exp(U(0, ln max_m))), 1, max_m), weight uniform; waits for the drain and reports requests
 * that arrived after warmup_s: nearest-rank p50 / p99 of (done - arrival), throughput. */
typedef struct sg_serve_report {
    int64_t offered, rejected, failed, measured, launches;
    double window_s, req_per_s, tflops, p50_ms, p99_ms, mean_ms, peak_bytes;
} sg_serve_report;
int sg_serve_poisson(sg_server* server, double rate, double duration_s, double warmup_s,
                     uint64_t seed, int64_t max_m, sg_serve_report* rep);
/* Closed-loop load (saturation): keeps `outstanding` requests in the server -- a new one is
 * submitted as each completes -- for duration_s, requests drawn as in sg_serve_poisson; reports
 * the requests that arrived in [warmup_s, duration_s): throughput and nearest-rank p50 / p99 of
 * (done - submit).  `launches` counts this run's launches only. */
int sg_serve_closed(sg_server* server, int outstanding, double duration_s, double warmup_s,
                    uint64_t seed, int64_t max_m, sg_serve_report* rep);

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
