// Internal declarations shared by the smoothgemm host runtime and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>
#include <string>
#include <vector>

#include "../../include/smoothgemm.h"

namespace sg {

// Thread-local error message; every C entry point records its failure through this.
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

#define SG_HIP(call)                                   \
    do {                                               \
        hipError_t e_ = (call);                        \
        if (e_ != hipSuccess) return ::sg::hip_fail(e_, #call); \
    } while (0)

// Buffer read / write kernels of the memory study (membench.hip).  Length a multiple of 16
// bytes, 16-byte aligned buffer; the read writes mem_blocks(bytes) partial XORs to sink.
int64_t mem_blocks(int64_t bytes);
int launch_mem_read(const void* buf, int64_t bytes, uint32_t* sink, hipStream_t s, hipEvent_t start,
                    hipEvent_t stop);
int launch_mem_write(void* buf, int64_t bytes, uint32_t seed, hipStream_t s, hipEvent_t start, hipEvent_t stop);

// One GEMM kernel launch of the tile family.
//  data dims (M, N, K) bound every load and store; the launch covers (Ml, Nl) in whole tiles
//  and runs the K loop over Kl >= K (padding: beyond K the operands read as zero).
struct LaunchDesc {
    int64_t M, N, K;
    int64_t Ml, Nl, Kl;
    const uint16_t* A; int64_t lda;
    const uint16_t* B; int64_t ldb;
    void* C; int64_t ldc;
    int out_bf16;                  // 1: C is BF16, 0: FP32
    const void* add; int64_t ldadd;
    int add_kind;                  // 0 none, 1 FP32 addend, 2 BF16 addend (may alias C)
    // Timing events stamped by the dispatch packets (may be null): ev_start at the start of the
    // tile kernel, ev_mid at its end when a split-K reduction follows, ev_stop at the end of
    // the launch's last kernel.
    hipEvent_t ev_start = nullptr, ev_mid = nullptr, ev_stop = nullptr;
    int mem_only = 0;              // 1: run the tile's memory-only twin (no MFMA work, C = addend or 0)
};

enum { ADD_NONE = 0, ADD_F32 = 1, ADD_BF16 = 2 };

constexpr int kNumTiles = 8;
constexpr int kSplitLevels = 4;               // S = 1, 2, 4, 8
constexpr int kNumSplitVariants = kNumTiles * kSplitLevels;
// Stream-K variants follow the split-K ones: variant kSkBase + t runs tile t (0..6) with the K
// iterations of all its tiles shared evenly by every resident work-group.
constexpr int kSkBase = kNumSplitVariants;
constexpr int kNumSkTiles = 7;
constexpr int kNumVariants = kNumSplitVariants + kNumSkTiles;
constexpr int kBK = 64;
// Tile 7 is 64 x 64 with 128-deep K stages (tile 6 with 64-deep ones): per call only, the
// persistent grouped kernel carries tiles 0 .. kNumGroupTiles - 1.
constexpr int kDeepTile = 7;
constexpr int kNumGroupTiles = 7;
constexpr int kDeepBK = 128;

struct TileShape { int bm, bn; };
extern const TileShape kTiles[kNumTiles];

inline bool variant_is_sk(int v) { return v >= kSkBase; }
inline int variant_tile(int v) { return variant_is_sk(v) ? v - kSkBase : v / kSplitLevels; }
// Parallel split-K factor (1 for stream-K variants, which split K across work-groups their own way).
inline int variant_splits(int v) { return variant_is_sk(v) ? 1 : 1 << (v % kSplitLevels); }
// K granularity of a split (a K stage never straddles two split ranges).
inline int tile_split_granule(int tile) { return tile == kDeepTile ? kDeepBK : kBK; }

// Number of non-empty K splits and the K extent of each for a launch of K extent Kl.
void split_geometry(int variant, int64_t Kl, int* splits, int64_t* k_chunk);
// Workspace bytes the variant needs for this launch: split-K partials, plus zero-padded copies
// of operands the direct-to-LDS kernel cannot read in place (0 when neither applies).
size_t launch_workspace_bytes(int variant, const LaunchDesc& d);
// Whether the launch runs a second kernel after the tile kernel (a split-K reduction, or the
// fix-up of a stream-K launch whose work-group ranges split a tile).
bool launch_has_second_kernel(int variant, const LaunchDesc& d);
// Enqueue one launch (operand copies if any, the tile kernel, and for S > 1 its reduction).
// ws must hold launch_workspace_bytes, or be null: then a split-K launch fails and operands
// that need a copy are read by the element-wise body instead.
int launch_variant(int variant, const LaunchDesc& d, void* ws, hipStream_t stream);
int lds_bytes_of_tile(int tile);

// Device descriptor of one problem of a grouped launch.
struct GroupProblem {
    const uint16_t* A;
    const uint16_t* B;
    void* C;
    int64_t lda, ldb, ldc;
    int M, N, K;
    int tile_begin;      // first queue index of this problem's tiles
    int tiles_m, tiles_n;
    int aligned;
    int vec_ok;          // C rows allow 4-wide vector stores
    int a_bytes, b_bytes;
};

// Grouped launch building blocks (also used by the server, which stages descriptors itself).
// Fill host descriptors for tile shape `tile`; order[i] receives the caller's index of queue
// entry i (longest K first when lpt, else as given).
// *all_aligned: every problem can take the aligned fast path.
int grouped_fill(const sg_problem* probs, int G, int tile, int c_dtype, bool lpt, GroupProblem* out,
                 int* order, int* total_tiles, double* flops, bool* all_aligned);
// Resident work-groups for the tile shape on `device` (capped at the tile count).
int grouped_grid(int tile, bool all_aligned, int device, int total_tiles, int grid_wgs, int* grid);
// Enqueue one persistent launch over device descriptors; counters: 2 ints, zero before the
// first launch, returned to zero by every launch.
int grouped_enqueue(int tile, bool all_aligned, const GroupProblem* d_probs, int G, int total_tiles,
                    int grid, int c_dtype, int* d_counters, hipStream_t s, hipEvent_t start,
                    hipEvent_t stop);

// The dispatch table a context borrows (NULL if none); defined with the context.
const struct ::sg_table* ctx_table(const struct ::sg_ctx* ctx);

// Device generator launcher.
int launch_fill(uint16_t* dst, int64_t n, uint64_t seed, uint64_t stream_id, int64_t offset,
                int kind, double scale, hipStream_t stream);

}  // namespace sg
