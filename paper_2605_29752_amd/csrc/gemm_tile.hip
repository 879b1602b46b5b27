// BF16 NN GEMM tile family for gfx950 (CDNA4).
//
// C = A * B, A M x K row-major (K contiguous), B K x N row-major (N contiguous); the problem
// statement of the paper's Sec. 2.2 / Sec. 7.1.  Each work-group (256 threads = 4 wave64 in a
// 2 x 2 arrangement) computes one BM x BN tile of C with v_mfma_f32_16x16x32_bf16 and FP32
// accumulators in registers.  Two bodies:
//
//  * aligned operands (leading dimensions, K and N multiples of 8, 16-byte bases: every shape
//    of the landscape), or operands first copied zero-padded into the workspace so that they
//    are: tile_body_dma.h, operands loaded HBM -> LDS directly into a ring of K stages whose
//    depth is chosen per tile (DmaTile), B fragments read with transposing LDS reads;
//  * anything else (no workspace, or an operand extent beyond the loads' 31-bit offsets):
//    tile_body.h, element-wise predicated loads into registers, B transposed in registers, two
//    padded LDS stages of 64-deep K steps.
//
// Each direct-to-LDS kernel has a memory-only twin (sg_gemm_tile_dma_mem) with the same loads,
// waits and stores and no matrix work: the measured memory surface of the paper's Sec. 4.
//
// The MFMA is issued with B^T as its first operand, so each lane ends up holding four
// consecutive N columns of one C row and stores them as one vector.
//
// Edges are predicated: rows / columns / depth beyond the data dims read as zero and are never
// stored.  The launch may be larger than the data (the pad action of the dispatch table):
// tiles wholly outside the data exit at once, depth beyond K is multiplied as zeros.
//
// Parallel split-K (S > 1): grid.z = S, each z covers one K range and writes an FP32 partial to
// its own workspace slice; sg_splitk_reduce then adds the S slices in fixed order (no atomics,
// bit-reproducible) and applies the epilogue.
#include <hip/hip_ext.h>

#include "sg_internal.h"
#include "tile_body.h"
#include "tile_body_dma.h"

namespace sg {

const TileShape kTiles[kNumTiles] = {{256, 256}, {256, 128}, {128, 256}, {128, 128},
                                     {128, 64},  {64, 128},  {64, 64},   {64, 64}};

// Aligned fast path with direct-to-LDS operand loads (see tile_body_dma.h).
template <int BM, int BN>
__global__ __launch_bounds__((64 * call_waves<BM, BN>())) void sg_gemm_tile_dma(KArgs p) {
    constexpr int NW = call_waves<BM, BN>();
    __shared__ __attribute__((aligned(1024))) uint16_t smem[dma_smem_bytes<BM, BN, false, NW>() / 2];
    int tm, tn;
    tile_coords(p.tiles_m, p.tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= p.M || n0 >= p.N) return;            // padding-only tile
    tile_body_dma<BM, BN, false, false, NW>(p, m0, n0, blockIdx.z, smem);
}

// Memory-only twin of sg_gemm_tile_dma: the same loads, waits and stores, no MFMA work.
template <int BM, int BN>
__global__ __launch_bounds__((64 * call_waves<BM, BN>())) void sg_gemm_tile_dma_mem(KArgs p) {
    constexpr int NW = call_waves<BM, BN>();
    __shared__ __attribute__((aligned(1024))) uint16_t smem[dma_smem_bytes<BM, BN, false, NW>() / 2];
    int tm, tn;
    tile_coords(p.tiles_m, p.tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= p.M || n0 >= p.N) return;
    tile_body_dma<BM, BN, true, false, NW>(p, m0, n0, blockIdx.z, smem);
}

// The 64 x 64 tile with 128-deep K stages (tile 7), and its memory-only twin.
template <int BM, int BN>
__global__ __launch_bounds__(256) void sg_gemm_tile_dma_k128(KArgs p) {
    __shared__ __attribute__((aligned(1024))) uint16_t smem[dma_smem_bytes<BM, BN, true>() / 2];
    int tm, tn;
    tile_coords(p.tiles_m, p.tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= p.M || n0 >= p.N) return;
    tile_body_dma<BM, BN, false, true>(p, m0, n0, blockIdx.z, smem);
}

template <int BM, int BN>
__global__ __launch_bounds__(256) void sg_gemm_tile_dma_k128_mem(KArgs p) {
    __shared__ __attribute__((aligned(1024))) uint16_t smem[dma_smem_bytes<BM, BN, true>() / 2];
    int tm, tn;
    tile_coords(p.tiles_m, p.tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= p.M || n0 >= p.N) return;
    tile_body_dma<BM, BN, true, true>(p, m0, n0, blockIdx.z, smem);
}

typedef void (*TileKernel)(KArgs);

// Direct-to-LDS kernel of a tile and its memory-only twin.
template <int BM, int BN, bool DEEP>
static TileKernel dma_kernel(bool twin) {
    if constexpr (DEEP) return twin ? sg_gemm_tile_dma_k128_mem<BM, BN> : sg_gemm_tile_dma_k128<BM, BN>;
    else return twin ? sg_gemm_tile_dma_mem<BM, BN> : sg_gemm_tile_dma<BM, BN>;
}

template <int BM, int BN>
__global__ __launch_bounds__(256) void sg_gemm_tile(KArgs p) {
    __shared__ __attribute__((aligned(16))) uint16_t smem[smem_elems<BM, BN>()];
    int tm, tn;
    tile_coords(p.tiles_m, p.tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= p.M || n0 >= p.N) return;            // padding-only tile
    tile_body<BM, BN>(p, m0, n0, blockIdx.z, smem);
}

// ---- stream-K: the K iterations of all tiles shared evenly by the resident work-groups ------
//
// The launch's work is the list of (tile, K stage) iterations, tile-major (tiles M-fastest, the
// stages of a tile in K order).  Work-group g of G takes iterations [g T / G, (g + 1) T / G) of
// the T in total, so every work-group does the same amount of MFMA work whatever the tile count
// (no wave-quantization tail).  A tile whose stages all fall to one work-group is written to C
// directly; the other tiles are split between consecutive work-groups, each writing its FP32
// partial of the tile to a slot of the workspace (slot 2 g for the first tile of g's range, 2 g + 1
// for its last), and a fix-up kernel sums a split tile's partials in work-group order (so in K
// order: bit-reproducible) and applies the epilogue.  Work-group g is the logical index of the
// dispatch order remapped so that consecutive logical work-groups -- which share tiles and
// operand panels -- run on one XCD.
struct SkArgs {
    float* partial;     // 2 G slots of BM x BN FP32, tile-local rows of BN
    int tiles;          // tiles_m * tiles_n (data tiles)
    int ipt;            // K stages per tile
};

__device__ __forceinline__ int sk_logical(int b, int G) {
    const int x = b & 7, q = G >> 3, r = G & 7;
    return x * q + (x < r ? x : r) + (b >> 3);
}

template <int BM, int BN>
__global__ __launch_bounds__((64 * call_waves<BM, BN>())) void sg_gemm_tile_dma_sk(KArgs p, SkArgs s) {
    constexpr int NW = call_waves<BM, BN>();
    __shared__ __attribute__((aligned(1024))) uint16_t smem[dma_smem_bytes<BM, BN, false, NW>() / 2];
    constexpr int BKD = DmaTile<BM, BN, false, NW>::BKD;
    const int G = gridDim.x;
    const int g = sk_logical(blockIdx.x, G);
    const int64_t total = (int64_t)s.tiles * s.ipt;
    const int64_t begin = (int64_t)g * total / G, end = (int64_t)(g + 1) * total / G;
    for (int64_t it = begin; it < end;) {
        const int t = (int)(it / s.ipt);
        const int k0 = (int)(it - (int64_t)t * s.ipt);
        const int k1 = (int)min<int64_t>(s.ipt, k0 + (end - it));
        const int m0 = (t % p.tiles_m) * BM, n0 = (t / p.tiles_m) * BN;
        if (it != begin) __syncthreads();       // the previous segment is done with the LDS
        // a whole tile goes to C; a partial goes to this work-group's slot, addressed as rows of
        // BN from (m0, n0) (one tile body for both, its output arguments selected)
        const bool whole = (k0 == 0 && k1 == s.ipt);
        KArgs q = p;
        if (!whole) {
            const int slot = (it == begin) ? 2 * g : 2 * g + 1;
            q.C = s.partial + (int64_t)slot * BM * BN - ((int64_t)m0 * BN + n0);
            q.ldc = BN; q.out_bf16 = 0;
            q.add = nullptr; q.add_kind = ADD_NONE; q.vec_ok = 1;
        }
        // (no cross-stage fragment prefetch for 256 x 256 here: its registers would spill)
        tile_body_dma_range<BM, BN, false, false, NW, !(BM == 256 && BN == 256)>(q, m0, n0, 0, k0 * BKD,
                                                                                 min(p.Kl, k1 * BKD), smem);
        it += k1 - k0;
    }
}

// Fix-up of a stream-K launch: one work-group per tile; a tile whose stages span work-groups
// g_lo .. g_hi gets the sum of their partials (g ascending), plus the addend, stored to C.
template <int BM, int BN>
__global__ __launch_bounds__(256) void sg_sk_fixup(KArgs p, SkArgs s, int G) {
    const int t = blockIdx.x;
    const int64_t total = (int64_t)s.tiles * s.ipt;
    // the work-group whose range holds iteration i: the last g with g T / G <= i
    auto wg_of = [&](int64_t i) { return (int)(((i + 1) * G + total - 1) / total) - 1; };
    const int64_t lo = (int64_t)t * s.ipt;
    const int g_lo = wg_of(lo), g_hi = wg_of(lo + s.ipt - 1);
    if (g_lo == g_hi) return;                   // written whole by one work-group
    const int m0 = (t % p.tiles_m) * BM, n0 = (t / p.tiles_m) * BN;
    constexpr int C4 = BN / 4;
    for (int q = threadIdx.x; q < BM * C4; q += 256) {
        const int r = q / C4, c = (q - r * C4) * 4;
        const int m = m0 + r, n = n0 + c;
        if (m >= p.M || n >= p.N) continue;
        f32x4_t v = {0.f, 0.f, 0.f, 0.f};
        for (int g = g_lo; g <= g_hi; ++g) {
            const int64_t gb = (int64_t)g * total / G;
            if (gb == (int64_t)(g + 1) * total / G) continue;      // empty range
            const int slot = (gb / s.ipt == t) ? 2 * g : 2 * g + 1;
            v += *(const f32x4_t*)(s.partial + (int64_t)slot * BM * BN + r * BN + c);
        }
        const bool full = p.vec_ok && (n + 3 < p.N);
        if (p.add_kind == ADD_F32) {
            const float* ap = (const float*)p.add + (int64_t)m * p.ldadd + n;
            for (int e = 0; e < 4; ++e)
                if (n + e < p.N) v[e] += ap[e];
        } else if (p.add_kind == ADD_BF16) {
            const uint16_t* ap = (const uint16_t*)p.add + (int64_t)m * p.ldadd + n;
            for (int e = 0; e < 4; ++e)
                if (n + e < p.N) v[e] += bf16_to_f32(ap[e]);
        }
        if (p.out_bf16) {
            uint16_t* cp = (uint16_t*)p.C + (int64_t)m * p.ldc + n;
            if (full) {
                u32x2_t o;
                o[0] = (uint32_t)f32_to_bf16_rne(v[0]) | ((uint32_t)f32_to_bf16_rne(v[1]) << 16);
                o[1] = (uint32_t)f32_to_bf16_rne(v[2]) | ((uint32_t)f32_to_bf16_rne(v[3]) << 16);
                *(u32x2_t*)cp = o;
            } else {
                for (int e = 0; e < 4; ++e)
                    if (n + e < p.N) cp[e] = f32_to_bf16_rne(v[e]);
            }
        } else {
            float* cp = (float*)p.C + (int64_t)m * p.ldc + n;
            if (full) {
                *(f32x4_t*)cp = v;
            } else {
                for (int e = 0; e < 4; ++e)
                    if (n + e < p.N) cp[e] = v[e];
            }
        }
    }
}

// Fixed-order sum of S FP32 partial slices (M x N, ld = N) plus the epilogue.
__global__ __launch_bounds__(256) void sg_splitk_reduce(const float* ws, int64_t slice, int S,
                                                         int M, int N, void* C, int64_t ldc,
                                                         int out_bf16, const void* add,
                                                         int64_t ldadd, int add_kind) {
    const int64_t total = (int64_t)M * N;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < total;
         idx += (int64_t)gridDim.x * blockDim.x) {
        const int m = (int)(idx / N), n = (int)(idx - (int64_t)m * N);
        float s = ws[idx];
        for (int z = 1; z < S; ++z) s += ws[(int64_t)z * slice + idx];
        if (add_kind == ADD_F32) s += ((const float*)add)[(int64_t)m * ldadd + n];
        else if (add_kind == ADD_BF16) s += bf16_to_f32(((const uint16_t*)add)[(int64_t)m * ldadd + n]);
        if (out_bf16) ((uint16_t*)C)[(int64_t)m * ldc + n] = f32_to_bf16_rne(s);
        else ((float*)C)[(int64_t)m * ldc + n] = s;
    }
}

// The same, four consecutive columns per thread (N, ldc and ldadd multiples of 4, C and the
// addend aligned to four elements): 16-byte partial loads, one index
// division per four elements (launched for M * N / 4 < 2^30, so indices stay in int range).
// Summation order and rounding are those of sg_splitk_reduce.
__global__ __launch_bounds__(256) void sg_splitk_reduce4(const float* ws, int64_t slice, int S,
                                                          int M, int N, void* C, int64_t ldc,
                                                          int out_bf16, const void* add,
                                                          int64_t ldadd, int add_kind) {
    const int n4 = N >> 2;
    const int total4 = M * n4;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total4; q += gridDim.x * blockDim.x) {
        const int m = q / n4, n = (q - m * n4) * 4;
        const int64_t idx = (int64_t)m * N + n;
        f32x4_t s = *(const f32x4_t*)(ws + idx);
        for (int z = 1; z < S; ++z) s += *(const f32x4_t*)(ws + (int64_t)z * slice + idx);
        if (add_kind == ADD_F32) {
            s += *(const f32x4_t*)((const float*)add + (int64_t)m * ldadd + n);
        } else if (add_kind == ADD_BF16) {
            const u32x2_t a2 = *(const u32x2_t*)((const uint16_t*)add + (int64_t)m * ldadd + n);
            s[0] += bf16_to_f32(a2[0] & 0xFFFFu); s[1] += bf16_to_f32(a2[0] >> 16);
            s[2] += bf16_to_f32(a2[1] & 0xFFFFu); s[3] += bf16_to_f32(a2[1] >> 16);
        }
        if (out_bf16) {
            u32x2_t o;
            o[0] = (uint32_t)f32_to_bf16_rne(s[0]) | ((uint32_t)f32_to_bf16_rne(s[1]) << 16);
            o[1] = (uint32_t)f32_to_bf16_rne(s[2]) | ((uint32_t)f32_to_bf16_rne(s[3]) << 16);
            *(u32x2_t*)((uint16_t*)C + (int64_t)m * ldc + n) = o;
        } else {
            *(f32x4_t*)((float*)C + (int64_t)m * ldc + n) = s;
        }
    }
}

// LDS of the aligned (direct-to-LDS) kernel of a tile: its ring of K stages.
int lds_bytes_of_tile(int tile) {
    switch (tile) {
        case 0: return dma_smem_bytes<256, 256, false, call_waves<256, 256>()>();
        case 1: return dma_smem_bytes<256, 128, false, call_waves<256, 128>()>();
        case 2: return dma_smem_bytes<128, 256, false, call_waves<128, 256>()>();
        case 3: return dma_smem_bytes<128, 128, false, call_waves<128, 128>()>();
        case 4: return dma_smem_bytes<128, 64>();
        case 5: return dma_smem_bytes<64, 128>();
        case 6: return dma_smem_bytes<64, 64>();
        default: return dma_smem_bytes<64, 64, true>();
    }
}

void split_geometry(int variant, int64_t Kl, int* splits, int64_t* k_chunk) {
    const int S = variant_splits(variant);
    const int64_t g = tile_split_granule(variant_tile(variant));
    int64_t per = (Kl + S - 1) / S;
    per = (per + g - 1) / g * g;
    if (per < g) per = g;
    *k_chunk = per;
    int64_t s = (Kl + per - 1) / per;
    *splits = (int)(s < 1 ? 1 : s);
}

// Zero-padded copy of a row-major BF16 matrix: dst[r][c] = src[r][c] for c < cols, 0 for
// cols <= c < ldd (ldd a multiple of 8, rows * ldd < 2^31).  One 16-byte store per thread.
__global__ __launch_bounds__(256) void sg_pack_bf16(const uint16_t* src, int64_t lds, int rows, int cols,
                                                     uint16_t* dst, int ldd) {
    const int n8 = ldd >> 3;
    const int total = rows * n8;
    for (int q = blockIdx.x * blockDim.x + threadIdx.x; q < total; q += gridDim.x * blockDim.x) {
        const int r = q / n8, c0 = (q - r * n8) * 8;
        const uint16_t* sp = src + (int64_t)r * lds;
        uint32_t w[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int c = c0 + 2 * e;
            const uint32_t lo = c < cols ? sp[c] : 0u;
            const uint32_t hi = c + 1 < cols ? sp[c + 1] : 0u;
            w[e] = lo | (hi << 16);
        }
        *(u32x4_t*)(dst + (int64_t)r * ldd + c0) = u32x4_t{w[0], w[1], w[2], w[3]};
    }
}

// Operands the direct-to-LDS kernel cannot read in place (leading dimension, K or N not a
// multiple of 8, or a base not 16-byte aligned) are first copied to the workspace, zero-padded
// to 8-element rows: A as M x roundup(K, 8), B as K x roundup(N, 8).  A chunk of 8 elements
// that straddles the data edge then reads zeros beyond it, so the kernel's per-chunk checks
// stay exact.  Layout in the workspace: split-K partials, then A', then B' (256-byte aligned).
struct Packing {
    bool pack_a = false, pack_b = false;
    int64_t k8 = 0, n8 = 0;
    size_t part_bytes = 0, a_off = 0, b_off = 0, total = 0;
};

static size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

static bool in_place_a(const LaunchDesc& d) {
    return d.lda % 8 == 0 && d.K % 8 == 0 && (uintptr_t)d.A % 16 == 0;
}
static bool in_place_b(const LaunchDesc& d) {
    return d.ldb % 8 == 0 && d.N % 8 == 0 && (uintptr_t)d.B % 16 == 0;
}

// Geometry of a stream-K launch of tile t: data tiles, K stages per tile, resident work-groups
// G (occupancy on every CU, at most one per iteration) and whether any tile is split between
// work-groups (then the fix-up runs).
struct SkGeom {
    int tiles = 0, ipt = 0, G = 0;
    bool fixup = false;
};

template <int BM, int BN>
static int sk_occupancy() {
    static int occ = -1;
    if (occ < 0) {
        int o = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&o, sg_gemm_tile_dma_sk<BM, BN>, 64 * call_waves<BM, BN>(), 0) !=
                hipSuccess || o < 1) {
            (void)hipGetLastError();
            o = 1;
        }
        occ = o;
    }
    return occ;
}

static int sk_occupancy_of(int tile) {
    switch (tile) {
        case 0: return sk_occupancy<256, 256>();
        case 1: return sk_occupancy<256, 128>();
        case 2: return sk_occupancy<128, 256>();
        case 3: return sk_occupancy<128, 128>();
        case 4: return sk_occupancy<128, 64>();
        case 5: return sk_occupancy<64, 128>();
        default: return sk_occupancy<64, 64>();
    }
}

static int device_cus() {
    static int cus[64] = {0};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
    if (cus[dev] == 0) {
        int c = 0;
        if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1) c = 256;
        cus[dev] = c;
    }
    return cus[dev];
}

static int stage_depth_of(int tile) {
    switch (tile) {
        case 0: return DmaTile<256, 256>::BKD;
        case 1: return DmaTile<256, 128>::BKD;
        case 2: return DmaTile<128, 256>::BKD;
        case 3: return DmaTile<128, 128>::BKD;
        case 4: return DmaTile<128, 64>::BKD;
        case 5: return DmaTile<64, 128>::BKD;
        case 6: return DmaTile<64, 64>::BKD;
        default: return DmaTile<64, 64, true>::BKD;
    }
}

static SkGeom sk_geometry(int variant, const LaunchDesc& d) {
    SkGeom g;
    const int tile = variant_tile(variant);
    const TileShape ts = kTiles[tile];
    const int bkd = stage_depth_of(tile);
    g.tiles = (int)(((d.M + ts.bm - 1) / ts.bm) * ((d.N + ts.bn - 1) / ts.bn));
    g.ipt = (int)((d.Kl + bkd - 1) / bkd);
    const int64_t total = (int64_t)g.tiles * g.ipt;
    g.G = (int)std::min<int64_t>(total, (int64_t)sk_occupancy_of(tile) * device_cus());
    if (g.G < 1) g.G = 1;
    for (int64_t w = 1; w < g.G && !g.fixup; ++w)
        if ((w * total / g.G) % g.ipt != 0) g.fixup = true;     // a range boundary inside a tile
    return g;
}

static Packing packing_of(int variant, const LaunchDesc& d) {
    Packing pk;
    int S;
    int64_t kc;
    split_geometry(variant, d.Kl, &S, &kc);
    pk.part_bytes = S > 1 ? round256((size_t)S * (size_t)d.M * (size_t)d.N * sizeof(float)) : 0;
    if (variant_is_sk(variant)) {
        const TileShape ts = kTiles[variant_tile(variant)];
        pk.part_bytes = round256((size_t)2 * sk_geometry(variant, d).G * ts.bm * ts.bn * sizeof(float));
    }
    pk.total = pk.part_bytes;
    if (d.K <= 0 || (in_place_a(d) && in_place_b(d))) return pk;
    pk.k8 = (d.K + 7) / 8 * 8;
    pk.n8 = (d.N + 7) / 8 * 8;
    pk.pack_a = !in_place_a(d);
    pk.pack_b = !in_place_b(d);
    // every byte offset of the (packed or in-place) operands must fit the 31-bit buffer range
    const int64_t a_ext = pk.pack_a ? d.M * pk.k8 * 2 : ((d.M - 1) * d.lda + d.K) * 2;
    const int64_t b_ext = pk.pack_b ? d.K * pk.n8 * 2 : ((d.K - 1) * d.ldb + d.N) * 2;
    if (a_ext >= 0x7FFFFFFF || b_ext >= 0x7FFFFFFF) {
        pk.pack_a = pk.pack_b = false;                  // the element-wise body handles it
        return pk;
    }
    pk.a_off = pk.total;
    if (pk.pack_a) pk.total += round256((size_t)a_ext);
    pk.b_off = pk.total;
    if (pk.pack_b) pk.total += round256((size_t)b_ext);
    return pk;
}

size_t launch_workspace_bytes(int variant, const LaunchDesc& d) { return packing_of(variant, d).total; }

static int launch_pack(const uint16_t* src, int64_t lds, int64_t rows, int64_t cols, uint16_t* dst,
                       int64_t ldd, hipEvent_t start, hipStream_t stream) {
    const int64_t total = rows * (ldd / 8);
    int64_t blocks = (total + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) return SG_OK;
    hipExtLaunchKernelGGL(sg_pack_bf16, dim3((unsigned)blocks), dim3(256), 0, stream, start, nullptr, 0,
                          src, lds, (int)rows, (int)cols, dst, (int)ldd);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

// Dynamic LDS to reserve for the memory-only twin of a tile so that it runs as many
// work-groups per CU as its GEMM kernel (the twin needs far fewer registers, which alone would
// let more of it share a CU and overstate the bandwidth the GEMM's loads can draw).  -1 if the
// occupancy query fails.
template <int BM, int BN, bool DEEP>
static int twin_extra_lds() {
    constexpr int threads = DEEP ? 256 : 64 * call_waves<BM, BN>();
    int occ_gemm = 0, occ_twin = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_gemm, dma_kernel<BM, BN, DEEP>(false), threads, 0) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_twin, dma_kernel<BM, BN, DEEP>(true), threads, 0) != hipSuccess ||
        occ_gemm < 1)
        return -1;
    if (occ_twin <= occ_gemm) return 0;
    int smem = 0;
    if constexpr (DEEP) smem = dma_smem_bytes<BM, BN, true>();
    else smem = dma_smem_bytes<BM, BN, false, call_waves<BM, BN>()>();
    const int budget = 160 * 1024 - smem;
    for (int extra = 1024; extra <= budget; extra += 1024) {
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_twin, dma_kernel<BM, BN, DEEP>(true), threads,
                                                         (size_t)extra) != hipSuccess)
            return -1;
        if (occ_twin <= occ_gemm) return extra;
    }
    return -1;
}

// Whether the direct-to-LDS body can run the launch: operands aligned in place, or packed into
// the workspace, with every byte offset inside the loads' 31-bit range.
static bool dma_feasible(int variant, const LaunchDesc& d, bool have_ws) {
    const Packing pk = packing_of(variant, d);
    const bool packed = (pk.pack_a || pk.pack_b) && have_ws;
    const int64_t a_bytes = pk.pack_a && packed ? d.M * pk.k8 * 2 : ((d.M - 1) * d.lda + d.K) * 2;
    const int64_t b_bytes = d.K <= 0 ? 0 : pk.pack_b && packed ? d.K * pk.n8 * 2 : ((d.K - 1) * d.ldb + d.N) * 2;
    return (packed || (in_place_a(d) && in_place_b(d))) && a_bytes < 0x7FFFFFFF && b_bytes < 0x7FFFFFFF;
}

bool launch_has_second_kernel(int variant, const LaunchDesc& d) {
    if (variant_is_sk(variant))
        return dma_feasible(variant, d, true) && !d.mem_only && sk_geometry(variant, d).fixup;
    int S = 1;
    int64_t kc = 0;
    split_geometry(variant, d.Kl, &S, &kc);
    return S > 1;
}

template <int BM, int BN, bool DEEP = false>
static int launch_tile(const LaunchDesc& d, int variant, void* ws, hipStream_t stream);

// A stream-K launch: operand packing as for the other variants, the stream-K tile kernel over
// the data tiles, and the fix-up when a tile is split between work-groups.  Operands the
// direct-to-LDS body cannot load run the tile's plain (one-split) variant instead.
template <int BM, int BN>
static int launch_sk(const LaunchDesc& d, int variant, void* ws, hipStream_t stream) {
    if (d.mem_only) return fail(SG_EINVAL, "stream-K variants have no memory-only twin");
    if (ws == nullptr) return fail(SG_EINVAL, "stream-K launch without workspace");
    const int tile = variant_tile(variant);
    if (!dma_feasible(variant, d, true)) return launch_tile<BM, BN>(d, tile * kSplitLevels, ws, stream);
    const Packing pk = packing_of(variant, d);
    const SkGeom gm = sk_geometry(variant, d);
    KArgs a;
    a.A = d.A; a.B = d.B;
    a.lda = d.lda; a.ldb = d.ldb;
    hipEvent_t start = d.ev_start;
    if (pk.pack_a) {
        uint16_t* ap = (uint16_t*)((char*)ws + pk.a_off);
        int rc = launch_pack(d.A, d.lda, d.M, d.K, ap, pk.k8, start, stream);
        if (rc) return rc;
        start = nullptr;
        a.A = ap; a.lda = pk.k8;
    }
    if (pk.pack_b) {
        uint16_t* bp = (uint16_t*)((char*)ws + pk.b_off);
        int rc = launch_pack(d.B, d.ldb, d.K, d.N, bp, pk.n8, start, stream);
        if (rc) return rc;
        start = nullptr;
        a.B = bp; a.ldb = pk.n8;
    }
    a.a_bytes = (int)(pk.pack_a ? d.M * pk.k8 * 2 : ((d.M - 1) * d.lda + d.K) * 2);
    a.b_bytes = (int)(pk.pack_b ? d.K * pk.n8 * 2 : ((d.K - 1) * d.ldb + d.N) * 2);
    a.M = (int)d.M; a.N = (int)d.N; a.K = (int)d.K; a.Kl = (int)d.Kl;
    a.tiles_m = (int)((d.M + BM - 1) / BM);
    a.tiles_n = (int)((d.N + BN - 1) / BN);
    a.k_chunk = (int)d.Kl;
    a.C = d.C; a.ldc = d.ldc; a.ws_slice = 0;
    a.out_bf16 = d.out_bf16; a.add = d.add; a.ldadd = d.ldadd; a.add_kind = d.add_kind;
    const size_t esz = d.out_bf16 ? 2 : 4;
    bool vec_c = (d.ldc % 4 == 0) && ((uintptr_t)d.C % (4 * esz) == 0);
    if (d.add_kind == ADD_F32) vec_c = vec_c && (d.ldadd % 4 == 0) && ((uintptr_t)d.add % 16 == 0);
    if (d.add_kind == ADD_BF16) vec_c = vec_c && (d.ldadd % 4 == 0) && ((uintptr_t)d.add % 8 == 0);
    a.vec_ok = vec_c ? 1 : 0;
    if (gm.tiles <= 0) return SG_OK;
    const SkArgs sk{(float*)ws, gm.tiles, gm.ipt};
    hipExtLaunchKernelGGL(sg_gemm_tile_dma_sk<BM, BN>, dim3((unsigned)gm.G), dim3(64 * call_waves<BM, BN>()), 0, stream, start,
                          gm.fixup ? d.ev_mid : d.ev_stop, 0, a, sk);
    SG_HIP(hipGetLastError());
    if (gm.fixup) {
        hipExtLaunchKernelGGL(sg_sk_fixup<BM, BN>, dim3((unsigned)gm.tiles), dim3(256), 0, stream, nullptr,
                              d.ev_stop, 0, a, sk, gm.G);
        SG_HIP(hipGetLastError());
    }
    return SG_OK;
}

template <int BM, int BN, bool DEEP>
static int launch_tile(const LaunchDesc& d, int variant, void* ws, hipStream_t stream) {
    if constexpr (!DEEP)
        if (variant_is_sk(variant)) return launch_sk<BM, BN>(d, variant, ws, stream);
    KArgs a;
    a.A = d.A; a.B = d.B;
    a.lda = d.lda; a.ldb = d.ldb;
    a.M = (int)d.M; a.N = (int)d.N; a.K = (int)d.K; a.Kl = (int)d.Kl;
    a.tiles_m = (int)((d.Ml + BM - 1) / BM);
    a.tiles_n = (int)((d.Nl + BN - 1) / BN);
    int S;
    int64_t kc;
    split_geometry(variant, d.Kl, &S, &kc);
    a.k_chunk = (int)kc;
    // Direct-to-LDS path: 16-byte chunks never straddle the data edge (or, for a packed
    // operand, straddle it into zeros), and every valid byte offset fits the 31-bit range the
    // buffer loads use.  Otherwise the element-wise body.
    const Packing pk = packing_of(variant, d);
    hipEvent_t start = d.ev_start;                  // stamped by the launch's first kernel
    if ((pk.pack_a || pk.pack_b) && ws != nullptr) {
        if (pk.pack_a) {
            uint16_t* ap = (uint16_t*)((char*)ws + pk.a_off);
            int rc = launch_pack(d.A, d.lda, d.M, d.K, ap, pk.k8, start, stream);
            if (rc) return rc;
            start = nullptr;
            a.A = ap; a.lda = pk.k8;
        }
        if (pk.pack_b) {
            uint16_t* bp = (uint16_t*)((char*)ws + pk.b_off);
            int rc = launch_pack(d.B, d.ldb, d.K, d.N, bp, pk.n8, start, stream);
            if (rc) return rc;
            start = nullptr;
            a.B = bp; a.ldb = pk.n8;
        }
    }
    const bool packed = (pk.pack_a || pk.pack_b) && ws != nullptr;
    const int64_t a_bytes = pk.pack_a && packed ? d.M * pk.k8 * 2 : ((d.M - 1) * d.lda + d.K) * 2;
    const int64_t b_bytes = d.K <= 0 ? 0 : pk.pack_b && packed ? d.K * pk.n8 * 2 : ((d.K - 1) * d.ldb + d.N) * 2;
    const bool aligned = (packed || (in_place_a(d) && in_place_b(d))) &&
                         a_bytes < 0x7FFFFFFF && b_bytes < 0x7FFFFFFF;
    a.a_bytes = aligned ? (int)a_bytes : 0;
    a.b_bytes = aligned ? (int)b_bytes : 0;
    // 4-wide vector access to C and the addend
    const size_t esz = d.out_bf16 ? 2 : 4;
    bool vec_c = (d.ldc % 4 == 0) && ((uintptr_t)d.C % (4 * esz) == 0);
    if (d.add_kind == ADD_F32) vec_c = vec_c && (d.ldadd % 4 == 0) && ((uintptr_t)d.add % 16 == 0);
    if (d.add_kind == ADD_BF16) vec_c = vec_c && (d.ldadd % 4 == 0) && ((uintptr_t)d.add % 8 == 0);
    if (S > 1) {                                   // partials at the workspace start
        a.C = ws; a.ldc = d.N; a.ws_slice = d.M * d.N;
        a.out_bf16 = 0; a.add = nullptr; a.ldadd = 0; a.add_kind = ADD_NONE;
        a.vec_ok = (d.N % 4 == 0) && ((uintptr_t)ws % 16 == 0);
    } else {
        a.C = d.C; a.ldc = d.ldc; a.ws_slice = 0;
        a.out_bf16 = d.out_bf16; a.add = d.add; a.ldadd = d.ldadd; a.add_kind = d.add_kind;
        a.vec_ok = vec_c ? 1 : 0;
    }
    const int64_t nwg = (int64_t)a.tiles_m * a.tiles_n;
    if (nwg <= 0) return SG_OK;
    if (nwg > 0x7FFFFFFF) return fail(SG_EINVAL, "launch grid too large");
    // the direct-to-LDS kernels and their twins run call_waves() waves (the deep-K tile four);
    // the element-wise body always four
    dim3 grid((unsigned)nwg, 1, (unsigned)S), block(256), block_dma(DEEP ? 256 : 64 * call_waves<BM, BN>());
    hipEvent_t stop1 = (S > 1) ? d.ev_mid : d.ev_stop;
    if (d.mem_only && !aligned)
        return fail(SG_EINVAL, "memory-only twin: operands the direct-to-LDS path cannot load "
                               "(an extent of 2^31 bytes or more, or no workspace to pack into)");
    if (d.mem_only) {
        static const int extra = twin_extra_lds<BM, BN, DEEP>();
        if (extra < 0) { (void)hipGetLastError(); return fail(SG_EHIP, "occupancy query for the memory-only twin failed"); }
        hipExtLaunchKernelGGL(dma_kernel<BM, BN, DEEP>(true), grid, block_dma, (size_t)extra, stream, start, stop1, 0, a);
    }
    else if (aligned)
        hipExtLaunchKernelGGL(dma_kernel<BM, BN, DEEP>(false), grid, block_dma, 0, stream, start, stop1, 0, a);
    else
        hipExtLaunchKernelGGL((sg_gemm_tile<BM, BN>), grid, block, 0, stream, start, stop1, 0, a);
    SG_HIP(hipGetLastError());
    if (S > 1) {
        const int64_t total = d.M * d.N;
        const bool vec4 = vec_c && (d.N % 4 == 0) && ((uintptr_t)ws % 16 == 0) && total / 4 < (1 << 30);
        const int64_t items = vec4 ? total / 4 : total;
        int64_t blocks = (items + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        if (vec4)
            hipExtLaunchKernelGGL(sg_splitk_reduce4, dim3((unsigned)blocks), dim3(256), 0, stream,
                                  nullptr, d.ev_stop, 0, (const float*)ws, (int64_t)(d.M * d.N), S,
                                  (int)d.M, (int)d.N, d.C, d.ldc, d.out_bf16, d.add, d.ldadd, d.add_kind);
        else
            hipExtLaunchKernelGGL(sg_splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, stream,
                                  nullptr, d.ev_stop, 0, (const float*)ws, (int64_t)(d.M * d.N), S,
                                  (int)d.M, (int)d.N, d.C, d.ldc, d.out_bf16, d.add, d.ldadd, d.add_kind);
        SG_HIP(hipGetLastError());
    }
    return SG_OK;
}

int launch_variant(int variant, const LaunchDesc& d, void* ws, hipStream_t stream) {
    if (variant < 0 || variant >= kNumVariants) return fail(SG_EINVAL, "variant out of range");
    if (d.M <= 0 || d.N <= 0) return SG_OK;
    if (d.M > 0x7FFFFFFF || d.N > 0x7FFFFFFF || d.Kl > 0x7FFFFFFF)
        return fail(SG_EINVAL, "dimension exceeds 2^31 - 1");
    if (d.Ml < d.M || d.Nl < d.N || d.Kl < d.K) return fail(SG_EINVAL, "launch dims below data dims");
    if (d.Kl <= 0) return fail(SG_EINVAL, "empty K extent");
    if (packing_of(variant, d).part_bytes > 0 && ws == nullptr)
        return fail(SG_EINVAL, "split-K launch without workspace");
    switch (variant_tile(variant)) {
        case 0: return launch_tile<256, 256>(d, variant, ws, stream);
        case 1: return launch_tile<256, 128>(d, variant, ws, stream);
        case 2: return launch_tile<128, 256>(d, variant, ws, stream);
        case 3: return launch_tile<128, 128>(d, variant, ws, stream);
        case 4: return launch_tile<128, 64>(d, variant, ws, stream);
        case 5: return launch_tile<64, 128>(d, variant, ws, stream);
        case 6: return launch_tile<64, 64>(d, variant, ws, stream);
        default: return launch_tile<64, 64, true>(d, variant, ws, stream);
    }
}

// ---- device operand generator: SplitMix64 counter words -> uniform / normal -> BF16 ----------
__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void sg_fill_kernel(uint16_t* dst, int64_t n, uint64_t key,
                                                       int64_t offset, int kind, double scale) {
    const uint64_t gamma = 0x9E3779B97F4A7C15ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t idx = (uint64_t)(i + offset);
        float f;
        if (kind == 0) {
            const int64_t u = (int64_t)(sm_mix(key + (idx + 1) * gamma) >> 40);
            f = (float)((double)(2 * u + 1 - (1ll << 24)) * 0x1p-24);
        } else {
            const uint64_t w1 = sm_mix(key + (2 * idx + 1) * gamma);
            const uint64_t w2 = sm_mix(key + (2 * idx + 2) * gamma);
            const double u1 = ((double)(w1 >> 11) + 0.5) * 0x1p-53;
            const double u2 = ((double)(w2 >> 11) + 0.5) * 0x1p-53;
            const double z = sqrt(-2.0 * log(u1)) * cos(2.0 * 3.141592653589793 * u2);
            f = (float)(z * scale);
        }
        dst[i] = f32_to_bf16_rne(f);
    }
}

static uint64_t host_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

int launch_fill(uint16_t* dst, int64_t n, uint64_t seed, uint64_t stream_id, int64_t offset,
                int kind, double scale, hipStream_t stream) {
    if (n < 0 || (n > 0 && dst == nullptr) || (kind != 0 && kind != 1))
        return fail(SG_EINVAL, "sg_fill_bf16: bad argument");
    if (n == 0) return SG_OK;
    const uint64_t key = host_mix(seed + (stream_id + 1) * 0x9E3779B97F4A7C15ull);
    int64_t blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(sg_fill_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, dst, n, key,
                       offset, kind, scale);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

}  // namespace sg
