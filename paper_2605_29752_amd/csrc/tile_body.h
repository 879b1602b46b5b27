// Tile body of the BF16 NN GEMM family for gfx950: one BM x BN tile of C = A * B over a K range.
// Shared by the per-call kernel (one tile per work-group) and the persistent grouped kernel
// (many tiles of many problems per work-group).  The design notes are in gemm_tile.hip.
#pragma once

#include "sg_internal.h"

namespace sg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));


struct KArgs {
    const uint16_t* A;
    const uint16_t* B;
    void* C;
    const void* add;
    int64_t lda, ldb, ldc, ldadd;
    int64_t ws_slice;   // elements between split-K partial slices
    int M, N, K;        // data bounds
    int Kl;             // K extent of the launch
    int k_chunk;        // K elements per split (multiple of 64)
    int tiles_m, tiles_n;
    int out_bf16;
    int add_kind;
    int vec_ok;         // C / addend rows allow 4-wide vector access
    int a_bytes, b_bytes;   // readable extents of A and B from their base (buffer range checks)
};

constexpr int LDK = kBK + 8;   // padded LDS row (elements)

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __builtin_bit_cast(uint32_t, f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0;   // NaN stays NaN
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __builtin_bit_cast(float, ((uint32_t)h) << 16);
}

// Tile index of this work-group.  Work-groups are handed to the 8 XCDs round robin; the
// remap gives each XCD one contiguous run of tiles (so tiles sharing operand panels share an
// L2), and the run is rastered in groups of 8 tile rows.
__device__ __forceinline__ void tile_coords(int tiles_m, int tiles_n, int& tm, int& tn) {
    const int nwg = tiles_m * tiles_n;
    const int b = blockIdx.x;
    const int x = b & 7, q = nwg >> 3, r = nwg & 7;
    const int logical = x * q + (x < r ? x : r) + (b >> 3);
    constexpr int GM = 8;
    const int group = GM * tiles_n;
    const int g = logical / group;
    const int first_m = g * GM;
    const int gm = min(tiles_m - first_m, GM);
    const int local = logical - g * group;
    tm = first_m + local % gm;
    tn = local / gm;
}

// Operand staging of one K step in registers.  A: A_CHUNKS 16-byte chunks along K.  B: an
// 8 (K) x NB (N) block, one row of NB elements per register group.
template <int BM, int BN>
struct Stage {
    static constexpr int A_CHUNKS = BM * (kBK / 8) / 256;
    static constexpr int NB = BN / 32;
    u32x4_t a[A_CHUNKS];
    uint32_t b[8][NB / 2];
};

template <int BM, int BN>
constexpr int smem_elems() { return 2 * (BM + BN) * LDK; }

// Fast epilogue of a tile that lies wholly inside C, with 4-wide vector access to C and no
// addend (every tile of an aligned landscape shape without a K split into C): each lane stores
// its four consecutive columns of one row straight from the accumulators, 8 bytes (BF16) or
// 16 bytes (FP32) per fragment, with no LDS round trip.  Returns false (nothing stored) when
// the tile does not qualify.
template <int BM, int BN, int NW = 4>
__device__ __forceinline__ bool epilogue_direct(const KArgs& p, const int m0, const int n0, const int kz,
                                                const f32x4_t (&acc)[BM / 32][BN / (8 * NW)]) {
    if (!(m0 + BM <= p.M && n0 + BN <= p.N && p.vec_ok && p.add_kind == ADD_NONE)) return false;
    constexpr int NWN = NW / 2;
    constexpr int WM = BM / 2, WN = BN / NWN;
    constexpr int FM = WM / 16, FN = WN / 16;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave / NWN, wn = wave % NWN;
    const int lr = lane & 15, lg = lane >> 4;
    const int64_t row0 = (int64_t)(m0 + wm * WM + lr);
    const int col0 = n0 + wn * WN + 4 * lg;
    if (p.out_bf16) {
        uint16_t* cp = (uint16_t*)p.C + (int64_t)kz * p.ws_slice + row0 * p.ldc + col0;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const f32x4_t v = acc[i][j];
                u32x2_t o;
                o[0] = (uint32_t)f32_to_bf16_rne(v[0]) | ((uint32_t)f32_to_bf16_rne(v[1]) << 16);
                o[1] = (uint32_t)f32_to_bf16_rne(v[2]) | ((uint32_t)f32_to_bf16_rne(v[3]) << 16);
                *(u32x2_t*)(cp + (int64_t)(i * 16) * p.ldc + j * 16) = o;
            }
    } else {
        float* cp = (float*)p.C + (int64_t)kz * p.ws_slice + row0 * p.ldc + col0;
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
                *(f32x4_t*)(cp + (int64_t)(i * 16) * p.ldc + j * 16) = acc[i][j];
    }
    return true;
}

// Epilogue shared by both tile bodies.  Each wave stages one 16-row band of its C sub-tile at
// a time in its own LDS slice (the caller's main loop ended with a barrier, so the operand
// stages are free), then writes the band out row by row: lanes cover 4 consecutive columns
// each, so a wave stores whole row segments.  acc[i][j] holds rows 16 i + (lane % 16) and
// columns 16 j + 4 (lane / 16) .. + 3 of the wave's sub-tile.
template <int BM, int BN, int NW = 4>
__device__ __forceinline__ void epilogue(const KArgs& p, const int m0, const int n0, const int kz,
                                         uint16_t* __restrict__ smem,
                                         const f32x4_t (&acc)[BM / 32][BN / (8 * NW)]) {
    constexpr int NWN = NW / 2;                           // waves along N (2 along M)
    constexpr int WM = BM / 2, WN = BN / NWN;
    constexpr int FM = WM / 16, FN = WN / 16;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / NWN, wn = wave % NWN;
    const int lr = lane & 15, lg = lane >> 4;
    constexpr int EPAD = WN + 4;                          // f32 row of the band, padded
    float* band = (float*)smem + wave * 16 * EPAD;
    const int64_t zoff = (int64_t)kz * p.ws_slice;
    constexpr int COLS4 = WN / 4;                         // 4-column groups per band row
    constexpr int ROWS_PER_PASS = 64 / COLS4;             // band rows written per pass
#pragma unroll
    for (int i = 0; i < FM; ++i) {
#pragma unroll
        for (int j = 0; j < FN; ++j)
            *(f32x4_t*)(band + lr * EPAD + j * 16 + lg * 4) = acc[i][j];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int mb = m0 + wm * WM + i * 16;
        const int nbase = n0 + wn * WN + (lane % COLS4) * 4;
#pragma unroll 1
        for (int r = lane / COLS4; r < 16; r += ROWS_PER_PASS) {
            const int m = mb + r;
            const int n = nbase;
            if (m >= p.M || n >= p.N) continue;
            f32x4_t v = *(const f32x4_t*)(band + r * EPAD + (lane % COLS4) * 4);
            const bool full = p.vec_ok && (n + 3 < p.N);
            if (p.add_kind == ADD_F32) {
                const float* ap = (const float*)p.add + (int64_t)m * p.ldadd + n;
                if (full) {
                    v += *(const f32x4_t*)ap;
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (n + e < p.N) v[e] += ap[e];
                }
            } else if (p.add_kind == ADD_BF16) {
                const uint16_t* ap = (const uint16_t*)p.add + (int64_t)m * p.ldadd + n;
                if (full) {
                    const u32x2_t a2 = *(const u32x2_t*)ap;
                    v[0] += bf16_to_f32(a2[0] & 0xFFFFu); v[1] += bf16_to_f32(a2[0] >> 16);
                    v[2] += bf16_to_f32(a2[1] & 0xFFFFu); v[3] += bf16_to_f32(a2[1] >> 16);
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (n + e < p.N) v[e] += bf16_to_f32(ap[e]);
                }
            }
            if (p.out_bf16) {
                uint16_t* cp = (uint16_t*)p.C + zoff + (int64_t)m * p.ldc + n;
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
                float* cp = (float*)p.C + zoff + (int64_t)m * p.ldc + n;
                if (full) {
                    *(f32x4_t*)cp = v;
                } else {
                    for (int e = 0; e < 4; ++e)
                        if (n + e < p.N) cp[e] = v[e];
                }
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// One BM x BN tile of C at (m0, n0) over the K range of split kz for operands that do not meet
// the aligned path's conditions (odd leading dimensions, K or N not a multiple of 8, unaligned
// bases): element-wise predicated loads into registers, then LDS.  Called by all 256 threads
// of a work-group; smem holds smem_elems<BM, BN>() elements.
template <int BM, int BN>
__device__ __forceinline__ void tile_body(const KArgs& p, const int m0, const int n0, const int kz,
                                          uint16_t* __restrict__ smem) {
    constexpr int WM = BM / 2, WN = BN / 2;        // per-wave tile
    constexpr int FM = WM / 16, FN = WN / 16;      // MFMA fragments per wave
    constexpr int A_CHUNKS = Stage<BM, BN>::A_CHUNKS;
    constexpr int NB = Stage<BM, BN>::NB;          // B block width (columns) per thread
    constexpr int STAGE = (BM + BN) * LDK;         // elements per LDS stage
    static_assert(A_CHUNKS >= 1 && NB >= 2 && NB <= 8, "tile shape");

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lg = lane >> 4;

    const int kb = kz * p.k_chunk;
    const int ke = min(p.Kl, kb + p.k_chunk);
    const int nk = (ke - kb + kBK - 1) / kBK;

    // Per-thread load geometry.  c: the thread's 8-wide K chunk (same for A and B).
    const int c = tid & 7;
    const int nb = tid >> 3;                       // B column block
    const int gn = n0 + nb * NB;

    auto load = [&](Stage<BM, BN>& s, int kt) {
        const int k0 = kb + kt * kBK;
#pragma unroll
        for (int i = 0; i < A_CHUNKS; ++i) {
            const int gm = m0 + ((tid + i * 256) >> 3), gk = k0 + c * 8;
            const uint16_t* rowp = p.A + (int64_t)gm * p.lda;
            uint32_t w[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k_lo = gk + 2 * e, k_hi = k_lo + 1;
                uint32_t lo = (gm < p.M && k_lo < p.K) ? rowp[k_lo] : 0u;
                uint32_t hi = (gm < p.M && k_hi < p.K) ? rowp[k_hi] : 0u;
                w[e] = lo | (hi << 16);
            }
            s.a[i] = u32x4_t{w[0], w[1], w[2], w[3]};
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int gk = k0 + c * 8 + r;
            const uint16_t* src = p.B + (int64_t)gk * p.ldb + gn;
#pragma unroll
            for (int w = 0; w < NB / 2; ++w) {
                const int n_lo = gn + 2 * w, n_hi = n_lo + 1;
                uint32_t lo = (gk < p.K && n_lo < p.N) ? src[2 * w] : 0u;
                uint32_t hi = (gk < p.K && n_hi < p.N) ? src[2 * w + 1] : 0u;
                s.b[r][w] = lo | (hi << 16);
            }
        }
    };

    // registers -> LDS: A as is; B transposed in registers to K-contiguous rows.
    auto store = [&](const Stage<BM, BN>& s, int buf) {
        uint16_t* As = smem + buf * STAGE;
        uint16_t* Bs = As + BM * LDK;
#pragma unroll
        for (int i = 0; i < A_CHUNKS; ++i) {
            const int row = (tid + i * 256) >> 3;
            *(u32x4_t*)(As + row * LDK + c * 8) = s.a[i];
        }
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const int w = e >> 1, sh = (e & 1) * 16;
            u32x4_t o;
#pragma unroll
            for (int pr = 0; pr < 4; ++pr) {
                const uint32_t lo = (s.b[2 * pr][w] >> sh) & 0xFFFFu;
                const uint32_t hi = (s.b[2 * pr + 1][w] >> sh) & 0xFFFFu;
                o[pr] = lo | (hi << 16);
            }
            *(u32x4_t*)(Bs + (nb * NB + e) * LDK + c * 8) = o;
        }
    };

    f32x4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    auto compute = [&](int buf) {
        const uint16_t* As = smem + buf * STAGE;
        const uint16_t* Bs = As + BM * LDK;
#pragma unroll
        for (int ks = 0; ks < kBK / 32; ++ks) {
            // all fragments of this 32-deep slice are read first, so their LDS latency overlaps
            bf16x8_t af[FM], bfr[FN];
#pragma unroll
            for (int i = 0; i < FM; ++i)
                af[i] = *(const bf16x8_t*)(As + (wm * WM + i * 16 + lr) * LDK + ks * 32 + lg * 8);
#pragma unroll
            for (int j = 0; j < FN; ++j)
                bfr[j] = *(const bf16x8_t*)(Bs + (wn * WN + j * 16 + lr) * LDK + ks * 32 + lg * 8);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
            // the largest tile would otherwise keep both slices' fragments live and spill
            // issue order: every fragment read of the slice, then its MFMAs
            __builtin_amdgcn_sched_group_barrier(0x100, FM + FN, 0);
            __builtin_amdgcn_sched_group_barrier(0x008, FM * FN, 0);
            if constexpr (FM * FN >= 64) __builtin_amdgcn_sched_barrier(0);
        }
    };

    // Pipeline: the loads of step kt+1 are in flight while step kt is multiplied, then they are
    // written to the other LDS stage.
    Stage<BM, BN> s0;
    if (nk > 0) {
        load(s0, 0);
        store(s0, 0);
    }
    __syncthreads();
    for (int kt = 0; kt < nk; ++kt) {
        if (kt + 1 < nk) load(s0, kt + 1);
        compute(kt & 1);
        if (kt + 1 < nk) store(s0, (kt + 1) & 1);
        __syncthreads();
    }

    static_assert(4 * 16 * (WN + 4) * 4 <= 2 * STAGE * 2, "epilogue staging must fit the LDS");
    epilogue<BM, BN>(p, m0, n0, kz, smem, acc);
}

}  // namespace sg
