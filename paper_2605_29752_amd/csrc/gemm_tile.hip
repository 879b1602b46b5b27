// BF16 NN GEMM tile family for gfx950 (CDNA4).
//
// C = A * B, A M x K row-major (K contiguous), B K x N row-major (N contiguous); the problem
// statement of the paper's Sec. 2.2 / Sec. 7.1.  Each work-group (256 threads = 4 wave64 in a
// 2 x 2 arrangement) computes one BM x BN tile of C over a 64-deep K step:
//
//  * global -> registers: A in 16-byte chunks along K; B in 8-row x (BN/32)-column blocks so
//    that every thread can transpose its block in registers (B must reach the matrix cores
//    K-contiguous, but it is stored N-contiguous);
//  * registers -> LDS: both operands stored K-contiguous, rows padded to 72 elements
//    (144 bytes) so 16 consecutive rows of a fragment read hit 16 disjoint 4-bank groups;
//  * LDS -> matrix cores: v_mfma_f32_16x16x32_bf16, FP32 accumulators in registers;
//  * two LDS stages: the next K step's global loads are in flight while the current one is
//    multiplied, one barrier per K step.
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
#include "sg_internal.h"

namespace sg {

typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));

const TileShape kTiles[kNumTiles] = {{256, 256}, {256, 128}, {128, 256}, {128, 128},
                                     {128, 64},  {64, 128},  {64, 64}};

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

template <int BM, int BN, bool ALIGNED>
__global__ __launch_bounds__(256) void sg_gemm_tile(KArgs p) {
    constexpr int WM = BM / 2, WN = BN / 2;        // per-wave tile
    constexpr int FM = WM / 16, FN = WN / 16;      // MFMA fragments per wave
    constexpr int A_CHUNKS = BM * (kBK / 8) / 256; // 16-byte A chunks per thread
    constexpr int NB = BN / 32;                    // B block width (columns) per thread
    constexpr int STAGE = (BM + BN) * LDK;         // elements per LDS stage
    static_assert(A_CHUNKS >= 1 && NB >= 2 && NB <= 8, "tile shape");

    __shared__ __attribute__((aligned(16))) uint16_t smem[2 * STAGE];

    int tm, tn;
    tile_coords(p.tiles_m, p.tiles_n, tm, tn);
    const int m0 = tm * BM, n0 = tn * BN;
    if (m0 >= p.M || n0 >= p.N) return;            // padding-only tile

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int lr = lane & 15, lg = lane >> 4;

    const int kb = blockIdx.z * p.k_chunk;
    const int ke = min(p.Kl, kb + p.k_chunk);
    const int nk = (ke - kb + kBK - 1) / kBK;

    // ---- global -> register staging ------------------------------------------------------
    u32x4_t ra[A_CHUNKS];
    uint32_t rb[8][NB / 2];

    auto load_tiles = [&](int kt) {
        const int k0 = kb + kt * kBK;
#pragma unroll
        for (int i = 0; i < A_CHUNKS; ++i) {
            const int q = tid + i * 256;
            const int row = q >> 3, c = q & 7;
            const int gm = m0 + row, gk = k0 + c * 8;
            if constexpr (ALIGNED) {
                u32x4_t v = {0u, 0u, 0u, 0u};
                if (gm < p.M && gk < p.K) v = *(const u32x4_t*)(p.A + (int64_t)gm * p.lda + gk);
                ra[i] = v;
            } else {
                uint32_t w[4];
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int k_lo = gk + 2 * e, k_hi = k_lo + 1;
                    const uint16_t* rowp = p.A + (int64_t)gm * p.lda;
                    uint32_t lo = (gm < p.M && k_lo < p.K) ? rowp[k_lo] : 0u;
                    uint32_t hi = (gm < p.M && k_hi < p.K) ? rowp[k_hi] : 0u;
                    w[e] = lo | (hi << 16);
                }
                ra[i] = u32x4_t{w[0], w[1], w[2], w[3]};
            }
        }
        {
            const int c = tid & 7, nb = tid >> 3;
            const int gn = n0 + nb * NB;
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                const int gk = k0 + c * 8 + r;
                const uint16_t* src = p.B + (int64_t)gk * p.ldb + gn;
                if constexpr (ALIGNED) {
                    const bool ok = gk < p.K && gn < p.N;
                    if constexpr (NB == 8) {
                        u32x4_t v = {0u, 0u, 0u, 0u};
                        if (ok) v = *(const u32x4_t*)src;
                        rb[r][0] = v[0]; rb[r][1] = v[1]; rb[r][2] = v[2]; rb[r][3] = v[3];
                    } else if constexpr (NB == 4) {
                        u32x2_t v = {0u, 0u};
                        if (ok) v = *(const u32x2_t*)src;
                        rb[r][0] = v[0]; rb[r][1] = v[1];
                    } else {
                        rb[r][0] = ok ? *(const uint32_t*)src : 0u;
                    }
                } else {
#pragma unroll
                    for (int w = 0; w < NB / 2; ++w) {
                        const int n_lo = gn + 2 * w, n_hi = n_lo + 1;
                        uint32_t lo = (gk < p.K && n_lo < p.N) ? src[2 * w] : 0u;
                        uint32_t hi = (gk < p.K && n_hi < p.N) ? src[2 * w + 1] : 0u;
                        rb[r][w] = lo | (hi << 16);
                    }
                }
            }
        }
    };

    // ---- register -> LDS (A as is, B transposed to K-contiguous rows) -------------------------
    auto store_tiles = [&](int buf) {
        uint16_t* As = smem + buf * STAGE;
        uint16_t* Bs = As + BM * LDK;
#pragma unroll
        for (int i = 0; i < A_CHUNKS; ++i) {
            const int q = tid + i * 256;
            const int row = q >> 3, c = q & 7;
            *(u32x4_t*)(As + row * LDK + c * 8) = ra[i];
        }
        const int c = tid & 7, nb = tid >> 3;
#pragma unroll
        for (int e = 0; e < NB; ++e) {
            const int w = e >> 1, sh = (e & 1) * 16;
            u32x4_t o;
#pragma unroll
            for (int pr = 0; pr < 4; ++pr) {
                const uint32_t lo = (rb[2 * pr][w] >> sh) & 0xFFFFu;
                const uint32_t hi = (rb[2 * pr + 1][w] >> sh) & 0xFFFFu;
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

    if (nk > 0) {
        load_tiles(0);
        store_tiles(0);
    }
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
        const int buf = kt & 1;
        if (kt + 1 < nk) load_tiles(kt + 1);
        const uint16_t* As = smem + buf * STAGE;
        const uint16_t* Bs = As + BM * LDK;
#pragma unroll
        for (int ks = 0; ks < kBK / 32; ++ks) {
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
        }
        if (kt + 1 < nk) store_tiles(buf ^ 1);
        __syncthreads();
    }

    // ---- epilogue: lane holds C[m][n .. n+3] of each fragment ---------------------------------
    const int64_t zoff = (int64_t)blockIdx.z * p.ws_slice;
#pragma unroll
    for (int i = 0; i < FM; ++i) {
        const int m = m0 + wm * WM + i * 16 + lr;
        if (m >= p.M) continue;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int n = n0 + wn * WN + j * 16 + lg * 4;
            if (n >= p.N) continue;
            float v[4] = {acc[i][j][0], acc[i][j][1], acc[i][j][2], acc[i][j][3]};
            const bool full = p.vec_ok && (n + 3 < p.N);
            if (p.add_kind == ADD_F32) {
                const float* ap = (const float*)p.add + (int64_t)m * p.ldadd + n;
                if (full) {
                    f32x4_t a4 = *(const f32x4_t*)ap;
                    v[0] += a4[0]; v[1] += a4[1]; v[2] += a4[2]; v[3] += a4[3];
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (n + e < p.N) v[e] += ap[e];
                }
            } else if (p.add_kind == ADD_BF16) {
                const uint16_t* ap = (const uint16_t*)p.add + (int64_t)m * p.ldadd + n;
                if (full) {
                    u32x2_t a2 = *(const u32x2_t*)ap;
                    v[0] += bf16_to_f32(a2[0] & 0xFFFFu); v[1] += bf16_to_f32(a2[0] >> 16);
                    v[2] += bf16_to_f32(a2[1] & 0xFFFFu); v[3] += bf16_to_f32(a2[1] >> 16);
                } else {
#pragma unroll
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
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (n + e < p.N) cp[e] = f32_to_bf16_rne(v[e]);
                }
            } else {
                float* cp = (float*)p.C + zoff + (int64_t)m * p.ldc + n;
                if (full) {
                    *(f32x4_t*)cp = f32x4_t{v[0], v[1], v[2], v[3]};
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        if (n + e < p.N) cp[e] = v[e];
                }
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

int lds_bytes_of_tile(int tile) {
    return 2 * (kTiles[tile].bm + kTiles[tile].bn) * LDK * (int)sizeof(uint16_t);
}

void split_geometry(int variant, int64_t Kl, int* splits, int64_t* k_chunk) {
    const int S = variant_splits(variant);
    int64_t per = (Kl + S - 1) / S;
    per = (per + kBK - 1) / kBK * kBK;
    if (per < kBK) per = kBK;
    *k_chunk = per;
    int64_t s = (Kl + per - 1) / per;
    *splits = (int)(s < 1 ? 1 : s);
}

size_t launch_workspace_bytes(int variant, const LaunchDesc& d) {
    int S;
    int64_t kc;
    split_geometry(variant, d.Kl, &S, &kc);
    if (S <= 1) return 0;
    return (size_t)S * (size_t)d.M * (size_t)d.N * sizeof(float);
}

template <int BM, int BN>
static int launch_tile(const LaunchDesc& d, int variant, void* ws, hipStream_t stream) {
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
    const bool aligned = (d.lda % 8 == 0) && (d.ldb % 8 == 0) && (d.K % 8 == 0) && (d.N % 8 == 0) &&
                         ((uintptr_t)d.A % 16 == 0) && ((uintptr_t)d.B % 16 == 0);
    if (S > 1) {
        a.C = ws; a.ldc = d.N; a.ws_slice = d.M * d.N;
        a.out_bf16 = 0; a.add = nullptr; a.ldadd = 0; a.add_kind = ADD_NONE;
        a.vec_ok = (d.N % 4 == 0) && ((uintptr_t)ws % 16 == 0);
    } else {
        a.C = d.C; a.ldc = d.ldc; a.ws_slice = 0;
        a.out_bf16 = d.out_bf16; a.add = d.add; a.ldadd = d.ldadd; a.add_kind = d.add_kind;
        const size_t esz = d.out_bf16 ? 2 : 4;
        bool vec = (d.ldc % 4 == 0) && ((uintptr_t)d.C % (4 * esz) == 0);
        if (d.add_kind == ADD_F32) vec = vec && (d.ldadd % 4 == 0) && ((uintptr_t)d.add % 16 == 0);
        if (d.add_kind == ADD_BF16) vec = vec && (d.ldadd % 4 == 0) && ((uintptr_t)d.add % 8 == 0);
        a.vec_ok = vec ? 1 : 0;
    }
    const int64_t nwg = (int64_t)a.tiles_m * a.tiles_n;
    if (nwg <= 0) return SG_OK;
    if (nwg > 0x7FFFFFFF) return fail(SG_EINVAL, "launch grid too large");
    dim3 grid((unsigned)nwg, 1, (unsigned)S), block(256);
    if (aligned)
        hipLaunchKernelGGL((sg_gemm_tile<BM, BN, true>), grid, block, 0, stream, a);
    else
        hipLaunchKernelGGL((sg_gemm_tile<BM, BN, false>), grid, block, 0, stream, a);
    SG_HIP(hipGetLastError());
    if (S > 1) {
        const int64_t total = d.M * d.N;
        int64_t blocks = (total + 255) / 256;
        if (blocks > 65536) blocks = 65536;
        hipLaunchKernelGGL(sg_splitk_reduce, dim3((unsigned)blocks), dim3(256), 0, stream,
                           (const float*)ws, (int64_t)(d.M * d.N), S, (int)d.M, (int)d.N, d.C,
                           d.ldc, d.out_bf16, d.add, d.ldadd, d.add_kind);
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
    if (launch_workspace_bytes(variant, d) > 0 && ws == nullptr)
        return fail(SG_EINVAL, "split-K launch without workspace");
    switch (variant_tile(variant)) {
        case 0: return launch_tile<256, 256>(d, variant, ws, stream);
        case 1: return launch_tile<256, 128>(d, variant, ws, stream);
        case 2: return launch_tile<128, 256>(d, variant, ws, stream);
        case 3: return launch_tile<128, 128>(d, variant, ws, stream);
        case 4: return launch_tile<128, 64>(d, variant, ws, stream);
        case 5: return launch_tile<64, 128>(d, variant, ws, stream);
        default: return launch_tile<64, 64>(d, variant, ws, stream);
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
