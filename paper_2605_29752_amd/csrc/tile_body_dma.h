// Tile body with direct-to-LDS operand loads (aligned fast path).
//
// The same tile as tile_body.h (2 x 2 or 2 x 4 waves of 64 lanes, MFMA 16x16x32 BF16, B^T as
// the first MFMA operand, LDS-staged epilogue), but the operands travel HBM -> LDS with
// `buffer_load_dwordx4 ... lds`: no staging registers, so the loads of later K stages are in
// flight while a stage is multiplied, in a ring of LDS stages.  Stage depth BKD (32 or 64 of K,
// one or two MFMA K steps) and ring depth are chosen per tile (DmaTile).
//
// LDS layout per stage (no padding: one DMA instruction writes 1 KiB contiguously):
//  * A: BM rows x BKD BF16 (2 BKD bytes), 16-byte chunk c of row r stored at slot c ^ swz(r):
//    swz(r) = (r >> 1) & 3 for 64-byte rows, r & 7 for 128-byte rows.  A 16-byte-per-lane LDS
//    read is served eight lanes (128 bytes, the 32 four-byte banks) at a time; the eight rows
//    those lanes read from land in distinct banks (measured: no bank-conflict cycles, where
//    (r >> 2) & 3 on 64-byte rows had one conflict cycle per access cycle);
//  * B: BKD rows (K) x BN BF16 (N contiguous, as in HBM), the 16-byte chunk c of row k stored
//    at slot c ^ swz(k), swz(k) = (2 (k & 3)) ^ (8 ((k >> 3) & 3)) (within the row's chunks).
//    A B fragment (8 consecutive K at one N per lane) comes from two ds_read_b64_tr_b16: within
//    each 16-lane group, result[i][e] is element i % 4 of the 4 elements at the address given by
//    lane 4 e + i / 4, so lane j of group g points at B[8 g + j / 4 (+ 4)][n0 + 4 (j % 4)] and
//    receives column n0 + j at K rows 8 g .. 8 g + 7.  The swizzle puts the four K rows one read
//    touches, and the four groups, in distinct 16-byte slots.
// Out-of-range elements are fetched with an offset past the end of the buffer and land as zeros.
#pragma once

#include <type_traits>

#include "tile_body.h"

namespace sg {

// NW: waves per work-group, 4 (a 2 x 2 grid) or 8 (2 x 4: two waves on every SIMD).
template <int BM, int BN, bool DEEP = false, int NW = 4>
struct DmaTile {
    // Stage depth and ring depth per tile, from measurements (4096^3, TFLOP/s):
    //  * tiles up to 128 x 128: 64-deep stages (two MFMA K steps per barrier) in a two-stage ring;
    //    the per-step cost of waits, barrier and load issue is paid once per 64 of K
    //    (128 x 128: 912 -> 1,085; 64 x 64: 578 -> 738; 2048^3 gains 13-26 %);
    //  * 256 x 128 / 128 x 256: 32-deep stages, two-stage ring: 48 KiB lets two work-groups share
    //    a CU, which hides more latency than deeper prefetch in one (1,070-1,140 against 730
    //    with four stages; 64-deep stages would take 96 KiB and one work-group: 818);
    //  * 256 x 256: 32-deep stages, four-stage ring (one work-group per CU either way);
    //  * DEEP (the 64 x 64 variant for shapes with few tiles): 128-deep stages, two-stage ring
    //    (64 KiB: two work-groups per CU instead of five, but the per-stage waits and barrier
    //    are paid once per four MFMA K steps; against the 64-deep 64 x 64: 1024^3 213 -> 264,
    //    2048^3 498 -> 551, 4096^3 686 -> 649).
    static_assert(!DEEP || (BM == 64 && BN == 64), "deep stages are for the 64 x 64 tile");
    static constexpr bool SMALL = BM * BN <= 128 * 128;
    // Cross-stage fragment prefetch (the fragments of stage kt + 1 read under the MFMAs of
    // stage kt) for 256 x 256 only.  Measured on the smaller tiles with four 32-deep stages, it
    // lost badly (128 x 128 at 4096^3: 1,068 -> 672): their 256 MFMA cycles per stage are too
    // few to cover a barrier per 32 of K, and the two-work-group 256 x 128 / 128 x 256 cannot
    // hold a second fragment set within the 128 registers that two work-groups per CU allow.
    static constexpr bool XPF = !DEEP && BM == 256 && BN == 256;
    static constexpr int BKD = DEEP ? 128 : SMALL ? 64 : 32;   // K per stage
    static constexpr int SUB = BKD / 32;                 // MFMA K steps per stage
    static constexpr int A_CH = BKD / 8;                 // 16-byte chunks per A row
    static constexpr int A_ROWS_PER_INSTR = 512 / BKD;   // 1 KiB = 512 BF16
    static constexpr int STAGES = XPF ? 4 : 2;
    static constexpr int A_BYTES = BM * BKD * 2;
    static constexpr int B_BYTES = BKD * BN * 2;
    static constexpr int STAGE_BYTES = A_BYTES + B_BYTES;
    static constexpr int A_INSTR = A_BYTES / 1024 / NW;  // DMA instructions per wave per stage
    static constexpr int B_INSTR = B_BYTES / 1024 / NW;
    static constexpr int B_ROWS_PER_INSTR = 512 / BN;    // 1 KiB = 512 BF16
    static constexpr int B_CHUNKS = BN / 8;              // 16-byte chunks per B row
    static constexpr int LDS_BYTES = STAGES * STAGE_BYTES;
    static_assert(NW == 4 || NW == 8, "2 x 2 or 2 x 4 waves");
    static_assert(A_INSTR >= 1 && B_INSTR >= 1 && B_CHUNKS >= 8, "tile shape");
    static_assert(STAGES >= 2 && STAGES <= 4, "the main loop's waits cover at most two later steps");
    // A split-K range is a multiple of kBK long and a stage must not run past its end: the
    // loads check depth against K, not against the split's end.
    static_assert((DEEP ? kDeepBK : kBK) % BKD == 0, "a K stage would straddle two split-K ranges");
};

// Waves per work-group of the direct-to-LDS kernels that run one tile shape per launch: eight
// (2 x 4) for the 256-wide tiles and 128 x 128, four (2 x 2) for the 64-wide ones.  One wave on a SIMD draws LDS
// fragment reads at about 32 bytes per clock (a probe of conflict-free ds_read_b128 with eight
// reads in flight: 131 bytes per clock per CU with four waves, 262 with eight), so a wave that
// both reads its fragments and issues its MFMAs stalls on the reads; with two waves per SIMD one
// multiplies while the other reads.  Measured against four waves (TFLOP/s): 256 x 256 at 4096^3
// 976 -> 1,063 and at 4096 x 4096 x 1024 680 -> 785; 128 x 256 1,148 -> 1,205 at 4096^3 and
// +15-29 % on mid-size shapes (2048^3 307 -> 384); 256 x 128 1,102 -> 1,151.  The 128 x 128 tile
// lost 4-10 % on the large shapes with eight waves until its fragment reads were pipelined
// under its MFMAs; since then eight waves gain on average (over a seeded sample of 1,024
// landscape cells: no split 459.9 -> 468.8 TFLOP/s, two splits 372.6 -> 377.8; 4096^3 1,083 ->
// 1,095, 1024^3 156 -> 176; 4096 x 4096 x 128 loses, 244 -> 220).  The 64-wide tiles lose with
// eight: they stay at four.
template <int BM, int BN>
constexpr int call_waves() { return (BM * BN >= 128 * 128) ? 8 : 4; }

template <int BM, int BN, bool DEEP = false, int NW = 4>
constexpr int dma_smem_bytes() {
    constexpr int ring = DmaTile<BM, BN, DEEP, NW>::LDS_BYTES;
    constexpr int epi = NW * 16 * (BN / (NW / 2) + 4) * 4;   // one staged 16-row band per wave
    return ring > epi ? ring : epi;
}

// s_waitcnt with only the vector-memory counter constrained (gfx9 encoding: vmcnt in bits 3:0
// and 15:14, expcnt 6:4 and lgkmcnt 11:8 left at their maxima).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
    static_assert(N >= 0 && N < 64, "vmcnt");
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_waitcnt((N & 0xF) | ((N >> 4) << 14) | (0x7 << 4) | (0xF << 8));
    asm volatile("" ::: "memory");
}

typedef __attribute__((address_space(3))) void lds_void;
typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) bf16x4_t lds_bf16x4;
typedef int i32x4_t __attribute__((ext_vector_type(4)));

// Raw buffer resource over [base, base + bytes): stride 0, so the range check is offset < bytes
// and an out-of-range load returns zeros.
__device__ __forceinline__ i32x4_t dma_rsrc(const void* base, uint32_t bytes) {
    const uint64_t a = (uint64_t)base;
    i32x4_t r;
    r.x = __builtin_amdgcn_readfirstlane((int)(uint32_t)a);
    r.y = __builtin_amdgcn_readfirstlane((int)(uint32_t)(a >> 32) & 0xFFFF);
    r.z = __builtin_amdgcn_readfirstlane((int)bytes);
    r.w = 0x00020000;
    return r;
}

// One 16-byte-per-lane load from a buffer straight into LDS: lane i writes 16 bytes at LDS byte
// address lds + 16 i.  Written as inline asm on purpose: the compiler's wait-count pass cannot
// tell which ring stage a direct-to-LDS load writes, and for the builtin it waits for every
// outstanding load before each later LDS read, which drains the ring on every K step.  Here
// the loop's own counted waits and barrier order the LDS reads after the data lands.  The asm
// restores M0, which the compiler treats as its own; the load has no register result, so
// nothing is left in flight towards a register the compiler could reuse.
__device__ __forceinline__ void dma16(const i32x4_t rsrc, uint32_t voffset, uint32_t lds) {
    int saved;
    asm volatile(
        "s_mov_b32 %0, m0\n\t"
        "s_mov_b32 m0, %3\n\t"
        "s_nop 0\n\t"
        "buffer_load_dwordx4 %1, %2, 0 offen lds\n\t"
        "s_mov_b32 m0, %0"
        : "=&s"(saved)
        : "v"(voffset), "s"(rsrc), "s"(lds)
        : "memory");
}

// One tile over the K range [kb, ke) (kb a multiple of the stage depth); kz only selects the
// split-K output slice (kz * ws_slice).
// MEM = true gives the memory-only twin of the tile (the paper's memory surface, Sec. 4): the
// same operand loads into the same ring, the same waits and barriers, and the same stores of C,
// with the fragment reads and the matrix-core products left out (C is written as zeros, plus
// the addend if one is fused).
template <int BM, int BN, bool MEM = false, bool DEEP = false, int NW = 4, bool XPF_OK = true>
__device__ __forceinline__ void tile_body_dma_range(const KArgs& p, const int m0, const int n0, const int kz,
                                                    const int kb, const int ke, uint16_t* __restrict__ smem) {
    using T = DmaTile<BM, BN, DEEP, NW>;
    constexpr int NWN = NW / 2;                          // waves along N (2 along M)
    constexpr int WM = BM / 2, WN = BN / NWN;
    constexpr int FM = WM / 16, FN = WN / 16;
    constexpr int PER_STAGE = T::A_INSTR + T::B_INSTR;  // vmcnt units per stage per lane

    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave / NWN, wn = wave % NWN;
    const int lr = lane & 15, lg = lane >> 4;

    const int nk = (ke - kb + T::BKD - 1) / T::BKD;

    constexpr uint32_t kOut = 0x80000000u;
    const i32x4_t rA = dma_rsrc(p.A, p.a_bytes);
    const i32x4_t rB = dma_rsrc(p.B, p.b_bytes);
    lds_void* lds = (lds_void*)smem;
    const uint32_t lds_base = (uint32_t)(uintptr_t)lds;

    // Per-lane DMA geometry (fixed over the loop).
    // A instruction i of this wave covers tile rows 16 q .. 16 q + 15, q = wave * A_INSTR + i;
    // lane -> row 16 q + lane / 4, slot lane % 4, which holds chunk slot ^ a_swz(row).
    const int a_row0 = lane / T::A_CH;
    const int a_slot = lane % T::A_CH;
    // B instruction i covers K rows q * R .. q * R + R - 1, q = wave * B_INSTR + i.
    const int b_row0 = lane / T::B_CHUNKS;
    const int b_slot = lane % T::B_CHUNKS;
    auto a_swz = [](int row) { return T::BKD == 32 ? (row >> 1) & 3 : row & 7; };
    auto b_swz = [](int k) { return ((2 * (k & 3)) ^ (8 * ((k >> 3) & 3))) & (T::B_CHUNKS - 1); };

    typedef __attribute__((address_space(3))) char lds_char;
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);   // DMA destinations are per wave

    // Per-lane byte offsets of step 0, or kOut where the lane's row (A) or column chunk (B) lies
    // outside the data.  A later step adds a uniform stride; kOut plus any in-range stride stays
    // at or above 2^31, past every readable extent, so such lanes keep loading zeros.
    uint32_t a_off[T::A_INSTR], b_off[T::B_INSTR];
#pragma unroll
    for (int i = 0; i < T::A_INSTR; ++i) {
        const int row = (wave_u * T::A_INSTR + i) * T::A_ROWS_PER_INSTR + a_row0;
        const int chunk = a_slot ^ a_swz(row);
        a_off[i] = (m0 + row < p.M) ? (uint32_t)(((int64_t)(m0 + row) * p.lda + kb + chunk * 8) * 2) : kOut;
    }
#pragma unroll
    for (int i = 0; i < T::B_INSTR; ++i) {
        const int row = (wave_u * T::B_INSTR + i) * T::B_ROWS_PER_INSTR + b_row0;
        const int chunk = b_slot ^ b_swz(row);
        b_off[i] = (n0 + chunk * 8 < p.N) ? (uint32_t)(((int64_t)(kb + row) * p.ldb + n0 + chunk * 8) * 2) : kOut;
    }
    const uint32_t a_step = T::BKD * 2;                          // bytes per K step
    const uint32_t b_step = (uint32_t)(T::BKD * p.ldb * 2);

    // Load instruction d (A instructions first, then B) of step kt into ring slot `slot`.
    auto issue_one = [&](int kt, int slot, int d) {
        const int k0 = kb + kt * T::BKD;
        const int stage = slot * T::STAGE_BYTES;           // LDS byte offset of the stage
        // Whole step inside K (every step but a ragged last one): no per-lane depth check.
        const bool interior = k0 + T::BKD <= p.K;
        if (d < T::A_INSTR) {
            const int q = wave_u * T::A_INSTR + d;
            uint32_t o = a_off[d] + (uint32_t)kt * a_step;
            if (!interior) {
                const int chunk = a_slot ^ a_swz(q * T::A_ROWS_PER_INSTR + a_row0);
                if (k0 + chunk * 8 >= p.K) o = kOut;
            }
            asm volatile("" : "+v"(o));
            dma16(rA, o, lds_base + stage + q * 1024);
        } else {
            const int i = d - T::A_INSTR;
            const int q = wave_u * T::B_INSTR + i;
            uint32_t o = b_off[i] + (uint32_t)kt * b_step;
            if (!interior && k0 + q * T::B_ROWS_PER_INSTR + b_row0 >= p.K) o = kOut;
            asm volatile("" : "+v"(o));
            dma16(rB, o, lds_base + stage + T::A_BYTES + q * 1024);
        }
    };
    auto issue = [&](int kt, int slot) {
#pragma unroll
        for (int d = 0; d < PER_STAGE; ++d) issue_one(kt, slot, d);
    };

    f32x4_t acc[FM][FN];
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = f32x4_t{0.f, 0.f, 0.f, 0.f};

    // One fragment of MFMA K step h in ring slot `slot`: q < FM is A fragment q (one 16-byte
    // read), q >= FM is B fragment q - FM (two transposing 8-byte reads).
    auto read_frag = [&](int slot, int h, int q, bf16x8_t* af, bf16x8_t* bfr) {
        const char* stage = (const char*)smem + slot * T::STAGE_BYTES;
        if (q < FM) {
            const int row = wm * WM + q * 16 + lr;
            af[q] = *(const bf16x8_t*)(stage + row * (T::BKD * 2) + (((4 * h + lg) ^ a_swz(row)) << 4));
        } else {
            const int j = q - FM;
            const int tk = 32 * h + lg * 8 + (lr >> 2);
            const int n = wn * WN + j * 16 + 4 * (lr & 3);
            bf16x4_t hv[2];
#pragma unroll
            for (int r = 0; r < 2; ++r) {
                const int k = tk + 4 * r;
                const int off = T::A_BYTES + k * BN * 2 + (((n >> 3) ^ b_swz(k)) << 4) + (n & 7) * 2;
                hv[r] = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
                    (lds_bf16x4*)((lds_char*)lds + slot * T::STAGE_BYTES + off));
            }
            bfr[j] = bf16x8_t{hv[0][0], hv[0][1], hv[0][2], hv[0][3], hv[1][0], hv[1][1], hv[1][2], hv[1][3]};
        }
    };

    constexpr bool SPREAD = (BM == 256 && BN == 256);
    // Multiply step `slot`; with SPREAD, the loads of step kt_next into slot_next are issued
    // between the MFMA rows.  The CU's address unit takes a 1 KiB load instruction every 16
    // cycles or so, so the loads of a whole stage from four waves take as long as a good part
    // of the MFMA work.  For 256 x 256 (one work-group per CU, 128 MFMA cycles per row) they
    // are spread over the MFMA rows, where they overlap with them (4096^3: 986 against 882
    // TFLOP/s); the other tiles issue them in one burst before the MFMAs, which measures
    // faster for them (the two-stage 256 x 128 ring needs its loads out as early as possible,
    // and the smaller tiles' rows are too short to cover a load's issue).
    auto compute = [&](int slot, bool issue_next, int kt_next, int slot_next) {
      if constexpr (MEM) {
        // the loads the MFMA rows would carry go out in one burst
        if constexpr (SPREAD)
            if (issue_next)
#pragma unroll
                for (int d = 0; d < PER_STAGE; ++d) issue_one(kt_next, slot_next, d);
      } else {
        const char* stage = (const char*)smem + slot * T::STAGE_BYTES;
        // Fragment reads of MFMA K step h of this stage: FM A fragments (one 16-byte read each)
        // and FN B fragments (two transposing 8-byte reads each).
        auto read_frags = [&](int h, bf16x8_t* af, bf16x8_t* bfr) {
#pragma unroll
            for (int i = 0; i < FM; ++i) {
                const int row = wm * WM + i * 16 + lr;
                af[i] = *(const bf16x8_t*)(stage + row * (T::BKD * 2) + (((4 * h + lg) ^ a_swz(row)) << 4));
            }
            const int tk = 32 * h + lg * 8 + (lr >> 2);  // K row this lane points at (+4: second read)
#pragma unroll
            for (int j = 0; j < FN; ++j) {
                const int n = wn * WN + j * 16 + 4 * (lr & 3);  // first of 4 columns this lane points at
                bf16x4_t hv[2];
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int k = tk + 4 * r;
                    const int off = T::A_BYTES + k * BN * 2 + (((n >> 3) ^ b_swz(k)) << 4) + (n & 7) * 2;
                    hv[r] = __builtin_amdgcn_ds_read_tr16_b64_v4bf16(
                        (lds_bf16x4*)((lds_char*)lds + slot * T::STAGE_BYTES + off));
                }
                bfr[j] = bf16x8_t{hv[0][0], hv[0][1], hv[0][2], hv[0][3], hv[1][0], hv[1][1], hv[1][2], hv[1][3]};
            }
        };
        auto mfma_step = [&](const bf16x8_t* af, const bf16x8_t* bfr, int kt_next, int slot_next, int h, bool issue_next) {
#pragma unroll
            for (int i = 0; i < FM; ++i) {
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bfr[j], af[i], acc[i][j], 0, 0, 0);
                if constexpr (SPREAD) {
                    // loads ((i+1) PER_STAGE / FM) - (i PER_STAGE / FM) follow MFMA row i
                    __builtin_amdgcn_sched_barrier(0);
                    if (h == 0 && issue_next) {
#pragma unroll
                        for (int d = i * PER_STAGE / FM; d < (i + 1) * PER_STAGE / FM; ++d)
                            issue_one(kt_next, slot_next, d);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
        };
        if constexpr (T::SUB >= 2 && !SPREAD) {
            // Several MFMA K steps per stage: the fragments of step h + 1 are read while the
            // MFMAs of step h run (two fragment sets), one read after each MFMA, so that the
            // wave's LDS read latency is hidden behind its own matrix work within a stage.
            // Measured against reading each step's fragments just before its MFMAs (TFLOP/s,
            // 4096^3): 128 x 128 1,052 -> 1,080, 128 x 64 825 -> 888, 64 x 128 827 -> 865,
            // 64 x 64 716 -> 741; the 128-deep 64 x 64 at 1024 x 1024 x 4096 362 -> 373.  Only
            // K = 128 loses (4096 x 4096 x 128 on 128 x 128: 252 -> 240).  Giving the 256-wide
            // tiles 64-deep stages to pipeline the same way costs them their second work-group
            // per CU (96 KiB) and measured slower at 4096^3 (128 x 256: 1,166 -> 996).
            constexpr int NREAD = FM + 2 * FN, NMFMA = FM * FN;
            constexpr int NPAIR = NREAD < NMFMA ? NREAD : NMFMA;
            bf16x8_t af[2][FM], bfr[2][FN];
            read_frags(0, af[0], bfr[0]);
#pragma unroll
            for (int h = 0; h < T::SUB; ++h) {
                const int c = h & 1;
                __builtin_amdgcn_s_setprio(1);
                if (h + 1 < T::SUB) read_frags(h + 1, af[c ^ 1], bfr[c ^ 1]);
                mfma_step(af[c], bfr[c], 0, 0, h, false);
                if (h + 1 < T::SUB) {
#pragma unroll
                    for (int q = 0; q < NPAIR; ++q) {
                        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);   // one MFMA
                        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
                    }
                    if constexpr (NMFMA > NPAIR) __builtin_amdgcn_sched_group_barrier(0x008, NMFMA - NPAIR, 0);
                    if constexpr (NREAD > NPAIR) __builtin_amdgcn_sched_group_barrier(0x100, NREAD - NPAIR, 0);
                }
                __builtin_amdgcn_s_setprio(0);
            }
        } else {
#pragma unroll
            for (int h = 0; h < T::SUB; ++h) {
                bf16x8_t af[FM], bfr[FN];
                read_frags(h, af, bfr);
                // raised wave priority while the MFMAs issue, so that the waves of a CU that are
                // ready to multiply are preferred over those issuing loads
                __builtin_amdgcn_s_setprio(1);
                mfma_step(af, bfr, kt_next, slot_next, h, issue_next);
                __builtin_amdgcn_s_setprio(0);
            }
        }
      }
    };

    // Step kt waits until this wave's loads of step kt have landed (at most `later` later
    // steps' loads outstanding), meets the other waves, then multiplies step kt while the
    // loads of step kt + S - 1 go out into the slot of step kt - 1.
    // At the barrier every wave's step kt has landed and every wave has consumed step kt - 1
    // (its fragment reads fed its MFMAs before it got here).  A bare barrier: __syncthreads()
    // would add a fence that waits for all outstanding loads and empty the ring every step.
    // The empty asm statements keep the compiler from moving LDS accesses across it.
    auto sync_step = [&](int later) {
        if (later >= 2) wait_vmcnt<2 * PER_STAGE>();
        else if (later == 1) wait_vmcnt<PER_STAGE>();
        else wait_vmcnt<0>();
        asm volatile("" ::: "memory");
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
    };
    constexpr int S = T::STAGES;
#pragma unroll
    for (int s = 0; s < S - 1; ++s)
        if (s < nk) issue(s, s);
    if constexpr (T::XPF && XPF_OK && !MEM) {
        // Cross-stage fragment prefetch: the fragments of stage kt + 1 are read while the MFMAs
        // of stage kt run (two fragment sets), so a wave never waits on LDS between stages.
        // Stage kt + 1 must have landed for every wave before its fragments are read: the wait
        // and barrier for it come after the first MFMA row of stage kt.  The loads of stage
        // kt + S - 1 go into the slot of stage kt - 1, whose fragments every wave consumed in
        // its stage kt - 1 MFMAs, before that barrier.  Measured against reading each stage's
        // fragments after its barrier (TFLOP/s): 4096^3 1,042 -> 1,137, 3840 x 2048 x 4096
        // 494 -> 546, 4096 x 4096 x 1024 770 -> 831, 2048^3 265 -> 291.
        constexpr int NQ = FM + FN;
        bf16x8_t fa[2][FM], fb[2][FN];
        sync_step(min(S - 2, nk - 1));
#pragma unroll
        for (int q = 0; q < NQ; ++q) read_frag(0, 0, q, fa[0], fb[0]);
        auto xstep = [&](auto cc, int kt) {
            constexpr int c = decltype(cc)::value;
            const bool has_next = kt + 1 < nk;
            const bool load_next = kt + S - 1 < nk;
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int i = 0; i < FM; ++i) {
#pragma unroll
                for (int j = 0; j < FN; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fb[c][j], fa[c][i], acc[i][j], 0, 0, 0);
                __builtin_amdgcn_sched_barrier(0);
                if (i == 0 && has_next) {
                    __builtin_amdgcn_s_setprio(0);
                    sync_step(min(kt + S - 2, nk - 1) - (kt + 1));
                    __builtin_amdgcn_s_setprio(1);
                }
                if (has_next) {
#pragma unroll
                    for (int q = i * NQ / FM; q < (i + 1) * NQ / FM; ++q) read_frag((kt + 1) % S, 0, q, fa[c ^ 1], fb[c ^ 1]);
                }
                if (load_next) {
#pragma unroll
                    for (int d = i * PER_STAGE / FM; d < (i + 1) * PER_STAGE / FM; ++d)
                        issue_one(kt + S - 1, (kt + S - 1) % S, d);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
            __builtin_amdgcn_s_setprio(0);
        };
        int kt = 0;
        for (; kt + 1 < nk; kt += 2) {
            xstep(std::integral_constant<int, 0>{}, kt);
            xstep(std::integral_constant<int, 1>{}, kt + 1);
        }
        if (kt < nk) xstep(std::integral_constant<int, 0>{}, kt);
    } else if constexpr (SPREAD) {
        // A steady-state loop (loads issued inside the MFMA sequence, no branch there) and a
        // drain without loads.
        int kt = 0;
        for (; kt + S - 1 < nk; ++kt) {
            sync_step(S - 2);
            compute(kt % S, true, kt + S - 1, (kt + S - 1) % S);
        }
        for (; kt < nk; ++kt) {
            sync_step(nk - 1 - kt);
            compute(kt % S, false, 0, 0);
        }
    } else {
        // One loop with a uniform branch: for these tiles, accumulators that live across two
        // loops get copied through a temporary before every MFMA by the compiler.
        for (int kt = 0; kt < nk; ++kt) {
            sync_step(min(nk - 1, kt + S - 2) - kt);
            // The two-stage ring's one-step lookahead needs the loads out before anything else
            // (issuing them after the fragment reads, which hides the LDS read latency, measured
            // slower for these tiles; it helped only four-stage rings of 32-deep stages).
            if (kt + S - 1 < nk) issue(kt + S - 1, (kt + S - 1) % S);
            compute(kt % S, false, 0, 0);
        }
    }
    // Tiles up to 128x128 write interior, unfused results straight from the accumulators
    // (no barrier, no LDS round trip: it pays most at small K, where the epilogue is a large
    // share of the tile).  The 256-wide tiles keep the LDS-staged epilogue: the direct stores
    // raise them past 256 VGPRs and halve their occupancy.  A caller that runs tiles back to
    // back must put a barrier before the next tile's loads, as the persistent kernel does.
    if constexpr (T::SMALL)
        if (epilogue_direct<BM, BN, NW>(p, m0, n0, kz, acc)) return;
    __syncthreads();                            // ring no longer read: the epilogue reuses it
    epilogue<BM, BN, NW>(p, m0, n0, kz, smem, acc);
}

// One tile over the K range of split kz: [kz k_chunk, min(Kl, (kz + 1) k_chunk)).
template <int BM, int BN, bool MEM = false, bool DEEP = false, int NW = 4, bool XPF_OK = true>
__device__ __forceinline__ void tile_body_dma(const KArgs& p, const int m0, const int n0, const int kz,
                                              uint16_t* __restrict__ smem) {
    const int kb = kz * p.k_chunk;
    tile_body_dma_range<BM, BN, MEM, DEEP, NW, XPF_OK>(p, m0, n0, kz, kb, min(p.Kl, kb + p.k_chunk), smem);
}

}  // namespace sg
