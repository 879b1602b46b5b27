// Buffer read / write kernels of the memory-subsystem study (paper Sec. 5): the bandwidth
// microbenchmarks it runs over the (M, N, K) grid, read A (M x K), read B (K x N) and write D
// (M x N).  Streaming 16-byte accesses, several in flight per lane; the read folds every
// 32-bit word into an XOR (so nothing can be skipped and the result checks the bytes), the
// write stores a word pattern given by the word's index.
#include <hip/hip_ext.h>

#include <algorithm>

#include "sg_internal.h"

namespace sg {

constexpr int kMemThreads = 256;
constexpr int64_t kMemMaxBlocks = 2048;        // 8 work-groups per CU on 256 CUs
constexpr uint32_t kMemWordMul = 0x9E3779B1u;  // odd: word i -> i * mul is a bijection mod 2^32

int64_t mem_blocks(int64_t bytes) {
    const int64_t n16 = bytes / 16;
    const int64_t per_block = (int64_t)kMemThreads * 4;   // at least four 16-byte loads per lane
    return std::max<int64_t>(1, std::min<int64_t>(kMemMaxBlocks, (n16 + per_block - 1) / per_block));
}

__global__ __launch_bounds__(256) void sg_mem_read_kernel(const uint4* __restrict__ p, int64_t n16,
                                                          uint32_t* __restrict__ sink) {
    const int64_t stride = (int64_t)gridDim.x * kMemThreads;
    int64_t i = (int64_t)blockIdx.x * kMemThreads + threadIdx.x;
    uint32_t x = 0;
    for (; i + 3 * stride < n16; i += 4 * stride) {     // four loads in flight
        const uint4 a = p[i], b = p[i + stride], c = p[i + 2 * stride], d = p[i + 3 * stride];
        x ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w;
        x ^= c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n16; i += stride) {
        const uint4 a = p[i];
        x ^= a.x ^ a.y ^ a.z ^ a.w;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x ^= __shfl_xor(x, o);
    __shared__ uint32_t part[kMemThreads / 64];
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) sink[blockIdx.x] = part[0] ^ part[1] ^ part[2] ^ part[3];
}

__global__ __launch_bounds__(256) void sg_mem_write_kernel(uint4* __restrict__ p, int64_t n16, uint32_t seed) {
    const int64_t stride = (int64_t)gridDim.x * kMemThreads;
    for (int64_t i = (int64_t)blockIdx.x * kMemThreads + threadIdx.x; i < n16; i += stride) {
        const uint32_t w = (uint32_t)(4 * i);
        p[i] = make_uint4((w * kMemWordMul) ^ seed, ((w + 1) * kMemWordMul) ^ seed,
                          ((w + 2) * kMemWordMul) ^ seed, ((w + 3) * kMemWordMul) ^ seed);
    }
}

static int mem_check(const void* buf, int64_t bytes) {
    if (bytes < 0 || bytes % 16 != 0) return fail(SG_EINVAL, "buffer length must be a non-negative multiple of 16 bytes");
    if (bytes > 0 && (!buf || (uintptr_t)buf % 16 != 0)) return fail(SG_EINVAL, "buffer must be 16-byte aligned and non-NULL");
    return SG_OK;
}

int launch_mem_read(const void* buf, int64_t bytes, uint32_t* sink, hipStream_t s, hipEvent_t start,
                    hipEvent_t stop) {
    int rc = mem_check(buf, bytes);
    if (rc) return rc;
    if (!sink) return fail(SG_EINVAL, "NULL sink");
    hipExtLaunchKernelGGL(sg_mem_read_kernel, dim3((unsigned)mem_blocks(bytes)), dim3(kMemThreads), 0, s,
                          start, stop, 0, (const uint4*)buf, bytes / 16, sink);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

int launch_mem_write(void* buf, int64_t bytes, uint32_t seed, hipStream_t s, hipEvent_t start, hipEvent_t stop) {
    int rc = mem_check(buf, bytes);
    if (rc) return rc;
    hipExtLaunchKernelGGL(sg_mem_write_kernel, dim3((unsigned)mem_blocks(bytes)), dim3(kMemThreads), 0, s,
                          start, stop, 0, (uint4*)buf, bytes / 16, seed);
    SG_HIP(hipGetLastError());
    return SG_OK;
}

}  // namespace sg

extern "C" {

int64_t sg_mem_read_blocks(int64_t bytes) { return bytes < 0 ? 0 : sg::mem_blocks(bytes); }

int sg_mem_read(const void* buf, int64_t bytes, uint32_t* sink, void* stream) {
    return sg::launch_mem_read(buf, bytes, sink, (hipStream_t)stream, nullptr, nullptr);
}

int sg_mem_write(void* buf, int64_t bytes, uint32_t seed, void* stream) {
    return sg::launch_mem_write(buf, bytes, seed, (hipStream_t)stream, nullptr, nullptr);
}

}  // extern "C"
