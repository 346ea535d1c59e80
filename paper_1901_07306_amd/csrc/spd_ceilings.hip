// Microbenchmarks of the MI355X ceilings the scan's design rests on (libspd_ceilings.so, C ABI in
// include/spd_ceilings.h): streaming reads from HBM, random device-scope atomicOr into a table of
// a given footprint, random 16-bit stores (the sliding scan's stamps), and LDS atomicOr.  Every
// access is masked into its buffer, whose size the host checks; each kernel runs a fixed grid
// over a fixed operation count and ends.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spd_ceilings.h"

namespace {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 64-bit finaliser (multiply / xor-shift mixing, as in SplitMix64's output function): a
// well-spread pseudo-random address per operation index.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

constexpr uint32_t kBlock = 256;
constexpr uint32_t kGrid = 4096;

__global__ __launch_bounds__(kBlock) void k_stream_read(const u32x4 *__restrict__ p, uint64_t n16, uint32_t *sink) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    uint32_t acc = 0;
    uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x;
    for (; i + 3 * stride < n16; i += 4 * stride) {
        const u32x4 a = __builtin_nontemporal_load(p + i), b = __builtin_nontemporal_load(p + i + stride);
        const u32x4 c = __builtin_nontemporal_load(p + i + 2 * stride), d = __builtin_nontemporal_load(p + i + 3 * stride);
        acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^ d.z ^ d.w;
    }
    for (; i < n16; i += stride) {
        const u32x4 a = __builtin_nontemporal_load(p + i);
        acc ^= a.x ^ a.y ^ a.z ^ a.w;
    }
    if (acc == 0x9E3779B9u) sink[0] = acc;   // keeps the loads; practically never taken
}

__global__ __launch_bounds__(kBlock) void k_atomic_or(uint32_t *__restrict__ table, uint64_t mask, uint64_t n_ops,
                                                      uint64_t seed) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n_ops; i += stride) {
        const uint64_t h = mix64(i + seed);
        __hip_atomic_fetch_or(table + (h & mask), 1u << (h >> 59), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ __launch_bounds__(kBlock) void k_store16(uint16_t *__restrict__ table, uint64_t mask, uint64_t n_ops,
                                                    uint64_t seed) {
    const uint64_t stride = (uint64_t)gridDim.x * kBlock;
    for (uint64_t i = blockIdx.x * (uint64_t)kBlock + threadIdx.x; i < n_ops; i += stride) {
        const uint64_t h = mix64(i + seed);
        table[h & mask] = (uint16_t)(h >> 48);
    }
}

constexpr uint32_t kLdsWords = 32768;   // a 128 KiB bitmap, the scan's apply-phase bucket

__global__ __launch_bounds__(kBlock) void k_lds_atomic_or(uint32_t n_iter, uint32_t *sink) {
    __shared__ uint32_t bm[kLdsWords];
    for (uint32_t w = threadIdx.x; w < kLdsWords; w += kBlock) bm[w] = 0;
    __syncthreads();
    uint64_t h = mix64(((uint64_t)blockIdx.x << 32) | threadIdx.x);
    for (uint32_t k = 0; k < n_iter; ++k) {
        h = mix64(h + k);
        atomicOr(&bm[h & (kLdsWords - 1)], 1u << (h >> 59));
    }
    __syncthreads();
    if (threadIdx.x == 0 && bm[blockIdx.x & (kLdsWords - 1)] == 0x9E3779B9u) sink[0] = 1;
}

bool pow2(uint64_t v) { return v && !(v & (v - 1)); }

}  // namespace

extern "C" {

int spd_ceil_stream_read(const void *p, uint64_t bytes, uint32_t *sink, void *stream) {
    if (!p || !sink || bytes % 16 || reinterpret_cast<uintptr_t>(p) % 16) return -1;
    hipLaunchKernelGGL(k_stream_read, dim3(kGrid * 2), dim3(kBlock), 0, static_cast<hipStream_t>(stream),
                       static_cast<const u32x4 *>(p), bytes / 16, sink);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int spd_ceil_atomic_or(uint32_t *table, uint64_t words, uint64_t n_ops, uint64_t seed, void *stream) {
    if (!table || !pow2(words)) return -1;
    hipLaunchKernelGGL(k_atomic_or, dim3(kGrid), dim3(kBlock), 0, static_cast<hipStream_t>(stream), table, words - 1,
                       n_ops, seed);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int spd_ceil_store16(uint16_t *table, uint64_t elems, uint64_t n_ops, uint64_t seed, void *stream) {
    if (!table || !pow2(elems)) return -1;
    hipLaunchKernelGGL(k_store16, dim3(kGrid), dim3(kBlock), 0, static_cast<hipStream_t>(stream), table, elems - 1,
                       n_ops, seed);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int spd_ceil_lds_atomic_or(uint32_t blocks, uint32_t n_iter, uint32_t *sink, void *stream) {
    if (!sink || blocks == 0) return -1;
    hipLaunchKernelGGL(k_lds_atomic_or, dim3(blocks), dim3(kBlock), 0, static_cast<hipStream_t>(stream), n_iter, sink);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

uint32_t spd_ceil_block(void) { return kBlock; }

}  // extern "C"
