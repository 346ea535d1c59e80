// HIP kernels of libspd for gfx950 (MI355X).
//
// Scan (Sections 3.1-3.3, 4.1): every pair sets LR bits of the LDCA and, when sampled, SR bits of
// the SEAV.  Two kernels record a batch:
//   * direct:  one thread per pair, global atomicOr per bit.  Device-wide random atomics run at a
//              fixed rate on MI355X whatever the footprint, so this path serves small batches.
//   * binned:  a workgroup reads a tile of pairs, turns each pair into bit addresses and
//              counting-sorts them in LDS by sketch bucket (2^S bits); an apply kernel gives one
//              workgroup per bucket, replays the bucket's items into an LDS bitmap with LDS
//              atomicOr, and writes the bucket back with plain stores.  No global atomics on the
//              hot path.  Three item layouts: k_region writes each tile's segments into
//              fixed-capacity (chunk of tiles, bucket) regions, read by k_apply_rg (the default,
//              one pass over the pairs); k_count + k_place write one exact bucket-major stream,
//              read by k_apply_bm; k_bin writes per-tile regions, gathered by k_apply.
// End of window (Sections 3.2-3.3): k_close gives one wavefront per SEA (one RP): hot-SE lists
// by ballot, the candidate product with Eq. 3 consistency and the SEU weight test, then the
// ULDC of each candidate (AND over LR rows, popcount by wavefront reduction).
#include <hip/hip_ext.h>

#include "spd_internal.h"

namespace spd {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));

// A pair as the method sees it: (hip, oip) = the record, or the swapped record for a
// destination-keyed batch (uniform per batch).
__device__ __forceinline__ u32x2 keyed(u32x2 pr, uint32_t swap) { return swap ? u32x2{pr.y, pr.x} : pr; }
// Pair i of a batch, keyed.  Batch pointers come from descriptors in memory, so the compiler
// cannot tell their address space; naming it keeps these global (not flat) loads, which do not
// hold up the LDS wait counter.
typedef __attribute__((address_space(1))) const u32x2 global_u32x2;
__device__ __forceinline__ u32x2 load_pair(const u32x2 *pairs, uint64_t i, uint32_t swap) {
    return keyed(__builtin_nontemporal_load((const global_u32x2 *)pairs + i), swap);
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct BatchTable {
    BatchDesc b[kMaxGroup];
    uint32_t n;
};
// Index of the batch that tile belongs to: the last one whose first tile is <= tile.
__device__ __forceinline__ uint32_t find_batch(const BatchList &bl, uint32_t tile) {
    uint32_t lo = 0, hi = bl.n;   // b[lo].first_tile <= tile < b[hi].first_tile (b[n] = infinity)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (bl.b[mid].first_tile <= tile) lo = mid;
        else hi = mid;
    }
    return lo;
}
// The batch of a tile, from device memory or from the inline copies (constant indices only, so
// that the kernel-argument array is never copied to scratch memory).
__device__ __forceinline__ BatchDesc batch_of(const BatchList &bl, uint32_t tile) {
    if (bl.b) return bl.b[find_batch(bl, tile)];
    BatchDesc B = bl.inl[0];
#pragma unroll
    for (uint32_t i = 1; i < kInlineBatches; ++i)
        if (i < bl.n && bl.inl[i].first_tile <= tile) B = bl.inl[i];
    return B;
}
struct SlotTable {
    SlotPtrs s[kMaxGroup];
};
struct ApplyTable {
    ApplySlot s[kMaxGroup];
};
struct SrcTable {
    const uint32_t *p[kMaxGroup];
};
struct SrcTable16 {
    const uint16_t *p[kMaxGroup];
};

__device__ __forceinline__ void global_or(uint32_t *p, uint32_t v) {
    __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool sampled(uint32_t oip, const Consts &c) {
    // lsb(H1(oip)) >= tau, with lsb(0) = 32 (Section 3.1): the low tau bits are all zero.
    return (mas_hi(oip, c.mul[0], c.add[0]) & c.tau_mask) == 0u;
}

__device__ __forceinline__ uint32_t se_bit(uint32_t oip, const Consts &c) { return mas_hi(oip, c.mul[1], c.add[1]) >> 29; }

__device__ __forceinline__ uint32_t ldc_bit(uint32_t oip, const Consts &c) {
    return top_bits(mas_hi(oip, c.mul[2], c.add[2]), c.sh_k);
}

__device__ __forceinline__ uint32_t ldc_col(uint32_t hip, uint32_t i, const Consts &c) {
    return top_bits(mas_hi(hip, c.mul[3 + i], c.add[3 + i]), c.sh_lc);
}

// Per-row SEAV constants (ISB, IBN, byte offset of the row in a SEA) copied to LDS by one thread
// with constant indices: loops over a runtime row count then read LDS instead of indexing the
// kernel-argument block, which would otherwise be copied to scratch memory.
struct RowLds {
    uint32_t v[3 * kMaxRows];
};
__device__ __forceinline__ void rows_to_lds(RowLds &rl, const Consts &c) {
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < kMaxRows; ++k) {
            rl.v[3 * k] = c.isb[k];
            rl.v[3 * k + 1] = c.ibn[k];
            rl.v[3 * k + 2] = c.row_off[k];
        }
    }
}
__device__ __forceinline__ uint32_t seav_byte_l(uint32_t hip, uint32_t i, const RowLds &rl, const Consts &c) {
    const uint32_t rp = hip & c.rmask;
    const uint32_t lp = (uint32_t)((uint64_t)hip >> c.r);
    return rp * c.sea_bytes + rl.v[3 * i + 2] + row_index(lp, rl.v[3 * i], rl.v[3 * i + 1], c.L);
}

// ------------------------------------------------------------------------------ fill
__global__ void k_fill_u32(uint32_t *__restrict__ p, uint64_t n, uint32_t v) {
    uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t n4 = n / 4;
    u32x4 vv = {v, v, v, v};
    for (uint64_t j = i; j < n4; j += stride) reinterpret_cast<u32x4 *>(p)[j] = vv;
    for (uint64_t j = n4 * 4 + i; j < n; j += stride) p[j] = v;
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t n_words, uint32_t value, hipStream_t s) {
    if (n_words == 0) return hipSuccess;
    uint64_t blocks = (n_words / 4 + 255) / 256;
    uint32_t grid = (uint32_t)(blocks < 4096 ? (blocks ? blocks : 1) : 4096);
    hipLaunchKernelGGL(k_fill_u32, dim3(grid), dim3(256), 0, s, p, n_words, value);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------ direct scan
template <bool SEAV_LDS>
__global__ __launch_bounds__(1024) void k_scan_direct(Consts c, BatchTable bt, SlotTable st, uint32_t lds_words) {
    extern __shared__ uint32_t lds[];
    if (SEAV_LDS) {
        for (uint32_t w = threadIdx.x; w < lds_words; w += blockDim.x) lds[w] = 0;
        __syncthreads();
    }
    const uint64_t gtid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint32_t bi = 0; bi < bt.n; ++bi) {
        const BatchDesc B = bt.b[bi];
        const SlotPtrs S = st.s[B.slot];
        uint32_t *seav_w = reinterpret_cast<uint32_t *>(S.seav);
        const u32x2 *pairs = reinterpret_cast<const u32x2 *>(B.pairs);
        for (uint64_t i = gtid; i < B.n; i += stride) {
            const u32x2 pr = load_pair(pairs, i, B.swap);
            const uint32_t hip = pr.x, oip = pr.y;
            const uint32_t q = ldc_bit(oip, c);
            for (uint32_t r = 0; r < c.lr; ++r) {
                uint32_t bit = ldca_bit(r, ldc_col(hip, r, c), q, c);
                global_or(S.ldca + (bit >> 5), 1u << (bit & 31u));
            }
            if (sampled(oip, c)) {
                const uint32_t b = se_bit(oip, c);
                for (uint32_t r = 0; r < c.sr; ++r) {
                    uint32_t bit = seav_byte(hip, r, c) * 8u + b;
                    if (SEAV_LDS)
                        atomicOr(&lds[bit >> 5], 1u << (bit & 31u));
                    else
                        global_or(seav_w + (bit >> 5), 1u << (bit & 31u));
                }
            }
        }
    }
    if (SEAV_LDS) {
        // OR the workgroup's SEAV copy into the sketch; untouched words cost nothing.
        __syncthreads();
        uint32_t *seav_w = reinterpret_cast<uint32_t *>(st.s[0].seav);
        for (uint32_t w = threadIdx.x; w < lds_words; w += blockDim.x) {
            uint32_t v = lds[w];
            if (v) global_or(seav_w + w, v);
        }
    }
}

hipError_t launch_scan_direct(const Consts &c, const BatchDesc *batches, uint32_t n_batches, const SlotPtrs *slots,
                              uint32_t block, uint32_t grid, bool seav_lds, hipStream_t s) {
    BatchTable bt{};
    SlotTable st{};
    if (n_batches > (uint32_t)kMaxGroup) return hipErrorInvalidValue;
    for (uint32_t i = 0; i < n_batches; ++i) bt.b[i] = batches[i];
    bt.n = n_batches;
    for (int i = 0; i < kMaxGroup; ++i) st.s[i] = slots[i];
    if (seav_lds) {
        uint32_t words = (uint32_t)((c.seav_bytes + 3) / 4);
        hipLaunchKernelGGL(k_scan_direct<true>, dim3(grid), dim3(block), words * 4u, s, c, bt, st, words);
    } else {
        hipLaunchKernelGGL(k_scan_direct<false>, dim3(grid), dim3(block), 0, s, c, bt, st, 0u);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------------ sliding scan
// Every bit the discrete scan would set receives the slice's value: a 16-bit stamp, or an 8-bit
// AT code.  All writers of one slice store the same value, and slices are ordered by the stream,
// so plain stores suffice.
template <typename T>
__device__ __forceinline__ T *ldca_counters(const SlotPtrs &S);
template <>
__device__ __forceinline__ uint16_t *ldca_counters<uint16_t>(const SlotPtrs &S) { return S.ldca_ts; }
template <>
__device__ __forceinline__ uint8_t *ldca_counters<uint8_t>(const SlotPtrs &S) { return S.ldca_at; }
template <typename T>
__device__ __forceinline__ T *seav_counters(const SlotPtrs &S);
template <>
__device__ __forceinline__ uint16_t *seav_counters<uint16_t>(const SlotPtrs &S) { return S.seav_ts; }
template <>
__device__ __forceinline__ uint8_t *seav_counters<uint8_t>(const SlotPtrs &S) { return S.seav_at; }

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_stamp(Consts c, BatchTable bt, SlotTable st, uint32_t value) {
    const uint64_t gtid = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const T v = (T)value;
    for (uint32_t bi = 0; bi < bt.n; ++bi) {
        const BatchDesc B = bt.b[bi];
        const SlotPtrs S = st.s[B.slot];
        T *ldca = ldca_counters<T>(S), *seav = seav_counters<T>(S);
        const u32x2 *pairs = reinterpret_cast<const u32x2 *>(B.pairs);
        for (uint64_t i = gtid; i < B.n; i += stride) {
            const u32x2 pr = load_pair(pairs, i, B.swap);
            const uint32_t hip = pr.x, oip = pr.y;
            const uint32_t q = ldc_bit(oip, c);
            for (uint32_t r = 0; r < c.lr; ++r) ldca[ldca_bit(r, ldc_col(hip, r, c), q, c)] = v;
            if (sampled(oip, c)) {
                const uint32_t b = se_bit(oip, c);
                for (uint32_t r = 0; r < c.sr; ++r) seav[(uint64_t)seav_byte(hip, r, c) * 8u + b] = v;
            }
        }
    }
}

hipError_t launch_scan_stamp(const Consts &c, const BatchDesc *batches, uint32_t n_batches, const SlotPtrs *slots,
                             uint32_t value, bool at, uint32_t block, uint32_t grid, hipStream_t s, KTiming kt) {
    BatchTable bt{};
    SlotTable st{};
    if (n_batches > (uint32_t)kMaxGroup) return hipErrorInvalidValue;
    for (uint32_t i = 0; i < n_batches; ++i) bt.b[i] = batches[i];
    bt.n = n_batches;
    for (int i = 0; i < kMaxGroup; ++i) st.s[i] = slots[i];
    if (at) hipExtLaunchKernelGGL(k_scan_stamp<uint8_t>, dim3(grid), dim3(block), 0, s, kt.start, kt.stop, 0, c, bt, st, value);
    else hipExtLaunchKernelGGL(k_scan_stamp<uint16_t>, dim3(grid), dim3(block), 0, s, kt.start, kt.stop, 0, c, bt, st, value);
    return hipGetLastError();
}

// AT pool maintenance and views.  A pool is handled 16 counters (one 16-byte vector) per lane.
struct PoolTable {
    uint8_t *p[kMaxGroup];
};
struct CPoolTable {
    const uint8_t *p[kMaxGroup];
};

// Byte k of a 16-byte vector.
__device__ __forceinline__ uint32_t byte_of(const u32x4 &v, uint32_t k) { return (v[k >> 2] >> (8 * (k & 3))) & 0xFFu; }

// Activity of the four AT counters packed in one 32-bit word, four at a time (SIMD within a
// register): bit 7 of byte j of the result is set iff counter j is active, i.e. its age
// (ct - v) mod 256 is below K.  The per-byte difference is taken without borrows between bytes;
// the per-byte compare with K needs K <= 128, so larger windows decode byte by byte.
__device__ __forceinline__ uint32_t at_active_bytes(uint32_t w, uint32_t ct, uint32_t K) {
    constexpr uint32_t H = 0x80808080u, L = 0x7F7F7F7Fu;
    if (K <= 128u) {
        const uint32_t ct4 = ct * 0x01010101u, k4 = K * 0x01010101u;
        const uint32_t e = ((ct4 | H) - (w & L)) ^ ((ct4 ^ ~w) & H);   // (ct - v) mod 256 per byte
        const uint32_t d = ((e & L) | H) - k4;                          // top bit: low 7 bits of e >= K
        return ~(e | d) & H;
    }
    uint32_t r = 0;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) r |= at_active((w >> (8 * j)) & 0xFFu, ct, K) << (8 * j + 7);
    return r;
}

__global__ __launch_bounds__(256) void k_at_sweep(PoolTable pt, uint32_t n, uint64_t lo16, uint64_t hi16, uint32_t ct,
                                                  uint32_t K) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    const uint32_t ex = (ct - K) & (kAtCodes - 1u);   // the code of slice t - K: expired, age K
    for (uint32_t k = 0; k < n; ++k) {
        u32x4 *p = reinterpret_cast<u32x4 *>(pt.p[k]);
        for (uint64_t i = lo16 + blockIdx.x * (uint64_t)256 + threadIdx.x; i < hi16; i += stride) {
            const u32x4 v = p[i];
            u32x4 o = v;
            bool changed = false;
#pragma unroll
            for (uint32_t b = 0; b < 16; ++b) {
                const uint32_t x = byte_of(v, b);
                if (!at_active(x, ct, K) && x != ex) {
                    o[b >> 2] = (o[b >> 2] & ~(0xFFu << (8 * (b & 3)))) | (ex << (8 * (b & 3)));
                    changed = true;
                }
            }
            if (changed) p[i] = o;
        }
    }
}

hipError_t launch_at_sweep(uint8_t *const *pools, uint32_t n, uint64_t lo, uint64_t hi, uint32_t ct, uint32_t K,
                           hipStream_t s) {
    if (lo % 16 || hi % 16 || hi < lo) return hipErrorInvalidValue;
    for (uint32_t k0 = 0; k0 < n; k0 += kMaxGroup) {
        PoolTable pt{};
        const uint32_t m = n - k0 < (uint32_t)kMaxGroup ? n - k0 : (uint32_t)kMaxGroup;
        for (uint32_t k = 0; k < m; ++k) pt.p[k] = pools[k0 + k];
        const uint64_t vec = (hi - lo) / 16;
        if (vec == 0) return hipSuccess;
        const uint32_t grid = (uint32_t)((vec + 255) / 256 < 2048 ? (vec + 255) / 256 : 2048);
        hipLaunchKernelGGL(k_at_sweep, dim3(grid), dim3(256), 0, s, pt, m, lo / 16, hi / 16, ct, K);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Per counter, the most recent of the sources: the smallest age.  Every source is maintained, so
// every age read modulo 256 is the true age.
__global__ __launch_bounds__(256) void k_at_merge(uint8_t *__restrict__ dst, CPoolTable src, uint32_t n_src,
                                                  uint64_t n16, uint32_t ct) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = blockIdx.x * (uint64_t)256 + threadIdx.x; i < n16; i += stride) {
        u32x4 best = reinterpret_cast<const u32x4 *>(src.p[0])[i];
        for (uint32_t k = 1; k < n_src; ++k) {
            const u32x4 v = reinterpret_cast<const u32x4 *>(src.p[k])[i];
#pragma unroll
            for (uint32_t b = 0; b < 16; ++b) {
                const uint32_t x = byte_of(v, b), y = byte_of(best, b);
                if (((ct - x) & (kAtCodes - 1u)) < ((ct - y) & (kAtCodes - 1u)))
                    best[b >> 2] = (best[b >> 2] & ~(0xFFu << (8 * (b & 3)))) | (x << (8 * (b & 3)));
            }
        }
        reinterpret_cast<u32x4 *>(dst)[i] = best;
    }
}

hipError_t launch_at_merge(uint8_t *dst, const uint8_t *const *src, uint32_t n_src, uint64_t n_bytes, uint32_t ct,
                           hipStream_t s) {
    if (n_src == 0 || n_src > (uint32_t)kMaxGroup || n_bytes % 16) return hipErrorInvalidValue;
    CPoolTable t{};
    for (uint32_t k = 0; k < n_src; ++k) t.p[k] = src[k];
    const uint64_t n16 = n_bytes / 16;
    const uint32_t grid = (uint32_t)((n16 + 255) / 256 < 8192 ? (n16 + 255) / 256 : 8192);
    hipLaunchKernelGGL(k_at_merge, dim3(grid ? grid : 1), dim3(256), 0, s, dst, t, n_src, n16, ct);
    return hipGetLastError();
}

// Bit view of AT counters: 32 counters (two 16-byte vectors) per output word.
__global__ __launch_bounds__(256) void k_bit_view_at(const uint8_t *__restrict__ at, uint64_t n_words, uint32_t ct,
                                                     uint32_t K, uint32_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t w = blockIdx.x * (uint64_t)256 + threadIdx.x; w < n_words; w += stride) {
        const u32x4 a = reinterpret_cast<const u32x4 *>(at)[2 * w], b = reinterpret_cast<const u32x4 *>(at)[2 * w + 1];
        uint32_t v = 0;
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            // counters 4q..4q+3 of each vector: activity bits at 0, 8, 16, 24, gathered into 4 bits
            const uint32_t ma = at_active_bytes(a[q], ct, K) >> 7, mb = at_active_bytes(b[q], ct, K) >> 7;
            v |= ((ma | ma >> 7 | ma >> 14 | ma >> 21) & 0xFu) << (4 * q);
            v |= ((mb | mb >> 7 | mb >> 14 | mb >> 21) & 0xFu) << (16 + 4 * q);
        }
        out[w] = v;
    }
}

hipError_t launch_bit_view_at(const uint8_t *at, uint64_t n_bits, uint32_t ct, uint32_t K, uint32_t *out_words,
                              hipStream_t s) {
    if (n_bits % 32) return hipErrorInvalidValue;
    const uint64_t words = n_bits / 32;
    const uint32_t grid = (uint32_t)((words + 255) / 256 < 8192 ? (words + 255) / 256 : 8192);
    hipLaunchKernelGGL(k_bit_view_at, dim3(grid ? grid : 1), dim3(256), 0, s, at, words, ct, K, out_words);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------ binned scan
// Block-wide pass over the bucket counters: cl[b] = LDCA items, cs[b] = SEAV items of bucket b.
// Afterwards cl[b] = first slot of bucket b in the tile's item list, cs[b] = first SEAV slot
// (after the bucket's LDCA items), cl[nb] = total items.
template <int BLOCK>
__device__ void bucket_offsets(uint32_t *cl, uint32_t *cs, uint32_t nb, uint32_t *scratch) {
    constexpr int NW = BLOCK / 64;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
    const uint32_t per = (nb + BLOCK - 1) / BLOCK;
    const uint32_t beg = tid * per < nb ? tid * per : nb;
    const uint32_t end = beg + per < nb ? beg + per : nb;
    uint32_t local = 0;
    for (uint32_t b = beg; b < end; ++b) local += cl[b] + cs[b];
    uint32_t incl = local;
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(incl, o, 64);
        if ((int)lane >= o) incl += t;
    }
    if (lane == 63u) scratch[wid] = incl;
    __syncthreads();
    if (tid == 0) {
        uint32_t run = 0;
        for (int w = 0; w < NW; ++w) {
            uint32_t t = scratch[w];
            scratch[w] = run;
            run += t;
        }
        scratch[NW] = run;
    }
    __syncthreads();
    uint32_t run = scratch[wid] + incl - local;
    for (uint32_t b = beg; b < end; ++b) {
        uint32_t l = cl[b], s = cs[b];
        cl[b] = run;
        cs[b] = run + l;
        run += l + s;
    }
    if (tid == 0) cl[nb] = scratch[NW];
    __syncthreads();
}

// Bit addresses of a tile's pairs: LDCA items are counted per bucket in cl (the returned rank is
// kept per item), sampled pairs are staged in samp; once samp is full the rest are recorded directly
// (DEFER: only counted, the caller hands the whole tile's sampled pairs to a later pass).
template <int LR, int PPT, int BLOCK, bool FULL, bool DEFER>
__device__ __forceinline__ void bin_hash_pairs(const Consts &c, const RowLds &rl, const BinGeometry &g, const SlotPtrs &S,
                                               const u32x2 (&pr)[PPT], uint64_t p0, uint64_t n, uint32_t *cl,
                                               uint32_t *samp, uint32_t *misc, uint32_t (&bits)[PPT * LR],
                                               uint32_t (&rk)[(PPT * LR + 1) / 2]) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const bool valid = FULL || p0 + (uint64_t)j * BLOCK + tid < n;
        const uint32_t hip = pr[j].x, oip = pr[j].y;
        const uint32_t q = ldc_bit(oip, c);
#pragma unroll
        for (int r = 0; r < LR; ++r) {
            const int k = j * LR + r;
            const uint32_t bit = ldca_bit((uint32_t)r, ldc_col(hip, (uint32_t)r, c), q, c);
            const uint32_t rank = valid ? atomicAdd(&cl[bit >> g.S], 1u) : 0xFFFFu;
            bits[k] = bit;
            if (k & 1)
                rk[k / 2] |= rank << 16;
            else
                rk[k / 2] = rank;
        }
        if (valid && sampled(oip, c)) {
            const uint32_t b = se_bit(oip, c);
            uint32_t e = atomicAdd(&misc[0], 1u);
            if (e < g.scap) {
                samp[2 * e] = hip;
                samp[2 * e + 1] = b;
            } else if (!DEFER) {
                // more sampled pairs than the tile reserved: record them directly
                uint32_t *seav_w = reinterpret_cast<uint32_t *>(S.seav);
                for (uint32_t r = 0; r < c.sr; ++r) {
                    uint32_t bit = seav_byte_l(hip, r, rl, c) * 8u + b;
                    global_or(seav_w + (bit >> 5), 1u << (bit & 31u));
                }
            }
        }
    }
}

// Each tile writes its items bucket-major into its own region (item j of the tile in 64-bit word
// j / 3) plus its nb + 1 bucket offsets in meta[tile].
template <int LR, int PPT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_bin(Consts c, BinGeometry g, BatchTable bt, SlotTable st,
                                               uint32_t *__restrict__ items, uint32_t *__restrict__ meta) {
    extern __shared__ uint32_t lds[];
    __shared__ RowLds rl;   // read after the first barrier
    rows_to_lds(rl, c);
    const uint32_t nb = g.nb;
    uint32_t *cl = lds;                  // [nb + 1] LDCA counts, then offsets
    uint32_t *cs = cl + (nb + 1);        // [nb + 1] SEAV counts, then cursors
    uint32_t *stage = lds + ((2 * (nb + 1) + 3) & ~3u);  // [cap] bucket-major items (16-byte aligned)
    uint32_t *samp = stage + g.cap;      // [2 * scap] sampled (hip, H2 bit)
    uint32_t *misc = samp + 2 * g.scap;  // [0] sampled count, [1..] scan scratch
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = xcd_contiguous(blockIdx.x, gridDim.x);   // neighbouring tiles on one XCD
    uint32_t bi = 0;
    while (bi + 1 < bt.n && bt.b[bi + 1].first_tile <= tile) ++bi;
    const BatchDesc B = bt.b[bi];
    const SlotPtrs S = st.s[B.slot];
    const uint64_t p0 = (uint64_t)(tile - B.first_tile) * (uint64_t)(PPT * BLOCK);
    const uint32_t smask = (1u << g.S) - 1u;
    const uint32_t seav_base = (uint32_t)c.ldca_bits;   // SEAV bits follow the LDCA bits

    for (uint32_t i = tid; i < 2 * (nb + 1); i += BLOCK) cl[i] = 0;
    if (tid == 0) misc[0] = 0;
    // every lane loads unconditionally (past-the-end lanes re-read the last pair and are masked
    // out below), so all PPT loads of a lane are in flight together
    const u32x2 *pairs = reinterpret_cast<const u32x2 *>(B.pairs);
    const uint64_t last = B.n - 1;
    u32x2 pr[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint64_t idx = p0 + (uint64_t)j * BLOCK + tid;
        pr[j] = load_pair(pairs, idx < B.n ? idx : last, B.swap);
    }
    __syncthreads();

    // per item: its bit address, and its rank inside its bucket (16 bits, two per register;
    // 0xFFFF marks a lane past the end of the batch)
    uint32_t bits[PPT * LR], rk[(PPT * LR + 1) / 2];
    // a full tile (all but the last of a batch) needs no per-pair range test
    if (p0 + (uint64_t)(PPT * BLOCK) <= B.n)
        bin_hash_pairs<LR, PPT, BLOCK, true, false>(c, rl, g, S, pr, p0, B.n, cl, samp, misc, bits, rk);
    else
        bin_hash_pairs<LR, PPT, BLOCK, false, false>(c, rl, g, S, pr, p0, B.n, cl, samp, misc, bits, rk);
    __syncthreads();
    // a tile with more sampled pairs than it can stage records all of them directly (the decision
    // depends only on the tile's sampled count, so a counting pass can repeat it)
    uint32_t ns = misc[0];
    if (ns > g.scap) {
        uint32_t *seav_w = reinterpret_cast<uint32_t *>(S.seav);
        for (uint32_t e = tid; e < g.scap; e += BLOCK) {
            const uint32_t hip = samp[2 * e], b = samp[2 * e + 1];
            for (uint32_t r = 0; r < c.sr; ++r) {
                uint32_t bit = seav_byte_l(hip, r, rl, c) * 8u + b;
                global_or(seav_w + (bit >> 5), 1u << (bit & 31u));
            }
        }
        ns = 0;
    }
    for (uint32_t e = tid; e < ns; e += BLOCK) {
        const uint32_t hip = samp[2 * e], b = samp[2 * e + 1];
        for (uint32_t r = 0; r < c.sr; ++r) {
            uint32_t bit = seav_base + seav_byte_l(hip, r, rl, c) * 8u + b;
            atomicAdd(&cs[bit >> g.S], 1u);
        }
    }
    __syncthreads();
    bucket_offsets<BLOCK>(cl, cs, nb, misc + 1);

#pragma unroll
    for (int k = 0; k < PPT * LR; ++k) {
        const uint32_t rank = (rk[k / 2] >> (16 * (k & 1))) & 0xFFFFu;
        if (rank != 0xFFFFu) stage[cl[bits[k] >> g.S] + rank] = bits[k] & smask;
    }
    for (uint32_t e = tid; e < ns; e += BLOCK) {
        const uint32_t hip = samp[2 * e], b = samp[2 * e + 1];
        for (uint32_t r = 0; r < c.sr; ++r) {
            uint32_t bit = seav_base + seav_byte_l(hip, r, rl, c) * 8u + b;
            uint32_t pos = atomicAdd(&cs[bit >> g.S], 1u);
            stage[pos] = bit & smask;
        }
    }
    __syncthreads();
    // items are at most 21 bits (S <= 20): three per 64-bit word
    const uint32_t total = cl[nb];
    uint64_t *out = reinterpret_cast<uint64_t *>(items + (uint64_t)tile * g.region);
    const uint32_t n64 = (total + 2) / 3;
    for (uint32_t i = tid; i < n64; i += BLOCK) {
        const uint32_t j = 3 * i;
        uint64_t v = stage[j];
        if (j + 1 < total) v |= (uint64_t)stage[j + 1] << 21;
        if (j + 2 < total) v |= (uint64_t)stage[j + 2] << 42;
        out[i] = v;
    }
    uint32_t *mo = meta + (uint64_t)tile * (nb + 1);
    for (uint32_t i = tid; i <= nb; i += BLOCK) mo[i] = cl[i];
}

// The bucket counts of bin_hash_pairs without keeping the items.  NEEDQ = false: a bucket holds
// whole LDCs (at least k bits) and a row holds more than one bucket, so a bucket index is the top
// bits of LH_r alone (H3 is not needed).
template <int LR, int PPT, int BLOCK, bool FULL, bool NEEDQ>
__device__ __forceinline__ void count_hash_pairs(const Consts &c, const BinGeometry &g, const u32x2 (&pr)[PPT],
                                                 uint64_t p0, uint64_t n, uint32_t *hl, uint32_t *samp, uint32_t *misc) {
    const uint32_t tid = threadIdx.x;
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        if (!FULL && p0 + (uint64_t)j * BLOCK + tid >= n) continue;
        const uint32_t hip = pr[j].x, oip = pr[j].y;
        if (NEEDQ) {
            const uint32_t q = ldc_bit(oip, c);
#pragma unroll
            for (int r = 0; r < LR; ++r) {
                uint32_t bit = ldca_bit((uint32_t)r, ldc_col(hip, (uint32_t)r, c), q, c);
                atomicAdd(&hl[bit >> g.S], 1u);
            }
        } else {
            // bucket = (r * LC + col) >> (S - log2 k): the top nbits bits of LH_r, after r's rows
            const uint32_t nbits = c.log2lc + c.log2k - g.S;   // >= 1 on this path
#pragma unroll
            for (int r = 0; r < LR; ++r)
                atomicAdd(&hl[((uint32_t)r << nbits) + (mas_hi(hip, c.mul[3 + r], c.add[3 + r]) >> (32u - nbits))], 1u);
        }
        if (sampled(oip, c)) {   // staged; its SR items are counted by the whole workgroup later
            const uint32_t e = atomicAdd(&misc[0], 1u);
            if (e < g.scap) {
                samp[2 * e] = hip;
                samp[2 * e + 1] = se_bit(oip, c);
            }
        }
    }
}

// Exact per-tile item counts by bucket (the first pass of the bucket-major layout): the same bit
// addresses as k_bin, counted in LDS, SEAV items left out for tiles that record them directly.
template <int LR, int PPT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_count(Consts c, BinGeometry g, BatchList bl, ClearList clr,
                                                 uint32_t *__restrict__ cnt) {
    extern __shared__ uint32_t lds[];
    __shared__ RowLds rl;   // read after the first barrier
    rows_to_lds(rl, c);
    const uint32_t nb = g.nb;
    uint32_t *hl = lds;              // [nb] LDCA items
    uint32_t *hs = hl + nb;          // [nb] SEAV items
    uint32_t *misc = hs + nb;        // [0] sampled pairs
    uint32_t *samp = misc + 1;       // [2 * scap] sampled (hip, H2 bit)
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = blockIdx.x;
    const BatchDesc B = bl.b[find_batch(bl, tile)];   // descriptors in device memory
    const uint64_t p0 = (uint64_t)(tile - B.first_tile) * (uint64_t)(PPT * BLOCK);
    for (uint32_t i = tid; i < 2 * nb; i += BLOCK) hl[i] = 0;
    if (tid == 0) misc[0] = 0;
    const u32x2 *pairs = reinterpret_cast<const u32x2 *>(B.pairs);
    const uint64_t last = B.n - 1;
    u32x2 pr[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint64_t idx = p0 + (uint64_t)j * BLOCK + tid;
        pr[j] = load_pair(pairs, idx < B.n ? idx : last, B.swap);
    }
    // the SEAVs of fresh slots, spread over the whole grid (16-byte stores)
    {
        const uint64_t gt = (uint64_t)blockIdx.x * BLOCK + tid, stride = (uint64_t)gridDim.x * BLOCK;
        for (uint32_t k = 0; k < clr.n; ++k) {
            u32x4 *p4 = reinterpret_cast<u32x4 *>(clr.p[k]);
            for (uint64_t w = gt; w < clr.words[k] / 4; w += stride) p4[w] = u32x4{0u, 0u, 0u, 0u};
        }
    }
    __syncthreads();
    const bool full = p0 + (uint64_t)(PPT * BLOCK) <= B.n;
    if (g.S < c.log2k || g.S >= c.log2lc + c.log2k) {
        if (full) count_hash_pairs<LR, PPT, BLOCK, true, true>(c, g, pr, p0, B.n, hl, samp, misc);
        else count_hash_pairs<LR, PPT, BLOCK, false, true>(c, g, pr, p0, B.n, hl, samp, misc);
    } else {
        if (full) count_hash_pairs<LR, PPT, BLOCK, true, false>(c, g, pr, p0, B.n, hl, samp, misc);
        else count_hash_pairs<LR, PPT, BLOCK, false, false>(c, g, pr, p0, B.n, hl, samp, misc);
    }
    __syncthreads();
    const uint32_t ns = misc[0];
    const bool direct = ns > g.scap;
    if (!direct) {
        // one thread per (sampled pair, row)
        const uint32_t seav_base = (uint32_t)c.ldca_bits;
        for (uint32_t w = tid; w < ns * c.sr; w += BLOCK) {
            const uint32_t e = w / c.sr, r = w - e * c.sr;
            const uint32_t bit = seav_base + seav_byte_l(samp[2 * e], r, rl, c) * 8u + samp[2 * e + 1];
            atomicAdd(&hs[bit >> g.S], 1u);
        }
        __syncthreads();
    }
    uint32_t *co = cnt + (uint64_t)tile * nb;
    for (uint32_t b = tid; b < nb; b += BLOCK) co[b] = hl[b] + (direct ? 0u : hs[b]);
}

// Bit addresses of a tile's pairs placed straight into their bucket's segment of the stage: the
// cursors start at the segment bases, so the returning LDS atomic gives the final position.  All
// of a lane's LDCA bit addresses are computed first and all their atomics issued together, so the
// LDS round trips overlap; sampled pairs (about one in 2^tau) follow.
template <int LR, int PPT, int BLOCK, bool FULL>
__device__ __forceinline__ void place_hash_pairs(const Consts &c, const RowLds &rl, const BinGeometry &g, const SlotPtrs &S,
                                                 const u32x2 (&pr)[PPT], uint64_t p0, uint64_t n, uint32_t *cur,
                                                 uint32_t *stage, uint32_t *samp, uint32_t *nsamp) {
    const uint32_t tid = threadIdx.x;
    // pairs in chunks of CH: a chunk's LR * CH atomics are in flight together
    constexpr int CH = PPT < 4 ? PPT : 4;
#pragma unroll
    for (int j0 = 0; j0 < PPT; j0 += CH) {
        uint32_t bits[CH * LR], pos[CH * LR];
        uint32_t valid = 0;
#pragma unroll
        for (int jj = 0; jj < CH; ++jj) {
            const int j = j0 + jj;
            const bool v = FULL || p0 + (uint64_t)j * BLOCK + tid < n;
            valid |= (uint32_t)v << jj;
            const uint32_t hip = pr[j].x, oip = pr[j].y;
            const uint32_t q = ldc_bit(oip, c);
#pragma unroll
            for (int r = 0; r < LR; ++r) bits[jj * LR + r] = ldca_bit((uint32_t)r, ldc_col(hip, (uint32_t)r, c), q, c);
            if (v && sampled(oip, c)) {   // staged; placed by the whole workgroup later
                const uint32_t e = atomicAdd(nsamp, 1u);
                const uint32_t b = se_bit(oip, c);
                if (e < g.scap) {
                    samp[2 * e] = hip;
                    samp[2 * e + 1] = b;
                } else {
                    // only a tile whose SEAV items were left out of the counts gets here
                    uint32_t *seav_w = reinterpret_cast<uint32_t *>(S.seav);
                    for (uint32_t r = 0; r < c.sr; ++r) {
                        const uint32_t bit = seav_byte_l(hip, r, rl, c) * 8u + b;
                        global_or(seav_w + (bit >> 5), 1u << (bit & 31u));
                    }
                }
            }
        }
#pragma unroll
        for (int k = 0; k < CH * LR; ++k)
            pos[k] = (FULL || ((valid >> (k / LR)) & 1u)) ? atomicAdd(&cur[bits[k] >> g.S], 1u) : 0u;
#pragma unroll
        for (int k = 0; k < CH * LR; ++k)
            if (FULL || ((valid >> (k / LR)) & 1u)) stage[pos[k]] = bits[k];
    }
}

// Bucket-major binning (after k_count and the offset scans): a workgroup re-reads a tile, builds
// its padded segment bases from the tile's exact counts (cnt[tile]), places every item directly
// at its final position in an LDS stage, pads each segment to whole 64-bit words with copies of
// its last item, and writes segment b to global item offset off[tile][b].  A tile whose SEAV
// items were left out of the counts (more sampled pairs than the stage reserves) records them with
// global atomics instead, exactly as k_count decided.
template <int LR, int PPT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_place(Consts c, BinGeometry g, BatchList bl, SlotTable st, ChunkTable ct,
                                                 uint64_t *__restrict__ items, const uint32_t *__restrict__ cnt,
                                                 const uint32_t *__restrict__ off, const uint32_t *__restrict__ cstart) {
    extern __shared__ uint32_t lds[];
    __shared__ RowLds rl;   // read after the first barrier
    rows_to_lds(rl, c);
    const uint32_t nb = g.nb;
    uint32_t *cur = lds;                 // [nb + 1] padded counts, then cursors, then global offsets
    uint32_t *lb = cur + (nb + 1);       // [nb + 1] segment bases in the stage; lb[nb] = padded total
    uint32_t *stage = lds + ((2 * (nb + 1) + 3) & ~3u);   // [cap]
    uint32_t *misc = stage + g.cap;      // [0..16] scan scratch, [17] sampled pairs
    uint32_t *samp = misc + 18;          // [2 * scap] sampled (hip, H2 bit)
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = xcd_contiguous(blockIdx.x, gridDim.x);   // neighbouring tiles on one XCD
    const BatchDesc B = bl.b[find_batch(bl, tile)];   // descriptors in device memory
    const SlotPtrs S = st.s[B.slot];
    const uint64_t p0 = (uint64_t)(tile - B.first_tile) * (uint64_t)(PPT * BLOCK);

    // counts and global offsets of this tile (two per thread held in registers), and the pairs:
    // every load is issued before the first wait
    // this tile's offset of bucket b = its offset inside its chunk + the chunk's start
    const uint32_t chunk = ct.cbase[B.slot] + (tile - ct.lo[B.slot]) / kChunk;
    const uint32_t *ctr = cnt + (uint64_t)tile * nb;
    const uint32_t *ot = off + (uint64_t)tile * nb;
    const uint32_t *cs0 = cstart + (uint64_t)chunk * nb;
    // (the two parts of an offset are added where they are used, so no wait comes before the pairs)
    uint32_t c_pre[2] = {0u, 0u}, o_pre[2] = {0u, 0u}, s_pre[2] = {0u, 0u};
    if (tid < nb) {
        c_pre[0] = ctr[tid];
        o_pre[0] = ot[tid];
        s_pre[0] = cs0[tid];
    }
    if (tid + BLOCK < nb) {
        c_pre[1] = ctr[tid + BLOCK];
        o_pre[1] = ot[tid + BLOCK];
        s_pre[1] = cs0[tid + BLOCK];
    }
    const u32x2 *pairs = reinterpret_cast<const u32x2 *>(B.pairs);
    const uint64_t last = B.n - 1;
    u32x2 pr[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint64_t idx = p0 + (uint64_t)j * BLOCK + tid;
        pr[j] = load_pair(pairs, idx < B.n ? idx : last, B.swap);
    }
    for (uint32_t b = tid, m = 0; b < nb; b += BLOCK, ++m) {
        const uint32_t v = m == 0 ? c_pre[0] : m == 1 ? c_pre[1] : ctr[b];
        cur[b] = (v + 2) / 3 * 3;
        lb[b] = 0;
    }
    if (tid == 0) {
        cur[nb] = lb[nb] = 0;
        misc[17] = 0;
    }
    __syncthreads();
    // exclusive scan of the padded counts (lb is all zero: bucket_offsets adds cur[b] + lb[b])
    bucket_offsets<BLOCK>(cur, lb, nb, misc);
    // bucket_offsets leaves cur[b] = base, lb[b] = base + padded count (= the next base)
    for (uint32_t b = tid; b <= nb; b += BLOCK) {
        const uint32_t base = cur[b];
        lb[b] = base;
    }
    __syncthreads();
    const bool seav_direct = lb[nb] == lb[g.nb_ldca];   // no SEAV items were counted for this tile
    if (p0 + (uint64_t)(PPT * BLOCK) <= B.n)
        place_hash_pairs<LR, PPT, BLOCK, true>(c, rl, g, S, pr, p0, B.n, cur, stage, samp, misc + 17);
    else
        place_hash_pairs<LR, PPT, BLOCK, false>(c, rl, g, S, pr, p0, B.n, cur, stage, samp, misc + 17);
    __syncthreads();
    // the staged sampled pairs: one thread per (pair, row)
    {
        const uint32_t ns = misc[17] < g.scap ? misc[17] : g.scap;
        const uint32_t seav_base = (uint32_t)c.ldca_bits;
        uint32_t *seav_w = reinterpret_cast<uint32_t *>(S.seav);
        for (uint32_t w = tid; w < ns * c.sr; w += BLOCK) {
            const uint32_t e = w / c.sr, r = w - e * c.sr;
            const uint32_t byte = seav_byte_l(samp[2 * e], r, rl, c), b = samp[2 * e + 1];
            if (seav_direct) {
                const uint32_t bit = byte * 8u + b;
                global_or(seav_w + (bit >> 5), 1u << (bit & 31u));
            } else {
                const uint32_t bit = seav_base + byte * 8u + b;
                stage[atomicAdd(&cur[bit >> g.S], 1u)] = bit;
            }
        }
    }
    __syncthreads();
    // pad every segment to whole words with its last item; cur[b] becomes the distance in words
    // from the segment's place in the stage to its place in the item buffer
    for (uint32_t b = tid, m = 0; b < nb; b += BLOCK, ++m) {
        const uint32_t e = cur[b], s0 = lb[b], pe = lb[b + 1];
        if (e > s0)
            for (uint32_t p = e; p < pe; ++p) stage[p] = stage[e - 1];
        cur[b] = (m == 0 ? o_pre[0] + s_pre[0] : m == 1 ? o_pre[1] + s_pre[1] : ot[b] + cs0[b]) / 3 - s0 / 3;
    }
    __syncthreads();
    // one thread per stage word: the stage holds full bit addresses, so a word's first item names
    // its bucket; three 21-bit offsets per 64-bit word
    const uint32_t smask = (1u << g.S) - 1u;
    const uint32_t nwords = lb[nb] / 3;
    for (uint32_t w = tid; w < nwords; w += BLOCK) {
        const uint32_t s0 = stage[3 * w], s1 = stage[3 * w + 1], s2 = stage[3 * w + 2];
        items[w + cur[s0 >> g.S]] =
            (uint64_t)(s0 & smask) | ((uint64_t)(s1 & smask) << 21) | ((uint64_t)(s2 & smask) << 42);
    }
}

template <int LR, int PPT, int BLOCK>
static void launch_bin_t(int kind, const Consts &c, const BinGeometry &g, const BatchTable &bt, const BatchList &bl,
                         const SlotTable &st, const ClearList &clr, const ChunkTable &ct, const uint32_t *cstart,
                         uint32_t n_tiles, uint32_t *items, uint32_t *meta, const uint32_t *off, hipStream_t s) {
    if (kind == 0)
        hipLaunchKernelGGL((k_bin<LR, PPT, BLOCK>), dim3(n_tiles), dim3(BLOCK), g.lds_bytes, s, c, g, bt, st, items, meta);
    else if (kind == 1)
        hipLaunchKernelGGL((k_place<LR, PPT, BLOCK>), dim3(n_tiles), dim3(BLOCK), g.lds_bytes, s, c, g, bl, st, ct,
                           reinterpret_cast<uint64_t *>(items), meta, off, cstart);
    else
        hipLaunchKernelGGL((k_count<LR, PPT, BLOCK>), dim3(n_tiles), dim3(BLOCK), (2 * g.nb + 1 + 2 * g.scap) * 4u, s, c,
                           g, bl, clr, meta);
}

template <int LR>
static hipError_t launch_bin_lr(int kind, const Consts &c, const BinGeometry &g, const BatchTable &bt,
                                const BatchList &bl, const SlotTable &st, const ClearList &clr, const ChunkTable &ct,
                                const uint32_t *cstart, uint32_t n_tiles, uint32_t *items, uint32_t *meta,
                                const uint32_t *off, hipStream_t s) {
    const uint32_t ppt = g.tile_pairs / g.block;
#define SPD_BIN_CASE(B, P) \
    else if (g.block == B && ppt == P)                                                                             \
        launch_bin_t<LR, P, B>(kind, c, g, bt, bl, st, clr, ct, cstart, n_tiles, items, meta, off, s);
    if (false) {
    }
    SPD_BIN_CASE(1024, 16) SPD_BIN_CASE(1024, 8) SPD_BIN_CASE(1024, 4) SPD_BIN_CASE(512, 16) SPD_BIN_CASE(512, 8)
    SPD_BIN_CASE(512, 4) SPD_BIN_CASE(256, 16) SPD_BIN_CASE(256, 8)
#undef SPD_BIN_CASE
    else return hipErrorInvalidConfiguration;
    return hipGetLastError();
}

// kind: 0 = k_bin (tile regions; batches by value, at most kMaxGroup), 1 = k_place (bucket-major),
// 2 = k_count (both: batches in device memory, any number)
static hipError_t launch_bin_kind(int kind, const Consts &c, const BinGeometry &g, const BatchDesc *batches,
                                  uint32_t n_batches, uint32_t n_tiles, uint32_t *items, uint32_t *meta,
                                  const uint32_t *off, const SlotPtrs *slots, const ClearList *clear,
                                  const ChunkTable *chunks, const uint32_t *cstart, hipStream_t s) {
    ClearList clr{};
    if (clear) clr = *clear;
    ChunkTable ct{};
    if (chunks) ct = *chunks;
    BatchTable bt{};
    BatchList bl{};
    SlotTable st{};
    if (n_batches == 0) return hipErrorInvalidValue;
    if (kind == 0) {
        if (n_batches > (uint32_t)kMaxGroup) return hipErrorInvalidValue;
        for (uint32_t i = 0; i < n_batches; ++i) bt.b[i] = batches[i];
        bt.n = n_batches;
    } else {
        bl.b = batches;
        bl.n = n_batches;
    }
    if (slots)
        for (int i = 0; i < kMaxGroup; ++i) st.s[i] = slots[i];
    switch (c.lr) {
    case 1: return launch_bin_lr<1>(kind, c, g, bt, bl, st, clr, ct, cstart, n_tiles, items, meta, off, s);
    case 2: return launch_bin_lr<2>(kind, c, g, bt, bl, st, clr, ct, cstart, n_tiles, items, meta, off, s);
    case 3: return launch_bin_lr<3>(kind, c, g, bt, bl, st, clr, ct, cstart, n_tiles, items, meta, off, s);
    case 4: return launch_bin_lr<4>(kind, c, g, bt, bl, st, clr, ct, cstart, n_tiles, items, meta, off, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_bin(const Consts &c, const BinGeometry &g, const BatchDesc *batches, uint32_t n_batches,
                      uint32_t n_tiles, uint32_t *items, uint32_t *meta, const SlotPtrs *slots, hipStream_t s) {
    return launch_bin_kind(0, c, g, batches, n_batches, n_tiles, items, meta, nullptr, slots, nullptr, nullptr, nullptr, s);
}

hipError_t launch_place(const Consts &c, const BinGeometry &g, const BatchDesc *batches_dev, uint32_t n_batches,
                        uint32_t n_tiles, uint32_t *items, const uint32_t *cnt, const uint32_t *loc,
                        const uint32_t *cstart, const ChunkTable &ct, const SlotPtrs *slots, hipStream_t s) {
    return launch_bin_kind(1, c, g, batches_dev, n_batches, n_tiles, items, const_cast<uint32_t *>(cnt), loc, slots,
                           nullptr, &ct, cstart, s);
}

hipError_t launch_count(const Consts &c, const BinGeometry &g, const BatchDesc *batches_dev, uint32_t n_batches,
                        uint32_t n_tiles, uint32_t *cnt, const ClearList &clear, hipStream_t s) {
    return launch_bin_kind(2, c, g, batches_dev, n_batches, n_tiles, nullptr, cnt, nullptr, nullptr, &clear, nullptr,
                           nullptr, s);
}

// ---- region layout (one pass over the pairs)

// A tile's items binned in LDS as in k_bin (ranks per bucket, then segment bases), with each
// bucket's segment padded to whole 64-bit words (copies of its last item).  Each non-empty segment
// takes room in its (chunk, bucket) region with one atomic; the atomics are issued before the
// items are placed in the stage, so their round trip overlaps that work.  The stage holds full
// bit addresses, so a stage word's first item names its bucket at write-out, and the last two
// places of each segment are first filled with an address of another bucket: those still holding
// it after placement are the padding.
template <int LR, int PPT, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_region(Consts c, BinGeometry g, BatchList bl, SlotTable st, ChunkTable ct,
                                                  RegionArgs ra) {
    extern __shared__ uint32_t lds[];
    __shared__ RowLds rl;   // read after the first barrier
    rows_to_lds(rl, c);
    const uint32_t nb = g.nb;
    uint32_t *cl = lds;                  // [nb + 1] LDCA counts, then padded counts, then bases
    uint32_t *cs = cl + (nb + 1);        // [nb + 1] SEAV counts, then SEAV cursors
    uint32_t *stage = lds + ((2 * (nb + 1) + 3) & ~3u);   // [cap] full bit addresses, bucket-major
    uint32_t *samp = stage + g.cap;      // [2 * scap] sampled (hip, H2 bit)
    uint32_t *misc = samp + 2 * g.scap;  // [0] sampled count, [1..17] scan scratch
    const uint32_t tid = threadIdx.x;
    const uint32_t tile = xcd_contiguous(blockIdx.x, gridDim.x);   // neighbouring tiles on one XCD
    const BatchDesc B = batch_of(bl, tile);
    const SlotPtrs S = st.s[B.slot];
    const uint64_t p0 = (uint64_t)(tile - B.first_tile) * (uint64_t)(PPT * BLOCK);
    const uint32_t cc = (tile - ct.lo[B.slot]) / kChunk, chunk = ct.cbase[B.slot] + cc;
    const uint32_t seav_base = (uint32_t)c.ldca_bits;   // SEAV bits follow the LDCA bits

    for (uint32_t i = tid; i < 2 * (nb + 1); i += BLOCK) cl[i] = 0;
    if (tid == 0) misc[0] = 0;
    const u32x2 *pairs = reinterpret_cast<const u32x2 *>(B.pairs);
    const uint64_t last = B.n - 1;
    const bool full = p0 + (uint64_t)(PPT * BLOCK) <= B.n;
    u32x2 pr[PPT];
#pragma unroll
    for (int j = 0; j < PPT; ++j) {
        const uint64_t idx = p0 + (uint64_t)j * BLOCK + tid;
        pr[j] = load_pair(pairs, idx < B.n ? idx : last, B.swap);
    }
    __syncthreads();
    uint32_t bits[PPT * LR], rk[(PPT * LR + 1) / 2];
    if (full)
        bin_hash_pairs<LR, PPT, BLOCK, true, true>(c, rl, g, S, pr, p0, B.n, cl, samp, misc, bits, rk);
    else
        bin_hash_pairs<LR, PPT, BLOCK, false, true>(c, rl, g, S, pr, p0, B.n, cl, samp, misc, bits, rk);
    __syncthreads();
    // a tile with more sampled pairs than it can stage stages none: it is listed, and the spill
    // pass records all of its sampled pairs once the apply phase has written the buckets
    uint32_t ns = misc[0];
    if (ns > g.scap) {
        if (tid == 0) {
            const uint32_t k = atomicAdd(ra.ovf_n, 1u);
            if (k < ra.ovf_cap) ra.ovf[k] = tile;
        }
        ns = 0;
    }
    for (uint32_t w = tid; w < ns * c.sr; w += BLOCK) {
        const uint32_t e = w / c.sr, r = w - e * c.sr;
        const uint32_t bit = seav_base + seav_byte_l(samp[2 * e], r, rl, c) * 8u + samp[2 * e + 1];
        atomicAdd(&cs[bit >> g.S], 1u);
    }
    __syncthreads();
    // padded counts (whole words); bucket_offsets then leaves cl[b] = cs[b] = segment base
    for (uint32_t b = tid; b < nb; b += BLOCK) {
        const uint32_t n = cl[b] + cs[b];
        cl[b] = 0;
        cs[b] = (n + 2) / 3 * 3;
    }
    __syncthreads();
    bucket_offsets<BLOCK>(cl, cs, nb, misc + 1);
    // room in the regions (the offsets of a thread's first two buckets stay in flight), and the
    // padding marks
    // (two named registers: an array indexed by the loop counter would live in scratch memory)
    uint32_t *rcur = ra.cur + (uint64_t)chunk * nb;
    uint32_t o_pre0 = 0u, o_pre1 = 0u;
    for (uint32_t b = tid, m = 0; b < nb; b += BLOCK, ++m) {
        const uint32_t s0 = cl[b], pe = cl[b + 1];
        if (pe > s0) {
            if (m == 0) o_pre0 = atomicAdd(rcur + b, (pe - s0) / 3);
            else if (m == 1) o_pre1 = atomicAdd(rcur + b, (pe - s0) / 3);
            stage[pe - 2] = stage[pe - 1] = (b ^ 1u) << g.S;
        }
    }
    __syncthreads();
    if (full) {   // every lane's items are valid
#pragma unroll
        for (int k = 0; k < PPT * LR; ++k)
            stage[cl[bits[k] >> g.S] + ((rk[k / 2] >> (16 * (k & 1))) & 0xFFFFu)] = bits[k];
    } else {
#pragma unroll
        for (int k = 0; k < PPT * LR; ++k) {
            const uint32_t rank = (rk[k / 2] >> (16 * (k & 1))) & 0xFFFFu;
            if (rank != 0xFFFFu) stage[cl[bits[k] >> g.S] + rank] = bits[k];
        }
    }
    for (uint32_t w = tid; w < ns * c.sr; w += BLOCK) {
        const uint32_t e = w / c.sr, r = w - e * c.sr;
        const uint32_t bit = seav_base + seav_byte_l(samp[2 * e], r, rl, c) * 8u + samp[2 * e + 1];
        stage[atomicAdd(&cs[bit >> g.S], 1u)] = bit;
    }
    __syncthreads();
    // pad every segment with its last item (the room of a thread's buckets past its first two is
    // taken here, its offset kept in cs)
    for (uint32_t b = tid, m = 0; b < nb; b += BLOCK, ++m) {
        const uint32_t s0 = cl[b], pe = cl[b + 1];
        if (pe > s0) {
            if ((stage[pe - 2] >> g.S) != b) stage[pe - 2] = stage[pe - 3];
            if ((stage[pe - 1] >> g.S) != b) stage[pe - 1] = stage[pe - 2];
            if (m >= 2) cs[b] = atomicAdd(rcur + b, (pe - s0) / 3);
        }
    }
    __syncthreads();
    // per bucket, in stage words: cl[b] = the first word past the region's room, cs[b] = the
    // distance from a word's place in the stage to its place among the chunk's regions
    for (uint32_t b = tid, m = 0; b < nb; b += BLOCK, ++m) {
        const uint32_t w0 = cl[b] / 3, o = m == 0 ? o_pre0 : m == 1 ? o_pre1 : cs[b];
        uint32_t capw;
        const uint32_t in = region_in(ra, g.nb_ldca, B.slot, cc, b, &capw);
        cl[b] = w0 + (o < capw ? capw - o : 0u);
        cs[b] = in + o - w0;
    }
    __syncthreads();
    // one thread per stage word: three 21-bit offsets per 64-bit word
    const uint32_t smask = (1u << g.S) - 1u;
    const uint32_t nwords = cl[nb] / 3;
    uint64_t *dst = ra.items + chunk_at(ra, B.slot, cc);
    for (uint32_t w = tid; w < nwords; w += BLOCK) {
        const uint32_t s0 = stage[3 * w], s1 = stage[3 * w + 1], s2 = stage[3 * w + 2];
        const uint32_t b = s0 >> g.S;
        const uint32_t lo = (s0 & smask) | (s1 << 21), hi = ((s1 & smask) >> 11) | ((s2 & smask) << 10);
        const uint64_t v = (uint64_t)lo | ((uint64_t)hi << 32);
        if (w < cl[b]) {
            dst[w + cs[b]] = v;
        } else {
            const uint32_t k = atomicAdd(ra.spill_n, 1u);
            if (k < ra.spill_cap) {
                ra.spill_w[k] = v;
                ra.spill_tag[k] = (B.slot << 16) | b;
            }
        }
    }
}

template <int LR>
static hipError_t launch_region_lr(const Consts &c, const BinGeometry &g, const BatchList &bl, const SlotTable &st,
                                   const ChunkTable &ct, const RegionArgs &ra, uint32_t n_tiles, hipStream_t s,
                                   KTiming kt) {
    const uint32_t ppt = g.tile_pairs / g.block;
#define SPD_RG_CASE(B, P)                                                                                        \
    else if (g.block == B && ppt == P)                                                                         \
        hipExtLaunchKernelGGL((k_region<LR, P, B>), dim3(n_tiles), dim3(B), g.lds_bytes, s, kt.start, kt.stop, 0, c, g, \
                              bl, st, ct, ra);
    if (false) {
    }
    SPD_RG_CASE(1024, 16) SPD_RG_CASE(1024, 8) SPD_RG_CASE(1024, 4) SPD_RG_CASE(512, 16) SPD_RG_CASE(512, 8)
    SPD_RG_CASE(512, 4) SPD_RG_CASE(256, 16) SPD_RG_CASE(256, 8)
#undef SPD_RG_CASE
    else return hipErrorInvalidConfiguration;
    return hipGetLastError();
}

hipError_t launch_region(const Consts &c, const BinGeometry &g, const BatchList &bl, uint32_t n_tiles,
                         const ChunkTable &ct, const SlotPtrs *slots, const RegionArgs &ra, hipStream_t s, KTiming kt) {
    if (bl.n == 0 || n_tiles == 0 || (!bl.b && bl.n > kInlineBatches)) return hipErrorInvalidValue;
    SlotTable st{};
    for (uint32_t i = 0; i < ct.n; ++i) st.s[i] = slots[i];
    switch (c.lr) {
    case 1: return launch_region_lr<1>(c, g, bl, st, ct, ra, n_tiles, s, kt);
    case 2: return launch_region_lr<2>(c, g, bl, st, ct, ra, n_tiles, s, kt);
    case 3: return launch_region_lr<3>(c, g, bl, st, ct, ra, n_tiles, s, kt);
    case 4: return launch_region_lr<4>(c, g, bl, st, ct, ra, n_tiles, s, kt);
    default: return hipErrorInvalidValue;
    }
}

// Zeroes every buffer of a clear list (16-byte stores over the whole grid).
__global__ __launch_bounds__(256) void k_clear(ClearList clr) {
    const uint64_t gt = (uint64_t)blockIdx.x * 256 + threadIdx.x, stride = (uint64_t)gridDim.x * 256;
    for (uint32_t k = 0; k < clr.n; ++k) {
        u32x4 *p4 = reinterpret_cast<u32x4 *>(clr.p[k]);
        for (uint64_t w = gt; w < clr.words[k] / 4; w += stride) p4[w] = u32x4{0u, 0u, 0u, 0u};
    }
}

hipError_t launch_clear(const ClearList &clear, hipStream_t s) {
    uint64_t words = 0;
    for (uint32_t k = 0; k < clear.n; ++k) {
        if (clear.words[k] % 4 || reinterpret_cast<uintptr_t>(clear.p[k]) % 16) return hipErrorInvalidValue;
        words += clear.words[k];
    }
    if (words == 0) return hipSuccess;
    // about eight 16-byte stores per lane: few waves to launch
    const uint64_t want = (words / 4 + 2047) / 2048;
    const uint32_t grid = (uint32_t)(want < 1024 ? (want ? want : 1) : 1024);
    hipLaunchKernelGGL(k_clear, dim3(grid), dim3(256), 0, s, clear);
    return hipGetLastError();
}

// Apply phase of the region layout: one workgroup per (slot, bucket) ORs the used part of the
// bucket's region in each of the slot's chunks into an LDS bitmap.  Work is split into pieces of
// 64 * U words (one per wavefront at a time); a piece past its region's fill is skipped.
// Bucket b of slot si: loaded into the LDS bitmap bm (zero for a fresh slot: nothing but the
// spill pass, which runs after this, writes a slot's memory during a launch), the
// filled part of the bucket's region in every chunk of the slot applied with LDS atomicOr, the
// region counters read zeroed for the next launch, the bitmap stored back.  Ends with bm complete
// and visible to the whole workgroup.
template <int BLOCK, int U>
__device__ __forceinline__ void apply_bucket(const BinGeometry &g, const ApplySlot &A, uint32_t si, uint32_t b,
                                             const ChunkTable &ct, const RegionArgs &ra, uint32_t *bm) {
    constexpr uint32_t NW = BLOCK / 64, PIECE = 64 * U;
    const uint32_t words = 1u << (g.S - 5);
    const uint32_t tid = threadIdx.x, lane = tid & 63u;
    const uint32_t wid = __builtin_amdgcn_readfirstlane(tid >> 6);
    uint32_t *dst = b < g.nb_ldca ? A.ldca + (uint64_t)b * words : A.seav_w + (uint64_t)(b - g.nb_ldca) * words;
    if (A.fresh) {
        for (uint32_t w = tid; w < words; w += BLOCK) bm[w] = 0;
    } else {
        for (uint32_t w = tid; w < words; w += BLOCK) bm[w] = dst[w];
    }
    __syncthreads();
    const uint32_t c0 = ct.cbase[si], nch = ct.cbase[si + 1] - c0;
    uint32_t capw;
    (void)region_in(ra, g.nb_ldca, si, 0, b, &capw);   // the largest capacity of the slot's chunks
    const uint32_t ppc = (capw + PIECE - 1) / PIECE;
    for (uint32_t u = wid; u < nch * ppc; u += NW) {
        const uint32_t cc = u / ppc, w0 = (u - cc * ppc) * PIECE;
        uint32_t cap_c;
        const uint64_t at = chunk_at(ra, si, cc) + region_in(ra, g.nb_ldca, si, cc, b, &cap_c);
        uint32_t len = ra.cur[(uint64_t)(c0 + cc) * g.nb + b];
        len = len < cap_c ? len : cap_c;
        if (w0 >= len) continue;
        const uint64_t *src = ra.items + at;
        uint64_t v[U];
#pragma unroll
        for (uint32_t k = 0; k < U; ++k) {
            const uint32_t ww = w0 + k * 64 + lane;
            v[k] = __builtin_nontemporal_load(src + (ww < len ? ww : len - 1));   // unconditional loads
        }
#pragma unroll
        for (uint32_t k = 0; k < U; ++k) {
            if (w0 + k * 64 + lane >= len) continue;
#pragma unroll
            for (uint32_t f = 0; f < 3; ++f) {
                const uint32_t it = (uint32_t)(v[k] >> (21 * f)) & 0x1FFFFFu;
                atomicOr(&bm[it >> 5], 1u << (it & 31u));
            }
        }
    }
    __syncthreads();
    // the region counters of this (slot, bucket) start the next launch at zero
    for (uint32_t cc = tid; cc < nch; cc += BLOCK) ra.cur[(uint64_t)(c0 + cc) * g.nb + b] = 0u;
    const uint32_t words4 = words / 4;
    if (words4) {
        for (uint32_t w = tid; w < words4; w += BLOCK)
            reinterpret_cast<u32x4 *>(dst)[w] = reinterpret_cast<const u32x4 *>(bm)[w];
    } else {
        for (uint32_t w = tid; w < words; w += BLOCK) dst[w] = bm[w];
    }
}

// One workgroup per (slot, bucket).
template <int BLOCK, int U>
__global__ __launch_bounds__(BLOCK) void k_apply_rg(BinGeometry g, ApplyTable at, ChunkTable ct, RegionArgs ra) {
    extern __shared__ uint32_t bm[];
    const uint32_t blk = blockIdx.x;
    const uint32_t si = blk / g.nb, b = blk % g.nb;
    apply_bucket<BLOCK, U>(g, at.s[si], si, b, ct, ra, bm);
}

// The same with the router OR merge fused in (Section 4.2): one workgroup per bucket applies the
// bucket of every slot of the launch in turn and keeps their OR in registers (a 2^S-bit bucket is
// 32 words per lane of 1024), then writes it to the global sketch's bucket.  The global's previous
// content is replaced.
template <int U>
__global__ __launch_bounds__(1024) void k_apply_rg_merge(BinGeometry g, ApplyTable at, uint32_t n_slots, ChunkTable ct,
                                                         RegionArgs ra, ApplySlot gs) {
    extern __shared__ uint32_t bm[];
    constexpr uint32_t BLOCK = 1024, PER = 32;   // words per lane of a 2^20-bit bucket
    const uint32_t words = 1u << (g.S - 5);
    const uint32_t tid = threadIdx.x, b = blockIdx.x;
    uint32_t acc[PER];
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k) acc[k] = 0;
    for (uint32_t si = 0; si < n_slots; ++si) {
        apply_bucket<BLOCK, U>(g, at.s[si], si, b, ct, ra, bm);
#pragma unroll
        for (uint32_t k = 0; k < PER; ++k)
            if (k * BLOCK + tid < words) acc[k] |= bm[k * BLOCK + tid];
        __syncthreads();   // every lane has read bm before the next slot's bucket overwrites it
    }
    uint32_t *dst = b < g.nb_ldca ? gs.ldca + (uint64_t)b * words : gs.seav_w + (uint64_t)(b - g.nb_ldca) * words;
#pragma unroll
    for (uint32_t k = 0; k < PER; ++k)
        if (k * BLOCK + tid < words) dst[k * BLOCK + tid] = acc[k];
}

template <int U>
static void launch_apply_rg_u(const BinGeometry &g, const ApplyTable &at, const ChunkTable &ct, const RegionArgs &ra,
                              dim3 grid, uint32_t lds, uint32_t block, hipStream_t s, KTiming kt) {
    if (block == 1024)
        hipExtLaunchKernelGGL((k_apply_rg<1024, U>), grid, dim3(1024), lds, s, kt.start, kt.stop, 0, g, at, ct, ra);
    else if (block == 512)
        hipExtLaunchKernelGGL((k_apply_rg<512, U>), grid, dim3(512), lds, s, kt.start, kt.stop, 0, g, at, ct, ra);
    else hipExtLaunchKernelGGL((k_apply_rg<256, U>), grid, dim3(256), lds, s, kt.start, kt.stop, 0, g, at, ct, ra);
}

hipError_t launch_apply_rg(const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots, const ChunkTable &ct,
                           const RegionArgs &ra, uint32_t block, uint32_t unroll, hipStream_t s, KTiming kt) {
    ApplyTable at{};
    if (n_slots == 0 || n_slots > (uint32_t)kMaxGroup || ct.n != n_slots) return hipErrorInvalidValue;
    if (block != 1024 && block != 512 && block != 256) return hipErrorInvalidConfiguration;
    for (uint32_t i = 0; i < n_slots; ++i) at.s[i] = slots[i];
    const uint32_t lds = (1u << (g.S - 5)) * 4u;
    dim3 grid(n_slots * g.nb);
    switch (unroll) {
    case 8: launch_apply_rg_u<4>(g, at, ct, ra, grid, lds, block, s, kt); break;
    case 16: launch_apply_rg_u<8>(g, at, ct, ra, grid, lds, block, s, kt); break;
    case 32: launch_apply_rg_u<16>(g, at, ct, ra, grid, lds, block, s, kt); break;
    default: return hipErrorInvalidConfiguration;
    }
    return hipGetLastError();
}

hipError_t launch_apply_rg_merge(const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots, const ChunkTable &ct,
                                 const RegionArgs &ra, const ApplySlot &global, uint32_t unroll, hipStream_t s,
                                 KTiming kt) {
    ApplyTable at{};
    if (n_slots == 0 || n_slots > (uint32_t)kMaxGroup || ct.n != n_slots || g.S > 20) return hipErrorInvalidValue;
    for (uint32_t i = 0; i < n_slots; ++i) at.s[i] = slots[i];
    const uint32_t lds = (1u << (g.S - 5)) * 4u;
    const dim3 grid(g.nb), block(1024);
    switch (unroll) {
    case 8: hipExtLaunchKernelGGL((k_apply_rg_merge<4>), grid, block, lds, s, kt.start, kt.stop, 0, g, at, n_slots, ct, ra, global); break;
    case 16: hipExtLaunchKernelGGL((k_apply_rg_merge<8>), grid, block, lds, s, kt.start, kt.stop, 0, g, at, n_slots, ct, ra, global); break;
    case 32: hipExtLaunchKernelGGL((k_apply_rg_merge<16>), grid, block, lds, s, kt.start, kt.stop, 0, g, at, n_slots, ct, ra, global); break;
    default: return hipErrorInvalidConfiguration;
    }
    return hipGetLastError();
}

// The spill pass, once the apply phase has written every bucket back (normally nothing to do): the
// words that did not fit their region, and the sampled pairs of the tiles the binning kernel listed
// (more than a tile could stage), re-read from the batch; both recorded with global atomics.  The
// counts of consecutive launches alternate between two words each: this launch clears the next
// one's.
__global__ __launch_bounds__(256) void k_spill(Consts c, BinGeometry g, ApplyTable at, RegionArgs ra, ApplySlot gs,
                                               uint32_t also_global, BatchList bl) {
    __shared__ RowLds rl;
    __shared__ uint32_t *lp[kMaxGroup];
    __shared__ uint32_t *sp[kMaxGroup];
    rows_to_lds(rl, c);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *ra.spill_next = 0u;
        *ra.ovf_next = 0u;
    }
    if (threadIdx.x < (uint32_t)kMaxGroup) {
        lp[threadIdx.x] = at.s[threadIdx.x].ldca;
        sp[threadIdx.x] = at.s[threadIdx.x].seav_w;
    }
    __syncthreads();
    const uint32_t n0 = *ra.spill_n, n = n0 < ra.spill_cap ? n0 : ra.spill_cap;
    const uint32_t words = 1u << (g.S - 5);
    for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
        const uint64_t v = ra.spill_w[i];
        const uint32_t tag = ra.spill_tag[i], si = tag >> 16, b = tag & 0xFFFFu;
        uint32_t *dst = b < g.nb_ldca ? lp[si] + (uint64_t)b * words : sp[si] + (uint64_t)(b - g.nb_ldca) * words;
        // (with the merge fused into the apply phase, the global sketch gets the word too)
        uint32_t *gd = b < g.nb_ldca ? gs.ldca + (uint64_t)b * words : gs.seav_w + (uint64_t)(b - g.nb_ldca) * words;
#pragma unroll
        for (uint32_t f = 0; f < 3; ++f) {
            const uint32_t it = (uint32_t)(v >> (21 * f)) & 0x1FFFFFu;
            global_or(dst + (it >> 5), 1u << (it & 31u));
            if (also_global) global_or(gd + (it >> 5), 1u << (it & 31u));
        }
    }
    // listed tiles, one workgroup per tile at a time
    const uint32_t t0 = *ra.ovf_n, nt = t0 < ra.ovf_cap ? t0 : ra.ovf_cap;
    for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
        const uint32_t tile = ra.ovf[t];
        const BatchDesc B = batch_of(bl, tile);
        const uint64_t p0 = (uint64_t)(tile - B.first_tile) * g.tile_pairs;
        const uint64_t p1 = p0 + g.tile_pairs < B.n ? p0 + g.tile_pairs : B.n;
        const u32x2 *pairs = reinterpret_cast<const u32x2 *>(B.pairs);
        uint32_t *seav_w = sp[B.slot];
        for (uint64_t i = p0 + threadIdx.x; i < p1; i += 256) {
            const u32x2 pr = load_pair(pairs, i, B.swap);
            if (!sampled(pr.y, c)) continue;
            const uint32_t b = se_bit(pr.y, c);
            for (uint32_t r = 0; r < c.sr; ++r) {
                const uint32_t bit = seav_byte_l(pr.x, r, rl, c) * 8u + b;
                global_or(seav_w + (bit >> 5), 1u << (bit & 31u));
                if (also_global) global_or(gs.seav_w + (bit >> 5), 1u << (bit & 31u));
            }
        }
    }
}

hipError_t launch_spill(const Consts &c, const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots,
                        const RegionArgs &ra, const BatchList &bl, hipStream_t s, const ApplySlot *global) {
    ApplyTable at{};
    if (n_slots == 0 || n_slots > (uint32_t)kMaxGroup) return hipErrorInvalidValue;
    for (uint32_t i = 0; i < n_slots; ++i) at.s[i] = slots[i];
    const ApplySlot gs = global ? *global : ApplySlot{};
    hipLaunchKernelGGL(k_spill, dim3(32), dim3(256), 0, s, c, g, at, ra, gs, global ? 1u : 0u, bl);   // normally nothing to do
    return hipGetLastError();
}

// ---- offsets of the bucket-major layout
// Per slot, bucket b's items are the concatenation over the slot's tiles of each tile's segment
// (count rounded up to a multiple of 3: whole 64-bit words); slots follow each other per bucket:
// base[s * nb + b] = start of (slot s, bucket b).  Tiles are scanned in chunks of kChunk that
// never span two slots: k_colscan writes each (tile, bucket) offset inside its chunk and each
// chunk's total, k_chunkscan turns the chunk totals into chunk starts (base included), and
// k_place adds a tile's chunk start to its offsets.
__device__ __forceinline__ uint32_t slot_of_chunk(const ChunkTable &ct, uint32_t c) {
    uint32_t si = 0;
    while (si + 1 < ct.n && ct.cbase[si + 1] <= c) ++si;
    return si;
}

// grid (ceil(nb / 64), chunks), 256 threads: 64 buckets x 4 groups of 32 tiles
__global__ __launch_bounds__(256) void k_colscan(const uint32_t *__restrict__ cnt, uint32_t *__restrict__ loc,
                                                 uint32_t *__restrict__ csum, ChunkTable ct, uint32_t nb) {
    static_assert(kChunk == 128, "four groups of 32 tiles");
    __shared__ uint32_t ps[4][64];
    const uint32_t c = blockIdx.y;
    const uint32_t si = slot_of_chunk(ct, c);
    const uint32_t t0 = ct.lo[si] + (c - ct.cbase[si]) * kChunk;
    const uint32_t t1 = t0 + kChunk < ct.hi[si] ? t0 + kChunk : ct.hi[si];   // > t0
    const uint32_t col = threadIdx.x & 63u, rg = threadIdx.x >> 6;
    const uint32_t b = blockIdx.x * 64 + col;
    const bool okb = b < nb;
    const uint32_t bb = okb ? b : nb - 1;
    const uint32_t r0 = t0 + rg * 32;
    uint32_t v[32];
#pragma unroll
    for (uint32_t k = 0; k < 32; ++k) {   // unconditional (clamped) loads, all in flight together
        const uint32_t t = r0 + k < t1 ? r0 + k : t1 - 1;
        v[k] = cnt[(uint64_t)t * nb + bb];
    }
    uint32_t sum = 0;
#pragma unroll
    for (uint32_t k = 0; k < 32; ++k) {
        const uint32_t x = (r0 + k < t1) ? (v[k] + 2) / 3 * 3 : 0u;
        v[k] = sum;
        sum += x;
    }
    ps[rg][col] = sum;
    __syncthreads();
    uint32_t pre = 0;
    for (uint32_t r = 0; r < rg; ++r) pre += ps[r][col];
    if (okb) {
#pragma unroll
        for (uint32_t k = 0; k < 32; ++k)
            if (r0 + k < t1) loc[(uint64_t)(r0 + k) * nb + b] = pre + v[k];
        if (rg == 3) csum[(uint64_t)c * nb + b] = pre + sum;
    }
}

// One workgroup: chunk totals -> chunk starts (in place, base included); base[s * nb + b] and
// base[n * nb] = all items.
__global__ __launch_bounds__(1024) void k_chunkscan(uint32_t *__restrict__ csum, uint32_t *__restrict__ base,
                                                    ChunkTable ct, uint32_t nb) {
    __shared__ uint32_t wsum[17];
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
    const uint32_t n = ct.n * nb;
    // 1. per (slot, bucket): exclusive prefix over the slot's chunks; the total goes to base
    for (uint32_t e = tid; e < n; e += 1024) {
        const uint32_t s = e / nb, b = e - s * nb;
        uint32_t run = 0;
        for (uint32_t c0 = ct.cbase[s]; c0 < ct.cbase[s + 1]; c0 += 8) {
            uint32_t x[8];
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) x[k] = c0 + k < ct.cbase[s + 1] ? csum[(uint64_t)(c0 + k) * nb + b] : 0u;
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) {
                if (c0 + k < ct.cbase[s + 1]) csum[(uint64_t)(c0 + k) * nb + b] = run;
                run += x[k];
            }
        }
        base[e] = run;
    }
    __syncthreads();
    // 2. exclusive prefix of the (slot, bucket) totals
    uint32_t carry = 0;
    for (uint32_t i0 = 0; i0 < n; i0 += 1024) {
        const uint32_t i = i0 + tid;
        const uint32_t v = i < n ? base[i] : 0u;
        uint32_t incl = v;
        for (int o = 1; o < 64; o <<= 1) {
            uint32_t x = __shfl_up(incl, o, 64);
            if ((int)lane >= o) incl += x;
        }
        if (lane == 63u) wsum[wid] = incl;
        __syncthreads();
        if (tid == 0) {
            uint32_t run = 0;
            for (uint32_t w = 0; w < 16; ++w) {
                uint32_t x = wsum[w];
                wsum[w] = run;
                run += x;
            }
            wsum[16] = run;
        }
        __syncthreads();
        if (i < n) base[i] = carry + wsum[wid] + incl - v;
        carry += wsum[16];
        __syncthreads();
    }
    if (tid == 0) base[n] = carry;
    __syncthreads();
    // 3. chunk starts become absolute
    for (uint32_t e = tid; e < n; e += 1024) {
        const uint32_t s = e / nb, b = e - s * nb, add = base[e];
        for (uint32_t c = ct.cbase[s]; c < ct.cbase[s + 1]; ++c) csum[(uint64_t)c * nb + b] += add;
    }
}

hipError_t launch_offsets(const uint32_t *cnt, uint32_t *loc, uint32_t *csum, uint32_t *base, const ChunkTable &ct,
                          uint32_t nb, hipStream_t s) {
    if (ct.n == 0 || ct.n > (uint32_t)kMaxGroup || ct.cbase[ct.n] == 0 || ct.cbase[ct.n] > 65535u)
        return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_colscan, dim3((nb + 63) / 64, ct.cbase[ct.n]), dim3(256), 0, s, cnt, loc, csum, ct, nb);
    hipLaunchKernelGGL(k_chunkscan, dim3(1), dim3(1024), 0, s, csum, base, ct, nb);
    return hipGetLastError();
}

// Phase 2 of the bucket-major layout: one workgroup per (slot, bucket) streams the bucket's
// contiguous items (three per 64-bit word) into an LDS bitmap and writes the bucket back.
template <int BLOCK, int U>
__global__ __launch_bounds__(BLOCK) void k_apply_bm(BinGeometry g, ApplyTable at, const uint64_t *__restrict__ items,
                                                    const uint32_t *__restrict__ base) {
    // U: 8-byte loads in flight per lane
    extern __shared__ uint32_t bm[];
    const uint32_t words = 1u << (g.S - 5);
    const uint32_t tid = threadIdx.x;
    const uint32_t blk = blockIdx.x;
    const uint32_t si = blk / g.nb, b = blk % g.nb;
    const ApplySlot A = at.s[si];
    uint32_t *dst = b < g.nb_ldca ? A.ldca + (uint64_t)b * words : A.seav_w + (uint64_t)(b - g.nb_ldca) * words;
    if (A.fresh && b < g.nb_ldca) {
        for (uint32_t w = tid; w < words; w += BLOCK) bm[w] = 0;
    } else {
        for (uint32_t w = tid; w < words; w += BLOCK) bm[w] = dst[w];
    }
    __syncthreads();
    const uint32_t w0 = base[blk] / 3, w1 = base[blk + 1] / 3;
    for (uint32_t w = w0 + tid; w < w1; w += BLOCK * U) {
        uint64_t v[U];
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            const uint32_t ww = w + u * BLOCK < w1 ? w + u * BLOCK : w1 - 1;   // unconditional loads
            v[u] = __builtin_nontemporal_load(items + ww);
        }
#pragma unroll
        for (uint32_t u = 0; u < U; ++u) {
            if (w + u * BLOCK >= w1) continue;
#pragma unroll
            for (uint32_t f = 0; f < 3; ++f) {
                const uint32_t it = (uint32_t)(v[u] >> (21 * f)) & 0x1FFFFFu;
                atomicOr(&bm[it >> 5], 1u << (it & 31u));
            }
        }
    }
    __syncthreads();
    const uint32_t words4 = words / 4;
    if (words4) {
        for (uint32_t w = tid; w < words4; w += BLOCK)
            reinterpret_cast<u32x4 *>(dst)[w] = reinterpret_cast<const u32x4 *>(bm)[w];
    } else {
        for (uint32_t w = tid; w < words; w += BLOCK) dst[w] = bm[w];
    }
}

template <int U>
static void launch_apply_bm_u(const BinGeometry &g, const ApplyTable &at, dim3 grid, uint32_t lds, const uint64_t *it,
                              const uint32_t *base, uint32_t block, hipStream_t s) {
    if (block == 1024) hipLaunchKernelGGL((k_apply_bm<1024, U>), grid, dim3(1024), lds, s, g, at, it, base);
    else if (block == 512) hipLaunchKernelGGL((k_apply_bm<512, U>), grid, dim3(512), lds, s, g, at, it, base);
    else hipLaunchKernelGGL((k_apply_bm<256, U>), grid, dim3(256), lds, s, g, at, it, base);
}

hipError_t launch_apply_bm(const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots, const uint32_t *items,
                           const uint32_t *base, uint32_t block, uint32_t unroll, hipStream_t s) {
    ApplyTable at{};
    if (n_slots == 0 || n_slots > (uint32_t)kMaxGroup) return hipErrorInvalidValue;
    if (block != 1024 && block != 512 && block != 256) return hipErrorInvalidConfiguration;
    for (uint32_t i = 0; i < n_slots; ++i) at.s[i] = slots[i];
    const uint32_t lds = (1u << (g.S - 5)) * 4u;
    const uint64_t *it = reinterpret_cast<const uint64_t *>(items);
    dim3 grid(n_slots * g.nb);
    switch (unroll) {
    case 8: launch_apply_bm_u<4>(g, at, grid, lds, it, base, block, s); break;
    case 16: launch_apply_bm_u<8>(g, at, grid, lds, it, base, block, s); break;
    case 32: launch_apply_bm_u<16>(g, at, grid, lds, it, base, block, s); break;
    default: return hipErrorInvalidConfiguration;
    }
    return hipGetLastError();
}

// meta[rows][cols] -> metaT[cols][rows]
__global__ __launch_bounds__(256) void k_transpose(const uint32_t *__restrict__ in, uint32_t *__restrict__ out,
                                                   uint32_t rows, uint32_t cols) {
    __shared__ uint32_t t[32][33];
    const uint32_t bx = blockIdx.y * 32, by = blockIdx.x * 32;   // bx: column block, by: row block
    const uint32_t tx = threadIdx.x & 31u, ty = threadIdx.x >> 5;   // 32 x 8
    for (uint32_t k = ty; k < 32; k += 8) {
        uint32_t r = by + k, col = bx + tx;
        if (r < rows && col < cols) t[k][tx] = in[(uint64_t)r * cols + col];
    }
    __syncthreads();
    for (uint32_t k = ty; k < 32; k += 8) {
        uint32_t col = bx + k, r = by + tx;
        if (r < rows && col < cols) out[(uint64_t)col * rows + r] = t[tx][k];
    }
}

hipError_t launch_transpose(const uint32_t *meta, uint32_t *metaT, uint32_t rows, uint32_t cols, hipStream_t s) {
    if (rows == 0 || cols == 0 || (cols + 31) / 32 > 65535u) return hipErrorInvalidValue;
    dim3 grid((rows + 31) / 32, (cols + 31) / 32);
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, meta, metaT, rows, cols);
    return hipGetLastError();
}

constexpr uint32_t kApplyChunk = 1024;

template <int BLOCK, int U>
__global__ __launch_bounds__(BLOCK) void k_apply(BinGeometry g, ApplyTable at, const uint32_t *__restrict__ items,
                                                 const uint32_t *__restrict__ metaT, uint32_t n_tiles) {
    // U: tiles per wavefront per step, i.e. U segment loads in flight per lane
    extern __shared__ uint32_t lds[];
    constexpr uint32_t NW = BLOCK / 64;
    const uint32_t words = 1u << (g.S - 5);
    uint32_t *bm = lds;
    uint32_t *mbeg = bm + words;
    uint32_t *mend = mbeg + kApplyChunk;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wid = tid >> 6;
    const uint32_t si = blockIdx.x / g.nb, b = blockIdx.x % g.nb;
    const ApplySlot A = at.s[si];
    uint32_t *dst = b < g.nb_ldca ? A.ldca + (uint64_t)b * words : A.seav_w + (uint64_t)(b - g.nb_ldca) * words;
    // LDCA buckets of a fresh slot start from zero; SEAV buckets always start from the sketch
    // (a tile with more sampled pairs than it staged records the rest there directly)
    if (A.fresh && b < g.nb_ldca) {
        for (uint32_t w = tid; w < words; w += BLOCK) bm[w] = 0;
    } else {
        for (uint32_t w = tid; w < words; w += BLOCK) bm[w] = dst[w];
    }
    const uint64_t *items64 = reinterpret_cast<const uint64_t *>(items);
    const uint32_t region64 = g.region / 2;
    for (uint32_t t0 = A.tile_lo; t0 < A.tile_hi; t0 += kApplyChunk) {
        const uint32_t nt = A.tile_hi - t0 < kApplyChunk ? A.tile_hi - t0 : kApplyChunk;
        __syncthreads();
        for (uint32_t k = tid; k < nt; k += BLOCK) {
            mbeg[k] = metaT[(uint64_t)b * n_tiles + t0 + k];
            mend[k] = metaT[(uint64_t)(b + 1) * n_tiles + t0 + k];
        }
        __syncthreads();
        for (uint32_t k0 = wid * U; k0 < nt; k0 += NW * U) {
            uint32_t v[U];
            bool ok[U];
            // unconditional loads (lanes without an item re-read the tile's first word and are
            // masked out), so all U loads of a lane are in flight together
            uint64_t w[U];
            uint32_t f[U];
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t k = k0 + u < nt ? k0 + u : nt - 1;
                const uint32_t j = mbeg[k] + lane;
                ok[u] = (k0 + u < nt) && (j < mend[k]);
                const uint32_t jj = ok[u] ? j : 0u;
                f[u] = jj % 3;
                w[u] = items64[(uint64_t)(t0 + k) * region64 + jj / 3];
            }
#pragma unroll
            for (uint32_t u = 0; u < U; ++u) v[u] = (uint32_t)(w[u] >> (21 * f[u])) & 0x1FFFFFu;
#pragma unroll
            for (uint32_t u = 0; u < U; ++u)
                if (ok[u]) atomicOr(&bm[v[u] >> 5], 1u << (v[u] & 31u));
            // segments longer than one wavefront
            for (uint32_t u = 0; u < U; ++u) {
                const uint32_t k = k0 + u;
                if (k >= nt) break;
                const uint32_t end = mend[k];
                for (uint32_t j = mbeg[k] + 64 + lane; j < end; j += 64) {
                    const uint64_t w = items64[(uint64_t)(t0 + k) * region64 + j / 3];
                    const uint32_t it = (uint32_t)(w >> (21 * (j % 3))) & 0x1FFFFFu;
                    atomicOr(&bm[it >> 5], 1u << (it & 31u));
                }
            }
        }
    }
    __syncthreads();
    const uint32_t words4 = words / 4;
    if (words4) {
        for (uint32_t w = tid; w < words4; w += BLOCK)
            reinterpret_cast<u32x4 *>(dst)[w] = reinterpret_cast<const u32x4 *>(bm)[w];
    } else {
        for (uint32_t w = tid; w < words; w += BLOCK) dst[w] = bm[w];
    }
}

template <int U>
static hipError_t launch_apply_u(const BinGeometry &g, const ApplyTable &at, uint32_t n_slots, const uint32_t *items,
                                 const uint32_t *metaT, uint32_t n_tiles, uint32_t block, hipStream_t s) {
    uint32_t lds = ((1u << (g.S - 5)) + 2 * kApplyChunk) * 4u;
    dim3 grid(n_slots * g.nb);
    if (block == 1024) hipLaunchKernelGGL((k_apply<1024, U>), grid, dim3(1024), lds, s, g, at, items, metaT, n_tiles);
    else if (block == 512) hipLaunchKernelGGL((k_apply<512, U>), grid, dim3(512), lds, s, g, at, items, metaT, n_tiles);
    else if (block == 256) hipLaunchKernelGGL((k_apply<256, U>), grid, dim3(256), lds, s, g, at, items, metaT, n_tiles);
    else return hipErrorInvalidConfiguration;
    return hipGetLastError();
}

hipError_t launch_apply(const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots, const uint32_t *items,
                        const uint32_t *metaT, uint32_t n_tiles, uint32_t block, uint32_t unroll, hipStream_t s) {
    ApplyTable at{};
    if (n_slots == 0 || n_slots > (uint32_t)kMaxGroup) return hipErrorInvalidValue;
    for (uint32_t i = 0; i < n_slots; ++i) at.s[i] = slots[i];
    switch (unroll) {
    case 8: return launch_apply_u<8>(g, at, n_slots, items, metaT, n_tiles, block, s);
    case 16: return launch_apply_u<16>(g, at, n_slots, items, metaT, n_tiles, block, s);
    case 32: return launch_apply_u<32>(g, at, n_slots, items, metaT, n_tiles, block, s);
    default: return hipErrorInvalidConfiguration;
    }
}

// ------------------------------------------------------------------------------ merge
__global__ void k_or_merge(uint32_t *__restrict__ dst, SrcTable src, uint32_t n_src, uint64_t n_words) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t n4 = n_words / 4;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n4; i += stride) {
        u32x4 v = {0u, 0u, 0u, 0u};
        for (uint32_t k = 0; k < n_src; ++k) v |= __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(src.p[k]) + i);
        reinterpret_cast<u32x4 *>(dst)[i] = v;
    }
    for (uint64_t i = n4 * 4 + blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_words; i += stride) {
        uint32_t v = 0;
        for (uint32_t k = 0; k < n_src; ++k) v |= src.p[k][i];
        dst[i] = v;
    }
}

hipError_t launch_or_merge(uint32_t *dst, const uint32_t *const *srcp, uint32_t n_src, uint64_t n_words, hipStream_t s) {
    SrcTable src{};
    if (n_src == 0 || n_src > (uint32_t)kMaxGroup) return hipErrorInvalidValue;
    for (uint32_t i = 0; i < n_src; ++i) src.p[i] = srcp[i];
    uint64_t blocks = (n_words / 4 + 255) / 256;
    uint32_t grid = (uint32_t)(blocks < 8192 ? (blocks ? blocks : 1) : 8192);
    hipLaunchKernelGGL(k_or_merge, dim3(grid), dim3(256), 0, s, dst, src, n_src, n_words);
    return hipGetLastError();
}

__global__ void k_max_merge_u16(uint16_t *__restrict__ dst, SrcTable16 src, uint32_t n_src, uint64_t n) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        uint16_t v = 0;
        for (uint32_t k = 0; k < n_src; ++k) {
            uint16_t t = src.p[k][i];
            v = t > v ? t : v;
        }
        dst[i] = v;
    }
}

hipError_t launch_max_merge_u16(uint16_t *dst, const uint16_t *const *srcp, uint32_t n_src, uint64_t n, hipStream_t s) {
    SrcTable16 src{};
    if (n_src == 0 || n_src > (uint32_t)kMaxGroup) return hipErrorInvalidValue;
    for (uint32_t i = 0; i < n_src; ++i) src.p[i] = srcp[i];
    uint64_t blocks = (n + 255) / 256;
    uint32_t grid = (uint32_t)(blocks < 8192 ? (blocks ? blocks : 1) : 8192);
    hipLaunchKernelGGL(k_max_merge_u16, dim3(grid), dim3(256), 0, s, dst, src, n_src, n);
    return hipGetLastError();
}

// Shift every stamp down by off; stamps at or below off (outside every future window) become 0.
__global__ void k_renormalize_u16(uint16_t *__restrict__ p, uint64_t n, uint16_t off) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
        uint16_t v = p[i];
        p[i] = v > off ? (uint16_t)(v - off) : (uint16_t)0;
    }
}

hipError_t launch_renormalize_u16(uint16_t *p, uint64_t n, uint16_t off, hipStream_t s) {
    uint64_t blocks = (n + 255) / 256;
    uint32_t grid = (uint32_t)(blocks < 8192 ? (blocks ? blocks : 1) : 8192);
    hipLaunchKernelGGL(k_renormalize_u16, dim3(grid), dim3(256), 0, s, p, n, off);
    return hipGetLastError();
}

// Bit view of stamps: bit j of word w is 1 iff ts[32 w + j] >= thr.
__global__ void k_bit_view(const uint16_t *__restrict__ ts, uint64_t n_words, uint16_t thr, uint32_t *__restrict__ out) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t w = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; w < n_words; w += stride) {
        uint32_t v = 0;
        for (uint32_t j = 0; j < 32; ++j) v |= (ts[w * 32 + j] >= thr ? 1u : 0u) << j;
        out[w] = v;
    }
}

hipError_t launch_bit_view(const uint16_t *ts, uint64_t n_bits, uint16_t thr, uint32_t *out_words, hipStream_t s) {
    uint64_t n_words = n_bits / 32;
    uint64_t blocks = (n_words + 255) / 256;
    uint32_t grid = (uint32_t)(blocks < 8192 ? (blocks ? blocks : 1) : 8192);
    hipLaunchKernelGGL(k_bit_view, dim3(grid), dim3(256), 0, s, ts, n_words, thr, out_words);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------ end of window
// Bit view of the two 16-bit stamps packed in one 32-bit word (stamp j in half j).
__device__ __forceinline__ uint32_t ts_bits2(uint32_t w, uint32_t thr) {
    return ((w & 0xFFFFu) >= thr ? 1u : 0u) | ((w >> 16) >= thr ? 2u : 0u);
}

// at_active_bytes with the close's window.
__device__ __forceinline__ uint32_t at_active4(uint32_t w, const CloseArgs &a) { return at_active_bytes(w, a.at_ct, a.at_k); }

// One SEAV byte as bits.  With counters (sliding window) the end of window reads a bit view of
// the SEAV made by a streaming kernel just before it (a.seav), so every mode reads bytes here.
template <int MODE>
__device__ __forceinline__ uint32_t load_se(const CloseArgs &a, uint64_t byte) {
    return a.seav[byte];
}

// The counters behind one LDCA word (word < 2^27: a sketch has fewer than 2^32 bits), as loaded:
// 32 16-bit stamps (four 16-byte vectors) or 32 AT counters (two).
template <int MODE>
struct LdcRaw {
    u32x4 v[MODE == kCloseStamps ? 4 : 2];
};
template <int MODE>
__device__ __forceinline__ LdcRaw<MODE> load_ldc_raw(const CloseArgs &a, uint32_t word) {
    LdcRaw<MODE> r;
    const u32x4 *t = MODE == kCloseStamps ? reinterpret_cast<const u32x4 *>(a.ldca_ts + (uint64_t)word * 32)
                                          : reinterpret_cast<const u32x4 *>(a.ldca_at + (uint64_t)word * 32);
#pragma unroll
    for (uint32_t q = 0; q < (MODE == kCloseStamps ? 4u : 2u); ++q) r.v[q] = t[q];
    return r;
}
// Their bit view.
template <int MODE>
__device__ __forceinline__ uint32_t decode_ldc(const CloseArgs &a, const LdcRaw<MODE> &r) {
    uint32_t v = 0;
    if (MODE == kCloseStamps) {
#pragma unroll
        for (uint32_t q = 0; q < 4; ++q) {
            const u32x4 x = r.v[q];
            v |= (ts_bits2(x.x, a.thr) | ts_bits2(x.y, a.thr) << 2 | ts_bits2(x.z, a.thr) << 4 |
                  ts_bits2(x.w, a.thr) << 6) << (8 * q);
        }
    } else {
        // 32 counters in a fixed permuted order (counter 4h + j at bit 8j + h): the LDCs of a
        // candidate are all read the same way, so the AND of its rows and the popcount are unchanged
        const u32x4 x = r.v[0], y = r.v[1];
        v = (at_active4(x.x, a) >> 7) | (at_active4(x.y, a) >> 6) | (at_active4(x.z, a) >> 5) |
            (at_active4(x.w, a) >> 4) | (at_active4(y.x, a) >> 3) | (at_active4(y.y, a) >> 2) |
            (at_active4(y.z, a) >> 1) | at_active4(y.w, a);
    }
    return v;
}

// One LDCA word as bits.
template <int MODE>
__device__ __forceinline__ uint32_t load_ldc_word(const CloseArgs &a, uint32_t word) {
    if (MODE == kCloseBits) return a.ldca[word];
    return decode_ldc<MODE>(a, load_ldc_raw<MODE>(a, word));
}

// Orders LDS traffic between lanes of one wavefront (writes by some lanes, reads by others).
__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ULDC of every queued candidate: AND of its LR LDCs, z0 = k - popcount; report if z0 <= z_theta.
// Four candidates at a time, 16 lanes each; a lane reads 8 words of each of two LDCs before it
// waits, so one round trip to memory serves four candidates (k = 4096, LR = 2).
// Counter modes (a window of time stamps or AT counters): an LDC word is 32 counters (64 or 32
// bytes), so one candidate takes the whole wavefront: each lane reads two words of every row, all
// rows' loads in flight together (one round trip per candidate for k up to 4096).
template <int MODE>
__device__ void filter_queue_counters(const CloseArgs &a, const Consts &c, const uint32_t *queue, uint32_t qn,
                                      uint32_t lane) {
    const uint32_t words = 1u << (c.log2k - 5);
    for (uint32_t e = 0; e < qn; ++e) {
        const uint32_t h = queue[e];
        uint32_t ones = 0;
        for (uint32_t w0 = 0; w0 < words; w0 += 128) {
            const uint32_t wa = w0 + lane < words ? w0 + lane : words - 1;
            const uint32_t wb = w0 + 64 + lane < words ? w0 + 64 + lane : words - 1;
            uint32_t ua = 0xFFFFFFFFu, ub = 0xFFFFFFFFu;
            // a runtime loop over the rows keeps the decoding code small (instruction cache); AT
            // counters of two rows at a time are loaded before either is decoded (one round trip
            // per two rows; the larger 16-bit stamps go one row at a time)
            if constexpr (MODE == kCloseAt) {
                for (uint32_t r = 0; r < c.lr; r += 2) {
                    const uint32_t r1 = r + 1 < c.lr ? r + 1 : r;
                    const uint32_t b0 = ((r << c.log2lc) | ldc_col(h, r, c)) << (c.log2k - 5);
                    const uint32_t b1 = ((r1 << c.log2lc) | ldc_col(h, r1, c)) << (c.log2k - 5);
                    const LdcRaw<MODE> x0 = load_ldc_raw<MODE>(a, b0 + wa), y0 = load_ldc_raw<MODE>(a, b0 + wb);
                    const LdcRaw<MODE> x1 = load_ldc_raw<MODE>(a, b1 + wa), y1 = load_ldc_raw<MODE>(a, b1 + wb);
                    ua &= decode_ldc<MODE>(a, x0) & decode_ldc<MODE>(a, x1);
                    ub &= decode_ldc<MODE>(a, y0) & decode_ldc<MODE>(a, y1);
                }
            } else {
                for (uint32_t r = 0; r < c.lr; ++r) {
                    const uint32_t b0 = ((r << c.log2lc) | ldc_col(h, r, c)) << (c.log2k - 5);
                    ua &= load_ldc_word<MODE>(a, b0 + wa);
                    ub &= load_ldc_word<MODE>(a, b0 + wb);
                }
            }
            ones += (w0 + lane < words ? __popc(ua) : 0u) + (w0 + 64 + lane < words ? __popc(ub) : 0u);
        }
        ones = wave_sum(ones);
        const uint32_t z0 = (1u << c.log2k) - ones;
        if (lane == 0 && z0 <= c.z_theta) {
            const uint32_t slot = atomicAdd(&a.counters[0], 1u);
            if (slot < a.rec_cap) {
                a.rec[2 * slot] = h;
                a.rec[2 * slot + 1] = z0;
            }
        }
    }
}

template <int MODE>
__device__ void filter_queue(const CloseArgs &a, const Consts &c, const uint32_t *queue, uint32_t qn, uint32_t lane) {
    if (MODE != kCloseBits) {
        filter_queue_counters<MODE>(a, c, queue, qn, lane);
        return;
    }
    constexpr uint32_t G = 16, W = 8, RB = 2;
    const uint32_t words = 1u << (c.log2k - 5);
    const uint32_t grp = lane / G, sub = lane % G;
    for (uint32_t e0 = 0; e0 < qn; e0 += 64 / G) {
        const bool live = e0 + grp < qn;
        const uint32_t h = queue[live ? e0 + grp : e0];
        uint32_t ones = 0;
        for (uint32_t w0 = 0; w0 < words; w0 += G * W) {
            uint32_t u[W];
#pragma unroll
            for (uint32_t k = 0; k < W; ++k) u[k] = 0xFFFFFFFFu;
            for (uint32_t r0 = 0; r0 < c.lr; r0 += RB) {
                uint32_t v[RB][W];
#pragma unroll
                for (uint32_t rr = 0; rr < RB; ++rr) {
                    const uint32_t r = r0 + rr < c.lr ? r0 + rr : c.lr - 1;   // a repeated row is harmless
                    const uint32_t base = ((r << c.log2lc) | ldc_col(h, r, c)) << (c.log2k - 5);
#pragma unroll
                    for (uint32_t k = 0; k < W; ++k) {
                        const uint32_t w = w0 + k * G + sub;
                        v[rr][k] = load_ldc_word<MODE>(a, base + (w < words ? w : words - 1));
                    }
                }
#pragma unroll
                for (uint32_t rr = 0; rr < RB; ++rr)
#pragma unroll
                    for (uint32_t k = 0; k < W; ++k) u[k] &= v[rr][k];
            }
#pragma unroll
            for (uint32_t k = 0; k < W; ++k)
                if (w0 + k * G + sub < words) ones += __popc(u[k]);
        }
        for (uint32_t o = G / 2; o > 0; o >>= 1) ones += __shfl_xor(ones, o, 64);
        const uint32_t z0 = (1u << c.log2k) - ones;
        if (live && sub == 0 && z0 <= c.z_theta) {
            uint32_t slot = atomicAdd(&a.counters[0], 1u);
            if (slot < a.rec_cap) {
                a.rec[2 * slot] = h;
                a.rec[2 * slot + 1] = z0;
            }
        }
    }
}

template <int MODE, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(5))) void k_close(Consts c, CloseArgs a) {
    extern __shared__ uint32_t lds[];
    constexpr uint32_t NW = BLOCK / 64;
    const uint32_t lane = threadIdx.x & 63u, wid = threadIdx.x >> 6;
    const uint32_t per_wave = c.sr * a.list_stride + a.qcap + a.stage_words;
    uint32_t *lists = lds + wid * per_wave;      // row i: entries (cell << 8 | SE value)
    uint32_t *queue = lists + c.sr * a.list_stride;
    uint8_t *sea8 = reinterpret_cast<uint8_t *>(queue + a.qcap);   // the SEA of the current RP
    const bool staged = a.stage_words != 0;
    const uint64_t lane_lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const uint64_t lmask = (c.L == 32) ? 0xFFFFFFFFull : ((1ull << c.L) - 1ull);
    uint32_t n_cand = 0;
    // work items: (SEA, part); the 2^parts_log2 parts of a SEA take interleaved shares of its tuples
    // (or of its LPs), so they find disjoint candidates
    const uint32_t P = 1u << a.parts_log2, part_mask = P - 1u;
    const uint64_t n_items = (uint64_t)a.n_rp << a.parts_log2;

    for (uint64_t wi = (uint64_t)blockIdx.x * NW + wid; wi < n_items; wi += (uint64_t)gridDim.x * NW) {
        const uint32_t rp = (uint32_t)(wi >> a.parts_log2), part = (uint32_t)wi & part_mask;
        const uint64_t sea = (uint64_t)rp * c.sea_bytes;
        // stage the whole SEA in LDS (when it fits) with 32-bit loads, up to eight in flight per lane
        // (an SEA is a whole number of words, rows of 2^IBN >= 4 bytes, and so is its offset)
        auto se_at = [&](uint32_t byte) -> uint32_t { return staged ? sea8[byte] : load_se<MODE>(a, sea + byte); };
        const uint32_t sea_words = c.sea_bytes >> 2;
        const uint32_t *sea32 = reinterpret_cast<const uint32_t *>(a.seav + sea);
        uint32_t *stage32 = reinterpret_cast<uint32_t *>(sea8);
        for (uint32_t w0 = 0; staged && w0 < sea_words; w0 += 64 * 8) {
            uint32_t v[8];
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k) {
                const uint32_t w = w0 + k * 64 + lane;
                v[k] = w0 + k * 64 < sea_words ? sea32[w < sea_words ? w : sea_words - 1] : 0u;
            }
#pragma unroll
            for (uint32_t k = 0; k < 8; ++k)
                if (w0 + k * 64 + lane < sea_words) stage32[w0 + k * 64 + lane] = v[k];
        }
        wave_lds_sync();
        // Row loops run over kMaxRows with constant indices (guarded by the row count), so the
        // per-row arrays stay in registers and the row constants are read from the kernel
        // arguments directly.
        uint32_t cnt[kMaxRows];
        bool empty = false;
#pragma unroll
        for (uint32_t i = 0; i < (uint32_t)kMaxRows; ++i) {
            cnt[i] = 1;
            if (i >= c.sr || empty) continue;
            const uint32_t cells = 1u << c.ibn[i];
            uint32_t n_hot = 0;
            for (uint32_t c0 = 0; c0 < cells; c0 += 64) {
                const uint32_t cell = c0 + lane;
                uint32_t v = cell < cells ? se_at(c.row_off[i] + cell) : 0u;
                const bool hot = __popc(v) >= kSeHot;
                const uint64_t bal = __ballot(hot);
                if (hot) lists[i * a.list_stride + n_hot + __popcll(bal & lane_lt)] = (cell << 8) | v;
                n_hot += (uint32_t)__popcll(bal);
            }
            cnt[i] = n_hot;
            empty = n_hot == 0;
        }
        if (empty) continue;
        wave_lds_sync();
        uint64_t total = 1;
#pragma unroll
        for (uint32_t i = 0; i < (uint32_t)kMaxRows; ++i) total *= cnt[i];
        uint32_t qn = 0;
        if (total <= lmask + 1ull) {
            // the product CIS of the hot lists (Section 3.2), one tuple per lane.  A lane's tuple
            // index is kept as mixed-radix digits (row 0 least significant) and advanced by 64 each
            // round by adding the digits of 64, computed once per SEA: no division in the loop.
            uint32_t dg[kMaxRows], st[kMaxRows];
            {
                uint32_t rem = part * 64u + lane, inc = 64u * P;
#pragma unroll
                for (uint32_t i = 0; i < (uint32_t)kMaxRows; ++i) {
                    dg[i] = rem % cnt[i];
                    rem /= cnt[i];
                    st[i] = inc % cnt[i];
                    inc /= cnt[i];
                }
            }
            for (uint64_t u0 = (uint64_t)part * 64u; u0 < total; u0 += 64u * P) {
                const uint64_t u = u0 + lane;
                bool cand = false;
                uint32_t h = 0;
                if (u < total) {
                    uint32_t lp = 0, seu = 0xFFu;
                    uint32_t ci[kMaxRows];
#pragma unroll
                    for (uint32_t i = 0; i < (uint32_t)kMaxRows; ++i) {
                        ci[i] = 0;
                        if (i >= c.sr) continue;
                        uint32_t e = lists[i * a.list_stride + dg[i]];
                        ci[i] = e >> 8;
                        seu &= e & 0xFFu;
                        lp |= row_bits_in_lp(ci[i], c.isb[i], c.L);
                    }
                    // Eq. 3: the rebuilt LP must give back every row index (overlap bits agree)
                    bool ok = __popc(seu) >= kSeHot;
#pragma unroll
                    for (uint32_t i = 0; i < (uint32_t)kMaxRows; ++i)
                        if (i < c.sr) ok = ok && (row_index(lp, c.isb[i], c.ibn[i], c.L) == ci[i]);
                    if (ok) {
                        cand = true;
                        h = (uint32_t)(((uint64_t)lp << c.r) | rp);
                    }
                }
                // advance the digits by 64 P; each sum stays below twice its radix, so it wraps at
                // most once (rows past the row count have radix 1 and stay 0)
                uint32_t carry = 0;
#pragma unroll
                for (uint32_t i = 0; i < (uint32_t)kMaxRows; ++i) {
                    const uint32_t d = dg[i] + st[i] + carry;
                    carry = d >= cnt[i] ? 1u : 0u;
                    dg[i] = carry ? d - cnt[i] : d;
                }
                const uint64_t bal = __ballot(cand);
                if (cand) queue[qn + __popcll(bal & lane_lt)] = h;
                qn += (uint32_t)__popcll(bal);
                if (qn + 64 > a.qcap) {
                    wave_lds_sync();
                    filter_queue<MODE>(a, c, queue, qn, lane);
                    n_cand += qn;
                    qn = 0;
                }
            }
        } else {
            // more tuples than hosts in this SEA: test every LP directly (the candidate definition)
            for (uint64_t l0 = (uint64_t)part * 64u; l0 <= lmask; l0 += 64u * P) {
                const uint64_t l = l0 + lane;
                bool cand = false;
                if (l <= lmask) {
                    uint32_t seu = 0xFFu;
#pragma unroll
                    for (uint32_t i = 0; i < (uint32_t)kMaxRows; ++i)
                        if (i < c.sr) seu &= se_at(c.row_off[i] + row_index((uint32_t)l, c.isb[i], c.ibn[i], c.L));
                    cand = __popc(seu) >= kSeHot;
                }
                const uint64_t bal = __ballot(cand);
                if (cand) queue[qn + __popcll(bal & lane_lt)] = (uint32_t)((l << c.r) | rp);
                qn += (uint32_t)__popcll(bal);
                if (qn + 64 > a.qcap) {
                    wave_lds_sync();
                    filter_queue<MODE>(a, c, queue, qn, lane);
                    n_cand += qn;
                    qn = 0;
                }
            }
        }
        wave_lds_sync();
        filter_queue<MODE>(a, c, queue, qn, lane);
        n_cand += qn;
        wave_lds_sync();
    }
    // one global atomic per workgroup: atomics on one address are serialized device-wide
    __shared__ uint32_t wave_cand[NW];
    if (lane == 0) wave_cand[wid] = n_cand;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sum = 0;
        for (uint32_t w = 0; w < NW; ++w) sum += wave_cand[w];
        if (sum) atomicAdd(&a.counters[1], sum);
    }
}

// After k_close (the launch boundary orders every workgroup's records before this): the counts
// and the first records go to host-visible memory, so that no copy follows, and the counters are
// zeroed for the next launch.  One workgroup.
// Last of all it writes the close's sequence number (counters[2] + 1, kept in counters[2]) to the
// host, after a system-scope fence, so that the host may poll that word instead of waiting for the
// stream.
__global__ __launch_bounds__(256) void k_close_out(CloseArgs a) {
    const uint32_t n = a.counters[0], cand = a.counters[1];
    const uint32_t m = min(min(n, a.rec_cap), a.host_recs);
    const uint2 *src = reinterpret_cast<const uint2 *>(a.rec);
    uint2 *dst = reinterpret_cast<uint2 *>(a.host_out + 4);
    for (uint32_t i = threadIdx.x; i < m; i += 256) dst[i] = src[i];
    __threadfence_system();   // this thread's records reach the host before the sequence number
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t seq = a.counters[2] + 1u;
        a.host_out[0] = n;
        a.host_out[1] = cand;
        a.counters[0] = 0u;
        a.counters[1] = 0u;
        a.counters[2] = seq;
        __threadfence_system();
        __hip_atomic_store(a.host_out + 2, seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

template <int MODE>
static uint32_t close_occupancy(uint32_t block, uint32_t lds_bytes) {
    int n = 0;
    hipError_t e = hipErrorInvalidValue;
    if (block == 256) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_close<MODE, 256>, 256, lds_bytes);
    else if (block == 128) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_close<MODE, 128>, 128, lds_bytes);
    else if (block == 64) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_close<MODE, 64>, 64, lds_bytes);
    return (e == hipSuccess && n > 0) ? (uint32_t)n : 1u;
}

uint32_t close_blocks_per_cu(int mode, uint32_t block, uint32_t lds_bytes) {
    if (mode == kCloseStamps) return close_occupancy<kCloseStamps>(block, lds_bytes);
    if (mode == kCloseAt) return close_occupancy<kCloseAt>(block, lds_bytes);
    return close_occupancy<kCloseBits>(block, lds_bytes);
}

template <int MODE>
static hipError_t launch_close_mode(const Consts &c, const CloseArgs &a, uint32_t block, uint32_t grid, uint32_t lds,
                                    hipStream_t s) {
    if (block == 256) hipLaunchKernelGGL((k_close<MODE, 256>), dim3(grid), dim3(256), lds, s, c, a);
    else if (block == 128) hipLaunchKernelGGL((k_close<MODE, 128>), dim3(grid), dim3(128), lds, s, c, a);
    else if (block == 64) hipLaunchKernelGGL((k_close<MODE, 64>), dim3(grid), dim3(64), lds, s, c, a);
    else return hipErrorInvalidConfiguration;
    return hipGetLastError();
}

hipError_t launch_close(const Consts &c, const CloseArgs &a, int mode, uint32_t block, uint32_t grid, hipStream_t s) {
    const uint32_t lds = (block / 64) * (c.sr * a.list_stride + a.qcap + a.stage_words) * 4u;
    hipError_t e = hipErrorInvalidValue;
    if (mode == kCloseStamps) e = launch_close_mode<kCloseStamps>(c, a, block, grid, lds, s);
    else if (mode == kCloseAt) e = launch_close_mode<kCloseAt>(c, a, block, grid, lds, s);
    else if (mode == kCloseBits) e = launch_close_mode<kCloseBits>(c, a, block, grid, lds, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_close_out, dim3(1), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace spd
