// Internal declarations shared by the kernels and the host runtime of libspd.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "spd.h"

namespace spd {

constexpr int kMaxRows = SPD_MAX_ROWS;
constexpr uint32_t kSeHot = 3;      // an SE of weight >= 3 is judged to have >= theta peers (Section 3.1)
constexpr int kMaxGroup = 32;       // batches / slots per fused launch (kernel-argument arrays)

// Method constants of one context, passed by value to every kernel.
struct Consts {
    uint64_t mul[3 + kMaxRows];     // hash multipliers: H1, H2, H3, LH_0..
    uint64_t add[3 + kMaxRows];     // hash addends
    uint32_t tau_mask;              // (1 << tau) - 1: sampled iff (H1(oip) & tau_mask) == 0
    uint32_t r, L, sr, lr;          // L = 32 - r bits of LP
    uint32_t rmask;                 // 2^r - 1
    uint32_t log2k, log2lc;
    uint32_t sh_k, sh_lc;           // (32 - output bits) mod 32 of H3 and of LH_i; a zero-bit LH_i
                                    // is given zero parameters, so its 32-bit value is already 0
    uint32_t isb[kMaxRows];
    uint32_t ibn[kMaxRows];
    uint32_t row_off[kMaxRows];     // byte offset of each row inside one SEA
    uint32_t sea_bytes;
    uint32_t z_theta;
    uint64_t ldca_bits;             // LR * LC * k
    uint64_t seav_bytes;            // canonical SEAV bytes (the allocation may be padded)
};

// ------------------------------------------------------------------------------ device math
// High 32 bits of (mul * x + add) mod 2^64: the multiply-add-shift hash before its final shift.
__device__ __forceinline__ uint32_t mas_hi(uint32_t x, uint64_t mul, uint64_t add) {
    uint64_t lo = (uint64_t)(uint32_t)mul * x + add;
    return (uint32_t)(lo >> 32) + (uint32_t)(mul >> 32) * x;
}

// Top bits of a 32-bit hash value; sh is (32 - bits) mod 32 (see Consts::sh_k).
__device__ __forceinline__ uint32_t top_bits(uint32_t h, uint32_t sh) { return h >> sh; }

// Eq. 2: Idx(i, LP) = IBN(i) consecutive bits of LP starting at ISB(i), wrapping modulo L.
// Rotating a doubled copy of LP gives the wrapped window in one shift.
__device__ __forceinline__ uint32_t row_index(uint32_t lp, uint32_t isb, uint32_t ibn, uint32_t L) {
    uint64_t d = (uint64_t)lp | ((uint64_t)lp << L);
    return (uint32_t)(d >> isb) & ((1u << ibn) - 1u);
}

// Inverse placement used by Eq. 3: the LP bits that a row index c of row (isb, ibn) stands for.
__device__ __forceinline__ uint32_t row_bits_in_lp(uint32_t c, uint32_t isb, uint32_t L) {
    uint64_t t = (uint64_t)c << isb;
    uint64_t lmask = (L == 32) ? 0xFFFFFFFFull : ((1ull << L) - 1ull);
    return (uint32_t)((t | (t >> L)) & lmask);
}

// LDCA bit address of (row i, column c, bit q): ((i * LC + c) * k) + q.
__device__ __forceinline__ uint32_t ldca_bit(uint32_t i, uint32_t col, uint32_t q, const Consts &k) {
    return (((i << k.log2lc) | col) << k.log2k) | q;
}

// SEAV byte offset of row i's cell for host hip (RP selects the SEA, LP the cell, Eq. 2).
__device__ __forceinline__ uint32_t seav_byte(uint32_t hip, uint32_t i, const Consts &k) {
    uint32_t rp = hip & k.rmask;
    uint32_t lp = (uint32_t)((uint64_t)hip >> k.r);
    return rp * k.sea_bytes + k.row_off[i] + row_index(lp, k.isb[i], k.ibn[i], k.L);
}

// Workgroups of a launch are dispatched to the XCDs round robin (workgroup i to XCD i mod 8).
// Renumbering them this way gives each XCD one contiguous range of [0, n), so that neighbouring
// indices (neighbouring buckets, neighbouring tiles) share one XCD's L2.  Any renumbering is a
// bijection of [0, n); only cache locality depends on the dispatch order.
constexpr uint32_t kXcds = 8;
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t i, uint32_t n) {
    const uint32_t x = i % kXcds, l = i / kXcds, q = n / kXcds, r = n % kXcds;
    return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// ------------------------------------------------------------------------------ launchers
struct SlotPtrs {
    uint8_t *seav;       // padded SEAV (word aligned)
    uint32_t *ldca;
    uint16_t *seav_ts;   // sliding mode, 16-bit time stamps
    uint16_t *ldca_ts;
    uint8_t *seav_at;    // sliding mode, AT pool (one 8-bit counter per bit)
    uint8_t *ldca_at;
};

// Sliding window with the AT pool: every bit is an 8-bit counter holding the code (slice mod 256)
// of a slice: the last slice that set it, or, once that is older than the window, a slice that is
// just outside it.  At slice t a counter v is active (bit 1) iff its age (t - v) mod 256 is below
// K.  Maintenance at every slice start re-stamps the expired counters of one of G = 255 - K groups
// of the pool with the code of slice t - K, so each counter is visited at least once every G
// slices and its true age stays below K + G = 255 < 256: the age read modulo 256 is the true age
// (never-set counters start with the code of slice -K, already expired).
constexpr uint32_t kAtCodes = 256;
__host__ __device__ __forceinline__ uint32_t at_code(uint32_t slice) { return slice & (kAtCodes - 1u); }
// An expired code at slice t: that of slice t - K.
__host__ __device__ __forceinline__ uint32_t at_expired_code(uint32_t slice, uint32_t K) {
    return (slice - K) & (kAtCodes - 1u);
}
__host__ __device__ __forceinline__ uint32_t at_active(uint32_t v, uint32_t ct, uint32_t K) {
    return ((ct - v) & (kAtCodes - 1u)) < K ? 1u : 0u;   // ct = at_code(t)
}
constexpr uint32_t kAtMaxK = 254;   // G = 255 - K >= 1

// What the end-of-window kernel reads: bits, 16-bit time stamps, or AT counters.
enum CloseMode : int { kCloseBits = 0, kCloseStamps = 1, kCloseAt = 2 };

struct BatchDesc {
    const uint32_t *pairs;
    uint64_t n;
    uint32_t first_tile;
    uint32_t slot;       // index into the launch's slot table
    uint32_t swap;       // 1: destination-keyed (each record read as (oip, hip))
    uint32_t pad;
};

// Batches of a launch: in device memory (b, any number), or, with b null, up to kInlineBatches
// copies carried in the kernel arguments; sorted by first_tile.
constexpr uint32_t kInlineBatches = 8;
struct BatchList {
    const BatchDesc *b;
    uint32_t n;
    BatchDesc inl[kInlineBatches];
};

struct BinGeometry {
    uint32_t S;          // log2 of bits per bucket
    uint32_t nb_ldca;    // buckets covering the LDCA
    uint32_t nb;         // total buckets (LDCA then padded SEAV)
    uint32_t tile_pairs;
    uint32_t scap;       // sampled pairs staged in LDS per tile
    uint32_t cap;        // items reserved per tile (multiple of 6)
    uint32_t region;     // 32-bit words per tile in the item buffer: items packed 3 per 64 bits
    uint32_t block;      // threads per binning workgroup
    uint32_t lds_bytes;  // dynamic LDS of the binning kernel
};

hipError_t launch_fill_u32(uint32_t *p, uint64_t n_words, uint32_t value, hipStream_t s);
hipError_t launch_scan_direct(const Consts &c, const BatchDesc *batches, uint32_t n_batches, const SlotPtrs *slots,
                              uint32_t block, uint32_t grid, bool seav_lds, hipStream_t s);
// Sliding scan: every bit the discrete scan would set receives `value` (a 16-bit stamp, or an AT
// code when at is set).
// Optional timing of one kernel launch: events that the dispatch itself stamps at the kernel's start
// and end (no separate event packets on the stream).  Null events: an ordinary launch.
struct KTiming {
    hipEvent_t start = nullptr;
    hipEvent_t stop = nullptr;
};
hipError_t launch_scan_stamp(const Consts &c, const BatchDesc *batches, uint32_t n_batches, const SlotPtrs *slots,
                             uint32_t value, bool at, uint32_t block, uint32_t grid, hipStream_t s, KTiming kt = {});
// AT pool maintenance: the counters of bytes [lo, hi) of each of n pools (hi <= pool bytes, lo and
// hi multiples of 16) that are expired at the slice of code ct are set to that slice's expired code.
hipError_t launch_at_sweep(uint8_t *const *pools, uint32_t n, uint64_t lo, uint64_t hi, uint32_t ct, uint32_t K,
                           hipStream_t s);
// dst = per counter the most recent of the n_src pools (the AT version of the OR merge).
hipError_t launch_at_merge(uint8_t *dst, const uint8_t *const *src, uint32_t n_src, uint64_t n_bytes, uint32_t ct,
                           hipStream_t s);
// Bit view of AT counters: bit j of word w is 1 iff counter 32 w + j is active.
hipError_t launch_bit_view_at(const uint8_t *at, uint64_t n_bits, uint32_t ct, uint32_t K, uint32_t *out_words,
                              hipStream_t s);
hipError_t launch_bin(const Consts &c, const BinGeometry &g, const BatchDesc *batches, uint32_t n_batches,
                      uint32_t n_tiles, uint32_t *items, uint32_t *meta, const SlotPtrs *slots, hipStream_t s);
hipError_t launch_transpose(const uint32_t *meta, uint32_t *metaT, uint32_t rows, uint32_t cols, hipStream_t s);
// Buffers the counting kernel zeroes on the way (the SEAVs of fresh slots); words a multiple of 4.
struct ClearList {
    uint32_t *p[kMaxGroup];
    uint64_t words[kMaxGroup];
    uint32_t n;
};

// Counting and placement of the bucket-major layout: batches_dev is a device array of n_batches
// descriptors (any number), sorted by first_tile.
hipError_t launch_count(const Consts &c, const BinGeometry &g, const BatchDesc *batches_dev, uint32_t n_batches,
                        uint32_t n_tiles, uint32_t *cnt, const ClearList &clear, hipStream_t s);
// Tiles of a bucket-major launch, per slot [lo, hi), scanned in chunks of kChunk tiles that never
// span two slots: chunks cbase[s] .. cbase[s + 1] - 1 belong to slot s.
constexpr uint32_t kChunk = 128;
struct ChunkTable {
    uint32_t lo[kMaxGroup], hi[kMaxGroup];
    uint32_t cbase[kMaxGroup + 1];
    uint32_t n;
};
// cnt [tiles][nb] -> loc [tiles][nb] (offset inside the tile's chunk), cstart [chunks][nb] (chunk
// start, absolute), base [n * nb + 1] (start of each (slot, bucket), then the total).
hipError_t launch_offsets(const uint32_t *cnt, uint32_t *loc, uint32_t *cstart, uint32_t *base, const ChunkTable &ct,
                          uint32_t nb, hipStream_t s);
hipError_t launch_place(const Consts &c, const BinGeometry &g, const BatchDesc *batches_dev, uint32_t n_batches,
                        uint32_t n_tiles, uint32_t *items, const uint32_t *cnt, const uint32_t *loc,
                        const uint32_t *cstart, const ChunkTable &ct, const SlotPtrs *slots, hipStream_t s);
// Region layout of the binned scan (one pass over the pairs): every (chunk, bucket) has a region of
// fixed capacity in `items`; a tile takes room for its padded segment of a bucket with one atomic
// on that region's word count, and words past a region's capacity go to the spill list, which is
// ORed into the sketches after the apply phase.  A slot's regions start at slot_base[s]: its full
// chunks (kChunk tiles) first, chunk_words each (the LDCA buckets, capw_l words each, then the SEAV
// buckets, capw_s words each), then its partial last chunk, if any, sized by its own tile count.
struct RegionArgs {
    uint64_t slot_base[kMaxGroup];
    uint32_t full[kMaxGroup];                      // full chunks of each slot
    uint32_t capl_last[kMaxGroup], caps_last[kMaxGroup];   // capacities of a partial last chunk
    uint64_t *items;
    uint32_t *cur;         // [chunks][nb] words taken in each region: zero before the launch, and
                           // zeroed again by the apply phase once read
    uint32_t *spill_n;     // overflow words of this launch (zero before the launch)
    uint32_t *spill_next;  // the next launch's count: zeroed by this launch's spill phase
    uint64_t *spill_w;     // [spill_cap] overflow words
    uint32_t *spill_tag;   // [spill_cap] (slot << 16) | bucket of each overflow word
    uint32_t *ovf_n;       // tiles listed by this launch (zero before the launch)
    uint32_t *ovf_next;    // the next launch's count: zeroed by this launch's spill phase
    uint32_t *ovf;         // [ovf_cap] tiles with more sampled pairs than they could stage
    uint64_t chunk_words;  // nb_ldca * capw_l + (nb - nb_ldca) * capw_s
    uint32_t capw_l, capw_s;
    uint32_t spill_cap;    // at least the launch's padded words: the spill list cannot overflow
    uint32_t ovf_cap;      // the launch's tiles: the tile list cannot overflow
};
hipError_t launch_clear(const ClearList &clear, hipStream_t s);
// Region of chunk cc (counted inside slot si) for bucket b: its first word counted from the chunk's
// first word (below 2^31: the host checks chunk sizes), and its capacity.
__host__ __device__ __forceinline__ uint32_t region_in(const RegionArgs &ra, uint32_t nb_ldca, uint32_t si,
                                                       uint32_t cc, uint32_t b, uint32_t *capw) {
    const bool last = cc >= ra.full[si];
    const uint32_t cl = last ? ra.capl_last[si] : ra.capw_l, cs = last ? ra.caps_last[si] : ra.capw_s;
    *capw = b < nb_ldca ? cl : cs;
    return b < nb_ldca ? b * cl : nb_ldca * cl + (b - nb_ldca) * cs;
}
// First word of chunk cc of slot si in items.
__host__ __device__ __forceinline__ uint64_t chunk_at(const RegionArgs &ra, uint32_t si, uint32_t cc) {
    return ra.slot_base[si] + (uint64_t)cc * ra.chunk_words;
}
hipError_t launch_region(const Consts &c, const BinGeometry &g, const BatchList &bl, uint32_t n_tiles,
                         const ChunkTable &ct, const SlotPtrs *slots, const RegionArgs &ra, hipStream_t s, KTiming kt = {});
struct ApplySlot {
    uint32_t *ldca;
    uint32_t *seav_w;
    uint32_t tile_lo, tile_hi;
    uint32_t fresh;
    uint32_t pad;
};
hipError_t launch_apply(const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots, const uint32_t *items,
                        const uint32_t *metaT, uint32_t n_tiles, uint32_t block, uint32_t unroll, hipStream_t s);
hipError_t launch_apply_bm(const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots, const uint32_t *items,
                           const uint32_t *base, uint32_t block, uint32_t unroll, hipStream_t s);
hipError_t launch_apply_rg(const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots, const ChunkTable &ct,
                           const RegionArgs &ra, uint32_t block, uint32_t unroll, hipStream_t s, KTiming kt = {});
// The apply phase with the router OR merge fused in: the global sketch (its LDCA and SEAV) :=
// OR of the launch's slots; 1024-lane workgroups, buckets of at most 2^20 bits.
hipError_t launch_apply_rg_merge(const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots, const ChunkTable &ct,
                                 const RegionArgs &ra, const ApplySlot &global, uint32_t unroll, hipStream_t s,
                                 KTiming kt = {});
// The spill pass of a region launch over the batches bl (which the listed tiles are read from again).
hipError_t launch_spill(const Consts &c, const BinGeometry &g, const ApplySlot *slots, uint32_t n_slots,
                        const RegionArgs &ra, const BatchList &bl, hipStream_t s, const ApplySlot *global = nullptr);
hipError_t launch_or_merge(uint32_t *dst, const uint32_t *const *src, uint32_t n_src, uint64_t n_words, hipStream_t s);
hipError_t launch_max_merge_u16(uint16_t *dst, const uint16_t *const *src, uint32_t n_src, uint64_t n_elems,
                                hipStream_t s);
hipError_t launch_renormalize_u16(uint16_t *p, uint64_t n, uint16_t off, hipStream_t s);
hipError_t launch_bit_view(const uint16_t *ts, uint64_t n_bits, uint16_t thr, uint32_t *out_words, hipStream_t s);

struct CloseArgs {
    const uint8_t *seav;     // the SEAV as bits (sliding: the bit view of its counters)
    const uint32_t *ldca;
    const uint16_t *ldca_ts;   // sliding: the LDCA's counters, read by the ULDC filter
    const uint8_t *ldca_at;
    uint32_t thr;        // sliding, 16-bit stamps: stamp threshold of the bit view
    uint32_t at_ct;      // sliding, AT pool: code of the current slice
    uint32_t at_k;       // sliding, AT pool: window length K
    uint32_t *rec;       // (ip, z0) pairs
    uint32_t *counters;  // [0] reported, [1] candidates; zero at launch, left zero by k_close_out
    uint32_t *host_out;  // host-visible: the counters, then the first host_recs records
    uint32_t host_recs;
    uint32_t rec_cap;
    uint32_t n_rp;
    uint32_t list_stride;
    uint32_t qcap;
    uint32_t stage_words;  // LDS words per wavefront holding one SEA
    uint32_t parts_log2;   // each SEA's candidates are searched by 2^parts_log2 wavefronts
};
hipError_t launch_close(const Consts &c, const CloseArgs &a, int mode, uint32_t block, uint32_t grid, hipStream_t s);
// Workgroups of the end-of-window kernel that one compute unit holds at once (registers and LDS).
uint32_t close_blocks_per_cu(int mode, uint32_t block, uint32_t lds_bytes);

}  // namespace spd
