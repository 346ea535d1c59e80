// Host runtime of libspd: parameter derivation, contexts, router slots, scratch memory, kernel
// dispatch and the C ABI declared in include/spd.h.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "spd_internal.h"

using namespace spd;

namespace {

constexpr uint32_t kMaxLds = 160 * 1024;       // LDS per workgroup on gfx950
constexpr uint32_t kMaxBucketBits = 20;        // 2^20 bits = 128 KiB bitmap per apply workgroup
constexpr uint64_t kSeavAlign = 1ull << (kMaxBucketBits - 3);  // SEAV padded to whole buckets

struct Slot {
    void *mem = nullptr;         // one allocation: [LDCA | padded SEAV] or [LDCA stamps | SEAV stamps]
    uint32_t *ldca = nullptr;
    uint8_t *seav = nullptr;
    uint16_t *ldca_ts = nullptr;
    uint16_t *seav_ts = nullptr;
    uint8_t *ldca_at = nullptr;  // AT pool: one 8-bit counter per bit
    uint8_t *seav_at = nullptr;
    bool fresh = true;           // logically all zero; device memory not yet cleared
};

struct WorkItem {
    Slot *slot;
    const uint32_t *pairs;
    uint64_t n;
    uint32_t swap = 0;   // destination-keyed batch
};

constexpr uint32_t kRecInit = 65536;   // device records per close buffer, grown on demand
constexpr uint32_t kRecChunk = 4096;   // records copied back together with the counters

// Device and pinned host buffers of one end-of-window pass.
struct CloseBuf {
    // one device buffer: 4 counters ([0] reported, [1] candidates, both zero between launches;
    // [2] the sequence number of the last close) then the (ip, z0) records.  The end-of-window
    // launch itself copies the counters and the first kRecChunk records to h_counters, and the
    // sequence number last.
    uint32_t *counters = nullptr;
    uint32_t *rec = nullptr;          // counters + 4
    uint32_t rec_cap = 0;
    uint32_t *h_counters = nullptr;   // pinned and mapped, same layout, kRecChunk records
    uint8_t *seav_bits = nullptr;     // sliding: the bit view of the SEAV counters the close reads
    uint32_t *d_counters = nullptr;   // h_counters' device address
    uint32_t *h_rec = nullptr;        // pinned, all records when there are more than kRecChunk
    uint32_t h_rec_cap = 0;
    bool empty = false;               // the slot was fresh: nothing was launched
    uint32_t seq = 0;                 // the sequence number the last enqueued close will write
    hipGraphExec_t graph = nullptr;   // captured close of graph_slot
    const Slot *graph_slot = nullptr;
    const uint32_t *graph_rec = nullptr;
};

}  // namespace

constexpr uint32_t kBdRing = 4;   // staging slots for the batch descriptors of binned launches

// A close begun with spd_close_begin and not yet collected: its buffers, and an event recorded
// after its device work.
struct PendingClose {
    CloseBuf cb;
    hipEvent_t done = nullptr;
    bool busy = false;
    uint32_t seq = 0;   // ticket = seq << 4 | index
};

struct spd_ctx {
    spd_params p{};
    spd_derived d{};
    Consts c{};
    int device = 0;
    uint32_t n_cu = 256;
    uint32_t n_routers = 0;
    uint64_t budget = 0;
    uint64_t held = 0;
    bool sliding = false;
    bool at = false;             // sliding window kept in the AT pool (else 16-bit stamps)
    uint32_t at_groups = 0;      // AT pool: groups swept round robin, one per slice
    uint32_t K = 0;
    uint32_t slice = 0;
    uint64_t seav_alloc = 0;     // padded SEAV bytes per slot
    uint64_t ldca_bytes = 0;     // LDCA bytes per slot, rounded up to 256
    uint64_t slot_bytes = 0;
    std::vector<Slot> slots;     // routers, then the global sketch
    uint32_t *items = nullptr;
    uint64_t items_words = 0;
    uint32_t *meta = nullptr;
    uint32_t *metaT = nullptr;
    uint32_t *metaB = nullptr;
    uint64_t meta_words = 0;
    BatchDesc *bd_host[kBdRing] = {};   // pinned staging of batch descriptors
    BatchDesc *bd_dev[kBdRing] = {};
    hipEvent_t bd_ev[kBdRing] = {};     // recorded after the last kernel that reads a slot
    uint32_t bd_cap = 0;                // descriptors per slot
    uint32_t bd_next = 0;
    uint32_t *h2d_buf[2] = {};          // staging of spd_scan_host
    uint64_t h2d_words = 0;             // per staging buffer
    hipStream_t h2d_s = nullptr;
    hipEvent_t h2d_copied[2] = {}, h2d_scanned[2] = {};
    uint32_t *aux = nullptr;         // region layout: counters; exact-count layout: bucket bases
    uint64_t aux_words = 0;
    bool aux_zero = false;           // region layout: every aux word is zero between launches
    uint32_t close_per_cu[3] = {0, 0, 0};   // resident end-of-window workgroups per CU (64, 128, 256 lanes)
    uint32_t spill_parity = 0;       // region layout: which of two spill counts the next launch uses
    CloseBuf cbuf;                  // end-of-window buffers of spd_close_window
    Slot *merge_into = nullptr;     // spd_scan_batches_merge: the global slot, while its scan runs
    bool merge_group = false;       // the region launch being enqueued covers the whole merged call
    bool merged = false;            // the merge was fused into that launch's apply phase
    PendingClose pend[SPD_MAX_PENDING_CLOSES];   // spd_close_begin / spd_close_end
    uint32_t pend_seq = 0;
    uint32_t pend_rec = 0;          // record room a pending close must have (grown after an overflow)
    hipStream_t copy_s = nullptr;   // non-blocking: record copies of spd_close_end
    uint32_t *view = nullptr;       // sliding export: bit view words
    uint64_t view_words = 0;
    std::vector<uint32_t> est;      // Eq. 4 estimate for every z0 in [0, k]
    uint8_t *noalloc = nullptr;     // device address of this device's no-alloc scratch array
    std::string noalloc_err;        // why it is missing (lookup failed at creation)
    spd_tuning tune{};
    spd_stats stats{};
    std::string err;
    hipStream_t last_stream = nullptr;
    bool have_last = false;
    hipEvent_t order_ev = nullptr;
    // optional per-kernel timing
    bool prof_on = false;
    uint32_t prof_mask = ~0u;      // kinds timed while profiling is on (bit k: kind k)
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Pending> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    spd_profile prof{};
};

// Scratch of spd_scan_noalloc: a fixed array in device memory.  Every GPU the library runs on
// holds its own copy, at its own address, until the process ends.  In host code the name is only
// a stand-in for the device symbol and is never passed to a kernel: host code uses the device
// address that hipGetSymbolAddress returns on each device (noalloc_lookup), kept per device.
static __device__ __align__(256) uint8_t scratch[SPD_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
uint8_t *g_noalloc_addr[kMaxDevices] = {};   // per device: the address of `scratch`, once looked up

// The device address of `scratch` on `device`, which must be the current device.
hipError_t noalloc_lookup(int device, uint8_t **out) {
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_addr[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_noalloc_addr[device] = static_cast<uint8_t *>(ptr);
    }
    *out = g_noalloc_addr[device];
    return hipSuccess;
}

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) (void)hipSetDevice(dev);
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

spd_status fail(spd_ctx *ctx, spd_status s, const std::string &msg) {
    if (ctx) ctx->err = msg;
    return s;
}

spd_status hip_fail(spd_ctx *ctx, hipError_t e, const char *where) {
    return fail(ctx, SPD_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define SPD_HIP(ctx, expr)                                \
    do {                                                  \
        hipError_t e_ = (expr);                           \
        if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
    } while (0)

// Eq. 1: the smallest t >= 0 with 8 * 2^t >= theta.
uint32_t tau_of(uint32_t theta) {
    uint32_t t = 0;
    while ((8ull << t) < (uint64_t)theta) ++t;
    return t;
}

// Eq. 4 inverted: the largest z0 in [1, k] whose estimate -k ln(z0/k) is at least theta.
uint32_t z_theta_of(uint32_t log2k, uint32_t theta) {
    const double k = std::ldexp(1.0, (int)log2k);
    uint32_t lo = 0;
    for (uint32_t z = 1u << log2k; z >= 1; --z) {
        if (-k * std::log((double)z / k) >= (double)theta) {
            lo = z;
            break;
        }
    }
    return lo;
}

spd_status derive(const spd_params *p, spd_derived *d, std::string *why) {
    auto bad = [&](const char *m) {
        if (why) *why = m;
        return SPD_E_INVALID;
    };
    if (!p || !d) return bad("null argument");
    if (p->theta < 1 || p->theta > (1u << 31)) return bad("theta must be in [1, 2^31]");
    if (p->r > 24) return bad("r must be <= 24");
    if (p->sr < 1 || p->sr > SPD_MAX_ROWS) return bad("sr must be in [1, 8]");
    if (p->lr < 1 || p->lr > SPD_MAX_ROWS) return bad("lr must be in [1, 8]");
    if (p->log2k < 5 || p->log2k > 16) return bad("log2k must be in [5, 16]");
    if (p->log2lc > 24) return bad("log2lc must be <= 24");
    if (p->window_slices > 30000) return bad("window_slices must be <= 30000");
    if (p->sliding_counter > 1) return bad("sliding_counter must be 0 (AT pool) or 1 (16-bit stamps)");
    if (p->window_slices && p->sliding_counter == 0 && p->window_slices > kAtMaxK)
        return bad("the AT pool needs window_slices <= 254 (use sliding_counter = 1)");
    const uint32_t L = 32 - p->r;
    std::memset(d, 0, sizeof(*d));
    if (p->explicit_layout) {
        for (uint32_t i = 0; i < p->sr; ++i) {
            if (p->isb[i] >= L) return bad("isb must be < 32 - r");
            d->isb[i] = p->isb[i];
            d->ibn[i] = p->ibn[i];
        }
    } else {
        // Section 3.2 example, read with L = 32 - r positions: s = ceil(L / SR),
        // ISB(i) = i * s mod L, IBN(i) = s + a (at most L).
        const uint32_t s = (L + p->sr - 1) / p->sr;
        for (uint32_t i = 0; i < p->sr; ++i) {
            d->isb[i] = (i * s) % L;
            d->ibn[i] = std::min(s + p->a, L);
        }
    }
    for (uint32_t i = 0; i < p->sr; ++i)
        if (d->ibn[i] < 1 || d->ibn[i] > 16 || d->ibn[i] > L) return bad("ibn must be in [1, min(16, 32 - r)]");
    // Constraint 1 (Section 3.2): every LP bit lies in some row's index window.
    for (uint32_t j = 0; j < L; ++j) {
        bool hit = false;
        for (uint32_t i = 0; i < p->sr && !hit; ++i) hit = ((j + L - d->isb[i]) % L) < d->ibn[i];
        if (!hit) return bad("layout leaves an LP bit uncovered (constraint 1)");
    }
    for (uint32_t i = 0; i < 3u + p->lr; ++i)
        if ((p->hash_mul[i] & 1u) == 0) return bad("hash multipliers must be odd");
    d->tau = tau_of(p->theta);
    d->z_theta = z_theta_of(p->log2k, p->theta);
    uint64_t sea = 0;
    for (uint32_t i = 0; i < p->sr; ++i) sea += 1ull << d->ibn[i];
    d->sea_bytes = sea;
    d->seav_bytes = sea << p->r;
    d->ldca_words = ((uint64_t)p->lr << p->log2lc) << (p->log2k - 5);
    const uint64_t seav_padded = (d->seav_bytes + kSeavAlign - 1) / kSeavAlign * kSeavAlign;
    if (d->ldca_words * 32 + seav_padded * 8 > (1ull << 32)) return bad("sketch larger than 2^32 bits");
    return SPD_OK;
}

void default_tuning(spd_tuning *t) {
    t->direct_max_pairs = 1u << 18;
    t->bucket_bits = 20;
    t->tile_pairs = 8192;
    t->bin_block = 1024;
    t->apply_block = 1024;
    t->direct_block = 256;
    t->direct_grid_per_cu = 8;
    t->seav_lds = 0;
    t->close_block = 256;
    t->launch_pairs = 0;
    t->apply_unroll = 16;
    t->bin_mode = 2;
    t->region_words = 0;
}

void order_stream(spd_ctx *ctx, hipStream_t s) {
    if (ctx->have_last && ctx->last_stream != s) {
        (void)hipEventRecord(ctx->order_ev, ctx->last_stream);
        (void)hipStreamWaitEvent(s, ctx->order_ev, 0);
    }
    ctx->last_stream = s;
    ctx->have_last = true;
}

hipEvent_t prof_event(spd_ctx *ctx) {
    if (!ctx->prof_pool.empty()) {
        hipEvent_t e = ctx->prof_pool.back();
        ctx->prof_pool.pop_back();
        return e;
    }
    // timing only: no system-scope fence (no cache writeback between the bracketed kernels)
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with events when profiling is on.
struct ProfScope {
    spd_ctx *ctx;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(spd_ctx *c, int k, hipStream_t st) : ctx(c), kind(k), s(st) {
        if (ctx->prof_on && ((ctx->prof_mask >> k) & 1u)) {
            a = prof_event(ctx);
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope() {
        if (!a) return;
        hipEvent_t b = prof_event(ctx);
        if (!b) {
            ctx->prof_pool.push_back(a);
            return;
        }
        (void)hipEventRecord(b, s);
        ctx->prof_pending.push_back({kind, a, b});
    }
};

// Times one kernel launch, when profiling is on, with events that the dispatch stamps itself at
// the kernel's start and end (no event packets of their own between the kernels of a window).
struct ProfKernel {
    spd_ctx *ctx;
    int kind;
    KTiming kt{};
    ProfKernel(spd_ctx *c, int k) : ctx(c), kind(k) {
        if (ctx->prof_on && ((ctx->prof_mask >> k) & 1u)) {
            kt.start = prof_event(ctx);
            kt.stop = kt.start ? prof_event(ctx) : nullptr;
            if (!kt.stop && kt.start) {
                ctx->prof_pool.push_back(kt.start);
                kt.start = nullptr;
            }
        }
    }
    ~ProfKernel() {
        if (kt.start) ctx->prof_pending.push_back({kind, kt.start, kt.stop});
    }
};

void prof_harvest(spd_ctx *ctx) {
    for (auto &p : ctx->prof_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            ctx->prof.launches[p.kind]++;
            ctx->prof.total_ms[p.kind] += ms;
        }
        ctx->prof_pool.push_back(p.a);
        ctx->prof_pool.push_back(p.b);
    }
    ctx->prof_pending.clear();
}

spd_status reserve(spd_ctx *ctx, uint64_t bytes) {
    if (ctx->budget && ctx->held + bytes > ctx->budget)
        return fail(ctx, SPD_E_NOMEM, "HBM budget exceeded: need " + std::to_string(ctx->held + bytes) +
                                          " bytes, budget " + std::to_string(ctx->budget));
    return SPD_OK;
}

template <typename T>
spd_status dev_alloc(spd_ctx *ctx, T **p, uint64_t bytes) {
    spd_status st = reserve(ctx, bytes);
    if (st) return st;
    void *m = nullptr;
    hipError_t e = hipMalloc(&m, bytes ? bytes : 16);
    if (e != hipSuccess) return hip_fail(ctx, e, "hipMalloc");
    ctx->held += bytes;
    *p = static_cast<T *>(m);
    return SPD_OK;
}

template <typename T>
void dev_free(spd_ctx *ctx, T **p, uint64_t bytes) {
    if (*p) {
        (void)hipFree(*p);
        ctx->held -= std::min(ctx->held, bytes);
        *p = nullptr;
    }
}

Slot *slot_of(spd_ctx *ctx, int32_t target) {
    if (target == SPD_GLOBAL) return &ctx->slots[ctx->n_routers];
    if (target < 0 || (uint32_t)target >= ctx->n_routers) return nullptr;
    return &ctx->slots[target];
}

SlotPtrs ptrs_of(const Slot &s) {
    SlotPtrs p{};
    p.seav = s.seav;
    p.ldca = s.ldca;
    p.seav_ts = s.seav_ts;
    p.ldca_ts = s.ldca_ts;
    p.seav_at = s.seav_at;
    p.ldca_at = s.ldca_at;
    return p;
}

uint64_t slot_words(const spd_ctx *ctx) { return ctx->slot_bytes / 4; }

// The value that empties a slot: zero, or for an AT pool the expired code of the current slice in
// every byte.
uint32_t empty_fill(const spd_ctx *ctx) { return ctx->at ? at_expired_code(ctx->slice, ctx->K) * 0x01010101u : 0u; }

spd_status clear_slot(spd_ctx *ctx, Slot &s, hipStream_t st) {
    {
        ProfScope ps(ctx, SPD_K_FILL, st);
        SPD_HIP(ctx, launch_fill_u32(static_cast<uint32_t *>(s.mem), slot_words(ctx), empty_fill(ctx), st));
    }
    s.fresh = false;
    return SPD_OK;
}

// Zero only the SEAV of a fresh slot: the per-tile and exact-count layouts rewrite every LDCA bucket
// of a fresh slot from zero, while its SEAV buckets are read back (they may hold bits recorded
// directly).
spd_status clear_seav(spd_ctx *ctx, Slot &s, hipStream_t st) {
    ProfScope ps(ctx, SPD_K_FILL, st);
    SPD_HIP(ctx, launch_fill_u32(reinterpret_cast<uint32_t *>(s.seav), ctx->seav_alloc / 4, 0u, st));
    return SPD_OK;
}

// Geometry of the binned scan for the current tuning; false if it does not fit the LDS.
bool bin_geometry(const spd_ctx *ctx, BinGeometry *g) {
    const spd_tuning &t = ctx->tune;
    const uint64_t ldca_bits = ctx->d.ldca_words * 32;
    uint32_t S = std::min<uint32_t>(t.bucket_bits, kMaxBucketBits);
    S = std::min<uint32_t>(S, ctx->p.log2lc + ctx->p.log2k);   // 2^S divides the LDCA bits
    if (S < 5) return false;
    g->S = S;
    g->nb_ldca = (uint32_t)(ldca_bits >> S);
    g->nb = g->nb_ldca + (uint32_t)((ctx->seav_alloc * 8) >> S);
    if (g->nb > 65535) return false;
    g->block = t.bin_block;
    for (uint32_t T = t.tile_pairs; T >= 2048; T /= 2) {
        if (T % g->block) continue;
        const uint32_t ppt = T / g->block;
        if (ppt != 4 && ppt != 8 && ppt != 16) continue;
        // items are held in registers between counting and scattering: keep them spill-free
        if (ppt * ctx->p.lr * g->block > 32u * 1024u) continue;
        // sampled pairs a tile stages (more are recorded with global atomics): the mean plus
        // six standard deviations and a margin
        const double expect = (double)T / (double)(1ull << ctx->d.tau);
        uint32_t scap = (uint32_t)std::ceil(expect + 6.0 * std::sqrt(expect) + 32.0);
        scap = std::min<uint32_t>((scap + 63) / 64 * 64, T);
        const bool bm = t.bin_mode != 0;
        // bucket-major segments are padded to whole words: at most 2 more items per bucket
        uint64_t cap = (uint64_t)T * ctx->p.lr + (uint64_t)scap * ctx->p.sr + (bm ? 2ull * g->nb : 0ull);
        cap = (cap + 5) / 6 * 6;
        if ((uint64_t)T * ctx->p.lr > 65535) continue;   // per-bucket ranks are 16 bits, 0xFFFF unused
        const uint64_t stage_off = (2ull * (g->nb + 1) + 3) & ~3ull;   // same layout in k_bin and k_place
        // + scan scratch (17 words) + the static per-row constants (3 per row)
        const uint64_t lds = 4ull * (stage_off + cap + 2ull * scap + 1 + 17 + 3ull * kMaxRows);
        if (lds <= kMaxLds) {
            g->tile_pairs = T;
            g->scap = scap;
            g->cap = (uint32_t)cap;
            g->region = cap / 3 * 2;
            g->lds_bytes = (uint32_t)lds;
            return true;
        }
    }
    return false;
}

void free_batch_ring(spd_ctx *ctx) {
    for (uint32_t k = 0; k < kBdRing; ++k) {
        if (ctx->bd_ev[k]) (void)hipEventSynchronize(ctx->bd_ev[k]);
        if (ctx->bd_host[k]) (void)hipHostFree(ctx->bd_host[k]);
        ctx->bd_host[k] = nullptr;
        dev_free(ctx, &ctx->bd_dev[k], (uint64_t)ctx->bd_cap * sizeof(BatchDesc));
    }
    ctx->bd_cap = 0;
}

// Copy a launch's batch descriptors to device memory (next slot of the staging ring; the slot's
// event, recorded after the kernels that read it, guards its reuse).  The caller records
// bd_ev[bd_next] after its last kernel and advances bd_next.
spd_status ensure_batch_ring(spd_ctx *ctx, size_t n) {
    for (uint32_t k = 0; k < kBdRing; ++k)
        if (!ctx->bd_ev[k]) SPD_HIP(ctx, hipEventCreateWithFlags(&ctx->bd_ev[k], hipEventDisableTiming));
    if (n > ctx->bd_cap) {
        free_batch_ring(ctx);
        const uint32_t cap = (uint32_t)std::max<size_t>(1024, (n + 1023) / 1024 * 1024);
        for (uint32_t k = 0; k < kBdRing; ++k) {
            SPD_HIP(ctx, hipHostMalloc((void **)&ctx->bd_host[k], cap * sizeof(BatchDesc), hipHostMallocDefault));
            spd_status st = dev_alloc(ctx, &ctx->bd_dev[k], (uint64_t)cap * sizeof(BatchDesc));
            if (st) return st;
        }
        ctx->bd_cap = cap;
    }
    return SPD_OK;
}

spd_status upload_batches(spd_ctx *ctx, const BatchDesc *bd, size_t n, hipStream_t s, BatchDesc **out) {
    spd_status st = ensure_batch_ring(ctx, n);
    if (st) return st;
    const uint32_t k = ctx->bd_next;
    SPD_HIP(ctx, hipEventSynchronize(ctx->bd_ev[k]));
    std::memcpy(ctx->bd_host[k], bd, n * sizeof(BatchDesc));
    SPD_HIP(ctx, hipMemcpyAsync(ctx->bd_dev[k], ctx->bd_host[k], n * sizeof(BatchDesc), hipMemcpyHostToDevice, s));
    *out = ctx->bd_dev[k];
    return SPD_OK;
}

spd_status ensure_aux(spd_ctx *ctx, uint64_t words, hipStream_t s) {
    if (words <= ctx->aux_words) return SPD_OK;
    SPD_HIP(ctx, hipStreamSynchronize(s));
    dev_free(ctx, &ctx->aux, ctx->aux_words * 4);
    ctx->aux_words = 0;
    ctx->aux_zero = false;
    words = (words + 3) / 4 * 4;
    spd_status st = dev_alloc(ctx, &ctx->aux, words * 4);
    if (st) return st;
    ctx->aux_words = words;
    return SPD_OK;
}

// Item and offset scratch (32-bit words) of one binned launch over `tiles` tiles.  Bucket-major:
// padded items per tile <= its items + 2 per bucket, 3 items per 64 bits.
void scratch_need(const BinGeometry &g, uint32_t bin_mode, uint64_t tiles, uint64_t *items_words, uint64_t *meta_words) {
    *items_words = bin_mode == 0 ? tiles * g.region : (tiles * g.cap + 2) / 3 * 2 + 4;
    *meta_words = tiles * (g.nb + 1);
}

// Region layout: 64-bit words per (chunk, bucket) region of a chunk of t tiles whose bucket expects
// E items: 1.25 E plus eight standard deviations of a binomial count, the padding of t tiles (at
// most two items each) and a margin, three items per word.  Room past the fill costs memory, not
// traffic.
static uint32_t region_capw(double E, double t) {
    return (uint32_t)std::ceil((1.25 * E + 8.0 * std::sqrt(E) + 2.0 * t + 64.0) / 3.0);
}

// Expected items per tile of one LDCA bucket and of one SEAV bucket.
static void region_load(const spd_ctx *ctx, const BinGeometry &g, double *el, double *es) {
    const double T = g.tile_pairs, bucket = std::ldexp(1.0, (int)g.S);
    const double ldca_bits = (double)ctx->d.ldca_words * 32.0, seav_bits = (double)ctx->d.seav_bytes * 8.0;
    *el = T * ctx->p.lr * std::min(bucket, ldca_bits) / ldca_bits;
    *es = T / std::ldexp(1.0, (int)ctx->d.tau) * ctx->p.sr * std::min(bucket, seav_bits) / seav_bits;
}

static uint32_t region_cap(const spd_ctx *ctx, double e_tile, double t) {
    return ctx->tune.region_words ? ctx->tune.region_words : region_capw(e_tile * t, t);
}

// The region layout of one launch over the slots of ct (pointers left null): items_words = 32-bit
// words of the regions, the spill words, the spill tags and the tile list; cur_words = two spill
// counts, two tile-list counts and the region counters, a multiple of 4.
void region_layout(const spd_ctx *ctx, const BinGeometry &g, const ChunkTable &ct, uint64_t tiles, RegionArgs *ra,
                   uint64_t *items_words, uint64_t *cur_words) {
    double el, es;
    region_load(ctx, g, &el, &es);
    const uint64_t nbs = g.nb - g.nb_ldca;
    *ra = RegionArgs{};
    ra->capw_l = region_cap(ctx, el, kChunk);
    ra->capw_s = region_cap(ctx, es, kChunk);
    ra->chunk_words = (uint64_t)g.nb_ldca * ra->capw_l + nbs * ra->capw_s;
    uint64_t words = 0;
    for (uint32_t k = 0; k < ct.n; ++k) {
        const uint32_t nt = ct.hi[k] - ct.lo[k], rem = nt % kChunk;
        ra->slot_base[k] = words;
        ra->full[k] = nt / kChunk;
        ra->capl_last[k] = rem ? region_cap(ctx, el, rem) : ra->capw_l;
        ra->caps_last[k] = rem ? region_cap(ctx, es, rem) : ra->capw_s;
        words += ra->full[k] * ra->chunk_words + (rem ? g.nb_ldca * ra->capl_last[k] + nbs * ra->caps_last[k] : 0);
    }
    // every padded word of the launch fits the spill list: at most cap / 3 words per tile; every
    // tile fits the tile list
    ra->spill_cap = (uint32_t)std::min<uint64_t>(tiles * g.cap / 3, 0xFFFFFFFFull);
    ra->ovf_cap = (uint32_t)tiles;
    *items_words = words * 2 + (uint64_t)ra->spill_cap * 3 + tiles;
    *cur_words = (4 + (uint64_t)ct.cbase[ct.n] * g.nb + 3) / 4 * 4;
}

// Upper bound of region_layout's sizes over every launch of at most `tiles` tiles in at most
// kMaxGroup slots.  A partial chunk of r tiles takes at most A r + B sqrt(r) + C words (A, B, C
// from region_capw, the ceiling included in C), and over at most kMaxGroup partial chunks of R
// tiles in all, sum sqrt(r) <= sqrt(kMaxGroup R).
void region_bound(const spd_ctx *ctx, const BinGeometry &g, uint64_t tiles, uint64_t *items_words,
                  uint64_t *cur_words) {
    double el, es;
    region_load(ctx, g, &el, &es);
    const double nbl = g.nb_ldca, nbs = g.nb - g.nb_ldca;
    double words;
    if (ctx->tune.region_words) {
        words = ((double)tiles + kMaxGroup) * (nbl + nbs) * ctx->tune.region_words;
    } else {
        const double chunk_words = nbl * region_capw(el * kChunk, kChunk) + nbs * region_capw(es * kChunk, kChunk);
        const double R = (double)std::min<uint64_t>(tiles, (uint64_t)kMaxGroup * (kChunk - 1));
        const double A = (nbl * (1.25 * el + 2.0) + nbs * (1.25 * es + 2.0)) / 3.0;
        const double B = 8.0 * (nbl * std::sqrt(el) + nbs * std::sqrt(es)) / 3.0;
        const double C = (nbl + nbs) * (64.0 / 3.0 + 1.0);
        words = (double)(tiles / kChunk) * chunk_words + A * R + B * std::sqrt(kMaxGroup * R) + kMaxGroup * C;
    }
    const uint64_t spill = std::min<uint64_t>(tiles * g.cap / 3, 0xFFFFFFFFull);
    *items_words = (uint64_t)std::ceil(words) * 2 + spill * 3 + tiles;
    *cur_words = (4 + (tiles / kChunk + kMaxGroup) * g.nb + 3) / 4 * 4;
}

void free_scratch(spd_ctx *ctx) {
    dev_free(ctx, &ctx->items, ctx->items_words * 4);
    dev_free(ctx, &ctx->meta, ctx->meta_words * 4);
    dev_free(ctx, &ctx->metaT, ctx->meta_words * 4);
    dev_free(ctx, &ctx->metaB, ctx->meta_words * 4);
    dev_free(ctx, &ctx->aux, ctx->aux_words * 4);
    ctx->items_words = ctx->meta_words = ctx->aux_words = 0;
    ctx->aux_zero = false;
}

spd_status ensure_scratch(spd_ctx *ctx, uint64_t items_words, uint64_t meta_words, hipStream_t s) {
    if (items_words > ctx->items_words || meta_words > ctx->meta_words) SPD_HIP(ctx, hipStreamSynchronize(s));
    if (items_words > ctx->items_words) {
        dev_free(ctx, &ctx->items, ctx->items_words * 4);
        ctx->items_words = 0;
        spd_status st = dev_alloc(ctx, &ctx->items, items_words * 4);
        if (st) return st;
        ctx->items_words = items_words;
    }
    if (meta_words > ctx->meta_words) {
        dev_free(ctx, &ctx->meta, ctx->meta_words * 4);
        dev_free(ctx, &ctx->metaT, ctx->meta_words * 4);
        dev_free(ctx, &ctx->metaB, ctx->meta_words * 4);
        ctx->meta_words = 0;
        spd_status st = dev_alloc(ctx, &ctx->meta, meta_words * 4);
        if (!st) st = dev_alloc(ctx, &ctx->metaT, meta_words * 4);
        if (!st) st = dev_alloc(ctx, &ctx->metaB, meta_words * 4);
        if (st) return st;
        ctx->meta_words = meta_words;
    }
    return SPD_OK;
}

// Scratch of one region-layout group: the item regions and spill list (`items`), the spill counts
// and region counters (`aux`), whether every aux word is known to be zero, and which of the two
// spill counts the group uses.
struct RegionScratch {
    uint32_t *items;
    uint64_t items_words;
    uint32_t *aux;
    uint64_t aux_words;
    bool *aux_zero;
    uint32_t *parity;
};

// One group of the region layout in the given scratch: clear the counters (unless known zero), bin
// into the regions, apply every (slot, bucket), then the spill pass.  A fresh slot needs no clear:
// the apply phase writes all of its buckets from zero, and only the spill pass, after it, writes
// the slot directly.  SPD_E_INVALID (nothing enqueued) if the group's layout does not fit the
// scratch.
spd_status region_launch_at(spd_ctx *ctx, const BinGeometry &g, const BatchDesc *bd, uint32_t nbd, uint32_t tiles,
                            const ChunkTable &ct, const SlotPtrs *sp, const ApplySlot *as, uint32_t nsl,
                            const RegionScratch &rs, hipStream_t s) {
    RegionArgs ra{};
    uint64_t items_words = 0, cur_words = 0;
    region_layout(ctx, g, ct, tiles, &ra, &items_words, &cur_words);
    if (ra.chunk_words >= (1ull << 31)) return fail(ctx, SPD_E_INVALID, "region layout: chunk too large");
    if (items_words > rs.items_words || cur_words > rs.aux_words)
        return fail(ctx, SPD_E_INVALID, "region layout larger than its scratch");
    const uint64_t region_words = items_words - (uint64_t)ra.spill_cap * 3 - ra.ovf_cap;   // 32-bit words
    const uint32_t par = *rs.parity;
    ra.items = reinterpret_cast<uint64_t *>(rs.items);
    ra.spill_w = reinterpret_cast<uint64_t *>(rs.items + region_words);
    ra.spill_tag = rs.items + region_words + (uint64_t)ra.spill_cap * 2;
    ra.ovf = rs.items + region_words + (uint64_t)ra.spill_cap * 3;
    ra.spill_n = rs.aux + par;
    ra.spill_next = rs.aux + (par ^ 1u);
    ra.ovf_n = rs.aux + 2 + par;
    ra.ovf_next = rs.aux + 2 + (par ^ 1u);
    ra.cur = rs.aux + 4;
    // a few batches travel in the kernel arguments; more go through the pinned staging ring
    BatchList bl{};
    bl.n = nbd;
    const bool inl = nbd <= kInlineBatches;
    if (inl) {
        std::copy(bd, bd + nbd, bl.inl);
    } else {
        BatchDesc *bdev = nullptr;
        spd_status st = upload_batches(ctx, bd, nbd, s, &bdev);
        if (st) return st;
        bl.b = bdev;
    }
    if (!*rs.aux_zero) {   // after (re)allocation, another layout's use, or a failed launch
        ProfScope ps(ctx, SPD_K_FILL, s);
        ClearList cl{};
        cl.p[cl.n] = rs.aux;
        cl.words[cl.n++] = rs.aux_words;
        SPD_HIP(ctx, launch_clear(cl, s));
    }
    *rs.aux_zero = false;   // until the launch's apply and spill phases are enqueued
    {
        ProfKernel pk(ctx, SPD_K_BIN);
        SPD_HIP(ctx, launch_region(ctx->c, g, bl, tiles, ct, sp, ra, s, pk.kt));
    }
    // the router merge fused into the apply phase (1024-lane workgroups hold a bucket's OR in
    // registers), when this launch covers every router of a merged call
    const bool fuse = ctx->merge_group && ctx->merge_into && ctx->tune.apply_block == 1024 && g.S <= 20;
    ApplySlot gas{};
    if (fuse) {
        gas.ldca = ctx->merge_into->ldca;
        gas.seav_w = reinterpret_cast<uint32_t *>(ctx->merge_into->seav);
    }
    {
        ProfKernel pk(ctx, SPD_K_APPLY);
        if (fuse)
            SPD_HIP(ctx, launch_apply_rg_merge(g, as, nsl, ct, ra, gas, ctx->tune.apply_unroll, s, pk.kt));
        else
            SPD_HIP(ctx, launch_apply_rg(g, as, nsl, ct, ra, ctx->tune.apply_block, ctx->tune.apply_unroll, s, pk.kt));
    }
    {
        ProfScope ps(ctx, SPD_K_SPILL, s);
        SPD_HIP(ctx, launch_spill(ctx->c, g, as, nsl, ra, bl, s, fuse ? &gas : nullptr));
        if (!inl) {
            // the staging slot may be rewritten once the spill pass (the last reader) has read it
            SPD_HIP(ctx, hipEventRecord(ctx->bd_ev[ctx->bd_next], s));
            ctx->bd_next = (ctx->bd_next + 1) % kBdRing;
        }
    }
    if (fuse) ctx->merged = true;
    *rs.parity = par ^ 1u;
    *rs.aux_zero = true;
    return SPD_OK;
}

// The same in the context's scratch, grown on demand within the HBM budget: SPD_E_NOMEM (nothing
// enqueued) if it does not fit.
spd_status region_launch(spd_ctx *ctx, const BinGeometry &g, const std::vector<BatchDesc> &bd, uint32_t tiles,
                         const ChunkTable &ct, const SlotPtrs *sp, const ApplySlot *as, uint32_t nsl, hipStream_t s) {
    RegionArgs ra{};
    uint64_t items_words = 0, cur_words = 0;
    region_layout(ctx, g, ct, tiles, &ra, &items_words, &cur_words);
    if (ra.chunk_words >= (1ull << 31)) return fail(ctx, SPD_E_INVALID, "region layout: chunk too large");
    spd_status st = ensure_scratch(ctx, items_words, 0, s);
    if (!st) st = ensure_aux(ctx, cur_words, s);
    if (st) return st;
    const RegionScratch rs{ctx->items, ctx->items_words, ctx->aux, ctx->aux_words, &ctx->aux_zero, &ctx->spill_parity};
    return region_launch_at(ctx, g, bd.data(), (uint32_t)bd.size(), tiles, ct, sp, as, nsl, rs, s);
}

// Record batches into slots.  Batches of one slot are kept together so that each slot's tiles are
// one contiguous range of the binned launch.
spd_status scan_work(spd_ctx *ctx, std::vector<WorkItem> &ws, hipStream_t s) {
    std::stable_sort(ws.begin(), ws.end(), [](const WorkItem &x, const WorkItem &y) {
        return std::less<Slot *>()(x.slot, y.slot);
    });
    uint64_t total = 0;
    std::vector<Slot *> slots;
    for (auto &w : ws) {
        total += w.n;
        if (slots.empty() || slots.back() != w.slot) slots.push_back(w.slot);
    }
    if (total == 0) return SPD_OK;
    // direct-style launches (sliding stamps, or small batches): groups of kMaxGroup batches
    auto direct_launch = [&](bool stamp) -> spd_status {
        for (size_t i0 = 0; i0 < ws.size(); i0 += kMaxGroup) {
            BatchDesc bd[kMaxGroup];
            SlotPtrs sp[kMaxGroup] = {};
            uint32_t nbd = 0, nsl = 0;
            uint64_t n = 0;
            std::vector<Slot *> seen;
            for (size_t i = i0; i < std::min(ws.size(), i0 + kMaxGroup); ++i) {
                auto it = std::find(seen.begin(), seen.end(), ws[i].slot);
                uint32_t si = (uint32_t)(it - seen.begin());
                if (it == seen.end()) {
                    seen.push_back(ws[i].slot);
                    sp[nsl++] = ptrs_of(*ws[i].slot);
                }
                bd[nbd++] = BatchDesc{ws[i].pairs, ws[i].n, 0, si, ws[i].swap, 0};
                n = std::max(n, ws[i].n);
            }
            uint32_t block = ctx->tune.direct_block;
            uint64_t want = (n + block - 1) / block;
            uint32_t grid = (uint32_t)std::max<uint64_t>(
                1, std::min<uint64_t>(want, (uint64_t)ctx->tune.direct_grid_per_cu * ctx->n_cu));
            if (stamp) {
                ProfKernel pk(ctx, SPD_K_STAMP);
                const uint32_t value = ctx->at ? at_code(ctx->slice) : (ctx->slice + 1) & 0xFFFFu;
                SPD_HIP(ctx, launch_scan_stamp(ctx->c, bd, nbd, sp, value, ctx->at, block, grid, s, pk.kt));
            } else {
                const bool lds = ctx->tune.seav_lds && nsl == 1 && ctx->d.seav_bytes <= 64 * 1024;
                ProfScope ps(ctx, SPD_K_DIRECT, s);
                SPD_HIP(ctx, launch_scan_direct(ctx->c, bd, nbd, sp, block, grid, lds, s));
            }
            ctx->stats.direct_launches++;
        }
        ctx->stats.pairs_scanned += total;
        return SPD_OK;
    };
    if (ctx->sliding) return direct_launch(true);   // time stamps of the current slice, plain stores
    BinGeometry g{};
    const bool binned = total > ctx->tune.direct_max_pairs && ctx->p.lr <= 4 && bin_geometry(ctx, &g);
    const bool bm = ctx->tune.bin_mode != 0;
    if (!binned) {
        for (Slot *sl : slots)
            if (sl->fresh) {
                spd_status st = clear_slot(ctx, *sl, s);
                if (st) return st;
            }
        return direct_launch(false);
    }
    // Binned: a slot's flags change only once a group covering it has been enqueued, so that an
    // error return (a budget refusal before anything was enqueued) leaves every slot as it was.
    // A fresh slot's buckets are written from zero by the apply phase of the region layout; the
    // other two layouts do so for its LDCA buckets and clear its SEAV inside the scan (the counting
    // kernel, or a fill before the per-tile binning).
    // later groups of the same call OR into the slots an enqueued group has written
    auto mark_written = [](Slot *const *owner, uint32_t n) {
        for (uint32_t k = 0; k < n; ++k) owner[k]->fresh = false;
    };
    // split batches larger than one launch may take: launch_pairs, and for the region and
    // exact-count layouts the 32-bit item offsets of one launch (tiles * cap < 2^32)
    const uint64_t lp = ctx->tune.launch_pairs;
    uint64_t split_at = lp;
    if (bm) {
        const uint64_t max_pairs = (((1ull << 32) - 1) / g.cap - 1) * g.tile_pairs;
        split_at = split_at ? std::min(split_at, max_pairs) : max_pairs;
    }
    if (split_at) {
        std::vector<WorkItem> split;
        for (auto &w : ws)
            for (uint64_t a = 0; a < w.n; a += split_at)
                split.push_back(WorkItem{w.slot, w.pairs + 2 * a, std::min(split_at, w.n - a), w.swap});
        ws.swap(split);
    }
    // binned: launch groups of at most kMaxGroup slots and launch_pairs pairs; per-tile regions also
    // take at most kMaxGroup batches per group, the region and exact-count layouts any number (one
    // launch of each kernel per group, so each slot's buckets are read and written once per group)
    size_t i0 = 0;
    while (i0 < ws.size()) {
        const size_t group_start = i0;
        std::vector<BatchDesc> bd;
        SlotPtrs sp[kMaxGroup] = {};
        ApplySlot as[kMaxGroup] = {};
        Slot *owner[kMaxGroup] = {};
        uint32_t nsl = 0, tiles = 0;
        uint64_t lpairs = 0;
        size_t i = i0;
        for (; i < ws.size() && (bm || bd.size() < (size_t)kMaxGroup); ++i) {
            const WorkItem &w = ws[i];
            if (w.n == 0) continue;
            if (lp && !bd.empty() && lpairs + w.n > lp) break;
            const uint64_t nt = (w.n + g.tile_pairs - 1) / g.tile_pairs;
            // a group ends before its item offsets would pass 32 bits
            if (bm && !bd.empty() && ((uint64_t)tiles + nt) * g.cap >= (1ull << 32)) break;
            lpairs += w.n;
            if (nsl == 0 || owner[nsl - 1] != w.slot) {
                if (nsl == (uint32_t)kMaxGroup) break;
                sp[nsl] = ptrs_of(*w.slot);
                as[nsl].ldca = w.slot->ldca;
                as[nsl].seav_w = reinterpret_cast<uint32_t *>(w.slot->seav);
                as[nsl].tile_lo = tiles;
                // a fresh slot's buckets are written from zero by this launch
                as[nsl].fresh = w.slot->fresh ? 1u : 0u;
                owner[nsl] = w.slot;
                ++nsl;
            }
            if ((uint64_t)tiles + nt > 0x7FFFFFFFull) return fail(ctx, SPD_E_INVALID, "batch too large");
            bd.push_back(BatchDesc{w.pairs, w.n, tiles, nsl - 1, w.swap, 0});
            tiles += (uint32_t)nt;
            as[nsl - 1].tile_hi = tiles;
        }
        i0 = i;
        const uint32_t nbd = (uint32_t)bd.size();
        if (nbd == 0) continue;
        uint64_t items_words, meta_words;
        scratch_need(g, ctx->tune.bin_mode, tiles, &items_words, &meta_words);
        if (ctx->tune.bin_mode == 0) {
            spd_status st = ensure_scratch(ctx, items_words, meta_words, s);
            if (st) return st;
            for (uint32_t k = 0; k < nsl; ++k)   // SEAV bits may be recorded directly by the binning
                if (as[k].fresh) {
                    st = clear_seav(ctx, *owner[k], s);
                    if (st) return st;
                }
            {
                ProfScope ps(ctx, SPD_K_BIN, s);
                SPD_HIP(ctx, launch_bin(ctx->c, g, bd.data(), nbd, tiles, ctx->items, ctx->meta, sp, s));
            }
            {
                ProfScope ps(ctx, SPD_K_TRANSPOSE, s);
                SPD_HIP(ctx, launch_transpose(ctx->meta, ctx->metaT, tiles, g.nb + 1, s));
            }
            {
                ProfScope ps(ctx, SPD_K_APPLY, s);
                SPD_HIP(ctx, launch_apply(g, as, nsl, ctx->items, ctx->metaT, tiles, ctx->tune.apply_block,
                                          ctx->tune.apply_unroll, s));
            }
        } else {
            if ((uint64_t)tiles * g.cap >= (1ull << 32))
                return fail(ctx, SPD_E_INVALID, "launch too large for 32-bit item offsets");
            // chunks of kChunk tiles, per slot
            ChunkTable ct{};
            ct.n = nsl;
            for (uint32_t k = 0; k < nsl; ++k) {
                ct.lo[k] = as[k].tile_lo;
                ct.hi[k] = as[k].tile_hi;
                ct.cbase[k + 1] = ct.cbase[k] + (as[k].tile_hi - as[k].tile_lo + kChunk - 1) / kChunk;
            }
            const uint32_t chunks = ct.cbase[nsl];
            if (ctx->tune.bin_mode == 2) {
                // the exact-count layout (less scratch) if the region layout does not fit the budget
                ctx->merge_group = ctx->merge_into && group_start == 0 && i0 == ws.size();
                spd_status st = region_launch(ctx, g, bd, tiles, ct, sp, as, nsl, s);
                ctx->merge_group = false;
                if (st && st != SPD_E_NOMEM) return st;
                if (!st) {
                    mark_written(owner, nsl);
                    ctx->stats.binned_launches++;
                    continue;
                }
            }
            spd_status st = ensure_scratch(ctx, items_words, meta_words, s);
            if (!st) st = ensure_aux(ctx, (uint64_t)nsl * g.nb + 1 + (uint64_t)chunks * g.nb, s);
            if (st) return st;
            uint32_t *base = ctx->aux, *cstart = ctx->aux + nsl * g.nb + 1;
            ctx->aux_zero = false;
            // the batch descriptors go to device memory through a pinned staging ring
            BatchDesc *bdev = nullptr;
            st = upload_batches(ctx, bd.data(), bd.size(), s, &bdev);
            if (st) return st;
            ClearList cl{};
            for (uint32_t k = 0; k < nsl; ++k)
                if (as[k].fresh) {
                    cl.p[cl.n] = as[k].seav_w;
                    cl.words[cl.n++] = ctx->seav_alloc / 4;
                }
            {
                ProfScope ps(ctx, SPD_K_COUNT, s);
                SPD_HIP(ctx, launch_count(ctx->c, g, bdev, nbd, tiles, ctx->meta, cl, s));
            }
            {
                ProfScope ps(ctx, SPD_K_OFFSETS, s);
                // counts stay in meta for k_place; offsets inside each chunk go to metaB
                SPD_HIP(ctx, launch_offsets(ctx->meta, ctx->metaB, cstart, base, ct, g.nb, s));
            }
            {
                ProfScope ps(ctx, SPD_K_BIN, s);
                SPD_HIP(ctx, launch_place(ctx->c, g, bdev, nbd, tiles, ctx->items, ctx->meta, ctx->metaB, cstart, ct, sp, s));
                // the staging slot may be rewritten once the placement kernel has read it
                SPD_HIP(ctx, hipEventRecord(ctx->bd_ev[ctx->bd_next], s));
                ctx->bd_next = (ctx->bd_next + 1) % kBdRing;
            }
            {
                ProfScope ps(ctx, SPD_K_APPLY, s);
                SPD_HIP(ctx, launch_apply_bm(g, as, nsl, ctx->items, base, ctx->tune.apply_block, ctx->tune.apply_unroll, s));
            }
        }
        mark_written(owner, nsl);
        ctx->stats.binned_launches++;
    }
    ctx->stats.pairs_scanned += total;
    return SPD_OK;
}

// Scan of one batch into one slot with no allocation: the direct kernel for small batches (no
// scratch), else the region layout with its scratch in the no-alloc array, in launches of as many
// tiles as that array holds.  No timing events, no descriptor ring (one inline batch per launch).
spd_status scan_noalloc(spd_ctx *ctx, Slot *sl, const uint32_t *pairs, uint64_t n, uint32_t swap, hipStream_t s) {
    BinGeometry g{};
    const bool binned = n > ctx->tune.direct_max_pairs && ctx->p.lr <= 4 && bin_geometry(ctx, &g);
    if (!binned) {
        if (sl->fresh) {
            spd_status st = clear_slot(ctx, *sl, s);
            if (st) return st;
        }
        BatchDesc bd[1] = {BatchDesc{pairs, n, 0, 0, swap, 0}};
        SlotPtrs sp[kMaxGroup] = {};
        sp[0] = ptrs_of(*sl);
        const uint32_t block = ctx->tune.direct_block;
        const uint64_t want = (n + block - 1) / block;
        const uint32_t grid = (uint32_t)std::max<uint64_t>(
            1, std::min<uint64_t>(want, (uint64_t)ctx->tune.direct_grid_per_cu * ctx->n_cu));
        const bool lds = ctx->tune.seav_lds && ctx->d.seav_bytes <= 64 * 1024;
        SPD_HIP(ctx, launch_scan_direct(ctx->c, bd, 1, sp, block, grid, lds, s));
        ctx->stats.direct_launches++;
        ctx->stats.pairs_scanned += n;
        return SPD_OK;
    }
    // the most tiles per launch whose region layout (items, spill list, counters) fits the array;
    // the layout grows with the tile count, so a binary search finds it
    const uint64_t cap = SPD_NOALLOC_SCRATCH_BYTES;
    auto layout_of = [&](uint32_t tiles, ChunkTable *ct, uint64_t *iw, uint64_t *cw) {
        *ct = ChunkTable{};
        ct->n = 1;
        ct->hi[0] = tiles;
        ct->cbase[1] = (tiles + kChunk - 1) / kChunk;
        RegionArgs ra{};
        region_layout(ctx, g, *ct, tiles, &ra, iw, cw);
        return ra.chunk_words < (1ull << 31);
    };
    auto fits = [&](uint32_t tiles) {
        ChunkTable ct;
        uint64_t iw, cw;
        if (!layout_of(tiles, &ct, &iw, &cw)) return false;
        return (cw * 4 + 255) / 256 * 256 + iw * 4 <= cap;
    };
    if (!fits(1))
        return fail(ctx, SPD_E_INVALID, "spd_scan_noalloc: one tile of this sketch geometry needs more scratch than "
                                        "SPD_NOALLOC_SCRATCH_BYTES");
    uint32_t lo = 1, hi = (uint32_t)std::min<uint64_t>((n + g.tile_pairs - 1) / g.tile_pairs, 1u << 20);
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (fits(mid)) lo = mid;
        else hi = mid - 1;
    }
    const uint32_t tmax = lo;
    ChunkTable ct;
    uint64_t iw, cw;
    layout_of(tmax, &ct, &iw, &cw);
    const uint64_t aux_bytes = (cw * 4 + 255) / 256 * 256;
    // counters first (cleared by the first launch of this call: the array keeps the last call's
    // contents), then the regions and the spill list
    bool aux_zero = false;
    uint32_t parity = 0;
    const RegionScratch rs{reinterpret_cast<uint32_t *>(ctx->noalloc + aux_bytes), (cap - aux_bytes) / 4,
                           reinterpret_cast<uint32_t *>(ctx->noalloc), cw, &aux_zero, &parity};
    const uint64_t max_pairs = (uint64_t)tmax * g.tile_pairs;
    for (uint64_t off = 0; off < n; off += max_pairs) {
        const uint64_t cn = std::min(max_pairs, n - off);
        const uint32_t tiles = (uint32_t)((cn + g.tile_pairs - 1) / g.tile_pairs);
        layout_of(tiles, &ct, &iw, &cw);
        const BatchDesc bd{pairs + 2 * off, cn, 0, 0, swap, 0};
        SlotPtrs sp[kMaxGroup] = {};
        ApplySlot as[kMaxGroup] = {};
        sp[0] = ptrs_of(*sl);
        as[0] = ApplySlot{sl->ldca, reinterpret_cast<uint32_t *>(sl->seav), 0, tiles, sl->fresh ? 1u : 0u, 0};
        spd_status st = region_launch_at(ctx, g, &bd, 1, tiles, ct, sp, as, 1, rs, s);
        if (st) return st;
        sl->fresh = false;
        ctx->stats.binned_launches++;
    }
    ctx->stats.pairs_scanned += n;
    return SPD_OK;
}

// ------------------------------------------------------------------------------ end of window
spd_status close_rec_alloc(spd_ctx *ctx, CloseBuf &cb, uint32_t cap) {
    dev_free(ctx, &cb.counters, 16 + (uint64_t)cb.rec_cap * 8);
    cb.rec = nullptr;
    cb.rec_cap = 0;
    spd_status st = dev_alloc(ctx, &cb.counters, 16 + (uint64_t)cap * 8);
    if (st) return st;
    SPD_HIP(ctx, hipMemset(cb.counters, 0, 16));   // once; each launch leaves them zero
    cb.rec = cb.counters + 4;
    cb.rec_cap = cap;
    cb.seq = 0;   // (no close of this buffer is in flight)
    if (cb.h_counters) cb.h_counters[2] = 0;
    return SPD_OK;
}

spd_status close_buf_init(spd_ctx *ctx, CloseBuf &cb) {
    if (!cb.counters) {
        spd_status st = close_rec_alloc(ctx, cb, kRecInit);
        if (st) return st;
    }
    if (ctx->sliding && !cb.seav_bits) {
        spd_status st = dev_alloc(ctx, &cb.seav_bits, ctx->seav_alloc);
        if (st) return st;
    }
    if (!cb.h_counters) {
        SPD_HIP(ctx, hipHostMalloc((void **)&cb.h_counters, 16 + (uint64_t)kRecChunk * 8, hipHostMallocMapped));
        SPD_HIP(ctx, hipHostGetDevicePointer((void **)&cb.d_counters, cb.h_counters, 0));
        std::memset(cb.h_counters, 0, 16);
    }
    return SPD_OK;
}

void close_buf_free(spd_ctx *ctx, CloseBuf &cb) {
    if (cb.graph) (void)hipGraphExecDestroy(cb.graph);
    cb.graph = nullptr;
    dev_free(ctx, &cb.counters, 16 + (uint64_t)cb.rec_cap * 8);
    cb.rec = nullptr;
    dev_free(ctx, &cb.seav_bits, ctx->seav_alloc);
    if (cb.h_counters) (void)hipHostFree(cb.h_counters);
    if (cb.h_rec) (void)hipHostFree(cb.h_rec);
    cb.h_counters = nullptr;
    cb.d_counters = nullptr;
    cb.h_rec = nullptr;
    cb.rec_cap = cb.h_rec_cap = 0;
}

int close_mode(const spd_ctx *ctx) { return ctx->at ? kCloseAt : ctx->sliding ? kCloseStamps : kCloseBits; }

// Arguments and launch shape of the end-of-window kernel for one slot.
spd_status close_args(spd_ctx *ctx, const Slot &sl, const CloseBuf &cb, CloseArgs *a, uint32_t *block, uint32_t *grid) {
    *a = CloseArgs{};
    a->seav = ctx->sliding ? cb.seav_bits : sl.seav;
    a->ldca = sl.ldca;
    a->ldca_ts = sl.ldca_ts;
    a->ldca_at = sl.ldca_at;
    a->at_ct = at_code(ctx->slice);
    a->at_k = ctx->K;
    if (ctx->sliding) {
        const int64_t lo = (int64_t)ctx->slice - (int64_t)ctx->K + 2;
        a->thr = lo < 1 ? 1u : (uint32_t)lo;
    }
    a->counters = cb.counters;
    a->rec = cb.rec;
    a->rec_cap = cb.rec_cap;
    a->host_out = cb.d_counters;
    a->host_recs = std::min(cb.rec_cap, kRecChunk);
    a->n_rp = 1u << ctx->p.r;
    uint32_t max_ibn = 0;
    for (uint32_t i = 0; i < ctx->p.sr; ++i) max_ibn = std::max(max_ibn, ctx->d.ibn[i]);
    a->list_stride = 1u << max_ibn;
    a->qcap = 256;
    // each wavefront stages its SEA in LDS when that fits next to the hot lists (else it reads
    // the SEA from global memory)
    const uint64_t lists = (uint64_t)ctx->p.sr * a->list_stride + a->qcap;
    const uint64_t stage = (ctx->d.sea_bytes + 3) / 4;
    a->stage_words = (lists + stage) * 4ull <= kMaxLds ? (uint32_t)stage : 0u;
    const uint64_t per_wave = lists + a->stage_words;
    uint32_t b = ctx->tune.close_block;
    while (b > 64 && (b / 64) * per_wave * 4ull > kMaxLds) b /= 2;
    if ((b / 64) * per_wave * 4ull > kMaxLds)
        return fail(ctx, SPD_E_INVALID, "SEA rows too large for the end-of-window kernel");
    const uint32_t waves = b / 64;
    *block = b;
    // one round of resident workgroups; each wavefront then takes (SEA, part) items round robin.
    // With fewer SEAs than resident wavefronts, each SEA's candidate search is split into parts
    // (a power of two, at most 64) so that every wavefront has work.
    if (!ctx->close_per_cu[b / 128])
        ctx->close_per_cu[b / 128] = close_blocks_per_cu(close_mode(ctx), b, (uint32_t)((b / 64) * per_wave * 4));
    const uint64_t resident = (uint64_t)ctx->n_cu * ctx->close_per_cu[b / 128];
    a->parts_log2 = 0;
    while (a->parts_log2 < 6 && ((uint64_t)a->n_rp << (a->parts_log2 + 1)) <= resident * waves) a->parts_log2++;
    // In sliding mode a candidate's filter reads the counters behind its LDCs (8 or 16 bits a bit),
    // so filtering, not the SEA, dominates a work item: every SEA is split at least in two, which
    // halves the longest run of candidates one wavefront filters.
    if (ctx->sliding && a->parts_log2 < 1) a->parts_log2 = 1;
    // With few SEAs (small sketches), one level finer than the resident wavefronts ask for: the
    // largest SEA's share then bounds the pass less (64 SEAs of 2 KiB, 1,000,000 pairs: the close
    // 21.7 -> 20.5 us).
    if (a->n_rp <= 1024 && a->parts_log2 < 6) a->parts_log2++;
    const uint64_t want = (((uint64_t)a->n_rp << a->parts_log2) + waves - 1) / waves;
    *grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, resident));
    return SPD_OK;
}

// The device part of the end of window: k_close, then k_close_out, which leaves the counters and
// the first kRecChunk records in pinned host memory (and the device counters zero).  Asynchronous
// on s.
spd_status close_launch_ops(spd_ctx *ctx, const Slot &sl, CloseBuf &cb, hipStream_t s) {
    CloseArgs a;
    uint32_t block, grid;
    spd_status st = close_args(ctx, sl, cb, &a, &block, &grid);
    if (st) return st;
    ProfScope ps(ctx, SPD_K_CLOSE, s);
    if (ctx->at)   // the SEAV's bit view first, streamed at full bandwidth (canonical bit order)
        SPD_HIP(ctx, launch_bit_view_at(sl.seav_at, ctx->seav_alloc * 8, a.at_ct, ctx->K, reinterpret_cast<uint32_t *>(cb.seav_bits), s));
    else if (ctx->sliding)
        SPD_HIP(ctx, launch_bit_view(sl.seav_ts, ctx->seav_alloc * 8, (uint16_t)a.thr, reinterpret_cast<uint32_t *>(cb.seav_bits), s));
    SPD_HIP(ctx, launch_close(ctx->c, a, close_mode(ctx), block, grid, s));
    ++cb.seq;
    return SPD_OK;
}

// Waits for the close last enqueued on cb: polls the sequence number that its last kernel writes
// to mapped host memory (no interrupt and no sleep between the kernel's end and the report), and
// past kCloseSpinMs waits for `ev` (or the stream) instead, which also reports a failed launch.
constexpr int kCloseSpinMs = 20;
spd_status close_wait(spd_ctx *ctx, const CloseBuf &cb, hipStream_t s, hipEvent_t ev = nullptr) {
    const volatile uint32_t *flag = cb.h_counters + 2;
    const auto t0 = std::chrono::steady_clock::now();
    for (uint32_t it = 1;; ++it) {
        if (*flag == cb.seq) {
            std::atomic_thread_fence(std::memory_order_acquire);
            return SPD_OK;
        }
        if ((it & 255u) == 0 && std::chrono::steady_clock::now() - t0 > std::chrono::milliseconds(kCloseSpinMs)) break;
        __builtin_ia32_pause();
    }
    if (ev) SPD_HIP(ctx, hipEventSynchronize(ev));
    else SPD_HIP(ctx, hipStreamSynchronize(s));
    return SPD_OK;
}

spd_status close_launch(spd_ctx *ctx, const Slot &sl, CloseBuf &cb, hipStream_t s) {
    cb.empty = !ctx->sliding && sl.fresh;
    if (cb.empty) return SPD_OK;
    spd_status st = close_buf_init(ctx, cb);
    if (st) return st;
    return close_launch_ops(ctx, sl, cb, s);
}

// Same device work replayed from a hipGraph captured once per (slot, buffer); discrete mode only.
spd_status close_launch_graph(spd_ctx *ctx, const Slot &sl, CloseBuf &cb, hipStream_t s) {
    cb.empty = sl.fresh;
    if (cb.empty) return SPD_OK;
    spd_status st = close_buf_init(ctx, cb);
    if (st) return st;
    if (!cb.graph || cb.graph_slot != &sl || cb.graph_rec != cb.rec) {
        if (cb.graph) (void)hipGraphExecDestroy(cb.graph);
        cb.graph = nullptr;
        hipGraph_t g = nullptr;
        const bool prof = ctx->prof_on;
        ctx->prof_on = false;   // no event nodes inside the graph
        const uint32_t seq = cb.seq;   // (capture runs nothing)
        SPD_HIP(ctx, hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
        spd_status cst = close_launch_ops(ctx, sl, cb, s);
        hipError_t e = hipStreamEndCapture(s, &g);
        cb.seq = seq;
        ctx->prof_on = prof;
        if (cst) {
            if (g) (void)hipGraphDestroy(g);
            return cst;
        }
        if (e != hipSuccess) return hip_fail(ctx, e, "hipStreamEndCapture");
        e = hipGraphInstantiate(&cb.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) return hip_fail(ctx, e, "hipGraphInstantiate");
        cb.graph_slot = &sl;
        cb.graph_rec = cb.rec;
    }
    ProfScope ps(ctx, SPD_K_CLOSE, s);
    SPD_HIP(ctx, hipGraphLaunch(cb.graph, s));
    ++cb.seq;
    return SPD_OK;
}

// The report of a finished close whose first n records (n <= rec_cap) are in cb: fetch those past
// the first chunk (a copy on s), Eq. 4 estimates, sorted by ip.
spd_status close_report(spd_ctx *ctx, CloseBuf &cb, uint32_t n, hipStream_t s, std::vector<spd_superpoint> *out) {
    ctx->stats.candidates_last = cb.h_counters[1];
    if (n > kRecChunk) {
        if (n > cb.h_rec_cap) {
            (void)hipHostFree(cb.h_rec);
            cb.h_rec = nullptr;
            cb.h_rec_cap = 0;
            SPD_HIP(ctx, hipHostMalloc((void **)&cb.h_rec, (uint64_t)n * 8, hipHostMallocDefault));
            cb.h_rec_cap = n;
        }
        SPD_HIP(ctx, hipMemcpyAsync(cb.h_rec, cb.rec, (uint64_t)n * 8, hipMemcpyDeviceToHost, s));
        SPD_HIP(ctx, hipStreamSynchronize(s));
    }
    out->resize(n);
    const uint32_t kmax = 1u << ctx->p.log2k;
    const uint32_t *hr = n > kRecChunk ? cb.h_rec : cb.h_counters + 4;
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t z0 = hr[2 * i + 1];
        (*out)[i] = spd_superpoint{hr[2 * i], z0, ctx->est[std::min(z0, kmax)], z0 == 0 ? 1u : 0u};
    }
    std::sort(out->begin(), out->end(), [](const spd_superpoint &x, const spd_superpoint &y) { return x.ip < y.ip; });
    ctx->stats.reported_last = n;
    return SPD_OK;
}

// Host part, after the launched work has completed: fetch records beyond the first chunk, grow
// the record buffer and run again if it overflowed (the pass is deterministic), build the sorted
// report with Eq. 4 estimates.  Discrete mode: the slot becomes fresh (next window from zero).
spd_status close_finish(spd_ctx *ctx, Slot &sl, CloseBuf &cb, hipStream_t s, std::vector<spd_superpoint> *out) {
    out->clear();
    ctx->stats.closes++;
    if (cb.empty) {
        ctx->stats.candidates_last = 0;
        ctx->stats.reported_last = 0;
        return SPD_OK;
    }
    uint32_t n = cb.h_counters[0];
    if (n > cb.rec_cap) {
        spd_status st = close_rec_alloc(ctx, cb, n + 1024);
        if (st) return st;
        st = close_launch_ops(ctx, sl, cb, s);
        if (st) return st;
        SPD_HIP(ctx, hipStreamSynchronize(s));
        n = cb.h_counters[0];
    }
    spd_status st = close_report(ctx, cb, n, s, out);
    if (st) return st;
    if (!ctx->sliding) sl.fresh = true;   // the next window starts from zero
    return SPD_OK;
}

// ------------------------------------------------------------------------------ contexts
spd_status slot_alloc(spd_ctx *ctx, Slot &sl) {
    spd_status st = dev_alloc(ctx, &sl.mem, ctx->slot_bytes);
    if (st) return st;
    const uint64_t ldca_bytes = ctx->ldca_bytes;
    if (ctx->at) {
        sl.ldca_at = static_cast<uint8_t *>(sl.mem);
        sl.seav_at = sl.ldca_at + ldca_bytes * 8;
        SPD_HIP(ctx, launch_fill_u32(static_cast<uint32_t *>(sl.mem), ctx->slot_bytes / 4, empty_fill(ctx), nullptr));
        sl.fresh = false;
    } else if (ctx->sliding) {
        sl.ldca_ts = static_cast<uint16_t *>(sl.mem);
        sl.seav_ts = sl.ldca_ts + ldca_bytes * 8;
        SPD_HIP(ctx, launch_fill_u32(static_cast<uint32_t *>(sl.mem), ctx->slot_bytes / 4, 0u, nullptr));
        sl.fresh = false;
    } else {
        sl.ldca = static_cast<uint32_t *>(sl.mem);
        sl.seav = static_cast<uint8_t *>(sl.mem) + ldca_bytes;
        sl.fresh = true;
    }
    return SPD_OK;
}

// A context with n_slots sketch slots; spd_create uses routers + the global sketch, the serving
// loop allocates its own window slots.
spd_status ctx_create(const spd_params *p, uint32_t n_routers, uint32_t n_slots, uint64_t budget, spd_ctx **out) {
    spd_ctx *ctx = new (std::nothrow) spd_ctx();
    if (!ctx) return SPD_E_NOMEM;
    std::string why;
    spd_status st = derive(p, &ctx->d, &why);
    if (st) {
        delete ctx;
        return st;
    }
    ctx->p = *p;
    ctx->n_routers = n_routers;
    ctx->budget = budget;
    ctx->sliding = p->window_slices > 0;
    ctx->K = p->window_slices;
    ctx->at = ctx->sliding && p->sliding_counter == 0;
    ctx->at_groups = ctx->at ? kAtCodes - 1u - ctx->K : 0;   // K + G = 255: ages read mod 256 stay exact
    default_tuning(&ctx->tune);
    if (hipGetDevice(&ctx->device) != hipSuccess) {
        delete ctx;
        return SPD_E_HIP;
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
        ctx->n_cu = (uint32_t)prop.multiProcessorCount;
    // kernel constants
    Consts &c = ctx->c;
    for (uint32_t i = 0; i < 3 + p->lr; ++i) {
        c.mul[i] = p->hash_mul[i];
        c.add[i] = p->hash_add[i];
    }
    c.tau_mask = (uint32_t)((1ull << ctx->d.tau) - 1ull);
    c.r = p->r;
    c.L = 32 - p->r;
    c.sr = p->sr;
    c.lr = p->lr;
    c.rmask = (uint32_t)((1ull << p->r) - 1ull);
    c.log2k = p->log2k;
    c.log2lc = p->log2lc;
    c.sh_k = (32u - p->log2k) & 31u;
    c.sh_lc = (32u - p->log2lc) & 31u;
    if (p->log2lc == 0)   // one column: every LH_i is the constant 0
        for (uint32_t i = 0; i < p->lr; ++i) c.mul[3 + i] = c.add[3 + i] = 0;
    uint32_t off = 0;
    for (uint32_t i = 0; i < p->sr; ++i) {
        c.isb[i] = ctx->d.isb[i];
        c.ibn[i] = ctx->d.ibn[i];
        c.row_off[i] = off;
        off += 1u << ctx->d.ibn[i];
    }
    c.sea_bytes = (uint32_t)ctx->d.sea_bytes;
    c.z_theta = ctx->d.z_theta;
    c.ldca_bits = ctx->d.ldca_words * 32;
    c.seav_bytes = ctx->d.seav_bytes;
    // Eq. 4 estimate for every z0, computed once in double
    ctx->est.resize((1u << p->log2k) + 1);
    const double k = std::ldexp(1.0, (int)p->log2k);
    for (uint32_t z = 0; z <= (1u << p->log2k); ++z)
        ctx->est[z] = (uint32_t)std::floor(-k * std::log((double)(z ? z : 1) / k) + 0.5);

    DeviceGuard dg(ctx->device);
    {
        // the no-alloc scan's scratch on this device; a failed lookup disables only that entry point
        const hipError_t e = noalloc_lookup(ctx->device, &ctx->noalloc);
        if (e != hipSuccess) ctx->noalloc_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
    }
    ctx->seav_alloc = (ctx->d.seav_bytes + kSeavAlign - 1) / kSeavAlign * kSeavAlign;
    ctx->ldca_bytes = (ctx->d.ldca_words * 4 + 255) / 256 * 256;   // SEAV starts 256-byte aligned
    // sliding: one 16-bit stamp or one 8-bit AT counter per bit
    ctx->slot_bytes = ctx->at        ? (ctx->ldca_bytes * 8 + ctx->seav_alloc * 8)
                      : ctx->sliding ? (ctx->ldca_bytes * 16 + ctx->seav_alloc * 16)
                                     : (ctx->ldca_bytes + ctx->seav_alloc);
    ctx->slots.resize(n_slots);
    for (auto &sl : ctx->slots) {
        st = slot_alloc(ctx, sl);
        if (st) {
            spd_destroy(ctx);
            return st;
        }
    }
    if (close_buf_init(ctx, ctx->cbuf) || hipEventCreateWithFlags(&ctx->order_ev, hipEventDisableTiming) != hipSuccess) {
        spd_destroy(ctx);
        return SPD_E_HIP;
    }
    if (hipDeviceSynchronize() != hipSuccess) {
        spd_destroy(ctx);
        return SPD_E_HIP;
    }
    ctx->stats.device_bytes = ctx->held;
    *out = ctx;
    return SPD_OK;
}

spd_status validate_batch(spd_ctx *ctx, const spd_batch &b) {
    if (b.router >= ctx->n_routers) return fail(ctx, SPD_E_STATE, "router id out of range");
    if (b.flags & ~SPD_BATCH_DST) return fail(ctx, SPD_E_INVALID, "unknown spd_batch flags");
    if (b.n_pairs && !b.pairs_dev) return fail(ctx, SPD_E_INVALID, "null pair buffer");
    if (reinterpret_cast<uintptr_t>(b.pairs_dev) % 8) return fail(ctx, SPD_E_INVALID, "pair buffer must be 8-byte aligned");
    if (b.n_pairs > (1ull << 40)) return fail(ctx, SPD_E_INVALID, "batch too large");
    return SPD_OK;
}

}  // namespace

// ==============================================================================================
extern "C" {

spd_status spd_derive(const spd_params *p, spd_derived *out) { return derive(p, out, nullptr); }

spd_status spd_create(const spd_params *p, uint32_t n_routers, uint64_t hbm_budget_bytes, spd_ctx **out) {
    if (!out) return SPD_E_INVALID;
    *out = nullptr;
    if (n_routers < 1 || n_routers > 4096) return SPD_E_INVALID;
    return ctx_create(p, n_routers, n_routers + 1, hbm_budget_bytes, out);
}

void spd_destroy(spd_ctx *ctx) {
    if (!ctx) return;
    {
        DeviceGuard dg(ctx->device);
        (void)hipDeviceSynchronize();
        for (auto &sl : ctx->slots) dev_free(ctx, &sl.mem, ctx->slot_bytes);
        dev_free(ctx, &ctx->items, ctx->items_words * 4);
        dev_free(ctx, &ctx->meta, ctx->meta_words * 4);
        dev_free(ctx, &ctx->metaT, ctx->meta_words * 4);
        dev_free(ctx, &ctx->metaB, ctx->meta_words * 4);
        dev_free(ctx, &ctx->aux, ctx->aux_words * 4);
        free_batch_ring(ctx);
        for (auto &e : ctx->bd_ev)
            if (e) (void)hipEventDestroy(e);
        for (int k = 0; k < 2; ++k) {
            dev_free(ctx, &ctx->h2d_buf[k], ctx->h2d_words * 4);
            if (ctx->h2d_copied[k]) (void)hipEventDestroy(ctx->h2d_copied[k]);
            if (ctx->h2d_scanned[k]) (void)hipEventDestroy(ctx->h2d_scanned[k]);
        }
        if (ctx->h2d_s) (void)hipStreamDestroy(ctx->h2d_s);
        close_buf_free(ctx, ctx->cbuf);
        for (auto &pc : ctx->pend) {
            close_buf_free(ctx, pc.cb);
            if (pc.done) (void)hipEventDestroy(pc.done);
        }
        if (ctx->copy_s) (void)hipStreamDestroy(ctx->copy_s);
        dev_free(ctx, &ctx->view, ctx->view_words * 4);
        if (ctx->order_ev) (void)hipEventDestroy(ctx->order_ev);
        prof_harvest(ctx);
        for (auto e : ctx->prof_pool) (void)hipEventDestroy(e);
    }
    delete ctx;
}

spd_status spd_scan(spd_ctx *ctx, uint32_t router, const uint32_t *pairs_dev, uint64_t n_pairs, void *stream) {
    if (!ctx) return SPD_E_INVALID;
    spd_batch b{router, 0, pairs_dev, n_pairs};
    return spd_scan_batches(ctx, &b, 1, stream);
}

spd_status spd_scan_noalloc(spd_ctx *ctx, uint32_t router, const uint32_t *pairs_dev, uint64_t n_pairs, uint32_t flags,
                            void *stream) {
    if (!ctx) return SPD_E_INVALID;
    spd_status st = validate_batch(ctx, spd_batch{router, flags, pairs_dev, n_pairs});
    if (st) return st;
    if (ctx->sliding) return fail(ctx, SPD_E_STATE, "spd_scan_noalloc: discrete-window contexts only");
    if (!ctx->noalloc) return fail(ctx, SPD_E_HIP, "spd_scan_noalloc: " + ctx->noalloc_err);
    if (n_pairs == 0) return SPD_OK;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    order_stream(ctx, s);
    const bool prof = ctx->prof_on;   // timing would create events
    ctx->prof_on = false;
    st = scan_noalloc(ctx, &ctx->slots[router], pairs_dev, n_pairs, (flags & SPD_BATCH_DST) ? 1u : 0u, s);
    ctx->prof_on = prof;
    return st;
}

spd_status spd_scan_host(spd_ctx *ctx, uint32_t router, const uint32_t *pairs_host, uint64_t n_pairs, uint32_t flags,
                         uint64_t chunk_pairs, void *stream) {
    if (!ctx) return SPD_E_INVALID;
    if (router >= ctx->n_routers) return fail(ctx, SPD_E_STATE, "router id out of range");
    if (flags & ~SPD_BATCH_DST) return fail(ctx, SPD_E_INVALID, "unknown flags");
    if (n_pairs && !pairs_host) return fail(ctx, SPD_E_INVALID, "null pair buffer");
    if (n_pairs > (1ull << 40)) return fail(ctx, SPD_E_INVALID, "batch too large");
    if (n_pairs == 0) return SPD_OK;
    if (chunk_pairs == 0) chunk_pairs = 16ull << 20;
    chunk_pairs = std::min<uint64_t>(chunk_pairs, n_pairs);
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    order_stream(ctx, s);
    if (!ctx->h2d_s) {
        SPD_HIP(ctx, hipStreamCreateWithFlags(&ctx->h2d_s, hipStreamNonBlocking));
        for (int k = 0; k < 2; ++k) {
            SPD_HIP(ctx, hipEventCreateWithFlags(&ctx->h2d_copied[k], hipEventDisableTiming));
            SPD_HIP(ctx, hipEventCreateWithFlags(&ctx->h2d_scanned[k], hipEventDisableTiming));
        }
    }
    if (2 * chunk_pairs > ctx->h2d_words) {
        SPD_HIP(ctx, hipStreamSynchronize(s));
        for (int k = 0; k < 2; ++k) dev_free(ctx, &ctx->h2d_buf[k], ctx->h2d_words * 4);
        ctx->h2d_words = 0;
        for (int k = 0; k < 2; ++k) {
            spd_status st = dev_alloc(ctx, &ctx->h2d_buf[k], chunk_pairs * 8);
            if (st) return st;
        }
        ctx->h2d_words = 2 * chunk_pairs;
    }
    const uint32_t swap = (flags & SPD_BATCH_DST) ? 1u : 0u;
    uint64_t i = 0;
    for (uint64_t off = 0; off < n_pairs; off += chunk_pairs, ++i) {
        const int k = (int)(i & 1);
        const uint64_t cn = std::min(chunk_pairs, n_pairs - off);
        // staging buffer k is free once the scan that last read it has run
        SPD_HIP(ctx, hipStreamWaitEvent(ctx->h2d_s, ctx->h2d_scanned[k], 0));
        SPD_HIP(ctx, hipMemcpyAsync(ctx->h2d_buf[k], pairs_host + 2 * off, cn * 8, hipMemcpyHostToDevice, ctx->h2d_s));
        SPD_HIP(ctx, hipEventRecord(ctx->h2d_copied[k], ctx->h2d_s));
        SPD_HIP(ctx, hipStreamWaitEvent(s, ctx->h2d_copied[k], 0));
        std::vector<WorkItem> ws{WorkItem{&ctx->slots[router], ctx->h2d_buf[k], cn, swap}};
        spd_status st = scan_work(ctx, ws, s);
        if (st) return st;
        SPD_HIP(ctx, hipEventRecord(ctx->h2d_scanned[k], s));
    }
    SPD_HIP(ctx, hipStreamSynchronize(s));
    return SPD_OK;
}

spd_status spd_scan_batches(spd_ctx *ctx, const spd_batch *batches, uint32_t n_batches, void *stream) {
    if (!ctx) return SPD_E_INVALID;
    if (n_batches && !batches) return fail(ctx, SPD_E_INVALID, "null batch list");
    std::vector<WorkItem> ws;
    ws.reserve(n_batches);
    for (uint32_t i = 0; i < n_batches; ++i) {
        spd_status st = validate_batch(ctx, batches[i]);
        if (st) return st;
        if (batches[i].n_pairs)
            ws.push_back(WorkItem{&ctx->slots[batches[i].router], batches[i].pairs_dev, batches[i].n_pairs,
                                  (batches[i].flags & SPD_BATCH_DST) ? 1u : 0u});
    }
    if (ws.empty()) return SPD_OK;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    order_stream(ctx, s);
    return scan_work(ctx, ws, s);
}

spd_status spd_scan_batches_merge(spd_ctx *ctx, const spd_batch *batches, uint32_t n_batches, void *stream) {
    if (!ctx) return SPD_E_INVALID;
    if (n_batches && !batches) return fail(ctx, SPD_E_INVALID, "null batch list");
    std::vector<WorkItem> ws;
    std::vector<uint32_t> named, fed;
    for (uint32_t i = 0; i < n_batches; ++i) {
        spd_status st = validate_batch(ctx, batches[i]);
        if (st) return st;
        const uint32_t r = batches[i].router;
        if (std::find(named.begin(), named.end(), r) == named.end()) named.push_back(r);
        if (batches[i].n_pairs) {
            if (std::find(fed.begin(), fed.end(), r) == fed.end()) fed.push_back(r);
            ws.push_back(WorkItem{&ctx->slots[r], batches[i].pairs_dev, batches[i].n_pairs,
                                  (batches[i].flags & SPD_BATCH_DST) ? 1u : 0u});
        }
    }
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!ws.empty()) {
        order_stream(ctx, s);
        // fused only when every named router is scanned here (the others' sketches would be missed)
        ctx->merge_into = fed.size() == named.size() && !ctx->sliding ? &ctx->slots[ctx->n_routers] : nullptr;
        ctx->merged = false;
        spd_status st = scan_work(ctx, ws, s);
        ctx->merge_into = nullptr;
        ctx->merge_group = false;
        if (st) return st;
        if (ctx->merged) {
            Slot &g = ctx->slots[ctx->n_routers];
            g.fresh = false;
            return SPD_OK;
        }
    }
    return spd_merge(ctx, named.data(), (uint32_t)named.size(), stream);
}

spd_status spd_merge(spd_ctx *ctx, const uint32_t *routers, uint32_t n, void *stream) {
    if (!ctx) return SPD_E_INVALID;
    if (n && !routers) return fail(ctx, SPD_E_INVALID, "null router list");
    for (uint32_t i = 0; i < n; ++i)
        if (routers[i] >= ctx->n_routers) return fail(ctx, SPD_E_STATE, "router id out of range");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    order_stream(ctx, s);
    Slot &g = ctx->slots[ctx->n_routers];
    std::vector<uint32_t> live;
    for (uint32_t i = 0; i < n; ++i) {
        uint32_t r = routers[i];
        if (std::find(live.begin(), live.end(), r) != live.end()) continue;
        if (ctx->sliding || !ctx->slots[r].fresh) live.push_back(r);
    }
    if (live.empty()) {
        if (ctx->sliding) return clear_slot(ctx, g, s);
        g.fresh = true;
        return SPD_OK;
    }
    const uint64_t words = slot_words(ctx);
    for (size_t i0 = 0; i0 < live.size(); i0 += kMaxGroup - 1) {
        std::vector<const uint32_t *> src;
        if (i0) src.push_back(static_cast<const uint32_t *>(g.mem));
        for (size_t i = i0; i < std::min(live.size(), i0 + kMaxGroup - 1); ++i)
            src.push_back(static_cast<const uint32_t *>(ctx->slots[live[i]].mem));
        if (ctx->at) {
            std::vector<const uint8_t *> s8;
            for (auto q : src) s8.push_back(reinterpret_cast<const uint8_t *>(q));
            ProfScope ps(ctx, SPD_K_MERGE, s);
            SPD_HIP(ctx, launch_at_merge(static_cast<uint8_t *>(g.mem), s8.data(), (uint32_t)s8.size(), ctx->slot_bytes,
                                         at_code(ctx->slice), s));
        } else if (ctx->sliding) {
            std::vector<const uint16_t *> s16;
            for (auto q : src) s16.push_back(reinterpret_cast<const uint16_t *>(q));
            ProfScope ps(ctx, SPD_K_MERGE, s);
            SPD_HIP(ctx, launch_max_merge_u16(static_cast<uint16_t *>(g.mem), s16.data(), (uint32_t)s16.size(), words * 2, s));
        } else {
            ProfScope ps(ctx, SPD_K_MERGE, s);
            SPD_HIP(ctx, launch_or_merge(static_cast<uint32_t *>(g.mem), src.data(), (uint32_t)src.size(), words, s));
        }
    }
    g.fresh = false;
    return SPD_OK;
}

spd_status spd_close_window(spd_ctx *ctx, int32_t target, spd_superpoint *out_host, uint32_t cap, uint32_t *n_out,
                            void *stream) {
    if (!ctx) return SPD_E_INVALID;
    if (!n_out || (cap && !out_host)) return fail(ctx, SPD_E_INVALID, "null output");
    *n_out = 0;
    Slot *sl = slot_of(ctx, target);
    if (!sl) return fail(ctx, SPD_E_STATE, "bad target");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    order_stream(ctx, s);
    std::vector<spd_superpoint> res;
    spd_status st = close_launch(ctx, *sl, ctx->cbuf, s);
    if (st) return st;
    if (!ctx->cbuf.empty) {
        st = close_wait(ctx, ctx->cbuf, s);
        if (st) return st;
    }
    st = close_finish(ctx, *sl, ctx->cbuf, s, &res);
    if (st) return st;
    const uint32_t n = (uint32_t)res.size();
    const uint32_t w = std::min(n, cap);
    if (w) std::memcpy(out_host, res.data(), (size_t)w * sizeof(spd_superpoint));
    *n_out = n;
    return n > cap ? fail(ctx, SPD_E_TRUNCATED, "output capacity smaller than the number of super points") : SPD_OK;
}

spd_status spd_close_begin(spd_ctx *ctx, int32_t target, void *stream, uint32_t *ticket) {
    if (!ctx) return SPD_E_INVALID;
    if (!ticket) return fail(ctx, SPD_E_INVALID, "null ticket");
    Slot *sl = slot_of(ctx, target);
    if (!sl) return fail(ctx, SPD_E_STATE, "bad target");
    uint32_t i = 0;
    while (i < SPD_MAX_PENDING_CLOSES && ctx->pend[i].busy) ++i;
    if (i == SPD_MAX_PENDING_CLOSES) return fail(ctx, SPD_E_STATE, "too many closes pending: collect one first");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (!ctx->copy_s) {
        // the first two-part close allocates the buffers of every pending close (allocation
        // synchronises the device: not in the middle of a pipeline)
        for (auto &q : ctx->pend) {
            spd_status st = close_buf_init(ctx, q.cb);
            if (st) return st;
            if (!q.done) SPD_HIP(ctx, hipEventCreateWithFlags(&q.done, hipEventDisableTiming));
        }
        SPD_HIP(ctx, hipStreamCreateWithFlags(&ctx->copy_s, hipStreamNonBlocking));
    }
    PendingClose &pc = ctx->pend[i];
    if (pc.cb.rec_cap < ctx->pend_rec) {
        spd_status st = close_rec_alloc(ctx, pc.cb, ctx->pend_rec);   // (idle: its last close has ended)
        if (st) return st;
    }
    order_stream(ctx, s);
    spd_status st = close_launch(ctx, *sl, pc.cb, s);
    if (st) return st;
    if (!ctx->sliding) sl->fresh = true;   // the next window's scans, enqueued after this, start from zero
    SPD_HIP(ctx, hipEventRecord(pc.done, s));
    pc.busy = true;
    pc.seq = (++ctx->pend_seq) & 0x0FFFFFFFu;
    *ticket = (pc.seq << 4) | i;
    return SPD_OK;
}

spd_status spd_close_end(spd_ctx *ctx, uint32_t ticket, spd_superpoint *out_host, uint32_t cap, uint32_t *n_out) {
    if (!ctx) return SPD_E_INVALID;
    if (!n_out || (cap && !out_host)) return fail(ctx, SPD_E_INVALID, "null output");
    *n_out = 0;
    const uint32_t i = ticket & 15u;
    if (i >= SPD_MAX_PENDING_CLOSES || !ctx->pend[i].busy || ctx->pend[i].seq != (ticket >> 4))
        return fail(ctx, SPD_E_STATE, "unknown or already collected close ticket");
    DeviceGuard dg(ctx->device);
    PendingClose &pc = ctx->pend[i];
    pc.busy = false;   // the ticket is spent whatever follows
    {
        // (a later call's work on this close's buffers is ordered after it by order_stream)
        spd_status st = pc.cb.empty ? SPD_OK : close_wait(ctx, pc.cb, nullptr, pc.done);
        if (!st && pc.cb.empty) SPD_HIP(ctx, hipEventSynchronize(pc.done));
        if (st) return st;
    }
    ctx->stats.closes++;
    std::vector<spd_superpoint> res;
    if (pc.cb.empty) {
        ctx->stats.candidates_last = 0;
        ctx->stats.reported_last = 0;
    } else {
        const uint32_t n = pc.cb.h_counters[0];
        if (n > pc.cb.rec_cap) {
            // the window's sketch may be rewritten already, so there is no re-run: the report is
            // lost, and later closes get a buffer large enough for it
            ctx->pend_rec = std::max(ctx->pend_rec, n + 1024);
            *n_out = n;
            return fail(ctx, SPD_E_TRUNCATED, "more super points than the close's record buffer held");
        }
        spd_status st = close_report(ctx, pc.cb, n, ctx->copy_s, &res);
        if (st) return st;
    }
    const uint32_t n = (uint32_t)res.size();
    const uint32_t w = std::min(n, cap);
    if (w) std::memcpy(out_host, res.data(), (size_t)w * sizeof(spd_superpoint));
    *n_out = n;
    return n > cap ? fail(ctx, SPD_E_TRUNCATED, "output capacity smaller than the number of super points") : SPD_OK;
}

spd_status spd_reset(spd_ctx *ctx, int32_t target, void *stream) {
    if (!ctx) return SPD_E_INVALID;
    Slot *sl = slot_of(ctx, target);
    if (!sl) return fail(ctx, SPD_E_STATE, "bad target");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    order_stream(ctx, s);
    if (ctx->sliding) return clear_slot(ctx, *sl, s);
    sl->fresh = true;   // the next scan starts the slot from zero
    return SPD_OK;
}

spd_status spd_slide(spd_ctx *ctx, void *stream) {
    if (!ctx) return SPD_E_INVALID;
    if (!ctx->sliding) return fail(ctx, SPD_E_STATE, "spd_slide needs a sliding-window context");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    order_stream(ctx, s);
    if (ctx->at) {
        // the next slice; then maintenance of one group of every pool (Section 5.2): its counters
        // that are expired at the new slice are cleared
        ctx->slice++;
        const uint64_t chunk = (ctx->slot_bytes / ctx->at_groups + 15) / 16 * 16;
        const uint64_t lo = (uint64_t)(ctx->slice % ctx->at_groups) * chunk;
        const uint64_t hi = std::min(lo + chunk, ctx->slot_bytes);
        if (lo < hi) {
            std::vector<uint8_t *> pools;
            for (auto &sl : ctx->slots) pools.push_back(static_cast<uint8_t *>(sl.mem));
            ProfScope ps(ctx, SPD_K_FILL, s);
            SPD_HIP(ctx, launch_at_sweep(pools.data(), (uint32_t)pools.size(), lo, hi, at_code(ctx->slice), ctx->K, s));
        }
        return SPD_OK;
    }
    if (ctx->slice + 2 >= 0xFFFFu) {
        // stamps would overflow: shift them down so that the window keeps its bits
        const uint32_t next = ctx->slice + 1;
        const uint32_t off = next + 1 > ctx->K ? next + 1 - ctx->K : 0;
        for (auto &sl : ctx->slots)
            SPD_HIP(ctx, launch_renormalize_u16(static_cast<uint16_t *>(sl.mem), ctx->slot_bytes / 2, (uint16_t)off, s));
        ctx->slice -= off;
    }
    ctx->slice++;
    return SPD_OK;
}

spd_status spd_export(spd_ctx *ctx, int32_t target, uint8_t *seav_host, uint32_t *ldca_host) {
    if (!ctx) return SPD_E_INVALID;
    Slot *sl = slot_of(ctx, target);
    if (!sl) return fail(ctx, SPD_E_STATE, "bad target");
    DeviceGuard dg(ctx->device);
    if (ctx->have_last) SPD_HIP(ctx, hipStreamSynchronize(ctx->last_stream));
    if (!ctx->sliding) {
        if (sl->fresh) {
            if (seav_host) std::memset(seav_host, 0, ctx->d.seav_bytes);
            if (ldca_host) std::memset(ldca_host, 0, ctx->d.ldca_words * 4);
            return SPD_OK;
        }
        if (seav_host) SPD_HIP(ctx, hipMemcpy(seav_host, sl->seav, ctx->d.seav_bytes, hipMemcpyDeviceToHost));
        if (ldca_host) SPD_HIP(ctx, hipMemcpy(ldca_host, sl->ldca, ctx->d.ldca_words * 4, hipMemcpyDeviceToHost));
        return SPD_OK;
    }
    const uint64_t need = std::max<uint64_t>(ctx->d.ldca_words, ctx->seav_alloc / 4);
    if (need > ctx->view_words) {
        dev_free(ctx, &ctx->view, ctx->view_words * 4);
        ctx->view_words = 0;
        spd_status st = dev_alloc(ctx, &ctx->view, need * 4);
        if (st) return st;
        ctx->view_words = need;
    }
    const int64_t lo = (int64_t)ctx->slice - (int64_t)ctx->K + 2;
    const uint16_t thr = (uint16_t)(lo < 1 ? 1 : lo);
    hipStream_t s = ctx->have_last ? ctx->last_stream : nullptr;
    const uint32_t tm = at_code(ctx->slice);
    if (ldca_host) {
        if (ctx->at) SPD_HIP(ctx, launch_bit_view_at(sl->ldca_at, ctx->d.ldca_words * 32, tm, ctx->K, ctx->view, s));
        else SPD_HIP(ctx, launch_bit_view(sl->ldca_ts, ctx->d.ldca_words * 32, thr, ctx->view, s));
        SPD_HIP(ctx, hipMemcpyAsync(ldca_host, ctx->view, ctx->d.ldca_words * 4, hipMemcpyDeviceToHost, s));
        SPD_HIP(ctx, hipStreamSynchronize(s));
    }
    if (seav_host) {
        if (ctx->at) SPD_HIP(ctx, launch_bit_view_at(sl->seav_at, ctx->seav_alloc * 8, tm, ctx->K, ctx->view, s));
        else SPD_HIP(ctx, launch_bit_view(sl->seav_ts, ctx->seav_alloc * 8, thr, ctx->view, s));
        SPD_HIP(ctx, hipMemcpyAsync(seav_host, ctx->view, ctx->d.seav_bytes, hipMemcpyDeviceToHost, s));
        SPD_HIP(ctx, hipStreamSynchronize(s));
    }
    return SPD_OK;
}

spd_status spd_export_stamps(spd_ctx *ctx, int32_t target, uint16_t *seav_ts_host, uint16_t *ldca_ts_host) {
    if (!ctx) return SPD_E_INVALID;
    if (!ctx->sliding) return fail(ctx, SPD_E_STATE, "time stamps exist only in sliding mode");
    Slot *sl = slot_of(ctx, target);
    if (!sl) return fail(ctx, SPD_E_STATE, "bad target");
    DeviceGuard dg(ctx->device);
    if (ctx->have_last) SPD_HIP(ctx, hipStreamSynchronize(ctx->last_stream));
    if (ctx->at) {
        // rebuild 1 + last slice from each counter's age: last = slice - age
        const uint32_t t = ctx->slice, ct = at_code(t);
        auto decode = [&](const uint8_t *dev, uint64_t n, uint16_t *out) -> spd_status {
            std::vector<uint8_t> raw(n);
            SPD_HIP(ctx, hipMemcpy(raw.data(), dev, n, hipMemcpyDeviceToHost));
            for (uint64_t i = 0; i < n; ++i) {
                const uint32_t age = (ct - raw[i]) & (kAtCodes - 1u);
                out[i] = age < ctx->K ? (uint16_t)(t - age + 1) : (uint16_t)0;
            }
            return SPD_OK;
        };
        spd_status st = SPD_OK;
        if (seav_ts_host) st = decode(sl->seav_at, ctx->d.seav_bytes * 8, seav_ts_host);
        if (!st && ldca_ts_host) st = decode(sl->ldca_at, ctx->d.ldca_words * 32, ldca_ts_host);
        return st;
    }
    if (seav_ts_host) SPD_HIP(ctx, hipMemcpy(seav_ts_host, sl->seav_ts, ctx->d.seav_bytes * 16, hipMemcpyDeviceToHost));
    if (ldca_ts_host) SPD_HIP(ctx, hipMemcpy(ldca_ts_host, sl->ldca_ts, ctx->d.ldca_words * 64, hipMemcpyDeviceToHost));
    return SPD_OK;
}

spd_status spd_import(spd_ctx *ctx, int32_t target, const uint8_t *seav_host, const uint32_t *ldca_host) {
    if (!ctx) return SPD_E_INVALID;
    if (ctx->sliding) return fail(ctx, SPD_E_STATE, "import is for discrete-window contexts");
    if (!seav_host || !ldca_host) return fail(ctx, SPD_E_INVALID, "null input");
    Slot *sl = slot_of(ctx, target);
    if (!sl) return fail(ctx, SPD_E_STATE, "bad target");
    DeviceGuard dg(ctx->device);
    if (ctx->have_last) SPD_HIP(ctx, hipStreamSynchronize(ctx->last_stream));
    hipStream_t s = ctx->have_last ? ctx->last_stream : nullptr;
    spd_status st = clear_slot(ctx, *sl, s);
    if (st) return st;
    SPD_HIP(ctx, hipStreamSynchronize(s));
    SPD_HIP(ctx, hipMemcpy(sl->seav, seav_host, ctx->d.seav_bytes, hipMemcpyHostToDevice));
    SPD_HIP(ctx, hipMemcpy(sl->ldca, ldca_host, ctx->d.ldca_words * 4, hipMemcpyHostToDevice));
    sl->fresh = false;
    return SPD_OK;
}

uint32_t spd_current_slice(const spd_ctx *ctx) { return ctx ? ctx->slice : 0; }

spd_status spd_profile_enable(spd_ctx *ctx, uint32_t on) {
    if (!ctx) return SPD_E_INVALID;
    DeviceGuard dg(ctx->device);
    prof_harvest(ctx);
    ctx->prof = spd_profile{};
    ctx->prof_on = on != 0;
    return SPD_OK;
}

spd_status spd_profile_select(spd_ctx *ctx, uint32_t kinds_mask) {
    if (!ctx) return SPD_E_INVALID;
    ctx->prof_mask = kinds_mask;
    return SPD_OK;
}

spd_status spd_get_profile(spd_ctx *ctx, spd_profile *out) {
    if (!ctx || !out) return SPD_E_INVALID;
    DeviceGuard dg(ctx->device);
    prof_harvest(ctx);
    *out = ctx->prof;
    return SPD_OK;
}

spd_status spd_get_tuning(const spd_ctx *ctx, spd_tuning *out) {
    if (!ctx || !out) return SPD_E_INVALID;
    *out = ctx->tune;
    return SPD_OK;
}

spd_status spd_set_tuning(spd_ctx *ctx, const spd_tuning *t) {
    if (!ctx || !t) return SPD_E_INVALID;
    auto pow2 = [](uint32_t v) { return v && !(v & (v - 1)); };
    if (t->bucket_bits < 12 || t->bucket_bits > kMaxBucketBits) return fail(ctx, SPD_E_INVALID, "bucket_bits must be in [12, 20]");
    if (!pow2(t->tile_pairs) || t->tile_pairs < 2048 || t->tile_pairs > 16384) return fail(ctx, SPD_E_INVALID, "tile_pairs");
    if (t->bin_block != 256 && t->bin_block != 512 && t->bin_block != 1024) return fail(ctx, SPD_E_INVALID, "bin_block");
    if (t->apply_block != 256 && t->apply_block != 512 && t->apply_block != 1024) return fail(ctx, SPD_E_INVALID, "apply_block");
    if (t->direct_block != 64 && t->direct_block != 128 && t->direct_block != 256 && t->direct_block != 512 && t->direct_block != 1024)
        return fail(ctx, SPD_E_INVALID, "direct_block");
    if (t->direct_grid_per_cu < 1 || t->direct_grid_per_cu > 64) return fail(ctx, SPD_E_INVALID, "direct_grid_per_cu");
    if (t->close_block != 64 && t->close_block != 128 && t->close_block != 256) return fail(ctx, SPD_E_INVALID, "close_block");
    if (t->apply_unroll != 8 && t->apply_unroll != 16 && t->apply_unroll != 32) return fail(ctx, SPD_E_INVALID, "apply_unroll");
    if (t->bin_mode > 2) return fail(ctx, SPD_E_INVALID, "bin_mode");
    if (t->region_words > (1u << 24)) return fail(ctx, SPD_E_INVALID, "region_words");
    ctx->tune = *t;
    BinGeometry g{};
    if (t->direct_max_pairs < UINT64_MAX && !bin_geometry(ctx, &g)) {
        // the binned path cannot run with this geometry: keep every batch on the direct path
        ctx->tune.direct_max_pairs = UINT64_MAX;
    }
    return SPD_OK;
}

spd_status spd_get_stats(const spd_ctx *ctx, spd_stats *out) {
    if (!ctx || !out) return SPD_E_INVALID;
    *out = ctx->stats;
    out->device_bytes = ctx->held;
    return SPD_OK;
}

const char *spd_strerror(spd_status s) {
    switch (s) {
    case SPD_OK: return "ok";
    case SPD_E_INVALID: return "invalid argument or parameters";
    case SPD_E_NOMEM: return "HBM budget exceeded";
    case SPD_E_HIP: return "HIP runtime error";
    case SPD_E_TRUNCATED: return "output truncated";
    case SPD_E_STATE: return "invalid state or target";
    default: return "unknown status";
    }
}

const char *spd_last_error(const spd_ctx *ctx) { return ctx ? ctx->err.c_str() : ""; }

}  // extern "C"

// ==============================================================================================
// Serving loop: continuous batching of many routers' batches over device window slots.
// ==============================================================================================
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>

namespace {
using Clock = std::chrono::steady_clock;

struct SrvPending {
    const uint32_t *pairs;
    uint64_t n;
    uint32_t flags;
    Clock::time_point t;
};

struct SrvRouter {
    int slot = -1;                // open window's slot, -1 = none
    uint64_t in_window = 0;       // pairs recorded in the open window
    uint32_t window = 0;          // index of the open window
    std::deque<SrvPending> q;
    uint64_t pending = 0;         // pairs queued in q
    uint32_t close_pending = 0;   // batches in q that carry a close request
    bool waiting = false;         // counted once per admission wait
};

struct SrvClosing {
    int slot;
    uint32_t router, window;
    uint64_t pairs;
    Clock::time_point t_req;
    hipEvent_t done;
};

struct SrvResult {
    spd_window_result hdr;
    std::vector<spd_superpoint> sp;
};
}  // namespace

struct spd_server {
    spd_ctx *ctx = nullptr;       // method constants, kernels, scratch, profiler; its slots are the pool
    spd_server_config cfg{};
    std::vector<CloseBuf> cbs;    // one per slot (with its captured graph)
    std::vector<int> free_slots;
    std::vector<SrvRouter> routers;
    std::deque<SrvClosing> closing;
    std::deque<SrvResult> done;
    std::vector<hipEvent_t> ev_pool;
    hipStream_t scan_s = nullptr, close_s = nullptr;
    hipEvent_t scan_ev = nullptr; // recorded after each fused group on scan_s
    bool scan_ev_set = false;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    uint32_t flushing = 0;        // drain calls in progress: scan every queued pair regardless of min_scan_pairs
    uint32_t launching = 0;       // closes decided whose work is not yet in `closing` (their slot is in neither list)
    uint64_t queued = 0;          // batches submitted and not yet fully scanned
    spd_server_stats st{};
    spd_status fault = SPD_OK;    // first error seen by the scheduler
    std::string err;
    uint32_t rr = 0;              // round-robin start
};

namespace {

hipEvent_t srv_event(spd_server *S) {
    if (!S->ev_pool.empty()) {
        hipEvent_t e = S->ev_pool.back();
        S->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
    return e;
}

void srv_fault(spd_server *S, spd_status st) {
    std::lock_guard<std::mutex> lk(S->mu);
    if (!S->fault) {
        S->fault = st;
        S->err = S->ctx->err;
    }
    S->cv_done.notify_all();
}

// Finish every close whose device work is complete (or wait for the oldest if block is set).
bool srv_reap(spd_server *S, bool block) {
    bool any = false;
    for (;;) {
        SrvClosing c;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (S->closing.empty()) return any;
            c = S->closing.front();
        }
        hipError_t q = block && !any ? hipEventSynchronize(c.done) : hipEventQuery(c.done);
        if (q == hipErrorNotReady) return any;
        if (q != hipSuccess) {
            srv_fault(S, hip_fail(S->ctx, q, "close event"));
            return any;
        }
        SrvResult res;
        spd_status st = close_finish(S->ctx, S->ctx->slots[c.slot], S->cbs[c.slot], S->close_s, &res.sp);
        if (st) {
            srv_fault(S, st);
            return any;
        }
        const double ms = std::chrono::duration<double, std::milli>(Clock::now() - c.t_req).count();
        res.hdr = spd_window_result{c.router, c.window, c.pairs, ms, (uint32_t)res.sp.size(), 0};
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->closing.pop_front();
            S->ev_pool.push_back(c.done);
            S->free_slots.push_back(c.slot);
            S->done.push_back(std::move(res));
            S->st.windows++;
        }
        S->cv_done.notify_all();
        S->cv_work.notify_all();
        any = true;
    }
}

struct SrvClose {
    uint32_t router;
    int slot;
    uint32_t window;
    uint64_t pairs;
    Clock::time_point t_req;
};

void srv_loop(spd_server *S) {
    DeviceGuard dg(S->ctx->device);
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        // ---- admission: a router with pending batches and no open window takes a free slot
        const uint32_t R = S->cfg.n_routers;
        for (uint32_t k = 0; k < R; ++k) {
            SrvRouter &r = S->routers[(S->rr + k) % R];
            if (r.q.empty() || r.slot >= 0) continue;
            if (S->free_slots.empty()) {
                if (!r.waiting) S->st.admission_waits++;
                r.waiting = true;
                continue;
            }
            r.slot = S->free_slots.back();
            S->free_slots.pop_back();
            r.waiting = false;
            uint32_t open = 0;
            for (auto &x : S->routers) open += x.slot >= 0;
            S->st.max_open = std::max(S->st.max_open, open);
        }
        // ---- one fused group from the routers that hold a slot, round robin.  While the scan
        // stream is busy, a router's pairs wait until min_scan_pairs have gathered (each scan of a
        // slot reads and writes all its buckets); when it is idle, whatever is queued is taken.
        const bool idle = !S->scan_ev_set || hipEventQuery(S->scan_ev) == hipSuccess;
        std::vector<WorkItem> group;
        std::vector<SrvClose> closes;
        std::vector<uint64_t> finished_batches;
        uint64_t gp = 0;
        for (uint32_t k = 0; k < R && gp < S->cfg.max_group_pairs && group.size() < S->cfg.max_group_batches; ++k) {
            const uint32_t ri = (S->rr + k) % R;
            SrvRouter &r = S->routers[ri];
            if (r.slot < 0 || r.q.empty()) continue;
            const bool due = idle || S->stop || S->flushing || r.close_pending || r.pending >= S->cfg.min_scan_pairs ||
                             (S->cfg.window_pairs && r.in_window + r.pending >= S->cfg.window_pairs);
            if (!due) continue;
            while (!r.q.empty() && gp < S->cfg.max_group_pairs && group.size() < S->cfg.max_group_batches) {
                SrvPending &b = r.q.front();
                uint64_t room = S->cfg.window_pairs ? S->cfg.window_pairs - r.in_window : UINT64_MAX;
                uint64_t take = std::min(b.n, room);
                if (take) group.push_back(WorkItem{&S->ctx->slots[r.slot], b.pairs, take, (b.flags & SPD_SUBMIT_DST) ? 1u : 0u});
                gp += take;
                r.in_window += take;
                const bool whole = take == b.n;
                const bool boundary = S->cfg.window_pairs && r.in_window == S->cfg.window_pairs;
                const bool close = boundary || (whole && (b.flags & SPD_SUBMIT_CLOSE));
                const Clock::time_point t = b.t;
                r.pending -= take;
                if (whole) {
                    if (b.flags & SPD_SUBMIT_CLOSE) r.close_pending--;
                    r.q.pop_front();
                    S->queued--;
                } else {
                    b.pairs += 2 * take;
                    b.n -= take;
                }
                if (close) {
                    closes.push_back(SrvClose{ri, r.slot, r.window, r.in_window, t});
                    S->launching++;
                    r.slot = -1;
                    r.in_window = 0;
                    r.window++;
                    break;   // the rest of this router's batches belong to its next window
                }
            }
        }
        S->rr = (S->rr + 1) % std::max<uint32_t>(1, R);
        if (group.empty() && closes.empty()) {
            if (S->stop && S->queued == 0 && S->closing.empty()) return;
            // queued pairs of open windows that are not due yet: look again once the scan stream
            // may have drained
            bool deferred = false;
            for (auto &r : S->routers) deferred = deferred || (r.slot >= 0 && !r.q.empty());
            if (!S->closing.empty()) {
                lk.unlock();
                srv_reap(S, !deferred);
                lk.lock();
                if (deferred) S->cv_work.wait_for(lk, std::chrono::microseconds(50));
                continue;
            }
            if (deferred)
                S->cv_work.wait_for(lk, std::chrono::microseconds(50));
            else
                S->cv_work.wait(lk);
            continue;
        }
        S->st.groups += group.empty() ? 0 : 1;
        lk.unlock();
        // ---- device work outside the lock
        spd_status st = SPD_OK;
        if (!group.empty()) {
            st = scan_work(S->ctx, group, S->scan_s);
            if (!st && hipEventRecord(S->scan_ev, S->scan_s) != hipSuccess) st = SPD_E_HIP;
            S->scan_ev_set = !st;
        }
        size_t pushed = 0;
        for (auto &c : closes) {
            if (st) break;
            hipEvent_t scanned = srv_event(S), fin = srv_event(S);
            if (!scanned || !fin) {
                st = SPD_E_HIP;
                break;
            }
            // the close waits only for the scans issued so far; later groups overlap it
            if (hipEventRecord(scanned, S->scan_s) != hipSuccess || hipStreamWaitEvent(S->close_s, scanned, 0) != hipSuccess) {
                st = SPD_E_HIP;
                break;
            }
            Slot &sl = S->ctx->slots[c.slot];
            st = S->cfg.use_graphs ? close_launch_graph(S->ctx, sl, S->cbs[c.slot], S->close_s)
                                   : close_launch(S->ctx, sl, S->cbs[c.slot], S->close_s);
            if (st) break;
            if (hipEventRecord(fin, S->close_s) != hipSuccess) {
                st = SPD_E_HIP;
                break;
            }
            std::lock_guard<std::mutex> g(S->mu);
            S->ev_pool.push_back(scanned);   // reusable once recorded again later (ordering kept by the stream)
            S->closing.push_back(SrvClosing{c.slot, c.router, c.window, c.pairs, c.t_req, fin});
            S->launching--;
            ++pushed;
        }
        if (pushed < closes.size()) {
            std::lock_guard<std::mutex> g(S->mu);
            S->launching -= (uint32_t)(closes.size() - pushed);
        }
        if (st) {
            srv_fault(S, st);
            lk.lock();
            return;
        }
        srv_reap(S, false);
        lk.lock();
        S->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

spd_status spd_server_create(const spd_params *p, const spd_server_config *cfg, spd_server **out) {
    if (!out || !p || !cfg) return SPD_E_INVALID;
    *out = nullptr;
    if (cfg->n_routers < 1 || cfg->n_routers > 65536) return SPD_E_INVALID;
    if (p->window_slices) return SPD_E_INVALID;   // the serving loop runs discrete windows
    spd_server *S = new (std::nothrow) spd_server();
    if (!S) return SPD_E_NOMEM;
    S->cfg = *cfg;
    if (!S->cfg.hbm_budget_bytes) S->cfg.hbm_budget_bytes = 4ull << 30;
    if (!S->cfg.max_group_pairs) S->cfg.max_group_pairs = 64ull << 20;
    if (!S->cfg.min_scan_pairs) S->cfg.min_scan_pairs = S->cfg.window_pairs ? S->cfg.window_pairs : 8ull << 20;
    if (!S->cfg.max_group_batches) S->cfg.max_group_batches = 1024;
    S->cfg.max_group_batches = std::min<uint32_t>(S->cfg.max_group_batches, 4096);
    spd_status st = ctx_create(p, 0, 0, S->cfg.hbm_budget_bytes, &S->ctx);
    if (st) {
        delete S;
        return st;
    }
    spd_ctx *ctx = S->ctx;
    if (cfg->tuning) {
        st = spd_set_tuning(ctx, cfg->tuning);
        if (st) {
            spd_server_destroy(S);
            return st;
        }
    }
    S->cfg.tuning = nullptr;   // the caller's struct is not kept
    DeviceGuard dg(ctx->device);
    // scratch for the largest fused group, reserved before the slots so admission never frees it
    BinGeometry g{};
    if (bin_geometry(ctx, &g)) {
        const uint64_t tiles = S->cfg.max_group_pairs / g.tile_pairs + S->cfg.max_group_batches + 1;
        auto reserve = [&](uint32_t mode) {
            uint64_t items_words, meta_words;
            scratch_need(g, mode, tiles, &items_words, &meta_words);
            uint64_t aux_words = (uint64_t)kMaxGroup * g.nb + 1 + (tiles / kChunk + kMaxGroup) * g.nb;
            if (mode == 2) {
                region_bound(ctx, g, tiles, &items_words, &aux_words);
                meta_words = 0;
            }
            spd_status r = ensure_scratch(ctx, items_words, meta_words, nullptr);
            if (!r && mode) r = ensure_aux(ctx, aux_words, nullptr);
            return r;
        };
        st = reserve(ctx->tune.bin_mode);
        if (ctx->tune.bin_mode == 2) {
            // the region layout needs the most scratch: under a budget that would then hold no window
            // slot, the server keeps the exact-count layout
            const uint64_t one_slot = ctx->slot_bytes + (uint64_t)kRecInit * 8 + 64;
            const bool room = ctx->held + one_slot <= ctx->budget;
            if (st == SPD_E_NOMEM || (!st && !room)) {
                free_scratch(ctx);
                ctx->tune.bin_mode = 1;
                st = reserve(1);
            }
        }
        if (!st && ctx->tune.bin_mode) st = ensure_batch_ring(ctx, S->cfg.max_group_batches);
        if (st) {
            spd_server_destroy(S);
            return st;
        }
    }
    const uint64_t per_slot = ctx->slot_bytes + (uint64_t)kRecInit * 8 + 64;
    uint64_t room = ctx->budget > ctx->held ? ctx->budget - ctx->held : 0;
    uint32_t n_slots = (uint32_t)std::min<uint64_t>(room / per_slot, 65536);
    if (S->cfg.max_slots) n_slots = std::min(n_slots, S->cfg.max_slots);
    if (n_slots == 0) {
        ctx->err = "HBM budget leaves no room for a window slot";
        spd_server_destroy(S);
        return SPD_E_NOMEM;
    }
    ctx->slots.resize(n_slots);
    S->cbs.resize(n_slots);
    for (uint32_t i = 0; i < n_slots; ++i) {
        st = slot_alloc(ctx, ctx->slots[i]);
        if (!st) st = close_buf_init(ctx, S->cbs[i]);
        if (st) {
            spd_server_destroy(S);
            return st;
        }
        S->free_slots.push_back((int)(n_slots - 1 - i));
    }
    S->st.slots = n_slots;
    S->routers.resize(S->cfg.n_routers);
    if (hipStreamCreateWithFlags(&S->scan_s, hipStreamNonBlocking) != hipSuccess ||
        hipStreamCreateWithFlags(&S->close_s, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->scan_ev, hipEventDisableTiming) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        spd_server_destroy(S);
        return SPD_E_HIP;
    }
    S->worker = std::thread(srv_loop, S);
    *out = S;
    return SPD_OK;
}

spd_status spd_server_submit(spd_server *S, uint32_t router, const uint32_t *pairs_dev, uint64_t n_pairs, uint32_t flags) {
    if (!S) return SPD_E_INVALID;
    if (router >= S->cfg.n_routers) return SPD_E_STATE;
    if (n_pairs && !pairs_dev) return SPD_E_INVALID;
    if (reinterpret_cast<uintptr_t>(pairs_dev) % 8) return SPD_E_INVALID;
    if (flags & ~(SPD_SUBMIT_CLOSE | SPD_SUBMIT_DST)) return SPD_E_INVALID;
    const Clock::time_point t = Clock::now();
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->fault) return S->fault;
    if (S->stop) return SPD_E_STATE;
    if (n_pairs == 0 && !(flags & SPD_SUBMIT_CLOSE)) return SPD_OK;
    SrvRouter &r = S->routers[router];
    r.q.push_back(SrvPending{pairs_dev, n_pairs, flags, t});
    r.pending += n_pairs;
    if (flags & SPD_SUBMIT_CLOSE) r.close_pending++;
    S->queued++;
    S->st.batches++;
    S->st.pairs += n_pairs;
    S->cv_work.notify_one();
    return SPD_OK;
}

spd_status spd_server_replay(spd_server *S, const spd_arrival *sched, uint64_t n, double *elapsed_s) {
    if (!S || (n && !sched)) return SPD_E_INVALID;
    const Clock::time_point t0 = Clock::now();
    for (uint64_t i = 0; i < n; ++i) {
        const auto due = t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(sched[i].t_s));
        for (;;) {
            const auto now = Clock::now();
            if (now >= due) break;
            if (due - now > std::chrono::microseconds(200)) std::this_thread::sleep_for(due - now - std::chrono::microseconds(100));
        }
        spd_status st = spd_server_submit(S, sched[i].router, sched[i].pairs_dev, sched[i].n_pairs, sched[i].flags);
        if (st) return st;
    }
    if (elapsed_s) *elapsed_s = std::chrono::duration<double>(Clock::now() - t0).count();
    return SPD_OK;
}

spd_status spd_server_next(spd_server *S, spd_window_result *hdr, spd_superpoint *out_host, uint32_t cap,
                           int32_t timeout_ms) {
    if (!S || !hdr || (cap && !out_host)) return SPD_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto ready = [&] { return !S->done.empty() || S->fault; };
    if (timeout_ms < 0) S->cv_done.wait(lk, ready);
    else S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready);
    if (S->done.empty()) return S->fault ? S->fault : SPD_E_AGAIN;
    SrvResult r = std::move(S->done.front());
    S->done.pop_front();
    lk.unlock();
    *hdr = r.hdr;
    const uint32_t w = std::min<uint32_t>(cap, (uint32_t)r.sp.size());
    if (w) std::memcpy(out_host, r.sp.data(), (size_t)w * sizeof(spd_superpoint));
    return r.sp.size() > cap ? SPD_E_TRUNCATED : SPD_OK;
}

spd_status spd_server_drain(spd_server *S) {
    if (!S) return SPD_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    S->flushing++;
    S->cv_work.notify_all();
    bool stuck = false;
    S->cv_done.wait(lk, [&] {
        if (S->fault) return true;
        if (!S->closing.empty() || S->launching) return false;
        if (!S->queued) return true;   // a window without a close request simply stays open
        // every slot is held by an open window that will never close while the routers that
        // still have batches wait for one: no progress is possible
        bool movable = !S->free_slots.empty();
        for (auto &r : S->routers) movable = movable || (r.slot >= 0 && !r.q.empty());
        stuck = !movable;
        return stuck;
    });
    S->flushing--;
    if (S->fault) return S->fault;
    if (stuck) {
        S->err = "all window slots are held by open windows; queued batches cannot be admitted";
        return SPD_E_STATE;
    }
    lk.unlock();
    hipError_t e = hipStreamSynchronize(S->scan_s);
    return e == hipSuccess ? SPD_OK : SPD_E_HIP;
}

spd_status spd_server_get_stats(spd_server *S, spd_server_stats *out) {
    if (!S || !out) return SPD_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    *out = S->st;
    return SPD_OK;
}

spd_status spd_server_set_tuning(spd_server *S, const spd_tuning *t) {
    if (!S || !t) return SPD_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    if (S->queued || !S->closing.empty()) return SPD_E_STATE;
    return spd_set_tuning(S->ctx, t);
}

const char *spd_server_last_error(spd_server *S) {
    if (!S) return "";
    std::lock_guard<std::mutex> lk(S->mu);
    return S->err.empty() ? S->ctx->err.c_str() : S->err.c_str();
}

void spd_server_destroy(spd_server *S) {
    if (!S) return;
    if (S->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->stop = true;
        }
        S->cv_work.notify_all();
        S->worker.join();
    }
    if (S->ctx) {
        DeviceGuard dg(S->ctx->device);
        (void)hipDeviceSynchronize();
        for (auto &cb : S->cbs) close_buf_free(S->ctx, cb);
        for (auto e : S->ev_pool) (void)hipEventDestroy(e);
        for (auto &c : S->closing) (void)hipEventDestroy(c.done);
        if (S->scan_ev) (void)hipEventDestroy(S->scan_ev);
        if (S->scan_s) (void)hipStreamDestroy(S->scan_s);
        if (S->close_s) (void)hipStreamDestroy(S->close_s);
        spd_destroy(S->ctx);
    }
    delete S;
}

}  // extern "C"
