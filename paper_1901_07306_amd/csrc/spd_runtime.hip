// Host runtime of libspd: parameter derivation, contexts, router slots, scratch memory, kernel
// dispatch and the C ABI declared in include/spd.h.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
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
    bool fresh = true;           // logically all zero; device memory not yet cleared
};

}  // namespace

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
    uint32_t K = 0;
    uint32_t slice = 0;
    uint64_t seav_alloc = 0;     // padded SEAV bytes per slot
    uint64_t slot_bytes = 0;
    std::vector<Slot> slots;     // routers, then the global sketch
    uint32_t *items = nullptr;
    uint64_t items_words = 0;
    uint32_t *meta = nullptr;
    uint32_t *metaT = nullptr;
    uint64_t meta_words = 0;
    uint32_t *rec = nullptr;
    uint32_t rec_cap = 0;
    uint32_t *counters = nullptr;   // device [4]
    uint32_t *h_counters = nullptr; // pinned host [4]
    uint32_t *h_rec = nullptr;      // pinned host records
    uint32_t h_rec_cap = 0;
    uint32_t *view = nullptr;       // sliding export: bit view words
    uint64_t view_words = 0;
    std::vector<uint32_t> est;      // Eq. 4 estimate for every z0 in [0, k]
    spd_tuning tune{};
    spd_stats stats{};
    std::string err;
    hipStream_t last_stream = nullptr;
    bool have_last = false;
    hipEvent_t order_ev = nullptr;
    // optional per-kernel timing
    bool prof_on = false;
    struct Pending {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Pending> prof_pending;
    std::vector<hipEvent_t> prof_pool;
    spd_profile prof{};
};

namespace {

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
    t->tile_pairs = 16384;
    t->bin_block = 1024;
    t->apply_block = 1024;
    t->direct_block = 256;
    t->direct_grid_per_cu = 8;
    t->seav_lds = 0;
    t->close_block = 256;
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
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Brackets one launch with events when profiling is on.
struct ProfScope {
    spd_ctx *ctx;
    int kind;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(spd_ctx *c, int k, hipStream_t st) : ctx(c), kind(k), s(st) {
        if (ctx->prof_on) {
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
    return p;
}

uint64_t slot_words(const spd_ctx *ctx) { return ctx->slot_bytes / 4; }

spd_status clear_slot(spd_ctx *ctx, Slot &s, hipStream_t st) {
    {
        ProfScope ps(ctx, SPD_K_FILL, st);
        SPD_HIP(ctx, launch_fill_u32(static_cast<uint32_t *>(s.mem), slot_words(ctx), 0u, st));
    }
    s.fresh = false;
    return SPD_OK;
}

// Zero only the SEAV of a fresh slot: the binned scan rewrites every LDCA bucket of a fresh slot
// from zero, while its SEAV buckets are read back (they may hold bits recorded directly).
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
        const double expect = (double)T / (double)(1ull << ctx->d.tau);
        uint32_t scap = (uint32_t)std::ceil(2.0 * expect + 8.0 * std::sqrt(expect) + 64.0);
        scap = std::min<uint32_t>((scap + 63) / 64 * 64, T);
        uint32_t cap = T * ctx->p.lr + scap * ctx->p.sr;
        cap = (cap + 5) / 6 * 6;
        if ((uint64_t)T * ctx->p.lr > 65536) continue;   // per-bucket ranks are 16 bits
        const uint64_t stage_off = (2ull * (g->nb + 1) + 3) & ~3ull;   // same layout as k_bin
        const uint64_t lds = 4ull * (stage_off + cap + 2ull * scap + 1 + 17);
        if (lds <= kMaxLds) {
            g->tile_pairs = T;
            g->scap = scap;
            g->cap = cap;
            g->region = cap / 3 * 2;
            g->lds_bytes = (uint32_t)lds;
            return true;
        }
    }
    return false;
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
        ctx->meta_words = 0;
        spd_status st = dev_alloc(ctx, &ctx->meta, meta_words * 4);
        if (st) return st;
        st = dev_alloc(ctx, &ctx->metaT, meta_words * 4);
        if (st) return st;
        ctx->meta_words = meta_words;
    }
    return SPD_OK;
}

// Record a group of batches whose routers are distinct-or-repeated; batches sorted by router.
spd_status scan_group(spd_ctx *ctx, std::vector<spd_batch> &bs, hipStream_t s) {
    std::stable_sort(bs.begin(), bs.end(), [](const spd_batch &x, const spd_batch &y) { return x.router < y.router; });
    uint64_t total = 0;
    std::vector<uint32_t> routers;
    for (auto &b : bs) {
        total += b.n_pairs;
        if (routers.empty() || routers.back() != b.router) routers.push_back(b.router);
    }
    if (total == 0) return SPD_OK;
    if (ctx->sliding) {
        // time stamps of the current slice, plain stores
        for (size_t i0 = 0; i0 < bs.size(); i0 += kMaxGroup) {
            BatchDesc bd[kMaxGroup];
            SlotPtrs sp[kMaxGroup] = {};
            uint32_t nbd = 0, nsl = 0;
            uint64_t n = 0;
            std::vector<uint32_t> seen;
            for (size_t i = i0; i < std::min(bs.size(), i0 + kMaxGroup); ++i) {
                auto it = std::find(seen.begin(), seen.end(), bs[i].router);
                uint32_t si = (uint32_t)(it - seen.begin());
                if (it == seen.end()) {
                    seen.push_back(bs[i].router);
                    sp[nsl++] = ptrs_of(ctx->slots[bs[i].router]);
                }
                bd[nbd++] = BatchDesc{bs[i].pairs_dev, bs[i].n_pairs, 0, si};
                n = std::max(n, bs[i].n_pairs);
            }
            uint32_t block = ctx->tune.direct_block;
            uint64_t want = (n + block - 1) / block;
            uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)ctx->tune.direct_grid_per_cu * ctx->n_cu));
            ProfScope ps(ctx, SPD_K_STAMP, s);
            SPD_HIP(ctx, launch_scan_stamp(ctx->c, bd, nbd, sp, (uint16_t)(ctx->slice + 1), block, grid, s));
        }
        ctx->stats.pairs_scanned += total;
        ctx->stats.direct_launches++;
        return SPD_OK;
    }
    BinGeometry g{};
    const bool binned = total > ctx->tune.direct_max_pairs && ctx->p.lr <= 4 && bin_geometry(ctx, &g);
    std::vector<uint32_t> fresh_routers;
    for (uint32_t r : routers) {
        Slot &sl = ctx->slots[r];
        if (!sl.fresh) continue;
        spd_status st = binned ? clear_seav(ctx, sl, s) : clear_slot(ctx, sl, s);
        if (st) return st;
        if (binned) fresh_routers.push_back(r);
        sl.fresh = false;
    }
    if (!binned) {
        for (size_t i0 = 0; i0 < bs.size(); i0 += kMaxGroup) {
            BatchDesc bd[kMaxGroup];
            SlotPtrs sp[kMaxGroup] = {};
            uint32_t nbd = 0, nsl = 0;
            uint64_t n = 0;
            std::vector<uint32_t> seen;
            for (size_t i = i0; i < std::min(bs.size(), i0 + kMaxGroup); ++i) {
                auto it = std::find(seen.begin(), seen.end(), bs[i].router);
                uint32_t si = (uint32_t)(it - seen.begin());
                if (it == seen.end()) {
                    seen.push_back(bs[i].router);
                    sp[nsl++] = ptrs_of(ctx->slots[bs[i].router]);
                }
                bd[nbd++] = BatchDesc{bs[i].pairs_dev, bs[i].n_pairs, 0, si};
                n = std::max(n, bs[i].n_pairs);
            }
            const bool lds = ctx->tune.seav_lds && nsl == 1 && ctx->d.seav_bytes <= 64 * 1024;
            uint32_t block = ctx->tune.direct_block;
            uint64_t want = (n + block - 1) / block;
            uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)ctx->tune.direct_grid_per_cu * ctx->n_cu));
            ProfScope ps(ctx, SPD_K_DIRECT, s);
            SPD_HIP(ctx, launch_scan_direct(ctx->c, bd, nbd, sp, block, grid, lds, s));
            ctx->stats.direct_launches++;
        }
        ctx->stats.pairs_scanned += total;
        return SPD_OK;
    }
    // binned: groups of at most kMaxGroup batches (and routers)
    size_t i0 = 0;
    while (i0 < bs.size()) {
        BatchDesc bd[kMaxGroup];
        SlotPtrs sp[kMaxGroup] = {};
        ApplySlot as[kMaxGroup] = {};
        uint32_t nbd = 0, nsl = 0, tiles = 0;
        size_t i = i0;
        for (; i < bs.size() && nbd < (uint32_t)kMaxGroup; ++i) {
            const spd_batch &b = bs[i];
            if (b.n_pairs == 0) continue;
            if (nsl == 0 || as[nsl - 1].pad != b.router) {
                if (nsl == (uint32_t)kMaxGroup) break;
                Slot &sl = ctx->slots[b.router];
                sp[nsl] = ptrs_of(sl);
                as[nsl].ldca = sl.ldca;
                as[nsl].seav_w = reinterpret_cast<uint32_t *>(sl.seav);
                as[nsl].tile_lo = tiles;
                // a fresh slot's LDCA buckets are written from zero by this launch
                as[nsl].fresh = std::find(fresh_routers.begin(), fresh_routers.end(), b.router) != fresh_routers.end();
                as[nsl].pad = b.router;
                ++nsl;
            }
            const uint64_t nt = (b.n_pairs + g.tile_pairs - 1) / g.tile_pairs;
            if ((uint64_t)tiles + nt > 0x7FFFFFFFull) return fail(ctx, SPD_E_INVALID, "batch too large");
            bd[nbd++] = BatchDesc{b.pairs_dev, b.n_pairs, tiles, nsl - 1};
            tiles += (uint32_t)nt;
            as[nsl - 1].tile_hi = tiles;
        }
        i0 = i;
        if (nbd == 0) continue;
        spd_status st = ensure_scratch(ctx, (uint64_t)tiles * g.region, (uint64_t)tiles * (g.nb + 1), s);
        if (st) return st;
        {
            ProfScope ps(ctx, SPD_K_BIN, s);
            SPD_HIP(ctx, launch_bin(ctx->c, g, bd, nbd, tiles, ctx->items, ctx->meta, sp, s));
        }
        {
            ProfScope ps(ctx, SPD_K_TRANSPOSE, s);
            SPD_HIP(ctx, launch_transpose(ctx->meta, ctx->metaT, tiles, g.nb + 1, s));
        }
        {
            ProfScope ps(ctx, SPD_K_APPLY, s);
            SPD_HIP(ctx, launch_apply(g, as, nsl, ctx->items, ctx->metaT, tiles, ctx->tune.apply_block, s));
        }
        // later groups of the same call OR into these slots
        for (uint32_t k = 0; k < nsl; ++k)
            fresh_routers.erase(std::remove(fresh_routers.begin(), fresh_routers.end(), as[k].pad), fresh_routers.end());
        ctx->stats.binned_launches++;
    }
    ctx->stats.pairs_scanned += total;
    return SPD_OK;
}

spd_status validate_batch(spd_ctx *ctx, const spd_batch &b) {
    if (b.router >= ctx->n_routers) return fail(ctx, SPD_E_STATE, "router id out of range");
    if (b.reserved != 0) return fail(ctx, SPD_E_INVALID, "spd_batch.reserved must be 0");
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
    ctx->budget = hbm_budget_bytes;
    ctx->sliding = p->window_slices > 0;
    ctx->K = p->window_slices;
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
    ctx->est.resize((1u << p->log2k) + 1);
    const double k = std::ldexp(1.0, (int)p->log2k);
    for (uint32_t z = 0; z <= (1u << p->log2k); ++z)
        ctx->est[z] = (uint32_t)std::floor(-k * std::log((double)(z ? z : 1) / k) + 0.5);

    DeviceGuard dg(ctx->device);
    ctx->seav_alloc = (ctx->d.seav_bytes + kSeavAlign - 1) / kSeavAlign * kSeavAlign;
    const uint64_t ldca_bytes = (ctx->d.ldca_words * 4 + 255) / 256 * 256;   // SEAV starts 256-byte aligned
    // sliding: one 16-bit stamp per bit
    ctx->slot_bytes = ctx->sliding ? (ldca_bytes * 16 + ctx->seav_alloc * 16) : (ldca_bytes + ctx->seav_alloc);
    ctx->slots.resize(n_routers + 1);
    hipStream_t s0 = nullptr;
    for (auto &sl : ctx->slots) {
        st = dev_alloc(ctx, &sl.mem, ctx->slot_bytes);
        if (st) {
            spd_destroy(ctx);
            return st;
        }
        if (ctx->sliding) {
            sl.ldca_ts = static_cast<uint16_t *>(sl.mem);
            sl.seav_ts = sl.ldca_ts + ldca_bytes * 8;
            if (launch_fill_u32(static_cast<uint32_t *>(sl.mem), ctx->slot_bytes / 4, 0u, s0) != hipSuccess) {
                spd_destroy(ctx);
                return SPD_E_HIP;
            }
            sl.fresh = false;
        } else {
            sl.ldca = static_cast<uint32_t *>(sl.mem);
            sl.seav = static_cast<uint8_t *>(sl.mem) + ldca_bytes;
            sl.fresh = true;
        }
    }
    if (dev_alloc(ctx, &ctx->counters, 16) || hipEventCreateWithFlags(&ctx->order_ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_counters, 16, hipHostMallocDefault) != hipSuccess) {
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

void spd_destroy(spd_ctx *ctx) {
    if (!ctx) return;
    {
        DeviceGuard dg(ctx->device);
        (void)hipDeviceSynchronize();
        for (auto &sl : ctx->slots) dev_free(ctx, &sl.mem, ctx->slot_bytes);
        dev_free(ctx, &ctx->items, ctx->items_words * 4);
        dev_free(ctx, &ctx->meta, ctx->meta_words * 4);
        dev_free(ctx, &ctx->metaT, ctx->meta_words * 4);
        dev_free(ctx, &ctx->rec, (uint64_t)ctx->rec_cap * 8);
        dev_free(ctx, &ctx->counters, 16);
        dev_free(ctx, &ctx->view, ctx->view_words * 4);
        if (ctx->h_counters) (void)hipHostFree(ctx->h_counters);
        if (ctx->h_rec) (void)hipHostFree(ctx->h_rec);
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

spd_status spd_scan_batches(spd_ctx *ctx, const spd_batch *batches, uint32_t n_batches, void *stream) {
    if (!ctx) return SPD_E_INVALID;
    if (n_batches && !batches) return fail(ctx, SPD_E_INVALID, "null batch list");
    std::vector<spd_batch> bs;
    bs.reserve(n_batches);
    for (uint32_t i = 0; i < n_batches; ++i) {
        spd_status st = validate_batch(ctx, batches[i]);
        if (st) return st;
        if (batches[i].n_pairs) bs.push_back(batches[i]);
    }
    if (bs.empty()) return SPD_OK;
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    order_stream(ctx, s);
    return scan_group(ctx, bs, s);
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
        if (ctx->sliding) {
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
    ctx->stats.closes++;
    if (!ctx->sliding && sl->fresh) {
        ctx->stats.candidates_last = 0;
        ctx->stats.reported_last = 0;
        return SPD_OK;
    }
    CloseArgs a{};
    a.seav = sl->seav;
    a.ldca = sl->ldca;
    a.seav_ts = sl->seav_ts;
    a.ldca_ts = sl->ldca_ts;
    if (ctx->sliding) {
        const int64_t lo = (int64_t)ctx->slice - (int64_t)ctx->K + 2;
        a.thr = lo < 1 ? 1u : (uint32_t)lo;
    }
    a.counters = ctx->counters;
    a.n_rp = 1u << ctx->p.r;
    uint32_t max_ibn = 0;
    for (uint32_t i = 0; i < ctx->p.sr; ++i) max_ibn = std::max(max_ibn, ctx->d.ibn[i]);
    a.list_stride = 1u << max_ibn;
    a.qcap = 256;
    uint32_t block = ctx->tune.close_block;
    while (block > 64 && (block / 64) * (ctx->p.sr * a.list_stride + a.qcap) * 4ull > kMaxLds) block /= 2;
    if ((block / 64) * (ctx->p.sr * a.list_stride + a.qcap) * 4ull > kMaxLds)
        return fail(ctx, SPD_E_INVALID, "SEA rows too large for the end-of-window kernel");
    const uint32_t waves = block / 64;
    const uint64_t want = ((uint64_t)a.n_rp + waves - 1) / waves;
    const uint32_t grid = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(want, (uint64_t)ctx->n_cu * 16));
    if (ctx->rec_cap == 0) {
        spd_status st = dev_alloc(ctx, &ctx->rec, 65536ull * 8);
        if (st) return st;
        ctx->rec_cap = 65536;
    }
    uint32_t n = 0;
    for (int attempt = 0; attempt < 2; ++attempt) {
        a.rec = ctx->rec;
        a.rec_cap = ctx->rec_cap;
        SPD_HIP(ctx, launch_fill_u32(ctx->counters, 4, 0u, s));
        {
            ProfScope ps(ctx, SPD_K_CLOSE, s);
            SPD_HIP(ctx, launch_close(ctx->c, a, ctx->sliding, block, grid, s));
        }
        SPD_HIP(ctx, hipMemcpyAsync(ctx->h_counters, ctx->counters, 16, hipMemcpyDeviceToHost, s));
        SPD_HIP(ctx, hipStreamSynchronize(s));
        n = ctx->h_counters[0];
        ctx->stats.candidates_last = ctx->h_counters[1];
        if (n <= ctx->rec_cap) break;
        // more reports than the record buffer holds: grow it and run the (deterministic) pass again
        dev_free(ctx, &ctx->rec, (uint64_t)ctx->rec_cap * 8);
        ctx->rec_cap = 0;
        uint32_t want_cap = n + 1024;
        spd_status st = dev_alloc(ctx, &ctx->rec, (uint64_t)want_cap * 8);
        if (st) return st;
        ctx->rec_cap = want_cap;
    }
    if (n > ctx->h_rec_cap) {
        if (ctx->h_rec) (void)hipHostFree(ctx->h_rec);
        ctx->h_rec = nullptr;
        ctx->h_rec_cap = 0;
        SPD_HIP(ctx, hipHostMalloc((void **)&ctx->h_rec, (uint64_t)std::max<uint32_t>(n, 1024) * 8, hipHostMallocDefault));
        ctx->h_rec_cap = std::max<uint32_t>(n, 1024);
    }
    if (n) {
        SPD_HIP(ctx, hipMemcpyAsync(ctx->h_rec, ctx->rec, (uint64_t)n * 8, hipMemcpyDeviceToHost, s));
        SPD_HIP(ctx, hipStreamSynchronize(s));
    }
    std::vector<spd_superpoint> res(n);
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t z0 = ctx->h_rec[2 * i + 1];
        res[i] = spd_superpoint{ctx->h_rec[2 * i], z0, ctx->est[std::min<uint32_t>(z0, 1u << ctx->p.log2k)], z0 == 0 ? 1u : 0u};
    }
    std::sort(res.begin(), res.end(), [](const spd_superpoint &x, const spd_superpoint &y) { return x.ip < y.ip; });
    const uint32_t w = std::min(n, cap);
    if (w) std::memcpy(out_host, res.data(), (size_t)w * sizeof(spd_superpoint));
    *n_out = n;
    ctx->stats.reported_last = n;
    if (!ctx->sliding) sl->fresh = true;   // the next window starts from zero
    return n > cap ? fail(ctx, SPD_E_TRUNCATED, "output capacity smaller than the number of super points") : SPD_OK;
}

spd_status spd_slide(spd_ctx *ctx, void *stream) {
    if (!ctx) return SPD_E_INVALID;
    if (!ctx->sliding) return fail(ctx, SPD_E_STATE, "spd_slide needs a sliding-window context");
    DeviceGuard dg(ctx->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    order_stream(ctx, s);
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
    if (ldca_host) {
        SPD_HIP(ctx, launch_bit_view(sl->ldca_ts, ctx->d.ldca_words * 32, thr, ctx->view, s));
        SPD_HIP(ctx, hipMemcpyAsync(ldca_host, ctx->view, ctx->d.ldca_words * 4, hipMemcpyDeviceToHost, s));
        SPD_HIP(ctx, hipStreamSynchronize(s));
    }
    if (seav_host) {
        SPD_HIP(ctx, launch_bit_view(sl->seav_ts, ctx->seav_alloc * 8, thr, ctx->view, s));
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
