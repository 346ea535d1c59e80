/*
 * libspd: super-point detection on AMD Instinct MI355X (gfx950).
 *
 * Implements the detection scheme of Xu, Ding and Hu, "Most memory efficient distributed super
 * points detection on core networks" (arXiv 1901.07306): every (hip, oip) IPv4 pair of a time
 * window is recorded in a short estimator array vector (SEAV, Section 3.2) and a linear distinct
 * counter array (LDCA, Section 3.3); each router (watch point) keeps its own pair of sketches,
 * the sketches are merged by OR (Section 4.2), and at the end of a window super-point candidates
 * are rebuilt from the SEAV and filtered by their LDCA estimate against the threshold theta
 * (Definition 2).  A sliding-window mode replaces every bit by a time stamp (Section 5).
 *
 * Conventions for every entry point:
 *  - Status codes: SPD_OK (0) or a negative SPD_E_* value; nothing is thrown across the ABI.
 *    spd_last_error() returns a message for the last failure on a context.
 *  - Pair buffers are DEVICE pointers owned by the caller: n_pairs records of two uint32
 *    (element 0 = hip, the monitored host; element 1 = oip, its opposite IP), 8-byte aligned.
 *    They must stay valid until the stream has passed the scan.
 *  - Streams are hipStream_t values passed as void* (NULL = the null stream).  Scans, merges
 *    and slides are asynchronous on that stream.  Close waits for its stream and builds the
 *    report; in discrete mode the closed window's reset needs no device work (the next scan
 *    writes the sketch from zero); export and import synchronise.
 *    Calls on one context are ordered among themselves whatever streams they name: the library
 *    makes each call's stream wait for the previous call's work.
 *  - The library owns all sketch state, in device memory of the device that was current at
 *    spd_create().  A context is not thread-safe: one host thread drives it, or callers lock.
 *  - Canonical layouts (export/import, also the device layouts):
 *      SEAV: uint8  [2^r][SR rows][2^IBN(row)]   (rows of one SEA stored one after another)
 *      LDCA: uint32 [LR][LC][k/32]               (bit q of LDC (i, c) = bit q%32 of word q/32)
 */
#ifndef SPD_H
#define SPD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t spd_status;

#define SPD_OK 0
#define SPD_E_INVALID (-1)    /* bad argument, parameter out of range or layout constraint broken */
#define SPD_E_NOMEM (-2)      /* the HBM budget given to spd_create() would be exceeded */
#define SPD_E_HIP (-3)        /* HIP runtime error; spd_last_error() has its text */
#define SPD_E_TRUNCATED (-4)  /* output capacity too small; *n_out holds the required count */
#define SPD_E_STATE (-5)      /* call not valid in the context's current state (e.g. bad router) */
#define SPD_E_AGAIN (-6)      /* serving loop: no finished window within the timeout */

#define SPD_MAX_ROWS 8        /* largest SR and LR */
#define SPD_GLOBAL (-1)       /* target id of the merged (global) sketch */

/* Method parameters.  Sections cited per field. */
typedef struct spd_params {
    uint32_t theta;            /* super-point threshold, Definition 2; 1 <= theta <= 2^31 */
    uint32_t r;                /* right-part bits: the SEAV holds 2^r SEAs (Section 3.2); r <= 24 */
    uint32_t sr;               /* rows per SEA, 1..SPD_MAX_ROWS */
    uint32_t a;                /* extra index bits per row (Section 3.2 example: IBN = ceil(L/SR) + a) */
    uint32_t explicit_layout;  /* 0: derive isb/ibn from (r, sr, a); 1: use isb/ibn as given */
    uint32_t isb[SPD_MAX_ROWS];/* index starting bit of each row, Definition 3 */
    uint32_t ibn[SPD_MAX_ROWS];/* index bit count of each row, Definition 4; 2..16 */
    uint32_t log2k;            /* LDC length k = 2^log2k bits (Section 3.3); 5..16 */
    uint32_t lr;               /* LDCA rows, 1..SPD_MAX_ROWS */
    uint32_t log2lc;           /* LDCA columns LC = 2^log2lc; 0..24 */
    uint32_t window_slices;    /* 0: discrete window; K > 0: sliding window of K slices (Section 5) */
    uint32_t sliding_counter;  /* sliding window, the counter that replaces each bit (Section 5.2):
                                  0 = AT pool, one 8-bit asynchronously maintained time stamp per bit
                                  (K <= 254); 1 = one exact 16-bit time stamp per bit (K <= 30000) */
    /* Multiply-add-shift hashes h(x) = ((mul * x + add) mod 2^64) >> (64 - bits), mul odd:
     * index 0 = H1 (32 bits), 1 = H2 (3 bits), 2 = H3 (log2k bits), 3 + i = LH_i (log2lc bits). */
    uint64_t hash_mul[3 + SPD_MAX_ROWS];
    uint64_t hash_add[3 + SPD_MAX_ROWS];
} spd_params;

/* Host-side constants derived from spd_params (Eq. 1, Definitions 3-4, Eq. 4). */
typedef struct spd_derived {
    uint32_t tau;              /* Eq. 1: smallest t >= 0 with 8 * 2^t >= theta */
    uint32_t z_theta;          /* Eq. 4: largest z0 in [1, k] with -k ln(z0/k) >= theta (0: none) */
    uint32_t isb[SPD_MAX_ROWS];
    uint32_t ibn[SPD_MAX_ROWS];
    uint64_t sea_bytes;        /* bytes of one SEA */
    uint64_t seav_bytes;       /* 2^r * sea_bytes */
    uint64_t ldca_words;       /* LR * LC * k / 32 */
} spd_derived;

/* One super point reported at the end of a window. */
typedef struct spd_superpoint {
    uint32_t ip;               /* the host */
    uint32_t z0;               /* zero bits of its ULDC (AND of its LR LDCs) */
    uint32_t est;              /* Eq. 4 estimate -k ln(z0/k) rounded to nearest (z0 = 0 read as 1) */
    uint32_t flags;            /* bit 0: saturated (z0 == 0) */
} spd_superpoint;

/* One batch of a fused multi-router scan. */
#define SPD_BATCH_DST 1u      /* spd_batch.flags: destination-keyed, each record read as (oip, hip) */
typedef struct spd_batch {
    uint32_t router;           /* router (watch point) id, 0..n_routers-1 */
    uint32_t flags;            /* 0: source-keyed (element 0 is the monitored host); SPD_BATCH_DST:
                                  destination-keyed, the super points of the opposite direction.
                                  Both directions of one stream: give each its own router id and
                                  the same pairs twice in one call (one fused launch). */
    const uint32_t *pairs_dev; /* device pointer to n_pairs (hip, oip) records */
    uint64_t n_pairs;
} spd_batch;

/* Launch tuning.  Every setting gives the same sketch bits; only speed changes. */
typedef struct spd_tuning {
    uint64_t direct_max_pairs; /* batches up to this size use the direct-atomic scan kernel */
    uint32_t bucket_bits;      /* binned scan: log2 of sketch bits per LDS bucket (12..20) */
    uint32_t tile_pairs;       /* binned scan: pairs per tile (power of two, 2048..16384) */
    uint32_t bin_block;        /* binned scan: threads per workgroup of the binning kernel (256..1024) */
    uint32_t apply_block;      /* binned scan: threads per workgroup of the apply kernel (256..1024) */
    uint32_t direct_block;     /* direct scan: threads per workgroup */
    uint32_t direct_grid_per_cu; /* direct scan: workgroups per compute unit */
    uint32_t seav_lds;         /* direct scan: 1 = keep a per-workgroup LDS copy of the SEAV when it fits */
    uint32_t close_block;      /* end-of-window kernel: threads per workgroup */
    uint64_t launch_pairs;     /* binned scan: at most this many pairs per bin/apply launch (0: no limit);
                                  smaller launches keep their items resident in the Infinity Cache */
    uint32_t apply_unroll;     /* binned scan: tile segments each wavefront loads at once (8, 16, 32);
                                  region and exact-count layouts: 4, 8 or 16 item words per lane */
    uint32_t bin_mode;         /* binned scan layout: 0 = per-tile regions (one pass over the pairs);
                                  1 = bucket-major (an exact counting pass first, then contiguous
                                  per-bucket items that the apply phase streams);
                                  2 = per-(chunk of 128 tiles, bucket) regions of fixed capacity
                                  (one pass over the pairs; words past a region's capacity are
                                  recorded from a spill list after the apply phase) */
    uint32_t region_words;     /* bin_mode 2: 64-bit words per region (0: derived from the expected
                                  load of a bucket with a wide margin; small values force spills) */
} spd_tuning;

typedef struct spd_stats {
    uint64_t pairs_scanned;
    uint64_t direct_launches;
    uint64_t binned_launches;
    uint64_t closes;
    uint64_t candidates_last;  /* candidates rebuilt at the last close (before the LDCA filter) */
    uint64_t reported_last;
    uint64_t device_bytes;     /* device memory held by the context */
} spd_stats;

/* Kernel kinds timed by the optional profiler. */
#define SPD_K_DIRECT 0     /* direct-atomic scan */
#define SPD_K_STAMP 1      /* sliding-window scan */
#define SPD_K_BIN 2        /* binned scan, phase 1: tile binning */
#define SPD_K_TRANSPOSE 3  /* binned scan: per-tile offsets transposed to per-bucket rows */
#define SPD_K_APPLY 4      /* binned scan, phase 2: bucket apply */
#define SPD_K_MERGE 5      /* router merge */
#define SPD_K_CLOSE 6      /* end-of-window candidate rebuild and filter */
#define SPD_K_FILL 7       /* clears (window reset, counters) */
#define SPD_K_COUNT 8      /* exact-count layout (bin_mode 1): per-tile bucket counts */
#define SPD_K_OFFSETS 9    /* exact-count layout (bin_mode 1): per-tile segment offsets */
#define SPD_K_SPILL 10     /* region layout: words past a region's capacity */
#define SPD_K_KINDS 11

typedef struct spd_profile {
    uint64_t launches[SPD_K_KINDS];
    double total_ms[SPD_K_KINDS];  /* summed device time between HIP events around each launch */
} spd_profile;

typedef struct spd_ctx spd_ctx;

/* Derive the host constants of p without touching the GPU (Eq. 1, Section 3.2 layout and its
 * two constraints, Eq. 4).  SPD_E_INVALID if p is out of range or the layout breaks a constraint. */
spd_status spd_derive(const spd_params *p, spd_derived *out);

/* Create a context for n_routers routers (watch points, Section 4) plus one global sketch, all
 * zero, on the current HIP device.  hbm_budget_bytes bounds the device memory the context may
 * hold (0 = no bound); SPD_E_NOMEM if the sketches alone exceed it.  *out receives the context. */
spd_status spd_create(const spd_params *p, uint32_t n_routers, uint64_t hbm_budget_bytes, spd_ctx **out);

/* Release every device and host resource of ctx (synchronises the device). */
void spd_destroy(spd_ctx *ctx);

/* Record n_pairs pairs seen at one router into its sketches (Sections 3.1-3.3, Section 4.1).
 * The scan is order-free and idempotent: the sketch depends only on the set of distinct pairs.
 * Sliding mode: the pairs belong to the current slice.  n_pairs = 0 is a no-op. */
spd_status spd_scan(spd_ctx *ctx, uint32_t router, const uint32_t *pairs_dev, uint64_t n_pairs, void *stream);

/* The same for pairs in HOST memory (the watch point's buffered copy to the GPU, Section 4.1):
 * copied in chunks of chunk_pairs (0: 16 Mi) through two device staging buffers on a copy stream of
 * the library, the copy of one chunk overlapping the scan of the previous one.  Page-locked host
 * memory gives asynchronous copies; pageable memory works, with the copies synchronous.  flags:
 * 0 or SPD_BATCH_DST.  Returns when every pair has been recorded (the host buffer may be reused). */
spd_status spd_scan_host(spd_ctx *ctx, uint32_t router, const uint32_t *pairs_host, uint64_t n_pairs, uint32_t flags,
                         uint64_t chunk_pairs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): spd_scan without any allocation.  Same result as
 * spd_scan.  flags: 0 or SPD_BATCH_DST.  Discrete-window contexts only (SPD_E_STATE otherwise).
 * Batches up to the tuning's direct_max_pairs take the direct kernel, which needs no scratch;
 * larger ones take the region layout of the binned scan with all of its scratch in one fixed array
 * of SPD_NOALLOC_SCRATCH_BYTES device bytes that the library holds on every GPU it runs on until
 * the process ends, in as many launches as that array requires (each launch reads and writes the
 * whole sketch, so this is slower than spd_scan for large batches).  SPD_E_INVALID if one tile of
 * the sketch geometry alone needs more scratch than the array.  No timing events are recorded.
 * Every no-alloc call on one GPU shares that GPU's array, from any context: calls whose work may
 * overlap on the device (different streams, no ordering between them) race and must be ordered
 * by the caller.  Each call clears the counters it needs before use. */
#define SPD_NOALLOC_SCRATCH_BYTES (64u << 20)
spd_status spd_scan_noalloc(spd_ctx *ctx, uint32_t router, const uint32_t *pairs_dev, uint64_t n_pairs, uint32_t flags,
                            void *stream);

/* Record several batches, from any routers and of any sizes, in one fused pass (same result as
 * calling spd_scan on each batch). */
spd_status spd_scan_batches(spd_ctx *ctx, const spd_batch *batches, uint32_t n_batches, void *stream);

/* spd_scan_batches, then spd_merge of the routers the batches name: the global sketch := OR of
 * their sketches (Section 4.2).  When every named router gets pairs here and the call is one launch
 * of the region layout, the merge is done by the apply phase itself (no pass over the router
 * sketches); otherwise an ordinary spd_merge follows.  Same results either way. */
spd_status spd_scan_batches_merge(spd_ctx *ctx, const spd_batch *batches, uint32_t n_batches, void *stream);

/* Merge (Section 4.2): global sketch = bitwise OR of the listed routers' sketches (sliding mode:
 * element-wise maximum of time stamps, whose bit view is the OR).  The previous global content
 * is replaced.  Order-free; listing a router twice changes nothing. */
spd_status spd_merge(spd_ctx *ctx, const uint32_t *routers, uint32_t n, void *stream);

/* End of window for a target (router id or SPD_GLOBAL): rebuild the candidates from the SEAV
 * (Section 3.2, Eq. 3), keep those whose ULDC estimate reaches theta (Section 3.3, Eq. 4), and
 * write them to out_host (host memory) sorted by ip ascending.  *n_out = number of super points;
 * if it exceeds cap the first cap are written and SPD_E_TRUNCATED is returned.
 * Discrete mode: the target's sketch is then reset to zero (a new window starts; no device work:
 * its next scan writes the sketch from zero).
 * Sliding mode: reports the window of the last K slices; nothing is reset. */
spd_status spd_close_window(spd_ctx *ctx, int32_t target, spd_superpoint *out_host, uint32_t cap,
                            uint32_t *n_out, void *stream);

/* The end of window in two halves, so that the next window's scans can be enqueued before the
 * report is collected (Sections 3.3, 4.2).  spd_close_begin enqueues on `stream` the device work of
 * spd_close_window for the target and, in discrete mode, resets the target at once (the next
 * scans start a new window); *ticket names the close.  spd_close_end waits for that close and
 * writes its report as spd_close_window does.  At most SPD_MAX_PENDING_CLOSES closes per context
 * are pending (begun, not ended; SPD_E_STATE beyond that); they are ended in any order, each once.
 * A pending close holds room for 65536 super points: if its window has more, spd_close_end returns
 * SPD_E_TRUNCATED with *n_out = their number and no report (spd_close_window re-runs instead),
 * and later closes get room for them.  The first spd_close_begin of a context allocates the
 * buffers of all pending closes (which synchronises the device). */
#define SPD_MAX_PENDING_CLOSES 4
spd_status spd_close_begin(spd_ctx *ctx, int32_t target, void *stream, uint32_t *ticket);
spd_status spd_close_end(spd_ctx *ctx, uint32_t ticket, spd_superpoint *out_host, uint32_t cap, uint32_t *n_out);

/* Start a new window for a target without reporting the current one: the re-initialisation of a
 * watch point's sketch at the start of each window (Sections 3.3, 4.2), e.g. once its sketch has
 * been merged into the global one.  Discrete mode: the slot is marked empty and its next scan
 * starts from zero (no device work here).  Sliding mode: every time stamp is cleared, enqueued on
 * `stream`. */
spd_status spd_reset(spd_ctx *ctx, int32_t target, void *stream);

/* Sliding mode only: the next scans belong to the next time slice (Section 5.2).  Exact stamps
 * older than the window simply drop out of the bit view.  With the AT pool, one of 255 - K groups
 * of every slot's counters is maintained, enqueued on `stream`: its counters outside the window
 * get the code of slice t - K, so that every counter's age read modulo 256 stays exact. */
spd_status spd_slide(spd_ctx *ctx, void *stream);

/* Copy a target's sketch to host memory in the canonical layouts (seav_host: seav_bytes bytes,
 * ldca_host: ldca_words words).  Sliding mode: the bit view of the current window. */
spd_status spd_export(spd_ctx *ctx, int32_t target, uint8_t *seav_host, uint32_t *ldca_host);

/* Replace a target's sketch by host data in the canonical layouts (discrete mode only). */
spd_status spd_import(spd_ctx *ctx, int32_t target, const uint8_t *seav_host, const uint32_t *ldca_host);

/* Sliding mode: copy a target's raw time stamps (1 + last slice that set the bit, 0 = never):
 * seav_ts_host holds seav_bytes * 8 entries (bit b of byte x at 8x + b), ldca_ts_host holds
 * ldca_words * 32 entries (one per LDCA bit).  With the AT pool the stamps are rebuilt from the
 * counters (modulo 2^16); a counter outside the window (set K or more slices ago, or never)
 * reads 0. */
spd_status spd_export_stamps(spd_ctx *ctx, int32_t target, uint16_t *seav_ts_host, uint16_t *ldca_ts_host);

/* Current slice index (sliding mode; 0 in discrete mode). */
uint32_t spd_current_slice(const spd_ctx *ctx);

/* Turn per-kernel timing on (1) or off (0) and reset its totals.  When on, every kernel launch
 * is bracketed by two HIP events recorded on the launch stream. */
spd_status spd_profile_enable(spd_ctx *ctx, uint32_t on);

/* Which kernel kinds are timed while profiling is on: bit k selects kind k (SPD_K_*); all by
 * default.  Timing fewer kinds records fewer events on the stream. */
spd_status spd_profile_select(spd_ctx *ctx, uint32_t kinds_mask);

/* Totals since the last spd_profile_enable(); waits for the recorded events. */
spd_status spd_get_profile(spd_ctx *ctx, spd_profile *out);

spd_status spd_get_tuning(const spd_ctx *ctx, spd_tuning *out);
spd_status spd_set_tuning(spd_ctx *ctx, const spd_tuning *t);
spd_status spd_get_stats(const spd_ctx *ctx, spd_stats *out);

const char *spd_strerror(spd_status s);
const char *spd_last_error(const spd_ctx *ctx);

/* ------------------------------------------------------------------------------------------
 * Serving loop.  Routers submit batches of pairs as they arrive; a scheduler thread keeps every
 * open router window in a device slot, admits windows while slots fit the HBM budget (others
 * wait), fuses whatever batches are pending, from any routers and of any sizes, into one scan
 * launch group, and closes a window when its router has seen window_pairs pairs (a batch that
 * crosses the boundary is split) or when a batch is submitted with SPD_SUBMIT_CLOSE.  Closes run
 * on their own stream, replayed from a hipGraph captured per slot, and overlap later scans.  A
 * window's result equals the result of scanning its pairs alone (Sections 3-4 are order-free).
 * ------------------------------------------------------------------------------------------ */
typedef struct spd_server spd_server;

#define SPD_SUBMIT_CLOSE 1u    /* close the router's window after this batch */
#define SPD_SUBMIT_DST 2u      /* destination-keyed batch (records read as (oip, hip)); a router's
                                  batches should all be keyed the same way */

typedef struct spd_server_config {
    uint32_t n_routers;
    uint32_t max_slots;            /* upper bound on open windows (0: as many as the budget allows) */
    uint64_t window_pairs;         /* close a router's window every this many pairs (0: on request only) */
    uint64_t hbm_budget_bytes;     /* device memory for slots and scratch (0: 4 GiB) */
    uint64_t max_group_pairs;      /* fused launch: at most this many pairs (0: 64 Mi) */
    uint32_t max_group_batches;    /* fused launch: at most this many batches (0: 1024) */
    uint32_t use_graphs;           /* 1: replay each slot's end-of-window work from a hipGraph */
    uint64_t min_scan_pairs;       /* while earlier scans are still running on the GPU, a router's queued
                                      pairs wait until this many are queued, its window can end, a close
                                      is requested or drain is called; an idle GPU takes whatever is
                                      queued (0: window_pairs, or 8 Mi without a window size: under
                                      load a window is then scanned whole, into a fresh sketch, instead
                                      of in parts that each read and rewrite the whole sketch) */
    const spd_tuning *tuning;      /* launch settings of the scans (NULL: the library's defaults); applied
                                      before the scratch of the largest group is reserved */
} spd_server_config;

typedef struct spd_window_result {
    uint32_t router;
    uint32_t window;               /* index of the window within its router, from 0 */
    uint64_t pairs;                /* pairs recorded in the window */
    double latency_ms;             /* submission of the batch that completed the window -> result on host */
    uint32_t n_super;              /* super points reported (the first cap are copied out) */
    uint32_t reserved;
} spd_window_result;

typedef struct spd_server_stats {
    uint64_t batches;
    uint64_t pairs;
    uint64_t groups;               /* fused scan launches */
    uint64_t windows;              /* windows closed */
    uint64_t admission_waits;      /* times a router waited for a free slot */
    uint32_t slots;                /* window slots that fit the budget */
    uint32_t max_open;             /* most windows open at once */
} spd_server_stats;

/* Start a serving loop with its own scheduler thread and streams on the current device. */
spd_status spd_server_create(const spd_params *p, const spd_server_config *cfg, spd_server **out);

/* Hand over one batch (device pointer; must stay valid until its window has been reported).
 * Returns at once. */
spd_status spd_server_submit(spd_server *srv, uint32_t router, const uint32_t *pairs_dev, uint64_t n_pairs,
                             uint32_t flags);

/* Next finished window: header in *hdr, its super points (sorted by ip) in out_host[0..cap).
 * Waits up to timeout_ms (negative: forever); SPD_E_AGAIN if none finished in time. */
spd_status spd_server_next(spd_server *srv, spd_window_result *hdr, spd_superpoint *out_host, uint32_t cap,
                           int32_t timeout_ms);

/* One arrival of a replayed traffic schedule. */
typedef struct spd_arrival {
    double t_s;                    /* arrival time in seconds from the start of the replay */
    uint32_t router;
    uint32_t flags;                /* SPD_SUBMIT_CLOSE and/or SPD_SUBMIT_DST, or 0 */
    const uint32_t *pairs_dev;
    uint64_t n_pairs;
} spd_arrival;

/* Submit a schedule of arrivals (sorted by t_s) from the calling thread, each at its time: a
 * native load generator for Poisson-like router traffic.  Returns the seconds it took. */
spd_status spd_server_replay(spd_server *srv, const spd_arrival *sched, uint64_t n, double *elapsed_s);

/* Wait until every submitted batch has been scanned and every requested close has finished. */
spd_status spd_server_drain(spd_server *srv);

spd_status spd_server_get_stats(spd_server *srv, spd_server_stats *out);
spd_status spd_server_set_tuning(spd_server *srv, const spd_tuning *t);
const char *spd_server_last_error(spd_server *srv);

/* Stop the scheduler (pending work is finished first) and release everything. */
void spd_server_destroy(spd_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* SPD_H */
