/*
 * Plain CPU oracle for super-point detection with a short-estimator array vector (SEAV) and a
 * linear-distinct-counter array (LDCA): Xu, Ding and Hu, "Most memory efficient distributed super
 * points detection on core networks" (arXiv 1901.07306).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously correct reference that the GPU
 * library is compared against.  Only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark may load it; the product path never does.  It shares no code, header or table
 * with the GPU library.
 *
 * Everything here is integer arithmetic except Eq. 4, whose threshold and estimate are evaluated
 * once per query in IEEE double with the C library's log().
 *
 * Readings of the paper used here (the paper is silent or garbled on these points):
 *  - lsb(x) is the index of the lowest set bit (trailing zeros); lsb(0) = 32 (Section 3.1).
 *  - sampling test is lsb(H1(oip)) >= tau, tau from Eq. 1 in integers, never below 0.
 *  - bit j of LP and of Idx counts from the least significant bit (Eq. 2).
 *  - RP = hip mod 2^r, LP = hip >> r, hip = (LP << r) | RP (Section 3.2).
 *  - Eq. 2 and Eq. 3 index LP modulo 32 - r; a row may wrap from the top of LP to bit 0.
 *  - A candidate tuple is kept only if every LP bit covered by several rows has the same value
 *    in all of them (the overlap bits remove fake candidates, Section 3.2, constraint 2), and the
 *    AND of its SR short estimators has weight >= 3 (SEU test, Section 3.2).
 *  - H1, H2, H3 hash the opposite IP and are shared by every row; LH_i hashes the host (3.1, 3.3).
 *  - Hashes are multiply-add-shift: ((a*x + b) mod 2^64) >> (64 - M) with odd 64-bit a.
 *  - The ULDC is the AND of a host's LR LDCs; z0 is its count of zero bits (Section 3.3, Lemma 1).
 *  - A host is reported iff -k ln(z0/k) >= theta (Definition 2 uses >=); z0 = 0 always passes and
 *    is flagged as saturated, with its estimate computed at z0 = 1.
 *  - Routers are merged with bitwise OR (Section 4.2).
 *  - Sliding window (Section 5): every bit becomes a time stamp holding 1 + the last slice that
 *    set it (0 = never).  The bit view of the window of K slices ending at slice t is
 *    stamp >= max(1, t - K + 2).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_ROWS 8
#define ORC_SE_BITS 8     /* g: bits per short estimator (Section 3.1) */
#define ORC_SE_HOT 3      /* weight at which an SE is judged >= theta (Section 3.1) */

typedef struct {
    uint32_t theta;                 /* super-point threshold (Definition 2) */
    uint32_t r;                     /* right-part bits: 2^r SEAs in the SEAV */
    uint32_t sr;                    /* rows per SEA */
    uint32_t isb[ORC_MAX_ROWS];     /* index starting bit per row (Definition 3) */
    uint32_t ibn[ORC_MAX_ROWS];     /* index bit count per row (Definition 4) */
    uint32_t log2k;                 /* LDC length k = 2^log2k bits */
    uint32_t lr;                    /* LDCA rows */
    uint32_t log2lc;                /* LDCA columns LC = 2^log2lc */
    uint64_t mul[3 + ORC_MAX_ROWS]; /* hash multipliers: H1, H2, H3, LH_0 .. LH_{lr-1} */
    uint64_t add[3 + ORC_MAX_ROWS]; /* hash addends, same order */
} orc_params;

typedef struct {
    uint32_t ip;
    uint32_t z0;
    uint32_t est;
    uint32_t flags;   /* bit 0: saturated (z0 == 0) */
} orc_record;

/* ---------------------------------------------------------------- constants (Eq. 1, Eq. 4) */

/* Eq. 1: tau = ceil(log2(theta / 8)), i.e. the smallest t >= 0 with 8 * 2^t >= theta. */
uint32_t orc_tau(uint32_t theta) {
    uint32_t t = 0;
    while (((uint64_t)ORC_SE_BITS << t) < (uint64_t)theta) t++;
    return t;
}

/* Eq. 4 estimate -k ln(z0/k), rounded to the nearest integer; z0 = 0 is evaluated at 1. */
uint32_t orc_est(uint32_t log2k, uint32_t z0) {
    double k = (double)(1u << log2k);
    double z = (double)(z0 == 0 ? 1u : z0);
    return (uint32_t)floor(-k * log(z / k) + 0.5);
}

/* Largest z in [1, k] whose Eq. 4 estimate reaches theta; 0 when none does. */
uint32_t orc_z_theta(uint32_t log2k, uint32_t theta) {
    uint32_t k = 1u << log2k;
    for (uint32_t z = k; z >= 1; z--)
        if (-(double)k * log((double)z / (double)k) >= (double)theta) return z;
    return 0;
}

/* ------------------------------------------------------------------ layout (Section 3.2) */

/* The example parameterisation of Section 3.2, read with L = 32 - r index positions:
 * s = ceil(L / SR), ISB(i) = i*s mod L, IBN(i) = min(s + a, L).  Returns 0 on success, -1 if
 * the constraints do not hold (every LP bit covered; consecutive rows, cyclically, share bits). */
int orc_layout(uint32_t r, uint32_t sr, uint32_t a, uint32_t *isb, uint32_t *ibn) {
    if (r > 30 || sr < 1 || sr > ORC_MAX_ROWS) return -1;
    uint32_t L = 32 - r;
    uint32_t s = (L + sr - 1) / sr;
    for (uint32_t i = 0; i < sr; i++) {
        isb[i] = (i * s) % L;
        ibn[i] = s + a < L ? s + a : L;
    }
    return 0;
}

/* Constraint 1: every position of LP lies in some row's index. */
int orc_covers_all(const orc_params *p) {
    uint32_t L = 32 - p->r;
    for (uint32_t j = 0; j < L; j++) {
        int hit = 0;
        for (uint32_t i = 0; i < p->sr; i++)
            if ((j + L - p->isb[i]) % L < p->ibn[i]) hit = 1;
        if (!hit) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------- hashes (Section 3.1) */

/* Multiply-add-shift hash to m bits (0 <= m <= 32); m = 0 has the single value 0. */
uint32_t orc_hash(uint32_t x, uint64_t mul, uint64_t add, uint32_t m) {
    uint64_t v = mul * (uint64_t)x + add;   /* mod 2^64 */
    return m == 0 ? 0u : (uint32_t)(v >> (64 - m));
}

static uint32_t lsb32(uint32_t x) {
    if (x == 0) return 32;
    uint32_t n = 0;
    while (!(x & 1u)) { x >>= 1; n++; }
    return n;
}

static uint32_t weight8(uint8_t v) {
    uint32_t n = 0;
    for (int b = 0; b < 8; b++) n += (v >> b) & 1u;
    return n;
}

static uint32_t weight32(uint32_t v) {
    uint32_t n = 0;
    for (int b = 0; b < 32; b++) n += (v >> b) & 1u;
    return n;
}

/* ------------------------------------------------------------ index maps (Eq. 2, Eq. 3) */

/* Eq. 2: bit j of Idx(i, LP) is bit (ISB(i) + j) mod L of LP. */
uint32_t orc_idx(uint32_t lp, uint32_t isb, uint32_t ibn, uint32_t L) {
    uint32_t idx = 0;
    for (uint32_t j = 0; j < ibn; j++) {
        uint32_t bit = (lp >> ((isb + j) % L)) & 1u;
        idx |= bit << j;
    }
    return idx;
}

/* Eq. 3: rebuild LP from the SR row indexes.  Bit j of LP is read from every row that covers
 * it; returns 1 and writes *lp when all of them agree, 0 when two rows disagree. */
int orc_lp_from_idx(const orc_params *p, const uint32_t *idx, uint32_t *lp) {
    uint32_t L = 32 - p->r;
    uint32_t out = 0;
    for (uint32_t j = 0; j < L; j++) {
        int seen = 0;
        uint32_t val = 0;
        for (uint32_t i = 0; i < p->sr; i++) {
            uint32_t off = (j + L - p->isb[i]) % L;
            if (off < p->ibn[i]) {
                uint32_t b = (idx[i] >> off) & 1u;
                if (seen && b != val) return 0;
                seen = 1;
                val = b;
            }
        }
        if (!seen) return 0;
        out |= val << j;
    }
    *lp = out;
    return 1;
}

/* ---------------------------------------------------------------------- sizes and offsets */

/* Bytes of one SEA: the rows are stored one after the other, row i holding 2^IBN(i) SEs. */
uint64_t orc_sea_bytes(const orc_params *p) {
    uint64_t n = 0;
    for (uint32_t i = 0; i < p->sr; i++) n += (uint64_t)1 << p->ibn[i];
    return n;
}

uint64_t orc_seav_bytes(const orc_params *p) { return orc_sea_bytes(p) << p->r; }

uint64_t orc_ldca_words(const orc_params *p) {
    return ((uint64_t)p->lr << p->log2lc) << (p->log2k - 5);
}

static uint64_t row_offset(const orc_params *p, uint32_t i) {
    uint64_t off = 0;
    for (uint32_t q = 0; q < i; q++) off += (uint64_t)1 << p->ibn[q];
    return off;
}

/* Byte offset of SE(RP, row i, column c) in the SEAV. */
static uint64_t se_offset(const orc_params *p, uint32_t rp, uint32_t i, uint32_t c) {
    return (uint64_t)rp * orc_sea_bytes(p) + row_offset(p, i) + c;
}

/* First word of LDC (row i, column c) in the LDCA. */
static uint64_t ldc_word(const orc_params *p, uint32_t i, uint32_t c) {
    return (((uint64_t)i << p->log2lc) + c) << (p->log2k - 5);
}

/* --------------------------------------------------------------- scan (Sections 3.1 - 3.3) */

/* Record n pairs (pairs[2j] = hip, pairs[2j+1] = oip) into one router's SEAV and LDCA. */
void orc_scan(const orc_params *p, uint8_t *seav, uint32_t *ldca, const uint32_t *pairs, uint64_t n) {
    uint32_t tau = orc_tau(p->theta);
    uint32_t L = 32 - p->r;
    for (uint64_t j = 0; j < n; j++) {
        uint32_t hip = pairs[2 * j], oip = pairs[2 * j + 1];
        /* short estimator: sampled by the lowest set bit of H1(oip), bit chosen by H2(oip) */
        if (lsb32(orc_hash(oip, p->mul[0], p->add[0], 32)) >= tau) {
            uint32_t b = orc_hash(oip, p->mul[1], p->add[1], 3);
            uint32_t rp = hip & ((1u << p->r) - 1u);
            uint32_t lp = (uint32_t)((uint64_t)hip >> p->r);
            for (uint32_t i = 0; i < p->sr; i++) {
                uint32_t c = orc_idx(lp, p->isb[i], p->ibn[i], L);
                seav[se_offset(p, rp, i, c)] |= (uint8_t)(1u << b);
            }
        }
        /* long estimator: one LDC per row picked by LH_i(hip), bit H3(oip) */
        uint32_t q = orc_hash(oip, p->mul[2], p->add[2], p->log2k);
        for (uint32_t i = 0; i < p->lr; i++) {
            uint32_t c = orc_hash(hip, p->mul[3 + i], p->add[3 + i], p->log2lc);
            ldca[ldc_word(p, i, c) + (q >> 5)] |= 1u << (q & 31u);
        }
    }
}

/* Merge of router sketches (Section 4.2): bitwise OR. */
void orc_merge(uint8_t *dst_seav, const uint8_t *src_seav, uint32_t *dst_ldca, const uint32_t *src_ldca,
               const orc_params *p) {
    uint64_t nb = orc_seav_bytes(p), nw = orc_ldca_words(p);
    for (uint64_t i = 0; i < nb; i++) dst_seav[i] |= src_seav[i];
    for (uint64_t i = 0; i < nw; i++) dst_ldca[i] |= src_ldca[i];
}

/* ------------------------------------------------------ restoring candidates (Section 3.2) */

/* The candidate list by the paper's procedure: per SEA, the hot SEs HSE(i) of every row, every
 * tuple of the product CIS, LP rebuilt by Eq. 3 (tuples whose overlap bits disagree dropped),
 * kept when the AND of the tuple's SEs has weight >= 3.  Writes up to cap hosts (ascending RP,
 * then tuple order) and returns how many there are. */
uint64_t orc_candidates(const orc_params *p, const uint8_t *seav, uint32_t *out, uint64_t cap) {
    uint64_t n = 0;
    uint32_t nrp = 1u << p->r;
    uint32_t *hse[ORC_MAX_ROWS];
    uint32_t cnt[ORC_MAX_ROWS];
    for (uint32_t i = 0; i < p->sr; i++) hse[i] = (uint32_t *)malloc(sizeof(uint32_t) << p->ibn[i]);
    for (uint32_t rp = 0; rp < nrp; rp++) {
        int empty = 0;
        for (uint32_t i = 0; i < p->sr; i++) {
            cnt[i] = 0;
            for (uint32_t c = 0; c < (1u << p->ibn[i]); c++)
                if (weight8(seav[se_offset(p, rp, i, c)]) >= ORC_SE_HOT) hse[i][cnt[i]++] = c;
            if (cnt[i] == 0) empty = 1;
        }
        if (empty) continue;
        uint32_t digit[ORC_MAX_ROWS] = {0};
        for (;;) {
            uint32_t idx[ORC_MAX_ROWS];
            uint8_t seu = 0xFF;
            for (uint32_t i = 0; i < p->sr; i++) {
                idx[i] = hse[i][digit[i]];
                seu &= seav[se_offset(p, rp, i, idx[i])];
            }
            uint32_t lp;
            if (orc_lp_from_idx(p, idx, &lp) && weight8(seu) >= ORC_SE_HOT) {
                if (n < cap) out[n] = (uint32_t)(((uint64_t)lp << p->r) | rp);
                n++;
            }
            /* next tuple of the product, row 0 varying fastest */
            uint32_t i = 0;
            while (i < p->sr && ++digit[i] == cnt[i]) digit[i++] = 0;
            if (i == p->sr) break;
        }
    }
    for (uint32_t i = 0; i < p->sr; i++) free(hse[i]);
    return n;
}

/* The candidate set by its definition: every host of RP in [rp_lo, rp_hi) whose SR SEs AND to
 * weight >= 3.  Ascending host order within each RP. */
uint64_t orc_candidates_brute(const orc_params *p, const uint8_t *seav, uint32_t rp_lo, uint32_t rp_hi,
                              uint32_t *out, uint64_t cap) {
    uint64_t n = 0;
    uint32_t L = 32 - p->r;
    for (uint32_t rp = rp_lo; rp < rp_hi; rp++) {
        for (uint64_t lp = 0; lp < ((uint64_t)1 << L); lp++) {
            uint8_t seu = 0xFF;
            for (uint32_t i = 0; i < p->sr; i++)
                seu &= seav[se_offset(p, rp, i, orc_idx((uint32_t)lp, p->isb[i], p->ibn[i], L))];
            if (weight8(seu) >= ORC_SE_HOT) {
                if (n < cap) out[n] = (uint32_t)((lp << p->r) | rp);
                n++;
            }
        }
    }
    return n;
}

/* ------------------------------------------------------------ filtering (Section 3.3) */

/* Zero bits of the host's ULDC: the AND of its LR LDCs. */
uint32_t orc_uldc_zeros(const orc_params *p, const uint32_t *ldca, uint32_t h) {
    uint32_t words = 1u << (p->log2k - 5);
    uint32_t ones = 0;
    for (uint32_t w = 0; w < words; w++) {
        uint32_t u = 0xFFFFFFFFu;
        for (uint32_t i = 0; i < p->lr; i++) {
            uint32_t c = orc_hash(h, p->mul[3 + i], p->add[3 + i], p->log2lc);
            u &= ldca[ldc_word(p, i, c) + w];
        }
        ones += weight32(u);
    }
    return (1u << p->log2k) - ones;
}

static int cmp_record(const void *a, const void *b) {
    uint32_t x = ((const orc_record *)a)->ip, y = ((const orc_record *)b)->ip;
    return (x > y) - (x < y);
}

/* End of window: candidates from the SEAV, kept when their ULDC estimate reaches theta, sorted by
 * ip.  Writes up to cap records and returns how many there are (-1 if the candidate list itself
 * could not be allocated). */
int64_t orc_detect(const orc_params *p, const uint8_t *seav, const uint32_t *ldca, orc_record *out, uint64_t cap) {
    uint64_t nc = orc_candidates(p, seav, NULL, 0);
    uint32_t *cand = (uint32_t *)malloc(sizeof(uint32_t) * (nc ? nc : 1));
    if (!cand) return -1;
    orc_candidates(p, seav, cand, nc);
    uint32_t zt = orc_z_theta(p->log2k, p->theta);
    orc_record *rec = (orc_record *)malloc(sizeof(orc_record) * (nc ? nc : 1));
    uint64_t n = 0;
    for (uint64_t j = 0; j < nc; j++) {
        uint32_t z0 = orc_uldc_zeros(p, ldca, cand[j]);
        if (z0 <= zt) {
            rec[n].ip = cand[j];
            rec[n].z0 = z0;
            rec[n].est = orc_est(p->log2k, z0);
            rec[n].flags = z0 == 0 ? 1u : 0u;
            n++;
        }
    }
    qsort(rec, n, sizeof(orc_record), cmp_record);
    for (uint64_t j = 0; j < n && j < cap; j++) out[j] = rec[j];
    free(rec);
    free(cand);
    return (int64_t)n;
}

/* ------------------------------------------------------------ sliding window (Section 5) */

/* Record the pairs of slice t: every bit the discrete scan would set gets time stamp t + 1.
 * seav_ts holds 8 stamps per SE byte (bit b of byte x at 8x + b); ldca_ts one stamp per bit. */
void orc_scan_slice(const orc_params *p, uint16_t *seav_ts, uint16_t *ldca_ts, const uint32_t *pairs,
                    uint64_t n, uint32_t t) {
    uint32_t tau = orc_tau(p->theta);
    uint32_t L = 32 - p->r;
    uint16_t stamp = (uint16_t)(t + 1);
    for (uint64_t j = 0; j < n; j++) {
        uint32_t hip = pairs[2 * j], oip = pairs[2 * j + 1];
        if (lsb32(orc_hash(oip, p->mul[0], p->add[0], 32)) >= tau) {
            uint32_t b = orc_hash(oip, p->mul[1], p->add[1], 3);
            uint32_t rp = hip & ((1u << p->r) - 1u);
            uint32_t lp = (uint32_t)((uint64_t)hip >> p->r);
            for (uint32_t i = 0; i < p->sr; i++) {
                uint32_t c = orc_idx(lp, p->isb[i], p->ibn[i], L);
                seav_ts[se_offset(p, rp, i, c) * 8 + b] = stamp;
            }
        }
        uint32_t q = orc_hash(oip, p->mul[2], p->add[2], p->log2k);
        for (uint32_t i = 0; i < p->lr; i++) {
            uint32_t c = orc_hash(hip, p->mul[3 + i], p->add[3 + i], p->log2lc);
            ldca_ts[((((uint64_t)i << p->log2lc) + c) << p->log2k) + q] = stamp;
        }
    }
}

/* Bit view of the window of K slices ending at slice t: a bit is 1 iff its stamp is at least
 * max(1, t - K + 2), i.e. it was set in one of the slices t-K+1 .. t. */
void orc_bit_view(const orc_params *p, const uint16_t *seav_ts, const uint16_t *ldca_ts, uint32_t t, uint32_t K,
                  uint8_t *seav, uint32_t *ldca) {
    int64_t lo = (int64_t)t - (int64_t)K + 2;
    uint32_t thr = lo < 1 ? 1u : (uint32_t)lo;
    uint64_t nb = orc_seav_bytes(p), nw = orc_ldca_words(p);
    for (uint64_t x = 0; x < nb; x++) {
        uint8_t v = 0;
        for (uint32_t b = 0; b < 8; b++)
            if (seav_ts[x * 8 + b] >= thr) v |= (uint8_t)(1u << b);
        seav[x] = v;
    }
    for (uint64_t w = 0; w < nw; w++) {
        uint32_t v = 0;
        for (uint32_t b = 0; b < 32; b++)
            if (ldca_ts[w * 32 + b] >= thr) v |= 1u << b;
        ldca[w] = v;
    }
}
