"""Seeded synthetic core-network traffic for super-point detection experiments.

This module produces inputs only: windows of IPv4 (hip, oip) pairs stored as ``uint32[n, 2]``
(column 0 = the monitored host, here the source; column 1 = its opposite IP, here the
destination), the ground truth of the hosts planted as super points, and the random hash
parameters the detection method draws.  It holds none of the detection arithmetic, so the CPU
oracle and the GPU library can both consume what it emits without sharing any method code.

Every random draw comes from a Philox counter-based generator keyed by (seed, stream id, ...),
so any router, window or time slice regenerates on its own.  Hash parameters are expanded from a
seed with SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014).

The workloads stand in for the paper's CAIDA OC192 windows (Section 6), which are not available
here: uniform random IPv4 addresses, background sources whose distinct-peer counts follow a
truncated Zipf law, and planted hosts with thousands of distinct peers.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from typing import Dict, List, Optional, Tuple

import numpy as np

MASK64 = (1 << 64) - 1
GOLDEN64 = 0x9E3779B97F4A7C15


# ----------------------------------------------------------------------------------------------
# SplitMix64 and the hash parameters the method draws
# ----------------------------------------------------------------------------------------------
def splitmix64(state: int) -> Tuple[int, int]:
    """One SplitMix64 step: returns (next_state, output)."""
    state = (state + GOLDEN64) & MASK64
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return state, z ^ (z >> 31)


def splitmix64_stream(seed: int, n: int) -> List[int]:
    out, s = [], seed & MASK64
    for _ in range(n):
        s, z = splitmix64(s)
        out.append(z)
    return out


def hash_params(seed: int, lr: int) -> Tuple[List[int], List[int]]:
    """Multipliers (odd) and addends for H1, H2, H3 and LH_0..LH_{lr-1}, in that order."""
    raw = splitmix64_stream(seed, 2 * (3 + lr))
    mul = [raw[2 * j] | 1 for j in range(3 + lr)]
    add = [raw[2 * j + 1] for j in range(3 + lr)]
    return mul, add


# ----------------------------------------------------------------------------------------------
# Method parameters (the same values are handed to the oracle and to the GPU library)
# ----------------------------------------------------------------------------------------------
@dataclass(frozen=True)
class MethodParams:
    """Sizes and threshold of the two estimators.

    theta   super-point threshold (Definition 2)
    r       bits of the host's right part that pick one SEA of the SEAV (Section 3.2)
    sr      rows per SEA
    a       extra index bits per row, so consecutive rows share bits (Section 3.2 example)
    log2k   log2 of the LDC length in bits (Section 3.3)
    lr      LDCA rows
    log2lc  log2 of the LDCA columns
    window_slices   sliding window length in slices (Section 5); 0 = discrete window
    sliding_counter the counter that replaces each bit under a sliding window: 0 = AT pool,
                    1 = exact 16-bit time stamps (a storage choice; every result is the same)
    hash_seed       seed for the hash parameters
    """
    theta: int = 1024
    r: int = 14
    sr: int = 4
    a: int = 2
    log2k: int = 12
    lr: int = 2
    log2lc: int = 16
    window_slices: int = 0
    sliding_counter: int = 0
    hash_seed: int = 0x51A7E5EED

    def hashes(self) -> Tuple[List[int], List[int]]:
        return hash_params(self.hash_seed, self.lr)

    def replace(self, **kw) -> "MethodParams":
        return dataclasses.replace(self, **kw)

    @property
    def seav_bytes_estimate(self) -> int:
        L = 32 - self.r
        s = -(-L // self.sr)
        return (1 << self.r) * self.sr * (1 << min(L, s + self.a))

    @property
    def ldca_bytes(self) -> int:
        return self.lr << (self.log2lc + self.log2k - 3)


# ----------------------------------------------------------------------------------------------
# Workloads
# ----------------------------------------------------------------------------------------------
@dataclass(frozen=True)
class Workload:
    name: str
    params: MethodParams
    n_packets: int                  # per router (and per slice for the sliding workload)
    n_sources: int
    zipf_s: float
    zipf_cap: int
    n_planted: int
    planted_lo: int                 # planted distinct peers drawn uniformly from [lo, hi]
    planted_hi: int
    dup_frac: float = 0.0
    n_routers: int = 1
    multi_router_frac: float = 0.0  # fraction of sources seen at >= 2 routers
    n_slices: int = 0
    seed: int = 1


CONFIGS: Dict[str, Workload] = {
    # 1 router, 1 window of 1,000,000 pairs
    "plain_1m": Workload(
        name="plain_1m",
        params=MethodParams(theta=1024, r=6, sr=4, a=2, log2k=12, lr=2, log2lc=12),
        n_packets=1_000_000, n_sources=50_000, zipf_s=1.2, zipf_cap=200,
        n_planted=20, planted_lo=2000, planted_hi=2000, dup_frac=0.0, seed=101),
    # 1 router, 1 large window of 64 Mi pairs with 30 % duplicates
    "plain_64m": Workload(
        name="plain_64m",
        params=MethodParams(theta=1024, r=14, sr=4, a=2, log2k=12, lr=2, log2lc=16),
        n_packets=64 << 20, n_sources=2_000_000, zipf_s=1.1, zipf_cap=500,
        n_planted=500, planted_lo=1024, planted_hi=20000, dup_frac=0.30, seed=202),
    # 8 routers x 16 Mi pairs, overlapping source sets, planted peers split over routers
    "routers_8x16m": Workload(
        name="routers_8x16m",
        params=MethodParams(theta=1024, r=15, sr=4, a=2, log2k=12, lr=2, log2lc=17),
        n_packets=16 << 20, n_sources=4_000_000, zipf_s=1.1, zipf_cap=500,
        n_planted=300, planted_lo=1024, planted_hi=20000, dup_frac=0.30,
        n_routers=8, multi_router_frac=0.40, seed=303),
    # 300 slices of 1,000,000 pairs, sliding window of 60 slices
    "sliding_300x1m": Workload(
        name="sliding_300x1m",
        params=MethodParams(theta=1024, r=14, sr=4, a=2, log2k=12, lr=2, log2lc=16,
                            window_slices=60),
        n_packets=1_000_000, n_sources=1_000_000, zipf_s=1.1, zipf_cap=500,
        n_planted=200, planted_lo=35, planted_hi=70, n_slices=300, seed=404),
    # 16 routers, batches of log-uniform size in [4Ki, 4Mi], close every 64 Mi pairs per router
    "serving_16r": Workload(
        name="serving_16r",
        params=MethodParams(theta=1024, r=14, sr=4, a=2, log2k=12, lr=2, log2lc=16),
        n_packets=64 << 20, n_sources=2_000_000, zipf_s=1.1, zipf_cap=500,
        n_planted=1000, planted_lo=1024, planted_hi=20000, dup_frac=0.30,
        n_routers=16, seed=505),
}


def scaled(w: Workload, **kw) -> Workload:
    """A smaller copy of a workload (same shape of traffic, same method parameters)."""
    return dataclasses.replace(w, **kw)


# ----------------------------------------------------------------------------------------------
# Random helpers
# ----------------------------------------------------------------------------------------------
def rng_for(seed: int, *stream: int) -> np.random.Generator:
    """Counter-based generator keyed by (seed, stream...)."""
    key = [int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF] + [int(s) & 0xFFFFFFFF for s in stream]
    return np.random.Generator(np.random.Philox(np.random.SeedSequence(key)))


def random_u32(rng: np.random.Generator, n: int) -> np.ndarray:
    return rng.integers(0, 0xFFFFFFFF, size=n, dtype=np.uint32, endpoint=True)


def distinct_ips(rng: np.random.Generator, n: int, exclude: Optional[np.ndarray] = None) -> np.ndarray:
    """n distinct uniform IPv4 addresses, none in ``exclude``, in random order."""
    out = np.empty(0, dtype=np.uint32)
    excl = None if exclude is None else np.unique(exclude.astype(np.uint32))
    while out.size < n:
        draw = random_u32(rng, int((n - out.size) * 1.02) + 16)
        out = np.unique(np.concatenate([out, draw]))
        if excl is not None and excl.size:
            out = out[~np.isin(out, excl, assume_unique=True)]
    return rng.permutation(out)[:n]


def zipf_counts(rng: np.random.Generator, s: float, cap: int, n: int) -> np.ndarray:
    """n i.i.d. draws from P(c) proportional to c^-s on [1, cap]."""
    c = np.arange(1, cap + 1, dtype=np.float64)
    cdf = np.cumsum(c ** -s)
    cdf /= cdf[-1]
    return (np.searchsorted(cdf, rng.random(n), side="right") + 1).astype(np.int64)


def zipf_mean(s: float, cap: int) -> float:
    c = np.arange(1, cap + 1, dtype=np.float64)
    p = c ** -s
    return float((c * p).sum() / p.sum())


@dataclass
class Window:
    """One window of one or more routers plus its ground truth."""
    pairs: List[np.ndarray]                 # per router: uint32[n, 2] (hip, oip)
    planted_ips: np.ndarray                 # uint32
    planted_card: np.ndarray                # int64: true distinct peers over all routers
    background_max: int                     # largest background distinct-peer count (upper bound)

    @property
    def all_pairs(self) -> np.ndarray:
        return self.pairs[0] if len(self.pairs) == 1 else np.concatenate(self.pairs)


def _planted_pairs(rng, ips: np.ndarray, cards: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    src = np.repeat(ips, cards).astype(np.uint32)
    dst = np.concatenate([distinct_ips(rng, int(c)) for c in cards]) if len(cards) else np.empty(0, np.uint32)
    return src, dst


def subset(rng: np.random.Generator, n: int, k: int) -> np.ndarray:
    """A uniformly random k-subset of range(n), ascending.  Bernoulli(k/n) selection, then
    uniformly random removals or additions to reach exactly k (each step keeps the subset
    uniform given its size)."""
    assert 0 <= k <= n
    if k == n:
        return np.arange(n, dtype=np.int64)
    keep = rng.random(n) < (k / n)
    m = int(keep.sum())
    if m > k:
        on = np.flatnonzero(keep)
        keep[on[rng.permutation(on.size)[: m - k]]] = False
    elif m < k:
        off = np.flatnonzero(~keep)
        keep[off[rng.permutation(off.size)[: k - m]]] = True
    return np.flatnonzero(keep)


def _finish(rng, src: np.ndarray, dst: np.ndarray, n_packets: int) -> np.ndarray:
    """Add uniform duplicates of the distinct pairs up to n_packets, then shuffle."""
    d = src.size
    assert d <= n_packets, (d, n_packets)
    packed = np.empty(n_packets, dtype=np.uint64)   # little endian: low word = hip, high = oip
    packed[:d] = src.astype(np.uint64) | (dst.astype(np.uint64) << np.uint64(32))
    if n_packets > d:
        packed[d:] = packed[rng.integers(0, d, size=n_packets - d)]
    packed = packed[rng.permutation(n_packets)]
    return packed.view(np.uint32).reshape(n_packets, 2)


def gen_plain(w: Workload, seed: Optional[int] = None) -> Window:
    """One router, one window: background Zipf sources thinned to the distinct-pair budget,
    planted hosts with distinct peers, uniform duplicates, random order."""
    seed = w.seed if seed is None else seed
    rng = rng_for(seed, 0)
    planted = distinct_ips(rng, w.n_planted)
    bg = distinct_ips(rng, w.n_sources, exclude=planted)
    counts = zipf_counts(rng, w.zipf_s, w.zipf_cap, w.n_sources)
    cards = rng.integers(w.planted_lo, w.planted_hi, size=w.n_planted, endpoint=True)
    n_distinct = w.n_packets - int(round(w.dup_frac * w.n_packets))
    p_src, p_dst = _planted_pairs(rng, planted, cards)
    need_bg = n_distinct - p_src.size
    assert need_bg > 0, "planted pairs exceed the distinct-pair budget"
    slots = np.repeat(np.arange(w.n_sources, dtype=np.int32), counts)
    if need_bg < slots.size:
        slots = slots[subset(rng, slots.size, need_bg)]
    src = np.concatenate([p_src, bg[slots]])
    dst = np.concatenate([p_dst, random_u32(rng, slots.size)])
    pairs = _finish(rng, src, dst, w.n_packets)
    kept = np.bincount(slots, minlength=w.n_sources)
    return Window([pairs], planted, cards.astype(np.int64), int(kept.max()) if kept.size else 0)


def gen_routers(w: Workload, seed: Optional[int] = None) -> Window:
    """Several routers of one window.  A fraction of the sources is seen at 2..R routers; each
    pair of such a source goes to one router of its set.  Planted hosts split their peers over
    2..R routers.  Every router carries exactly ``n_packets`` pairs."""
    seed = w.seed if seed is None else seed
    R = w.n_routers
    rng = rng_for(seed, 0)
    planted = distinct_ips(rng, w.n_planted)
    bg = distinct_ips(rng, w.n_sources, exclude=planted)
    counts = zipf_counts(rng, w.zipf_s, w.zipf_cap, w.n_sources)
    cards = rng.integers(w.planted_lo, w.planted_hi, size=w.n_planted, endpoint=True)
    # router sets: a random permutation of the routers truncated to the set size
    multi = rng.random(w.n_sources) < w.multi_router_frac
    set_size = np.where(multi, rng.integers(2, R, size=w.n_sources, endpoint=True), 1)
    perm = np.argsort(rng.random((w.n_sources, R)), axis=1).astype(np.int8)
    slots = np.repeat(np.arange(w.n_sources, dtype=np.int32), counts)
    pick = (rng.random(slots.size) * set_size[slots]).astype(np.int64)
    slot_router = perm[slots, pick]
    del pick
    # planted: peers split over 2..R routers
    p_src, p_dst = _planted_pairs(rng, planted, cards)
    p_size = rng.integers(2, R, size=w.n_planted, endpoint=True)
    p_perm = np.argsort(rng.random((w.n_planted, R)), axis=1).astype(np.int8)
    p_owner = np.repeat(np.arange(w.n_planted), cards)
    p_router = p_perm[p_owner, (rng.random(p_owner.size) * p_size[p_owner]).astype(np.int64)]
    n_distinct = w.n_packets - int(round(w.dup_frac * w.n_packets))
    # the background slots of each router, ascending (a stable sort groups them by router)
    by_router = np.argsort(slot_router, kind="stable")
    bounds = np.searchsorted(slot_router[by_router], np.arange(R + 1))

    def one_router(r):
        rr = rng_for(seed, 1, r)
        ps, pd = p_src[p_router == r], p_dst[p_router == r]
        mine = by_router[bounds[r]:bounds[r + 1]]
        need = n_distinct - ps.size
        assert 0 < need <= mine.size, (need, mine.size)
        mine = mine[subset(rr, mine.size, need)]
        s_idx = slots[mine]
        src = np.concatenate([ps, bg[s_idx]])
        dst = np.concatenate([pd, random_u32(rr, s_idx.size)])
        return _finish(rr, src, dst, w.n_packets), np.bincount(s_idx, minlength=w.n_sources)

    # every router draws from its own generator, so the threads give the same output in any order
    from concurrent.futures import ThreadPoolExecutor
    with ThreadPoolExecutor(max_workers=min(R, 8)) as ex:
        done = list(ex.map(one_router, range(R)))
    out = [d[0] for d in done]
    kept_all = np.sum([d[1] for d in done], axis=0)
    return Window(out, planted, cards.astype(np.int64), int(kept_all.max()))


# ----------------------------------------------------------------------------------------------
# Sliding-window traffic: a fixed population of sources, each with a universe of peers; every
# slice draws packets (source proportional to its universe size, peer uniform in the universe).
# Planted hosts are active on [on, off) slices and contact fresh peers in every active slice.
# ----------------------------------------------------------------------------------------------
def _peer_ip(src_ips: np.ndarray, j: np.ndarray, salt: int) -> np.ndarray:
    """Deterministic peer address number j of a source (SplitMix64 finaliser of a 64-bit key)."""
    z = (src_ips.astype(np.uint64) << np.uint64(32)) | j.astype(np.uint64)
    z = z ^ np.uint64(salt & MASK64)
    with np.errstate(over="ignore"):
        z = z + np.uint64(GOLDEN64)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return (z & np.uint64(0xFFFFFFFF)).astype(np.uint32)


@dataclass
class SlidingTraffic:
    w: Workload
    seed: int
    src_ips: np.ndarray
    counts: np.ndarray
    cdf: np.ndarray
    planted_ips: np.ndarray
    on: np.ndarray
    off: np.ndarray
    rate: np.ndarray      # fresh peers per active slice

    def slice(self, t: int) -> np.ndarray:
        w = self.w
        rng = rng_for(self.seed, 2, t)
        active = np.nonzero((self.on <= t) & (t < self.off))[0]
        n_pl = int(self.rate[active].sum())
        n_bg = w.n_packets - n_pl
        # sorted draws make the search sequential; the final permutation shuffles the pairs anyway
        s = np.searchsorted(self.cdf, np.sort(rng.random(n_bg)), side="right")
        j = (rng.random(n_bg) * self.counts[s]).astype(np.int64)
        bsrc = self.src_ips[s]
        bdst = _peer_ip(bsrc, j, self.seed)
        psrc = np.repeat(self.planted_ips[active], self.rate[active])
        owner = np.repeat(np.arange(active.size), self.rate[active])
        first = np.concatenate([[0], np.cumsum(self.rate[active])[:-1]]) if active.size else np.zeros(0, np.int64)
        jj = np.arange(n_pl) - np.repeat(first, self.rate[active])
        pdst = _peer_ip(psrc, t * 256 + jj, self.seed ^ 0x5A5A5A5A)
        pairs = np.empty((w.n_packets, 2), dtype=np.uint32)
        pairs[:n_bg, 0], pairs[:n_bg, 1] = bsrc, bdst
        pairs[n_bg:, 0], pairs[n_bg:, 1] = psrc, pdst
        del owner
        return pairs[rng.permutation(w.n_packets)]

    def planted_card(self, t_end: int, K: int) -> np.ndarray:
        """True distinct peers of every planted host over slices [t_end-K+1, t_end]."""
        lo = max(0, t_end - K + 1)
        span = np.clip(np.minimum(self.off, t_end + 1) - np.maximum(self.on, lo), 0, None)
        return span * self.rate


def gen_sliding(w: Workload, seed: Optional[int] = None) -> SlidingTraffic:
    seed = w.seed if seed is None else seed
    rng = rng_for(seed, 0)
    planted = distinct_ips(rng, w.n_planted)
    src = distinct_ips(rng, w.n_sources, exclude=planted)
    counts = zipf_counts(rng, w.zipf_s, w.zipf_cap, w.n_sources)
    cdf = np.cumsum(counts.astype(np.float64))
    cdf /= cdf[-1]
    a = rng.integers(0, w.n_slices, size=w.n_planted)
    b = rng.integers(0, w.n_slices, size=w.n_planted)
    on, off = np.minimum(a, b), np.maximum(a, b) + 1
    rate = rng.integers(w.planted_lo, w.planted_hi, size=w.n_planted, endpoint=True)
    assert w.planted_hi < 256
    return SlidingTraffic(w, seed, src, counts, cdf, planted, on, off, rate)


# ----------------------------------------------------------------------------------------------
# Ground truth helpers (exact distinct counting, Definition 1)
# ----------------------------------------------------------------------------------------------
def distinct_peer_counts(pairs: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Exact |OP(h)| for every host h seen: returns (hosts, counts), hosts ascending."""
    key = (pairs[:, 0].astype(np.uint64) << np.uint64(32)) | pairs[:, 1].astype(np.uint64)
    key = np.unique(key)
    hosts, cnt = np.unique((key >> np.uint64(32)).astype(np.uint32), return_counts=True)
    return hosts, cnt


def split_batches(n: int, rng: np.random.Generator, lo: int, hi: int) -> np.ndarray:
    """Cut [0, n) into consecutive batches of log-uniform size in [lo, hi]; returns boundaries."""
    cuts = [0]
    while cuts[-1] < n:
        size = int(np.exp(rng.uniform(np.log(lo), np.log(hi))))
        cuts.append(min(n, cuts[-1] + max(1, size)))
    return np.asarray(cuts, dtype=np.int64)
