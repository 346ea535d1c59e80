"""Pins of the CPU oracle to facts fixed by the paper and by mathematics, not by the oracle itself.

Each test names what it pins: a closed form worked by hand (golden files), an independent
formulation (bit strings instead of shifts, sets instead of bitmaps), brute force on tiny inputs,
an invariant of the method (order, duplicates, split, OR merge), or a probability derived from
first principles and compared with many random trials.
"""
import math
import os

import numpy as np
import pytest

import oracle
import synth_traffic as st

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if line:
                out.append(line.split())
    return out


def tiny_params(r=20, sr=3, a=1, log2k=10, lr=2, log2lc=6, theta=1024, seed=7):
    return st.MethodParams(theta=theta, r=r, sr=sr, a=a, log2k=log2k, lr=lr, log2lc=log2lc, hash_seed=seed)


def lsb(x):
    return 32 if x == 0 else (x & -x).bit_length() - 1


# ------------------------------------------------------------------------- Eq. 1, Eq. 4
def test_tau_eq1_golden():
    for theta, tau in _rows("eq1_tau.txt"):
        assert oracle.tau(int(theta)) == int(tau), theta


def test_z_theta_eq4_golden():
    for log2k, theta, z in _rows("eq4_threshold.txt"):
        assert oracle.z_theta(int(log2k), int(theta)) == int(z), (log2k, theta)


def test_estimate_eq4_golden():
    for log2k, z0, est in _rows("eq4_estimate.txt"):
        assert oracle.est(int(log2k), int(z0)) == int(est), (log2k, z0)


def test_z_theta_unreachable_threshold():
    # k ln k < theta: no z0 >= 1 can reach theta (k = 32: 32 ln 32 = 110.9)
    assert oracle.z_theta(5, 111) == 0
    assert oracle.z_theta(5, 110) == 1


# ------------------------------------------------------------------- Eq. 2, Eq. 3, layout
def test_layout_worked_example_golden():
    g = {row[0]: row[1:] for row in _rows("eq2_worked_example.txt")}
    r, sr, a = int(g["r"][0]), int(g["sr"][0]), int(g["a"][0])
    isb, ibn = oracle.layout(r, sr, a)
    assert isb == [int(v) for v in g["isb"]]
    assert ibn == [int(v) for v in g["ibn"]]
    host = int(g["host"][0], 16)
    lp, rp = host >> r, host & ((1 << r) - 1)
    assert rp == int(g["rp"][0], 16) and lp == int(g["lp"][0], 16)
    want = [int(v, 16) for v in g["idx"]]
    assert [oracle.idx(lp, isb[i], ibn[i], 32 - r) for i in range(sr)] == want
    p = oracle.params(st.MethodParams(r=r, sr=sr, a=a))
    assert oracle.lp_from_idx(p, want) == lp


def _idx_by_strings(lp, isb, ibn, L):
    """Eq. 2 through bit strings: position j of the string is LP bit j (LSB first)."""
    bits = format(lp, "0%db" % L)[::-1]
    idx_bits = "".join(bits[(isb + j) % L] for j in range(ibn))
    return int(idx_bits[::-1], 2)


@pytest.mark.parametrize("r,sr,a", [(6, 4, 2), (14, 4, 2), (15, 4, 2), (8, 3, 1), (20, 3, 1), (4, 5, 3)])
def test_idx_matches_string_model(r, sr, a):
    isb, ibn = oracle.layout(r, sr, a)
    L = 32 - r
    rng = np.random.default_rng(r * 100 + sr)
    for lp in [0, (1 << L) - 1] + [int(v) for v in rng.integers(0, 1 << L, size=200)]:
        for i in range(sr):
            assert oracle.idx(lp, isb[i], ibn[i], L) == _idx_by_strings(lp, isb[i], ibn[i], L)


def test_eq2_eq3_exhaustive_roundtrip_and_consistency():
    """For L = 12 every LP survives Eq. 2 -> Eq. 3, and the tuples that Eq. 3 accepts are exactly
    the index tuples of some LP (brute force over the whole product of row values)."""
    mp = tiny_params(r=20, sr=3, a=1)
    p = oracle.params(mp)
    isb, ibn = list(p.isb[:3]), list(p.ibn[:3])
    L = 12
    images = {}
    for lp in range(1 << L):
        t = tuple(oracle.idx(lp, isb[i], ibn[i], L) for i in range(3))
        assert oracle.lp_from_idx(p, t) == lp
        images[t] = lp
    assert len(images) == 1 << L
    accepted = 0
    for c0 in range(1 << ibn[0]):
        for c1 in range(1 << ibn[1]):
            for c2 in range(1 << ibn[2]):
                got = oracle.lp_from_idx(p, (c0, c1, c2))
                assert got == images.get((c0, c1, c2))
                accepted += got is not None
    assert accepted == 1 << L


def test_layout_constraints():
    for r in range(2, 24):
        for sr in (2, 3, 4, 5):
            for a in (1, 2, 3):
                isb, ibn = oracle.layout(r, sr, a)
                p = oracle.params(st.MethodParams(r=r, sr=sr, a=a))
                assert oracle.covers_all(p), (r, sr, a)
                L = 32 - r
                span = [{(isb[i] + j) % L for j in range(ibn[i])} for i in range(sr)]
                for i in range(sr):   # consecutive rows, cyclically, share at least one bit
                    assert span[i] & span[(i + 1) % sr], (r, sr, a, i)
    # a layout leaving LP bit 11 uncovered violates constraint 1 and no LP can be rebuilt
    p = oracle.params(st.MethodParams(r=20, sr=2, a=1), isb=[0, 5], ibn=[5, 6])
    assert not oracle.covers_all(p)
    assert oracle.lp_from_idx(p, (0, 0)) is None


# ----------------------------------------------------------------------------- hashes
def test_hash_closed_forms():
    # (2^32 + 1) x + 0 = x 2^32 + x: the top 32 bits are x itself
    for x in (0, 1, 0xDEADBEEF, 0xFFFFFFFF):
        assert oracle.hash32(x, (1 << 32) + 1, 0, 32) == x
    # 3 * 2^31 = 2^32 + 2^31: the carry out of the low word must reach the high word
    assert oracle.hash32(1 << 31, 3, 0, 32) == 1
    # b = 2^64 - 1, a = 1, x = 1: the sum wraps modulo 2^64 to 0
    assert oracle.hash32(1, 1, (1 << 64) - 1, 32) == 0
    # a = 2^63 + 1 (odd), b = 0, x odd: 2^63 x mod 2^64 = 2^63, plus x -> top bit set, top 3 bits 100
    assert oracle.hash32(5, (1 << 63) + 1, 0, 3) == 4
    assert oracle.hash32(5, (1 << 63) + 1, 0, 1) == 1
    # the shift keeps the top m bits: b = 0xABCD << 48, a = 1, x = 0 -> 0xABCD >> (16 - m)
    for m in (1, 4, 12, 16):
        assert oracle.hash32(0, 1, 0xABCD << 48, m) == 0xABCD >> (16 - m)


def test_hash_output_distribution():
    """H2 is uniform on [0, 8) and lsb(H1) is geometric: P(lsb >= t) = 2^-t (Section 3.1)."""
    mul, add = st.hash_params(12345, 2)
    rng = np.random.default_rng(1)
    xs = [int(v) for v in rng.integers(0, 1 << 32, size=40000)]
    h2 = np.bincount([oracle.hash32(x, mul[1], add[1], 3) for x in xs], minlength=8)
    chi2 = float(((h2 - 5000.0) ** 2 / 5000.0).sum())
    assert chi2 < 30.0  # 7 degrees of freedom: P(chi2 > 30) ~ 1e-4
    lsbs = np.array([lsb(oracle.hash32(x, mul[0], add[0], 32)) for x in xs])
    for t in range(1, 8):
        frac = float((lsbs >= t).mean())
        sd = math.sqrt(2.0 ** -t * (1 - 2.0 ** -t) / len(xs))
        assert abs(frac - 2.0 ** -t) < 5 * sd, t


# ----------------------------------------------------------------- scan: brute force
def _lone_host_pairs(host, n, seed):
    peers = st.distinct_ips(np.random.default_rng(seed), n)
    return np.stack([np.full(n, host, np.uint32), peers], axis=1)


@pytest.mark.parametrize("mp", [tiny_params(), st.CONFIGS["plain_1m"].params, tiny_params(r=8, sr=4, a=2, log2k=12, lr=3, log2lc=5)])
def test_scan_lone_host_brute_force(mp):
    """One host alone: its SR cells hold exactly {H2(o) : lsb(H1(o)) >= tau}, everything else in
    the SEAV is 0; its LR LDCs hold exactly {H3(o)}; z0 = k - |{H3(o)}| (Sections 3.1-3.3)."""
    p = oracle.params(mp)
    mul, add = mp.hashes()
    host = 0x9AF2506D
    pairs = _lone_host_pairs(host, 3000, 3)
    sk = oracle.Sketch(p).scan(pairs)
    tau = oracle.tau(mp.theta)
    want_bits = set()
    want_q = set()
    for o in pairs[:, 1].tolist():
        if lsb(oracle.hash32(o, mul[0], add[0], 32)) >= tau:
            want_bits.add(oracle.hash32(o, mul[1], add[1], 3))
        want_q.add(oracle.hash32(o, mul[2], add[2], mp.log2k))
    se = sum(1 << b for b in want_bits)
    # SEAV: cell (RP, row i, Idx(i, LP)) at byte RP * sea_bytes + sum_{q<i} 2^IBN(q) + Idx
    rp, lp, L = host & ((1 << mp.r) - 1), host >> mp.r, 32 - mp.r
    expect = np.zeros_like(sk.seav)
    off = rp * oracle.sea_bytes(p)
    for i in range(mp.sr):
        expect[off + _idx_by_strings(lp, p.isb[i], p.ibn[i], L)] = se
        off += 1 << p.ibn[i]
    np.testing.assert_array_equal(sk.seav, expect)
    # LDCA: row i, column LH_i(host), bit q at word ((i*LC + c) * k + q) / 32
    words = 1 << (mp.log2k - 5)
    expect = np.zeros_like(sk.ldca)
    for i in range(mp.lr):
        c = oracle.hash32(host, mul[3 + i], add[3 + i], mp.log2lc)
        for q in want_q:
            expect[(i * (1 << mp.log2lc) + c) * words + q // 32] |= np.uint32(1 << (q % 32))
    np.testing.assert_array_equal(sk.ldca, expect)
    assert sk.uldc_zeros(host) == (1 << mp.log2k) - len(want_q)


def test_scan_invariants_order_duplicates_split_merge():
    """The sketch is a function of the set of distinct pairs; routers merge by OR in any order
    (no access conflicts, Section 3.4; merge, Section 4.2)."""
    w = st.scaled(st.CONFIGS["plain_1m"], n_packets=200_000, n_sources=10_000, n_planted=4)
    pairs = st.gen_plain(w).pairs[0]
    p = oracle.params(w.params)
    base = oracle.Sketch(p).scan(pairs)
    rng = np.random.default_rng(5)
    perm = oracle.Sketch(p).scan(pairs[rng.permutation(len(pairs))])
    dup = oracle.Sketch(p).scan(np.concatenate([pairs, pairs[rng.integers(0, len(pairs), 50_000)]]))
    uniq = oracle.Sketch(p).scan(np.unique(pairs.view(np.uint64)).view(np.uint32).reshape(-1, 2))
    for s in (perm, dup, uniq):
        np.testing.assert_array_equal(s.seav, base.seav)
        np.testing.assert_array_equal(s.ldca, base.ldca)
    for parts in (2, 5, 16):
        owner = rng.integers(0, parts, size=len(pairs))
        sks = [oracle.Sketch(p).scan(pairs[owner == j]) for j in range(parts)]
        order = rng.permutation(parts)
        merged = oracle.Sketch(p)
        for j in order:
            merged.merge(sks[j])
        np.testing.assert_array_equal(merged.seav, base.seav)
        np.testing.assert_array_equal(merged.ldca, base.ldca)
        merged.merge(sks[order[0]])  # idempotent
        np.testing.assert_array_equal(merged.ldca, base.ldca)
    assert base.seav.any() and base.ldca.any()


# ---------------------------------------------------------- restoring candidates (3.2)
def _random_seav(p, density, seed, rp_lo, rp_hi):
    """Random SE bytes for the SEAs of RP in [rp_lo, rp_hi), zero elsewhere."""
    rng = np.random.default_rng(seed)
    sea = oracle.sea_bytes(p)
    out = np.zeros(oracle.seav_bytes(p), np.uint8)
    bits = rng.random(((rp_hi - rp_lo) * sea, 8)) < density
    out[rp_lo * sea: rp_hi * sea] = np.packbits(bits, axis=1, bitorder="little").reshape(-1)
    return out


@pytest.mark.parametrize("density,seed", [(0.3, 1), (0.45, 2), (0.6, 3)])
def test_candidates_join_equals_definition_tiny(density, seed):
    """The HSE/CIS join finds exactly the hosts whose SR SEs AND to weight >= 3 (brute force over
    every LP of each RP)."""
    mp = tiny_params(r=20, sr=3, a=1)
    p = oracle.params(mp)
    sk = oracle.Sketch(p)
    lo, hi = 4096, 4096 + 96
    sk.seav[:] = _random_seav(p, density, seed, lo, hi)
    join = np.sort(sk.candidates())
    brute = np.sort(sk.candidates_brute(lo, hi))
    np.testing.assert_array_equal(join, brute)
    assert brute.size > 0


def test_candidates_join_equals_definition_real_sketch():
    """Same check on a sketch built from traffic with planted hosts (cfg2-shaped layout)."""
    w = st.scaled(st.CONFIGS["plain_64m"], n_packets=1 << 20, n_sources=20_000, n_planted=12, dup_frac=0.3)
    win = st.gen_plain(w)
    p = oracle.params(w.params)
    sk = oracle.Sketch(p).scan(win.pairs[0])
    join = sk.candidates()
    rmask = (1 << w.params.r) - 1
    rps = sorted(set((join & rmask).tolist()) | {0, 1, 777, rmask})[:24]
    for rp in rps:
        brute = np.sort(sk.candidates_brute(rp, rp + 1))
        np.testing.assert_array_equal(np.sort(join[(join & rmask) == rp]), brute)
    assert set(win.planted_ips.tolist()) <= set(join.tolist())


# ------------------------------------------------------------------- filter (3.3) and report
def test_detect_lone_hosts_and_report_order():
    mp = st.MethodParams(theta=1024, r=6, sr=4, a=2, log2k=12, lr=2, log2lc=12, hash_seed=99)
    p = oracle.params(mp)
    rng = np.random.default_rng(8)
    hosts = st.distinct_ips(rng, 6)
    cards = [300, 900, 1500, 2500, 6000, 60000]
    pairs = np.concatenate([_lone_host_pairs(int(h), c, 10 + i) for i, (h, c) in enumerate(zip(hosts, cards))])
    sk = oracle.Sketch(p).scan(pairs)
    rec = sk.detect()
    assert list(rec["ip"]) == sorted(rec["ip"])
    got = dict(zip(rec["ip"].tolist(), zip(rec["z0"].tolist(), rec["est"].tolist(), rec["flags"].tolist())))
    k = 1 << mp.log2k
    zt = oracle.z_theta(mp.log2k, mp.theta)
    for h, c in zip(hosts.tolist(), cards):
        z0 = sk.uldc_zeros(h)
        passes = z0 <= zt
        if h in got:
            assert passes and got[h][0] == z0 and got[h][1] == oracle.est(mp.log2k, z0)
            assert got[h][2] == (1 if z0 == 0 else 0)
        if c >= 1500:   # SE hot with probability > 0.99 and the estimate far above theta
            assert h in got
        if c <= 900:    # linear counting: E z0 = k e^(-n/k) far above z_theta
            assert h not in got
        if c < 30000:   # linear counting error (Whang et al.): |est - n| < 6 sd
            t = c / k
            sd = math.sqrt(k * (math.exp(t) - t - 1))
            assert abs(-k * math.log(max(z0, 1) / k) - c) < 6 * sd + 2
    assert got[hosts[-1]][2] == 1 and got[hosts[-1]][0] == 0  # 60000 peers saturate k = 4096


def test_detect_plain_1m_finds_planted():
    """Sanity on the 1,000,000-pair window: the 20 planted hosts (2000 peers each) are reported,
    no background host (at most 200 peers) is."""
    w = st.CONFIGS["plain_1m"]
    win = st.gen_plain(w)
    rec = oracle.Sketch(oracle.params(w.params)).scan(win.pairs[0]).detect()
    assert sorted(rec["ip"].tolist()) == sorted(win.planted_ips.tolist())
    assert np.all(np.abs(rec["est"].astype(np.int64) - 2000) < 150)


# ---------------------------------------------------------------- sliding window (Section 5)
def test_sliding_window_is_discrete_sketch_of_slice_union():
    mp = st.MethodParams(theta=64, r=10, sr=4, a=2, log2k=9, lr=2, log2lc=8, window_slices=3, hash_seed=5)
    p = oracle.params(mp)
    K = 3
    rng = np.random.default_rng(3)
    slices = [np.stack([rng.integers(0, 1 << 32, 4000, dtype=np.uint64).astype(np.uint32) % 500,
                        rng.integers(0, 1 << 32, 4000, dtype=np.uint64).astype(np.uint32)], axis=1)
              for _ in range(7)]
    sl = oracle.SlidingSketch(p, K)
    one = oracle.SlidingSketch(p, 1)
    for t, s in enumerate(slices):
        sl.scan_slice(s, t)
        one.scan_slice(s, t)
        union = oracle.Sketch(p).scan(np.concatenate(slices[max(0, t - K + 1): t + 1]))
        view = sl.bit_view(t)
        np.testing.assert_array_equal(view.seav, union.seav)
        np.testing.assert_array_equal(view.ldca, union.ldca)
        # K = 1 is the discrete window (Section 5.1)
        alone = oracle.Sketch(p).scan(s)
        v1 = one.bit_view(t)
        np.testing.assert_array_equal(v1.seav, alone.seav)
        np.testing.assert_array_equal(v1.ldca, alone.ldca)


# ------------------------------------------------------------- statistics (first principles)
def _p_hot(n, tau, g=8, hot=3):
    """P(a lone host's SE has weight >= hot | n distinct peers): sampled peers ~ Bin(n, 2^-tau),
    each sets one of g bits uniformly (occupancy distribution by dynamic programming)."""
    p = 2.0 ** -tau
    xmax = min(n, 200)
    occ = np.zeros(g + 1)
    occ[0] = 1.0
    total = 0.0
    for x in range(0, xmax + 1):
        if x > 0:
            nxt = np.zeros(g + 1)
            for j in range(g + 1):
                nxt[j] += occ[j] * j / g
                if j < g:
                    nxt[j + 1] += occ[j] * (g - j) / g
            occ = nxt
        pmf = math.comb(n, x) * p ** x * (1 - p) ** (n - x)
        total += pmf * occ[hot:].sum()
    return total


def test_lone_host_hot_probability_matches_closed_form():
    mp = st.MethodParams(theta=1024, r=8, sr=8, a=1, log2k=5, lr=1, log2lc=0, hash_seed=31)
    p = oracle.params(mp)
    sk = oracle.Sketch(p)
    rng = np.random.default_rng(17)
    for n, trials in ((200, 1500), (400, 1500), (1024, 600)):
        hot = 0
        for _ in range(trials):
            sk.seav[:] = 0
            host = int(rng.integers(0, 1 << 32))
            peers = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
            sk.scan(np.stack([np.full(n, host, np.uint32), peers], axis=1))
            # a lone host: all its SR cells hold the same SE; its weight is that of their OR
            hot += int(np.unpackbits(np.bitwise_or.reduce(sk.seav)).sum() >= 3)
        q = _p_hot(n, oracle.tau(mp.theta))
        sd = math.sqrt(q * (1 - q) / trials)
        assert abs(hot / trials - q) < 5 * sd + 1e-3, (n, hot / trials, q)
    assert abs(_p_hot(400, 7) - 0.508) < 0.01 and abs(_p_hot(2000, 7) - 0.9998) < 1e-3


def test_lemma1_uldc_noise_density():
    """Lemma 1: a host that never appeared sees ULDC one-density (1 - (1 - 1/k)^(N/LC))^LR."""
    mp = st.MethodParams(theta=1024, r=8, sr=4, a=2, log2k=10, lr=2, log2lc=8, hash_seed=77)
    p = oracle.params(mp)
    rng = np.random.default_rng(23)
    N = 200_000
    pairs = np.stack([rng.integers(0, 1 << 32, N, dtype=np.uint64).astype(np.uint32),
                      rng.integers(0, 1 << 32, N, dtype=np.uint64).astype(np.uint32)], axis=1)
    sk = oracle.Sketch(p).scan(pairs)
    k, LC = 1 << mp.log2k, 1 << mp.log2lc
    seen = set(pairs[:, 0].tolist())
    probes = [h for h in rng.integers(0, 1 << 32, 400).tolist() if h not in seen][:300]
    dens = np.mean([1 - sk.uldc_zeros(h) / k for h in probes])
    psu = (1 - (1 - 1 / k) ** (N / LC)) ** mp.lr
    assert abs(dens - psu) < 0.01, (dens, psu)
