"""GPU parity on the edges of the method and of the context state, bit-exact against the oracle.

* A saturated ULDC (z0 = 0, Eq. 4 read at z0 = 1, flag bit 0) produced by a host with far more
  distinct peers than its LDC has bits.
* The sliding window past the point where the 16-bit time stamps are renormalised (more than
  65533 slices): the bit view and the report must equal the oracle's discrete detection on the
  union of the last K slices (the plain definition of the sliding window, Section 5).
* A scan refused by the HBM budget leaves the window as it was: retried in smaller batches it
  gives the oracle's sketch of those pairs alone.
* The window after a close starts from zero, for every scan layout, on the close's stream and on
  another stream, and for the merged sketch.
"""
import numpy as np
import pytest

import oracle
import synth_traffic as st
from gpu_util import assert_same_report, assert_same_sketch, heavy_hosts, log, oracle_sketch, set_tuning, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402

LAYOUTS = {
    "direct": dict(direct_max_pairs=1 << 62),
    "tiles": dict(direct_max_pairs=0, bin_mode=0),
    "exact_count": dict(direct_max_pairs=0, bin_mode=1),
    "regions": dict(direct_max_pairs=0, bin_mode=2),
}


def detector(mp, n_routers=1, budget=0, **tune):
    det = spd.Detector(spd.params_from(mp), n_routers=n_routers, hbm_budget_bytes=budget)
    if tune:
        set_tuning(det, **tune)
    return det


@pytest.mark.parametrize("layout", list(LAYOUTS))
def test_saturated_uldc(layout):
    """k = 32 bits per LDC and hosts with 3000 distinct peers: every bit of their LDCs is set, so
    z0 = 0; the record carries est(1) and the saturated flag (reading of Eq. 4 at ln 0)."""
    mp = st.MethodParams(theta=64, r=8, sr=4, a=2, log2k=5, lr=2, log2lc=6, hash_seed=29)
    rng = np.random.default_rng(3 + len(layout))
    pairs, hosts = heavy_hosts(rng, 3, 3000, noise=20_000)
    log(f"case saturated ULDC layout={layout}")
    ref = oracle_sketch(mp, pairs)
    want = ref.detect()
    sat = want[want["z0"] == 0]
    assert set(hosts.tolist()) <= set(sat["ip"].tolist())
    assert (sat["flags"] == 1).all() and (sat["est"] == oracle.est(mp.log2k, 1)).all()
    det = detector(mp, **LAYOUTS[layout])
    try:
        det.scan(0, to_dev(pairs))
        assert_same_sketch(det, 0, ref, f"saturated {layout}")
        got = det.close_window(0)
        assert_same_report(got, want, f"saturated {layout}")
    finally:
        det.close()


def test_sliding_stamps_renormalised():
    """Slides up to slice 65540 (empty slices cost the host only); the slices around the point where
    the library shifts every stamp down hold traffic.  Two routers; after every slice both routers'
    windows and their merge equal the oracle on the union of the last K slices."""
    K = 3
    mp = st.MethodParams(theta=256, r=10, sr=4, a=2, log2k=10, lr=2, log2lc=8, window_slices=K, sliding_counter=1,
                         hash_seed=59)
    rng = np.random.default_rng(61)
    det = detector(mp, n_routers=2)
    try:
        first, _ = heavy_hosts(rng, 2, 600, noise=5000)
        det.scan(0, to_dev(first))              # slice 0: long expired at the end
        torch.cuda.synchronize()
        t_start = 65529
        for _ in range(t_start):
            det.slide()
        assert spd.spd_current_slice(det.ctx) == t_start
        log("case sliding renormalisation: slices 65530..65540")
        slices = {}
        for t in range(t_start + 1, 65541):
            det.slide()
            pairs, _ = heavy_hosts(rng, 3, int(rng.integers(150, 400)), noise=8000 + t % 7)
            owner = rng.integers(0, 2, size=len(pairs))
            det.scan_batches([(r, to_dev(pairs[owner == r])) for r in range(2)])
            slices[t] = (pairs, owner)
            live = [slices[j] for j in range(t - K + 1, t + 1) if j in slices]
            for r in range(2):
                union = oracle_sketch(mp, np.concatenate([p[o == r] for p, o in live]))
                assert_same_sketch(det, r, union, f"router {r} slice {t}")
                assert_same_report(det.close_window(r), union.detect(), f"router {r} slice {t}")
            det.merge([0, 1])
            union = oracle_sketch(mp, np.concatenate([p for p, _ in live]))
            assert_same_sketch(det, spd.GLOBAL, union, f"merged slice {t}")
            assert_same_report(det.close_window(spd.GLOBAL), union.detect(), f"merged slice {t}")
        # the stamps were shifted: the slice counter restarted near K
        assert spd.spd_current_slice(det.ctx) < 64
    finally:
        det.close()


@pytest.mark.parametrize("K", [5, 60, 254])
def test_at_pool_across_code_periods(K):
    """The AT pool stores slice codes modulo 256 and re-stamps the expired counters of one of
    255 - K groups of the pool per slice (K = 254: the whole pool every slice).  Traffic in slices
    spread over four code periods, including slices whose code repeats that of earlier traffic;
    after every slice with traffic, and after runs of empty slices while that traffic expires, the
    bit view and the report of two routers and of their merge must equal the oracle on the union of
    the last K slices."""
    mp = st.MethodParams(theta=256, r=10, sr=4, a=2, log2k=10, lr=2, log2lc=8, window_slices=K, hash_seed=63)
    rng = np.random.default_rng(65 + K)
    busy = {0, 1, 2, 3, 200, 254, 255, 256, 257, 258, 511, 512, 513, 700, 767, 768, 769, 1023, 1024}
    check = busy | {t + d for t in busy for d in (K - 1, K, K + 1)} | {510, 766, 1022}
    det = detector(mp, n_routers=2)
    slices = {}
    try:
        log(f"case AT pool across code periods, K={K}")
        for t in range(max(check) + 1):
            if t:
                det.slide()
            if t in busy:
                pairs, _ = heavy_hosts(rng, 3, int(rng.integers(200, 500)), noise=6000)
                owner = rng.integers(0, 2, size=len(pairs))
                det.scan_batches([(r, to_dev(pairs[owner == r])) for r in range(2)])
                slices[t] = (pairs, owner)
            if t not in check:
                continue
            live = [slices[j] for j in range(t - K + 1, t + 1) if j in slices]
            for r in range(2):
                parts = [p[o == r] for p, o in live] or [np.zeros((0, 2), np.uint32)]
                union = oracle_sketch(mp, np.concatenate(parts))
                assert_same_sketch(det, r, union, f"router {r} slice {t}")
                assert_same_report(det.close_window(r), union.detect(), f"router {r} slice {t}")
            det.merge([0, 1])
            union = oracle_sketch(mp, np.concatenate([p for p, _ in live] or [np.zeros((0, 2), np.uint32)]))
            assert_same_sketch(det, spd.GLOBAL, union, f"merged slice {t}")
            assert_same_report(det.close_window(spd.GLOBAL), union.detect(), f"merged slice {t}")
        assert spd.spd_current_slice(det.ctx) == max(check)
    finally:
        det.close()


def test_budget_refusal_leaves_window_unchanged():
    """Window A is scanned and closed (the slot keeps A's LDCA words until its next scan rewrites
    them); a large scan of window B is refused by the HBM budget; B retried in small batches (direct
    and binned) must equal the oracle's sketch of B alone."""
    mp = st.CONFIGS["plain_1m"].params
    probe = detector(mp)
    held = probe.stats.device_bytes
    probe.close()
    rng = np.random.default_rng(71)
    a_pairs, _ = heavy_hosts(rng, 5, 2500, noise=150_000)
    b_pairs, _ = heavy_hosts(rng, 5, 2500, noise=2_000_000)
    for small in ("direct", "regions"):
        log(f"case budget refusal, retry {small}")
        det = detector(mp, budget=held + (8 << 20))
        try:
            det.scan(0, to_dev(a_pairs))
            det.close_window(0)
            xb = to_dev(b_pairs)
            with pytest.raises(spd.SpdError) as e:
                set_tuning(det, direct_max_pairs=0)
                det.scan(0, xb)
            assert e.value.status == spd.SPD_E_NOMEM
            set_tuning(det, **LAYOUTS[small])
            for a in range(0, len(b_pairs), 150_000):
                det.scan(0, xb[a:a + 150_000])
            ref = oracle_sketch(mp, b_pairs)
            assert_same_sketch(det, 0, ref, f"after refusal ({small})")
            assert_same_report(det.close_window(0), ref.detect(), f"after refusal ({small})")
        finally:
            det.close()


@pytest.mark.parametrize("layout", list(LAYOUTS))
@pytest.mark.parametrize("other_stream", [False, True])
def test_window_after_close_starts_from_zero(layout, other_stream):
    """Scan A, close, scan B into the same slot: B's sketch and report equal the oracle's on B
    alone, whether the next scan runs on the close's stream or on another one.  The same for the
    merged sketch: merge, close, reset the routers, scan, merge again."""
    mp = st.CONFIGS["plain_1m"].params
    rng = np.random.default_rng(81 + 2 * len(layout) + int(other_stream))
    a_pairs, _ = heavy_hosts(rng, 6, 2500, noise=300_000)
    b_pairs, _ = heavy_hosts(rng, 6, 2500, noise=300_000)
    log(f"case next window after close layout={layout} other_stream={other_stream}")
    det = detector(mp, n_routers=2, **LAYOUTS[layout])
    s1 = torch.cuda.Stream() if other_stream else None
    try:
        xa, xb = to_dev(a_pairs), to_dev(b_pairs)
        torch.cuda.synchronize()
        det.scan(0, xa)
        assert_same_report(det.close_window(0), oracle_sketch(mp, a_pairs).detect(), "window A")
        det.scan(0, xb, stream=s1)
        ref = oracle_sketch(mp, b_pairs)
        assert_same_sketch(det, 0, ref, "window B")
        assert_same_report(det.close_window(0, stream=s1), ref.detect(), "window B")
        # merged sketch: A split over two routers, then B
        half = len(a_pairs) // 2
        det.scan_batches([(0, xa[:half]), (1, xa[half:])])
        det.merge([0, 1])
        assert_same_report(det.close_window(spd.GLOBAL), oracle_sketch(mp, a_pairs).detect(), "merged A")
        det.close_window(0)
        det.close_window(1)
        det.scan_batches([(0, xb[:half]), (1, xb[half:])], stream=s1)
        det.merge([0, 1], stream=s1)
        assert_same_sketch(det, spd.GLOBAL, ref, "merged B")
        assert_same_report(det.close_window(spd.GLOBAL, stream=s1), ref.detect(), "merged B")
    finally:
        det.close()
        if s1 is not None:
            s1.synchronize()


def test_reset_starts_a_new_window():
    """spd_reset re-initialises a router's sketch without a report (a watch point's new window): a
    merge then leaves it out and its next scan starts from zero; in sliding mode every stamp is
    cleared."""
    mp = st.CONFIGS["plain_1m"].params
    rng = np.random.default_rng(91)
    a0, _ = heavy_hosts(rng, 4, 2500, noise=120_000)
    a1, _ = heavy_hosts(rng, 4, 2500, noise=120_000)
    b0, _ = heavy_hosts(rng, 4, 2500, noise=120_000)
    for layout in ("direct", "regions"):
        log(f"case reset layout={layout}")
        det = detector(mp, n_routers=2, **LAYOUTS[layout])
        try:
            det.scan(0, to_dev(a0))
            det.scan(1, to_dev(a1))
            det.reset(0)
            det.merge([0, 1])
            ref1 = oracle_sketch(mp, a1)
            assert_same_sketch(det, spd.GLOBAL, ref1, "merge after reset")
            det.scan(0, to_dev(b0))
            assert_same_sketch(det, 0, oracle_sketch(mp, b0), "scan after reset")
            assert_same_report(det.close_window(spd.GLOBAL), ref1.detect(), "global after reset")
        finally:
            det.close()
    K = 3
    ms = mp.replace(window_slices=K)
    det = detector(ms)
    try:
        det.scan(0, to_dev(a0))
        det.slide()
        det.reset(0)
        seav, ldca = det.export(0)
        assert not seav.any() and not ldca.any()
        det.scan(0, to_dev(b0))
        assert_same_sketch(det, 0, oracle_sketch(mp, b0), "sliding scan after reset")
    finally:
        det.close()
