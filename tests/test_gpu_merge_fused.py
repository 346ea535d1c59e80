"""GPU parity of the fused scan + router merge (spd_scan_batches_merge), bit-exact against the oracle.

The global sketch must equal the oracle's OR of the routers named by the call (Section 4.2), every
router's own sketch the oracle's sketch of its pairs, and the global report the oracle's detection
on the union: with the merge done by the apply phase (region layout, one launch, every named router
fed), with words forced through the spill list (which then ORs them into the global too), and on
the fallback paths (direct and exact-count layouts, a named router without pairs in the call whose
earlier pairs must count, several launches, a sliding window).
"""
import numpy as np
import pytest

import synth_traffic as st
from gpu_util import assert_same_report, assert_same_sketch, heavy_hosts, log, oracle_sketch, set_tuning, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402

MP = st.MethodParams(theta=256, r=10, sr=4, a=2, log2k=10, lr=2, log2lc=12, hash_seed=97)
TUNES = {
    "regions_fused": dict(direct_max_pairs=0, bin_mode=2),
    "regions_spill": dict(direct_max_pairs=0, bin_mode=2, region_words=3),
    "regions_small_buckets": dict(direct_max_pairs=0, bin_mode=2, bucket_bits=14, tile_pairs=2048, bin_block=512),
    "regions_apply512": dict(direct_max_pairs=0, bin_mode=2, apply_block=512),
    "regions_launches": dict(direct_max_pairs=0, bin_mode=2, launch_pairs=60_000),
    "exact_count": dict(direct_max_pairs=0, bin_mode=1),
    "direct": dict(direct_max_pairs=1 << 62),
}


def router_traffic(seed, R=4):
    rng = np.random.default_rng(seed)
    shared, _ = heavy_hosts(rng, 6, 700, noise=0)
    out = []
    for r in range(R):
        own, _ = heavy_hosts(rng, 3, 500, noise=40_000 + 7_001 * r)
        part = shared[r::R]
        out.append(np.concatenate([own, part])[rng.permutation(len(own) + len(part))])
    return out


@pytest.mark.parametrize("tune", list(TUNES))
def test_fused_merge_matches_oracle(tune):
    R = 4
    traffic = router_traffic(101 + list(TUNES).index(tune), R)
    det = spd.Detector(spd.params_from(MP), n_routers=R)
    set_tuning(det, **TUNES[tune])
    try:
        log(f"case fused scan + merge, {tune}")
        det.profile_enable(True)
        det.scan_batches([(r, to_dev(traffic[r])) for r in range(R)], merge=True)
        merges = det.profile().get("merge", (0, 0.0))[0]
        det.profile_enable(False)
        # the merge is fused into the apply phase exactly when one region launch with 1024-lane
        # workgroups covers the call; otherwise a merge kernel runs
        fused = tune in ("regions_fused", "regions_spill", "regions_small_buckets")
        assert (merges == 0) == fused, (tune, merges)
        union = oracle_sketch(MP, np.concatenate(traffic))
        assert_same_sketch(det, spd.GLOBAL, union, f"{tune} global")
        for r in range(R):
            assert_same_sketch(det, r, oracle_sketch(MP, traffic[r]), f"{tune} router {r}")
        assert_same_report(det.close_window(spd.GLOBAL), union.detect(), f"{tune} global report")
        # more pairs into the same routers (they were not closed: their sketches accumulate), merged
        # again into the global sketch, which its close has reset
        more = router_traffic(202 + list(TUNES).index(tune), R)
        det.scan_batches([(r, to_dev(more[r])) for r in range(R)], merge=True)
        union2 = oracle_sketch(MP, np.concatenate(traffic + more))
        assert_same_sketch(det, spd.GLOBAL, union2, f"{tune} global, accumulated")
        assert_same_report(det.close_window(spd.GLOBAL), union2.detect(), f"{tune} accumulated report")
    finally:
        det.close()


def test_named_router_without_pairs_still_counts():
    """Router 2 is named with an empty batch: its earlier pairs must be in the global (the merge
    falls back to an ordinary spd_merge)."""
    R = 3
    traffic = router_traffic(303, R)
    det = spd.Detector(spd.params_from(MP), n_routers=R)
    set_tuning(det, direct_max_pairs=0, bin_mode=2)
    try:
        log("case named router without pairs")
        det.scan(2, to_dev(traffic[2]))
        empty = to_dev(np.zeros((0, 2), np.uint32))
        det.scan_batches([(0, to_dev(traffic[0])), (1, to_dev(traffic[1])), (2, empty)], merge=True)
        union = oracle_sketch(MP, np.concatenate(traffic))
        assert_same_sketch(det, spd.GLOBAL, union, "global")
        # an unnamed router is not part of the global
        det.scan_batches([(0, to_dev(traffic[0]))], merge=True)
        assert_same_sketch(det, spd.GLOBAL, oracle_sketch(MP, traffic[0]), "global of router 0 only")
    finally:
        det.close()


def test_sliding_merge_falls_back():
    K = 3
    sp = st.MethodParams(theta=256, r=10, sr=4, a=2, log2k=10, lr=2, log2lc=12, window_slices=K, hash_seed=97)
    slices = [router_traffic(400 + t, 2) for t in range(5)]
    det = spd.Detector(spd.params_from(sp), n_routers=2)
    try:
        log("case sliding fused-merge call")
        for t, tr in enumerate(slices):
            if t:
                det.slide()
            det.scan_batches([(r, to_dev(tr[r])) for r in range(2)], merge=True)
            live = [p for s in slices[max(0, t - K + 1): t + 1] for p in s]
            union = oracle_sketch(sp, np.concatenate(live))
            assert_same_sketch(det, spd.GLOBAL, union, f"slice {t}")
            assert_same_report(det.close_window(spd.GLOBAL), union.detect(), f"slice {t}")
    finally:
        det.close()
