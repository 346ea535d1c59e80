"""GPU parity of binning tiles with more sampled pairs than they stage, bit-exact against the oracle.

The traffic holds a run of pairs whose destinations are all sampled (tau = 1, Section 3.1), so
every tile inside it overflows its staging room.  In the region layout such a tile stages none of
its sampled pairs: it is listed, and the spill pass re-reads its pairs and records their SEAV bits
once the apply phase has written the buckets.  The apply phase writes every bucket of a fresh slot
from zero, and no clear follows a close, so a slot's memory still holds the previous window when
the next one is scanned: windows in a row (with both kinds of close) must not leak into each
other.  Also: the router merge fused into the apply phase (listed tiles reach the global sketch
too), more batches than travel in the kernel arguments (the spill pass reads the batch list in
device memory), destination-keyed batches, and the entry point that allocates nothing.
"""
import ctypes

import numpy as np
import pytest

import synth_traffic as st
from gpu_util import (assert_same_report, assert_same_sketch, heavy_hosts, log, oracle_sketch, overflow_traffic,
                      set_tuning, to_dev)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402

# tau = 1: half of all pairs are sampled into a 128 KiB SEAV, so the inputs stay small (a dense SEAV
# makes the candidate product of Section 3.2, and the oracle's time, explode)
MP = st.CONFIGS["plain_1m"].params.replace(theta=16)
TUNES = {
    "region": dict(direct_max_pairs=0, bin_mode=2),
    "region_small": dict(direct_max_pairs=0, bin_mode=2, tile_pairs=2048, bucket_bits=12, bin_block=512,
                         apply_block=256, apply_unroll=8),
    "region_spill": dict(direct_max_pairs=0, bin_mode=2, region_words=5, apply_unroll=8),
}


def detector(n_routers=1, **tune):
    det = spd.Detector(spd.params_from(MP), n_routers=n_routers)
    set_tuning(det, **tune)
    return det


@pytest.mark.parametrize("tune", list(TUNES))
def test_windows_in_a_row(tune):
    """A plain window, an overflowing one (its report collected after the next scan is enqueued),
    then a plain one again, on one detector: each sketch and report equals the oracle's."""
    rng = np.random.default_rng(11 + list(TUNES).index(tune))
    a, _ = heavy_hosts(rng, 6, 1500, noise=20_000)
    b, _ = overflow_traffic(MP, rng, 10, 2200, noise=8_000)
    c, _ = heavy_hosts(rng, 5, 1700, noise=20_000)
    det = detector(**TUNES[tune])
    try:
        log(f"case windows in a row, {tune}")
        det.scan(0, to_dev(a))
        ref = oracle_sketch(MP, a)
        assert_same_sketch(det, 0, ref, "window a")
        assert_same_report(det.close_window(0), ref.detect(), "window a report")
        det.scan(0, to_dev(b))
        ref_b = oracle_sketch(MP, b)
        assert_same_sketch(det, 0, ref_b, "window b (overflowing tiles)")
        ticket = det.close_begin(0)
        det.scan(0, to_dev(c))
        got_b = det.close_end(ticket)
        assert_same_report(got_b, ref_b.detect(), "window b report")
        assert len(got_b) >= 10
        ref = oracle_sketch(MP, c)
        assert_same_sketch(det, 0, ref, "window c")
        assert_same_report(det.close_window(0), ref.detect(), "window c report")
    finally:
        det.close()


def test_fused_merge_with_listed_tiles():
    """Every router overflows; the merge fused into the apply phase: the global sketch is the OR of
    the routers', listed tiles included; then a second round of windows after the closes."""
    R = 3
    rng = np.random.default_rng(23)
    det = detector(n_routers=R, **TUNES["region"])
    try:
        for rnd in range(2):
            traffic = [overflow_traffic(MP, rng, 4, 2100, noise=4_000 + 1_001 * r)[0] for r in range(R)]
            log(f"case fused merge with listed tiles, round {rnd}")
            det.profile_enable(True)
            det.scan_batches([(r, to_dev(traffic[r])) for r in range(R)], merge=True)
            merges = det.profile().get("merge", (0, 0.0))[0]
            det.profile_enable(False)
            assert merges == 0, "the merge was not fused into the apply phase"
            union = oracle_sketch(MP, np.concatenate(traffic))
            assert_same_sketch(det, spd.GLOBAL, union, "global")
            for r in range(R):
                ref = oracle_sketch(MP, traffic[r])
                assert_same_sketch(det, r, ref, f"router {r}")
                assert_same_report(det.close_window(r), ref.detect(), f"router {r} report")
            assert_same_report(det.close_window(spd.GLOBAL), union.detect(), "global report")
    finally:
        det.close()


def test_batches_in_device_memory():
    """Twelve batches of two routers in one call (more than the kernel arguments carry), most of
    them overflowing."""
    rng = np.random.default_rng(31)
    pairs, _ = overflow_traffic(MP, rng, 12, 2400, noise=8_000)
    cuts = np.sort(rng.choice(np.arange(1, len(pairs)), size=11, replace=False))
    parts = np.split(pairs, cuts)
    owner = [i % 2 for i in range(len(parts))]
    det = detector(n_routers=2, **TUNES["region_small"])
    try:
        log("case 12 batches with listed tiles")
        x = to_dev(pairs)
        starts = np.concatenate([[0], cuts])
        det.scan_batches([(o, x[s:s + len(p)]) for o, s, p in zip(owner, starts, parts)])
        for r in range(2):
            ref = oracle_sketch(MP, np.concatenate([p for o, p in zip(owner, parts) if o == r]))
            assert_same_sketch(det, r, ref, f"router {r}")
            assert_same_report(det.close_window(r), ref.detect(), f"router {r} report")
    finally:
        det.close()


def test_destination_keyed():
    """Records read as (oip, hip): the sampled destinations are in the first column."""
    rng = np.random.default_rng(37)
    pairs, _ = overflow_traffic(MP, rng, 8, 2300, noise=8_000)
    swapped = np.ascontiguousarray(pairs[:, ::-1])
    det = detector(**TUNES["region"])
    try:
        log("case destination-keyed batch with listed tiles")
        det.scan_batches([(0, to_dev(swapped), spd.BATCH_DST)])
        ref = oracle_sketch(MP, pairs)
        assert_same_sketch(det, 0, ref, "destination-keyed")
        assert_same_report(det.close_window(0), ref.detect(), "destination-keyed report")
    finally:
        det.close()


def test_noalloc_entry_point():
    """spd_scan_noalloc (its scratch in the library's fixed array, the tile list included) over a
    plain window, then an overflowing one."""
    rng = np.random.default_rng(41)
    det = detector(**TUNES["region"])
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    try:
        for k, pairs in enumerate((heavy_hosts(rng, 6, 1500, noise=20_000)[0],
                                   overflow_traffic(MP, rng, 10, 2200, noise=8_000)[0])):
            log(f"case spd_scan_noalloc window {k}")
            x = to_dev(pairs)
            st_ = spd.lib().spd_scan_noalloc(det.ctx, 0, ctypes.c_void_p(x.data_ptr()), x.shape[0], 0, stream)
            assert st_ == spd.SPD_OK, spd.lib().spd_last_error(det.ctx)
            ref = oracle_sketch(MP, pairs)
            assert_same_sketch(det, 0, ref, f"window {k}")
            assert_same_report(det.close_window(0), ref.detect(), f"window {k} report")
    finally:
        det.close()
