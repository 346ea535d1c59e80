"""GPU parity of the two-part end of window (spd_close_begin / spd_close_end), bit-exact against
the oracle.

* Windows pipelined the way a capture loop runs them: each window's close is begun, the next
  window's pairs are scanned, and only then is the previous report collected.  Every report must
  equal the oracle's detection on that window alone (the reset at the begin of the close is what
  keeps the windows apart), for the direct and the region scan layouts.
* Every pending slot in use at once, collected in reverse order; one more begin is refused; a
  ticket is collected only once.
* The merged sketch, an empty window, and a sliding window (nothing reset there) give the same
  report as the blocking close; sliding reports collected one slice behind (the next slide, its AT
  maintenance and its scan enqueued first) are those of their own windows.
* A window with more super points than a pending close holds: SPD_E_TRUNCATED with their number,
  then room in every pending close.
"""
import numpy as np
import pytest

import synth_traffic as st
from gpu_util import assert_same_report, heavy_hosts, log, oracle_sketch, set_tuning, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402

MP = st.MethodParams(theta=256, r=10, sr=4, a=2, log2k=10, lr=2, log2lc=10, hash_seed=91)


def windows(seed, n, heavy=6, peers=900, noise=120_000):
    rng = np.random.default_rng(seed)
    return [heavy_hosts(rng, heavy, peers, noise=noise)[0] for _ in range(n)]


@pytest.mark.parametrize("layout", ["direct", "regions"])
def test_pipelined_windows_match_oracle(layout):
    tune = dict(direct_max_pairs=1 << 62) if layout == "direct" else dict(direct_max_pairs=0, bin_mode=2)
    ws = windows(301 if layout == "direct" else 302, 6)
    det = spd.Detector(spd.params_from(MP))
    set_tuning(det, **tune)
    try:
        log(f"case pipelined closes, {layout}")
        xs = [to_dev(w) for w in ws]
        tickets, reports = [], []
        for i, x in enumerate(xs):
            det.scan(0, x)
            tickets.append(det.close_begin(0))
            if i:
                reports.append(det.close_end(tickets[i - 1]))
        reports.append(det.close_end(tickets[-1]))
        torch.cuda.synchronize()
        for i, (w, rep) in enumerate(zip(ws, reports)):
            want = oracle_sketch(MP, w).detect()
            assert len(want) > 0
            assert_same_report(rep, want, f"{layout} window {i}")
        assert det.stats.closes == len(ws)
    finally:
        det.close()


def test_all_pending_slots_and_refusals():
    ws = windows(303, spd.MAX_PENDING_CLOSES)
    det = spd.Detector(spd.params_from(MP), n_routers=spd.MAX_PENDING_CLOSES)
    try:
        log("case every pending close in use")
        for r, w in enumerate(ws):
            det.scan(r, to_dev(w))
        tickets = [det.close_begin(r) for r in range(len(ws))]
        with pytest.raises(spd.SpdError) as e:
            det.close_begin(0)
        assert e.value.status == spd.SPD_E_STATE
        for r in reversed(range(len(ws))):
            assert_same_report(det.close_end(tickets[r]), oracle_sketch(MP, ws[r]).detect(), f"router {r}")
        with pytest.raises(spd.SpdError) as e:
            det.close_end(tickets[0])
        assert e.value.status == spd.SPD_E_STATE
        # every router was reset by its close: the next windows start from zero
        for r, w in enumerate(ws[::-1]):
            det.scan(r, to_dev(w))
        for r, w in enumerate(ws[::-1]):
            assert_same_report(det.close_end(det.close_begin(r)), oracle_sketch(MP, w).detect(), f"again {r}")
    finally:
        det.close()


def test_global_empty_and_sliding_match_blocking_close():
    ws = windows(304, 2)
    det = spd.Detector(spd.params_from(MP), n_routers=2)
    try:
        log("case merged sketch and empty window")
        for r, w in enumerate(ws):
            det.scan(r, to_dev(w))
        det.merge([0, 1])
        got = det.close_end(det.close_begin(spd.GLOBAL))
        assert_same_report(got, oracle_sketch(MP, np.concatenate(ws)).detect(), "merged")
        assert len(det.close_end(det.close_begin(spd.GLOBAL))) == 0   # reset by the close
        assert len(det.close_end(det.close_begin(1))) > 0
    finally:
        det.close()
    K = 4
    slices = windows(305, 7, heavy=4, peers=300, noise=20_000)
    for counter in (spd.SLIDING_AT, spd.SLIDING_STAMPS):
        log(f"case sliding window, counter {counter}")
        sp = st.MethodParams(theta=256, r=10, sr=4, a=2, log2k=10, lr=2, log2lc=10, window_slices=K,
                             sliding_counter=counter, hash_seed=91)
        det = spd.Detector(spd.params_from(sp))
        try:
            for t, w in enumerate(slices):
                if t:
                    det.slide()
                det.scan(0, to_dev(w))
                tk = det.close_begin(0)
                blocking = det.close_window(0)
                got = det.close_end(tk)
                want = oracle_sketch(sp, np.concatenate(slices[max(0, t - K + 1): t + 1])).detect()
                assert_same_report(got, want, f"slice {t}")
                assert_same_report(blocking, want, f"slice {t}, blocking")
        finally:
            det.close()


def test_pending_close_record_overflow_then_room():
    """A window with more super points than a pending close's record room (65536): spd_close_end
    reports SPD_E_TRUNCATED with their number (the window may already be rewritten, so nothing is
    re-run); every later close has room, and the same window scanned again is reported in full."""
    mp = st.MethodParams(theta=8, r=16, sr=4, a=2, log2k=6, lr=2, log2lc=16, hash_seed=41)
    rng = np.random.default_rng(43)
    pairs, _ = heavy_hosts(rng, 90_000, 24)
    want = oracle_sketch(mp, pairs).detect()
    assert len(want) > 65536
    det = spd.Detector(spd.params_from(mp))
    set_tuning(det, direct_max_pairs=0)
    try:
        log("case pending close past its record room")
        x = to_dev(pairs)
        det.scan(0, x)
        with pytest.raises(spd.SpdError) as e:
            det.close_end(det.close_begin(0), cap=200_000)
        assert e.value.status == spd.SPD_E_TRUNCATED
        assert str(len(want)) in str(e.value)
        # every pending slot (all in use at once) now has room
        tickets = []
        for _ in range(spd.MAX_PENDING_CLOSES):
            det.scan(0, x)
            tickets.append(det.close_begin(0))
        for k, t in enumerate(tickets):
            assert_same_report(det.close_end(t, cap=200_000), want, f"again {k}")
    finally:
        det.close()


def test_sliding_reports_collected_one_slice_behind():
    """Sliding window as a capture loop runs it: each slice's close is begun, the next slice is
    slid to and scanned (AT maintenance included), and only then is the previous report collected;
    every report must be the oracle's for the window that ended at its own slice."""
    K = 6
    slices = windows(306, 14, heavy=5, peers=200, noise=30_000)
    for counter in (spd.SLIDING_AT, spd.SLIDING_STAMPS):
        log(f"case sliding reports one slice behind, counter {counter}")
        sp = st.MethodParams(theta=256, r=10, sr=4, a=2, log2k=10, lr=2, log2lc=10, window_slices=K,
                             sliding_counter=counter, hash_seed=93)
        det = spd.Detector(spd.params_from(sp))
        try:
            reps, prev = [], None
            for t, w in enumerate(slices):
                if t:
                    det.slide()
                det.scan(0, to_dev(w))
                tk = det.close_begin(0)
                if prev is not None:
                    reps.append(det.close_end(prev))
                prev = tk
            reps.append(det.close_end(prev))
            for t, got in enumerate(reps):
                want = oracle_sketch(sp, np.concatenate(slices[max(0, t - K + 1): t + 1])).detect()
                assert_same_report(got, want, f"counter {counter} slice {t}")
        finally:
            det.close()
