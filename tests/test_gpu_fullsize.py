"""GPU parity at the full sizes of the multi-router and sliding-window workloads.

routers_8x16m: 8 routers x 16 Mi pairs scanned in one fused call, every router's sketch and the
merged sketch bit-exact against the oracle, the global report equal to the oracle's.
sliding_300x1m: 300 slices of 1,000,000 pairs with a 60-slice window; the GPU reports after
every slice; at sampled slices the exported bit view and the report must equal the oracle's
discrete detection on the union of the window's slices (the plain definition of the sliding
window), and the first full window is also checked against the oracle's time-stamp counters.
"""
import numpy as np
import pytest

import oracle
import synth_traffic as st
from gpu_util import assert_same_report, assert_same_sketch, log, oracle_sketch, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402


def test_routers_8x16m_full():
    w = st.CONFIGS["routers_8x16m"]
    log("case routers_8x16m: generating")
    win = st.gen_routers(w)
    R = w.n_routers
    det = spd.Detector(spd.params_from(w.params), n_routers=R)
    try:
        log("case routers_8x16m: fused scan of 8 routers")
        xs = [to_dev(win.pairs[r]) for r in range(R)]
        det.scan_batches([(r, xs[r]) for r in range(R)])
        torch.cuda.synchronize()
        merged = None
        for r in range(R):
            log(f"case routers_8x16m: oracle router {r}")
            ref = oracle_sketch(w.params, win.pairs[r])
            assert_same_sketch(det, r, ref, f"router {r}")
            merged = ref if merged is None else merged.merge(ref)
        det.merge(list(range(R)))
        assert_same_sketch(det, spd.GLOBAL, merged, "merged")
        got = det.close_window(spd.GLOBAL)
        assert_same_report(got, merged.detect(), "global report")
        assert len(got) >= 0.95 * w.n_planted
    finally:
        det.close()


def test_sliding_300x1m_full_sampled():
    w = st.CONFIGS["sliding_300x1m"]
    K = w.params.window_slices
    log("case sliding_300x1m: setup")
    tr = st.gen_sliding(w)
    samples = {K - 1, 173, w.n_slices - 1}
    keep = set()
    for t in samples:
        keep.update(range(max(0, t - K + 1), t + 1))
    kept = {}
    det = spd.Detector(spd.params_from(w.params))
    stamps = oracle.SlidingSketch(oracle.params(w.params), K)
    n_reports = 0
    try:
        for t in range(w.n_slices):
            if t:
                det.slide()
            p = tr.slice(t)
            det.scan(0, to_dev(p))
            if t < K:
                stamps.scan_slice(p, t)
            if t in keep:
                kept[t] = p
            got = det.close_window(0)
            n_reports += 1
            if t == K - 1:
                log("case sliding_300x1m: raw stamps at the first full window")
                ts_seav, ts_ldca = det.export_stamps(0)
                np.testing.assert_array_equal(ts_seav, stamps.seav_ts)
                np.testing.assert_array_equal(ts_ldca, stamps.ldca_ts)
                del stamps
            if t in samples:
                log(f"case sliding_300x1m: oracle window ending at slice {t}")
                union = oracle_sketch(w.params, np.concatenate([kept[j] for j in range(t - K + 1, t + 1)]))
                assert_same_sketch(det, 0, union, f"window {t}")
                want = union.detect()
                assert_same_report(got, want, f"window {t}")
                truth = tr.planted_card(t, K)
                strong = set(tr.planted_ips[truth >= 2 * w.params.theta].tolist())
                assert len(strong - set(got["ip"].tolist())) <= max(1, len(strong) // 20)
            for j in [j for j in kept if j < t - K + 1 and all(j < s - K + 1 or j > s for s in samples)]:
                del kept[j]
        assert n_reports == w.n_slices
    finally:
        det.close()
