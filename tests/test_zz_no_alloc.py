"""The scan entry point that allocates nothing, spd_scan_noalloc, against spd_scan through the C ABI.

Two windows in a row per case, the second smaller than the first: after each, both contexts'
sketches (SEAV bytes, LDCA words) and end-of-window reports must be identical, and the no-alloc
context must hold exactly the device memory it held before the call.  The first window of the
plain_1m and plain_64m cases needs several launches of the fixed scratch array.
"""
import ctypes

import numpy as np
import pytest

import synth_traffic as st
from gpu_util import assert_same_report, heavy_hosts, log, oracle_sketch, set_tuning, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402


def noalloc(det, router, x, flags=0):
    """spd_scan_noalloc through the C ABI, on torch's current stream; returns the status."""
    n = x.shape[0]
    return spd.lib().spd_scan_noalloc(det.ctx, router, ctypes.c_void_p(x.data_ptr() if n else None), n, flags,
                                      ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def same_window(a, b, what):
    sa, la = a.export(0)
    sb, lb = b.export(0)
    assert np.array_equal(sa, sb), f"{what}: SEAV differs"
    assert np.array_equal(la, lb), f"{what}: LDCA differs"
    ra, rb = a.close_window(0), b.close_window(0)
    assert_same_report(ra, rb, what)
    return ra


def run_case(mp, windows, flags=0, tune=None, oracle_last=False):
    """Scans each window through both entry points; returns the binned launches of each no-alloc call."""
    a = spd.Detector(spd.params_from(mp))
    b = spd.Detector(spd.params_from(mp))
    per_call = []
    try:
        if tune:
            set_tuning(a, **tune)
            set_tuning(b, **tune)
        for k, pairs in enumerate(windows):
            x = to_dev(pairs)
            torch.cuda.synchronize()
            held = a.stats.device_bytes
            launches = a.stats.binned_launches
            log(f"  window {k}: {len(pairs)} pairs, flags {flags}")
            assert noalloc(a, 0, x, flags) == spd.SPD_OK, spd.lib().spd_last_error(a.ctx)
            b.scan_batches([(0, x, flags)])
            torch.cuda.synchronize()
            assert a.stats.device_bytes == held, "spd_scan_noalloc allocated device memory"
            per_call.append(a.stats.binned_launches - launches)
            rep = same_window(a, b, f"window {k}")
            if oracle_last and k == len(windows) - 1:
                view = pairs if not flags else np.ascontiguousarray(pairs[:, ::-1])
                assert_same_report(rep, oracle_sketch(mp, view).detect(), f"window {k} vs oracle")
        return per_call
    finally:
        a.close()
        b.close()


def test_noalloc_plain_1m_two_windows():
    mp = st.CONFIGS["plain_1m"].params
    rng = np.random.default_rng(1001)
    big, _ = heavy_hosts(rng, 8, 3000, noise=5_000_001)
    small, _ = heavy_hosts(rng, 5, 2500, noise=700_003)
    log("case no-alloc plain_1m: 5 Mi then 0.7 Mi pairs")
    launches = run_case(mp, [big, small], oracle_last=True)
    assert launches[0] >= 2 and launches[1] >= 1, launches


def test_noalloc_plain_64m_geometry_many_launches():
    mp = st.CONFIGS["plain_64m"].params
    rng = np.random.default_rng(1002)
    big, _ = heavy_hosts(rng, 20, 4000, noise=12_000_000)
    small, _ = heavy_hosts(rng, 10, 3000, noise=3_000_000)
    log("case no-alloc plain_64m sizes: 12 Mi then 3 Mi pairs")
    launches = run_case(mp, [big, small])
    assert launches[0] >= 3 and launches[1] >= 1, launches


def test_noalloc_direct_and_destination_keyed():
    mp = st.CONFIGS["plain_1m"].params
    rng = np.random.default_rng(1003)
    w1, _ = heavy_hosts(rng, 4, 2500, noise=200_000)
    w2, _ = heavy_hosts(rng, 3, 2500, noise=60_000)
    log("case no-alloc direct kernel (batches below direct_max_pairs)")
    assert run_case(mp, [w1, w2], oracle_last=True) == [0, 0]
    log("case no-alloc destination-keyed, binned")
    run_case(mp, [w1, w2], flags=spd.BATCH_DST, tune=dict(direct_max_pairs=0), oracle_last=True)


def test_noalloc_refusals():
    mp = st.CONFIGS["plain_1m"].params
    x = to_dev(np.zeros((16, 2), np.uint32))
    det = spd.Detector(spd.params_from(mp), n_routers=2)
    try:
        assert noalloc(det, 2, x) == spd.SPD_E_STATE          # no such router
        assert noalloc(det, 0, x, flags=4) == spd.SPD_E_INVALID
    finally:
        det.close()
    sl = spd.Detector(spd.params_from(mp.replace(window_slices=4)))
    try:
        assert noalloc(sl, 0, x) == spd.SPD_E_STATE           # sliding contexts are refused
    finally:
        sl.close()
