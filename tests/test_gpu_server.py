"""GPU tests of the serving loop: continuous batching over router-window slots.

Routers submit batches of log-uniform sizes in an interleaved order; windows close every W pairs
per router (batches crossing the boundary are split); fewer window slots fit the HBM budget than
there are routers, so routers wait for admission.  Every window's report must equal the oracle's
detection on exactly that window's pairs, and must be the same when the router runs alone, with
and without hipGraph replay of the end-of-window work.
"""
import numpy as np
import pytest

import oracle
import synth_traffic as st
from gpu_util import assert_same_report, heavy_hosts, log, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402

MP = st.CONFIGS["plain_1m"].params
W = 1 << 20


def router_streams(R, windows, seed):
    rng = np.random.default_rng(seed)
    streams = []
    for r in range(R):
        parts = []
        for w in range(windows):
            pairs, _ = heavy_hosts(rng, 4, int(rng.integers(1500, 4000)), noise=0)
            noise = rng.integers(0, 1 << 32, size=(W - len(pairs), 2), dtype=np.uint64).astype(np.uint32)
            win = np.concatenate([pairs, noise])
            parts.append(win[rng.permutation(W)])
        streams.append(np.concatenate(parts))
    return streams


def batches_of(stream_len, rng, lo=4096, hi=300_000):
    cuts = st.split_batches(stream_len, rng, lo, hi)
    return list(zip(cuts[:-1], cuts[1:]))


def run_server(streams, routers, seed, use_graphs=True, max_slots=2):
    """Submit the given routers' streams interleaved; return {(router, window): report}."""
    rng = np.random.default_rng(seed)
    dev = {r: to_dev(streams[r]) for r in routers}
    plan = {r: batches_of(len(streams[r]), rng) for r in routers}
    order = []
    cursor = {r: 0 for r in routers}
    while any(cursor[r] < len(plan[r]) for r in routers):
        live = [r for r in routers if cursor[r] < len(plan[r])]
        r = live[int(rng.integers(0, len(live)))]
        order.append((r, plan[r][cursor[r]]))
        cursor[r] += 1
    srv = spd.Server(spd.params_from(MP), n_routers=max(routers) + 1, window_pairs=W, max_slots=max_slots,
                     hbm_budget_bytes=512 << 20, max_group_pairs=2 << 20, use_graphs=use_graphs)
    try:
        for r, (a, b) in order:
            srv.submit(r, dev[r][a:b])
        srv.drain()
        out = {}
        expect = sum(len(streams[r]) // W for r in routers)
        while len(out) < expect:
            got = srv.next(timeout_ms=20000)
            assert got is not None, "a window never finished"
            hdr, sp = got
            out[(hdr["router"], hdr["window"])] = (hdr, sp)
        stats = srv.stats
    finally:
        srv.close()
    return out, stats


def test_serving_windows_match_oracle_and_alone():
    R, windows = 4, 2
    log("case serving: 4 routers x 2 windows of 1Mi pairs, 2 slots")
    streams = router_streams(R, windows, 7)
    mixed, stats = run_server(streams, list(range(R)), seed=11)
    assert stats["slots"] == 2 and stats["admission_waits"] > 0
    assert stats["windows"] == R * windows
    p = oracle.params(MP)
    for r in range(R):
        for w in range(windows):
            hdr, sp = mixed[(r, w)]
            assert hdr["pairs"] == W
            want = oracle.Sketch(p).scan(streams[r][w * W:(w + 1) * W]).detect()
            assert_same_report(sp, want, f"router {r} window {w}")
            assert hdr["latency_ms"] > 0
    # the same router alone, and without graph replay: identical reports
    alone, _ = run_server(streams, [2], seed=3, use_graphs=False)
    for w in range(windows):
        assert np.array_equal(alone[(2, w)][1], mixed[(2, w)][1])


def test_serving_slots_follow_hbm_budget():
    """Window slots are admitted by the HBM budget: two more slots' worth of budget gives exactly
    two more slots."""
    det = spd.Detector(spd.params_from(MP))
    d = det.derived
    det.close()
    # per slot: LDCA (256-byte aligned) + SEAV padded to 128 KiB + its record buffer + counters
    per_slot = (d.ldca_words * 4 + 255) // 256 * 256 + (-(-d.seav_bytes // (1 << 17)) << 17) + 65536 * 8 + 64
    budget = 64 << 20
    counts = []
    for extra in (0, 2):
        srv = spd.Server(spd.params_from(MP), n_routers=2, hbm_budget_bytes=budget + extra * per_slot,
                         max_group_pairs=1 << 20)
        try:
            counts.append(srv.stats["slots"])
        finally:
            srv.close()
    assert counts[0] >= 1 and counts[1] == counts[0] + 2, counts


def test_serving_close_flag_and_repeated_graph_replays():
    """Windows closed by request (no fixed size): many replays of each slot's captured graph, with
    eager scans between them, every replay equal to the oracle."""
    rng = np.random.default_rng(21)
    det = spd.Detector(spd.params_from(MP))
    slot_bytes = det.derived.ldca_words * 4 + (1 << 17) + 65536 * 8
    det.close()
    srv = spd.Server(spd.params_from(MP), n_routers=2, window_pairs=0, hbm_budget_bytes=(64 << 20) + 3 * slot_bytes,
                     max_group_pairs=2 << 20, use_graphs=True)
    p = oracle.params(MP)
    try:
        wants = []
        for k in range(6):
            r = k % 2
            pairs, _ = heavy_hosts(rng, 3, 2500, noise=int(rng.integers(10_000, 200_000)))
            x = to_dev(pairs)
            half = len(pairs) // 2
            srv.submit(r, x[:half])
            srv.submit(r, x[half:], close=True)
            wants.append((r, oracle.Sketch(p).scan(pairs).detect()))
            hdr, sp = srv.next(timeout_ms=20000)
            assert hdr["router"] == r and hdr["pairs"] == len(pairs)
            assert_same_report(sp, wants[-1][1], f"request close {k}")
    finally:
        srv.close()


def test_serving_rejects_bad_requests():
    srv = spd.Server(spd.params_from(MP), n_routers=2, window_pairs=W, hbm_budget_bytes=256 << 20,
                     max_group_pairs=1 << 20)
    try:
        with pytest.raises(spd.SpdError):
            srv.submit(5, to_dev(np.zeros((4, 2), np.uint32)))
    finally:
        srv.close()
    with pytest.raises(spd.SpdError):
        spd.Server(spd.params_from(MP), n_routers=2, hbm_budget_bytes=1 << 20)


def test_serving_destination_keyed_router():
    """A router fed destination-keyed batches reports the super points of the opposite direction."""
    rng = np.random.default_rng(31)
    srv = spd.Server(spd.params_from(MP), n_routers=2, window_pairs=0, hbm_budget_bytes=512 << 20,
                     max_group_pairs=2 << 20)
    p = oracle.params(MP)
    try:
        pairs, _ = heavy_hosts(rng, 3, 2500, noise=150_000)
        x = to_dev(pairs)
        srv.submit(0, x, close=True)
        srv.submit(1, x, close=True, dst=True)
        got = {}
        for _ in range(2):
            hdr, sp = srv.next(timeout_ms=20000)
            got[hdr["router"]] = sp
        assert_same_report(got[0], oracle.Sketch(p).scan(pairs).detect(), "source-keyed")
        assert_same_report(got[1], oracle.Sketch(p).scan(np.ascontiguousarray(pairs[:, ::-1])).detect(),
                           "destination-keyed")
    finally:
        srv.close()
