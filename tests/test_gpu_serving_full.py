"""The serving loop at the serving_16r configuration itself: method parameters r = 14, LC = 2^16,
k = 4096, windows of 64 Mi pairs, 16 routers, batches of log-uniform size in [4 Ki, 4 Mi] pairs
submitted in an interleaved order.  Router r's window w carries pool window (r + w) mod 4 of
plain_64m-shaped traffic (1000 planted super points over the pool), so each of the 32 windows is
checked against the oracle's detection on its pool window, and windows sharing a pool window must
report the same list whatever else ran beside them."""
import numpy as np
import pytest

import synth_traffic as st
from gpu_util import assert_same_report, log, oracle_sketch_threads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402


def test_serving_16r_full_configuration():
    from concurrent.futures import ThreadPoolExecutor
    w = st.CONFIGS["serving_16r"]
    R, W, windows = w.n_routers, w.n_packets, 2
    log("case serving_16r full: generating 4 pool windows of 64 Mi pairs")
    with ThreadPoolExecutor(max_workers=4) as ex:
        pool_np = list(ex.map(lambda k: st.gen_plain(st.scaled(w, n_planted=w.n_planted // 4, seed=w.seed + k)).pairs[0],
                              range(4)))
    pool = [torch.from_numpy(p.view(np.int32)).to("cuda") for p in pool_np]
    log("case serving_16r full: oracle on the pool windows")
    with ThreadPoolExecutor(max_workers=4) as ex:
        wants = list(ex.map(lambda p: oracle_sketch_threads(w.params, np.array_split(p, 4), 4).detect(), pool_np))
    rng = np.random.default_rng(5051)
    plan = []
    for r in range(R):
        for wi in range(windows):
            cuts = st.split_batches(W, rng, 4096, 4 << 20)
            plan.append([(r, pool[(r + wi) % 4][a:b]) for a, b in zip(cuts[:-1], cuts[1:])])
    per_router = [[b for k, seq in enumerate(plan) if k // windows == r for b in seq] for r in range(R)]
    order, cursor = [], [0] * R
    while any(cursor[r] < len(per_router[r]) for r in range(R)):
        live = [r for r in range(R) if cursor[r] < len(per_router[r])]
        r = live[int(rng.integers(0, len(live)))]
        order.append(per_router[r][cursor[r]])
        cursor[r] += 1
    log(f"case serving_16r full: {len(order)} batches, {R} routers x {windows} windows")
    srv = spd.Server(spd.params_from(w.params), n_routers=R, window_pairs=W, hbm_budget_bytes=16 << 30,
                     max_slots=24, max_group_pairs=64 << 20)
    try:
        for r, x in order:
            srv.submit(r, x)
        srv.drain()
        got = {}
        while len(got) < R * windows:
            res = srv.next(timeout_ms=60000)
            assert res is not None, "a window never finished"
            got[(res[0]["router"], res[0]["window"])] = res
        stats = srv.stats
    finally:
        srv.close()
    assert stats["windows"] == R * windows and stats["slots"] == 24
    for (r, wi), (hdr, sp) in sorted(got.items()):
        assert hdr["pairs"] == W
        assert_same_report(sp, wants[(r + wi) % 4], f"router {r} window {wi}")
    assert all(len(x) >= 240 for x in wants)
