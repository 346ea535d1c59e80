#!/usr/bin/env python3
"""Benchmark of the super-point detection hot path on one MI355X.

One step = one window of the 64 Mi-pair workload (1 router): the scan of every pair into the
short estimator array vector and the long estimator array, then the end of window (candidate
rebuild from the SEAV, LDCA filter against theta, report, reset).  Inputs are seeded synthetic
traffic already resident in HBM when the timed region starts.  The launch settings are the ones
the autotuner picks for this GPU and shape.

Prints ONE JSON line: throughput in packets (pairs) per second of the default (binned) scan, the
roofline of the dominant kernel (HIP events on the launch stream), p50/p99 end-of-window latency,
the same figures for the plain per-batch kernel (one thread per pair, global atomics), the other
workloads (1 Mi-pair window, 8 routers fused + merge, sliding window of 60 one-million-pair
slices), the serving loop on 16 routers, and the CPU oracle timed on the host (P threads and one).
`--ceilings` instead prints one JSON line of the hardware ceilings the design rests on.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, public figure
BYTES_PER_PAIR = 8             # algorithmic HBM bytes per pair: one uint32 (hip, oip) record
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "region_kernel_plain_64m_traffic.txt")
SCAN_KINDS = ("bin", "transpose", "apply", "fill", "direct", "count", "offsets", "spill", "stamp")
CPU_THREADS_MAX = 16           # the host-core share of one GPU on the benchmark machines


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    """sha256[:16] of the kernel sources with comments, trailing blanks and blank lines removed:
    a change of the code invalidates the committed counters, a change of a comment does not."""
    import re
    h = hashlib.sha256()
    for f in ("spd_kernels.hip", "spd_internal.h"):
        with open(os.path.join(ROOT, "paper_1901_07306_amd", "csrc", f)) as fh:
            src = re.sub(r"/\*.*?\*/", "", fh.read(), flags=re.S)
        lines = [re.sub(r"//.*$", "", ln).rstrip() for ln in src.split("\n")]
        h.update("\n".join(ln for ln in lines if ln.strip()).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3 counter summary,
    or None if the summary is missing or was taken on a different kernel source."""
    try:
        kv = {}
        with open(PROFILE_TRAFFIC) as f:
            for line in f:
                if ":" in line and not line.startswith("#"):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("kernel_source_sha") != kernel_source_sha():
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def pct(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q)) if len(v) else None


def set_tuning(det, settings):
    t = det.tuning
    for k, v in settings.items():
        setattr(t, k, v)
    det.tuning = t


def roofline(kind, n_pairs, launches, total_ms, traffic=None):
    """Roofline entry of one kernel kind whose every launch covers n_pairs pairs (8 B each)."""
    avg = total_ms / launches
    alg = BYTES_PER_PAIR * n_pairs
    ach = alg / (avg * 1e-3) / 1e9
    return {"kernel": kind, "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": traffic, "alg_bytes_per_launch": alg, "avg_launch_ms": avg,
            "launches": launches}


def run_detector(spd, torch, params, x, steps, warmup, tune):
    """Four passes of `steps` windows each (scan + end of window, the report on the host):
    1. every kernel kind timed with the library's HIP events: the per-kernel breakdown and the
       dominant kernel;
    2. the timed region: back-to-back windows as a capture loop runs them, each window's close
       begun (spd_close_begin) before the next window's scan is enqueued and its report collected
       (spd_close_end) after it, so that the GPU does not wait for the host between windows; only
       the dominant kernel timed (two events per launch, so the timing hardly disturbs the run);
    3. the same windows with the blocking close (spd_close_window after each scan);
    4. untimed, a synchronisation after each scan: the end-of-window latency alone."""
    import numpy as np
    det = spd.Detector(params)
    set_tuning(det, tune)
    for _ in range(warmup):
        det.scan(0, x)
        det.close_window(0)
        det.close_end(det.close_begin(0))   # (an empty window: warms up the two-part close)
    torch.cuda.synchronize()
    det.profile_enable(True)
    for _ in range(steps):
        det.scan(0, x)
        det.close_window(0)
    breakdown = {k: v for k, v in det.profile().items() if v[0]}
    scan_only = {k: v for k, v in breakdown.items() if k in SCAN_KINDS}
    dom = max(scan_only, key=lambda k: scan_only[k][1])
    det.profile_enable(True, kinds=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec, prev = None, None
    for _ in range(steps):
        det.scan(0, x)
        t = det.close_begin(0)
        if prev is not None:
            rec = det.close_end(prev)
        prev = t
    rec = det.close_end(prev)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed = det.profile()[dom]
    det.profile_enable(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        det.scan(0, x)
        brec = det.close_window(0)
    torch.cuda.synchronize()
    elapsed_blocking = time.perf_counter() - t0
    assert np.array_equal(brec, rec), "blocking and two-part closes disagree"
    close_ms, window_ms = [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        det.scan(0, x)
        torch.cuda.synchronize()
        c0 = time.perf_counter()
        det.close_window(0)
        c1 = time.perf_counter()
        close_ms.append((c1 - c0) * 1e3)
        window_ms.append((c1 - s0) * 1e3)
    stats = det.stats
    det.close()
    return elapsed, close_ms, window_ms, breakdown, (dom, timed), rec, stats, elapsed_blocking


def config_entry(n, steps, el, close_ms, window_ms, kinds, dom, dom_launches, dom_ms, traffic=None):
    scan_ms = sum(v[1] for k, v in kinds.items() if k in SCAN_KINDS) / steps
    return {"value": n * steps / el, "unit": "packets/s", "ms_per_step": el / steps * 1e3,
            "roofline": roofline(dom, n, dom_launches, dom_ms, traffic),
            "scan_ms_per_window": scan_ms,
            "scan_roofline_frac": (BYTES_PER_PAIR * n / (scan_ms * 1e-3) / 1e9) / HBM_PEAK_GBS,
            "close_latency_ms": {"p50": pct(close_ms, 50), "p99": pct(close_ms, 99)},
            "window_latency_ms": {"p50": pct(window_ms, 50), "p99": pct(window_ms, 99)},
            "kernel_ms_per_step": {k: v[1] / steps for k, v in kinds.items()}}


def run_both_directions(spd, torch, params, x, steps, warmup, tune):
    """Source- and destination-keyed super points of the same window: one fused scan call with the
    pairs as given (router 0) and swapped (router 1), then both ends of window.  Returns pairs/s
    (each pair counted once) and the two report sizes."""
    det = spd.Detector(params, n_routers=2)
    set_tuning(det, tune)
    rep = None
    for i in range(warmup + steps):
        if i == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        det.scan_batches([(0, x), (1, x, spd.BATCH_DST)])
        rep = (det.close_window(0), det.close_window(1))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    det.close()
    return x.shape[0] * steps / el, el / steps * 1e3, [int(len(r)) for r in rep]


def run_host_ingest(spd, torch, params, pairs_np, steps, warmup, tune):
    """The window handed over in page-locked host memory: spd_scan_host copies it in 16 Mi-pair
    chunks on its own stream, each copy overlapping the scan of the previous chunk, then the end of
    window.  PCIe-inclusive pairs/s (the host link, not HBM, bounds this figure)."""
    import numpy as np
    host = torch.from_numpy(pairs_np.view(np.int32)).pin_memory()
    det = spd.Detector(params)
    set_tuning(det, tune)
    for i in range(warmup + steps):
        if i == warmup:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        det.scan_host(0, host)
        det.close_window(0)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    det.close()
    return host.shape[0] * steps / el, el / steps * 1e3


def bench_plain_1m(spd, torch, np, st, at, steps, warmup):
    """1,000,000-pair window of one router: scan + end of window (tuned), and the plain kernel."""
    w = st.CONFIGS["plain_1m"]
    win = st.gen_plain(w)
    x = torch.from_numpy(win.pairs[0].view(np.int32)).to("cuda")
    params = spd.params_from(w.params)
    probe = spd.Detector(params)
    tuned = at.autotune(probe, x, quick=True)
    probe.close()
    el, close_ms, window_ms, kinds, (dom, (dl, dms)), rec, _, _ = run_detector(spd, torch, params, x, steps, warmup,
                                                                               tuned)
    e = config_entry(x.shape[0], steps, el, close_ms, window_ms, kinds, dom, dl, dms)
    pel, _, _, _, _, prec, _, _ = run_detector(spd, torch, params, x, steps, warmup, {"direct_max_pairs": 1 << 62})
    assert np.array_equal(prec, rec), "plain_1m: plain and tuned scans disagree"
    e["plain"] = {"value": x.shape[0] * steps / pel, "unit": "packets/s", "ms_per_step": pel / steps * 1e3}
    e["batched_over_plain"] = e["value"] / e["plain"]["value"]
    e["tuning"] = tuned
    e["reported_super_points"] = int(len(rec))
    e["workload"] = "plain_1m: 1 router, 1 window of 1,000,000 pairs; 50k Zipf(1.2)<=200 sources, 20 planted x 2000"
    return e, win.pairs[0], rec


def bench_routers(spd, torch, np, st, at, steps, warmup):
    """8 routers x 16 Mi pairs: one fused scan call over the 8 routers' batches that also ORs them
    into the global sketch (spd_scan_batches_merge: the merge done by the apply phase), global end
    of window, each router's sketch reset for its next window."""
    w = st.CONFIGS["routers_8x16m"]
    g0 = time.perf_counter()
    win = st.gen_routers(w)
    log(f"routers_8x16m generated in {time.perf_counter() - g0:.1f} s")
    R = w.n_routers
    xs = [torch.from_numpy(p.view(np.int32)).to("cuda") for p in win.pairs]
    params = spd.params_from(w.params)
    det = spd.Detector(params, n_routers=R)
    batches = [(r, xs[r]) for r in range(R)]
    tuned = at.autotune(det, xs[0], quick=True, batches=batches, merge=True)   # timed on the fused call itself

    def step():
        det.scan_batches(batches, merge=True)
        rep = det.close_window(spd.GLOBAL)
        for r in range(R):
            det.reset(r)
        return rep

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    det.profile_enable(True)
    for _ in range(steps):
        step()
    kinds = {k: v for k, v in det.profile().items() if v[0]}
    scan_only = {k: v for k, v in kinds.items() if k in SCAN_KINDS}
    dom = max(scan_only, key=lambda k: scan_only[k][1])
    det.profile_enable(True, kinds=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rec = step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    dl, dms = det.profile()[dom]
    det.profile_enable(False)
    det.close()
    n = R * xs[0].shape[0]
    scan_ms = sum(v[1] for k, v in scan_only.items()) / steps
    e = {"value": n * steps / el, "unit": "packets/s", "ms_per_step": el / steps * 1e3,
         "roofline": roofline(dom, n, dl, dms), "scan_ms_per_window": scan_ms,
         "scan_roofline_frac": (BYTES_PER_PAIR * n / (scan_ms * 1e-3) / 1e9) / HBM_PEAK_GBS,
         "kernel_ms_per_step": {k: v[1] / steps for k, v in kinds.items()},
         "tuning": tuned, "reported_super_points": int(len(rec)),
         "workload": "routers_8x16m: 8 routers x 16Mi pairs, 40% of 4M sources at >=2 routers, 300 planted "
                     "split over routers; fused scan of the 8 routers + OR merge + global end of window",
         "step": "scan_batches_merge(8 routers: scan + OR merge into the global sketch) + close(global) + "
                 "reset(routers)"}
    del xs
    return e, win, rec


def bench_sliding(spd, torch, np, st):
    """sliding_300x1m: 300 slices of 1,000,000 pairs, window of 60 slices; one step = slide + scan of
    the slice + report of the window ending there.  Two passes over all slices: every kernel kind
    timed (breakdown), then the timed pass with only the dominant scan kernel timed."""
    from concurrent.futures import ThreadPoolExecutor
    w = st.CONFIGS["sliding_300x1m"]
    g0 = time.perf_counter()
    tr = st.gen_sliding(w)
    with ThreadPoolExecutor(max_workers=8) as ex:
        slices = list(ex.map(tr.slice, range(w.n_slices)))
    log(f"sliding_300x1m generated in {time.perf_counter() - g0:.1f} s")
    xs = [torch.from_numpy(p.view(np.int32)).to("cuda") for p in slices]
    params = spd.params_from(w.params)

    def run(kinds_mask, count=False):
        # each slice's report is collected after the next slice is enqueued (the two-part close)
        det = spd.Detector(params)
        det.close_end(det.close_begin(0))   # allocates the two-part close's buffers
        det.profile_enable(True, kinds=kinds_mask)
        reps, cands = [], []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        prev = None
        for t, x in enumerate(xs):
            if t:
                det.slide()
            det.scan(0, x)
            tk = det.close_begin(0)
            if prev is not None:
                reps.append(det.close_end(prev))
                if count:
                    cands.append(det.stats.candidates_last)
            prev = tk
        reps.append(det.close_end(prev))
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        if count:
            cands.append(det.stats.candidates_last)
        prof = {k: v for k, v in det.profile().items() if v[0]}
        det.close()
        return el, prof, reps, cands

    _, kinds, _, cands = run(None, count=True)
    scan_only = {k: v for k, v in kinds.items() if k in SCAN_KINDS}
    dom = max(scan_only, key=lambda k: scan_only[k][1])
    el, timed, reps, _ = run([dom])
    n, T = xs[0].shape[0], len(xs)
    dl, dms = timed[dom]
    e = {"value": n * T / el, "unit": "packets/s", "ms_per_slice": el / T * 1e3,
         "roofline": dict(roofline(dom, n, dl, dms), bound="random stores (one 8-bit AT code per bit set)" if params.sliding_counter == spd.SLIDING_AT
                                             else "random stores (one 16-bit stamp per bit set)"),
         "kernel_ms_per_slice": {k: v[1] / T for k, v in kinds.items()},
         "reports": T, "mean_reported": float(np.mean([len(r) for r in reps])),
         "mean_candidates": float(np.mean(cands)),
         "workload": "sliding_300x1m: 300 slices x 1,000,000 pairs, window K = 60 slices, 1M Zipf(1.1)<=500 "
                     "sources, 200 planted with onset/offset; one report per slice",
         "step": "slide + scan of one slice + report of the window ending at it (collected after the next "
                 "slice is enqueued)"}
    del xs
    return e, slices, reps


def bench_serving(spd, torch, np, st, capacity_pps, windows_per_router, loads, tuned, budget, max_slots,
                  min_scan_pairs=0, use_graphs=True):
    """The serving loop on the 16-router workload: batches of log-uniform size in [4Ki, 4Mi] pairs,
    Poisson arrivals at load x capacity_pps, a window closed every 64Mi pairs per router.  Router
    r's window w replays pool window (r + w) mod 4 of plain_64m-shaped traffic (1000 planted super
    points spread over the pool).  Returns one entry per load, the pool (host arrays) and, per
    load, the reports {(router, window): records}."""
    from concurrent.futures import ThreadPoolExecutor
    w = st.CONFIGS["serving_16r"]
    R, W = w.n_routers, w.n_packets
    g0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=4) as ex:
        pool_np = list(ex.map(lambda k: st.gen_plain(st.scaled(w, n_planted=w.n_planted // 4, seed=w.seed + k)).pairs[0],
                              range(4)))
    log(f"serving pool generated in {time.perf_counter() - g0:.1f} s")
    pool = [torch.from_numpy(p.view(np.int32)).to("cuda") for p in pool_np]
    params = spd.params_from(w.params)
    t = spd.SpdTuning()
    probe = spd.Detector(params)
    t = probe.tuning
    for k, v in tuned.items():
        setattr(t, k, v)
    probe.close()
    results, reports = [], []
    for load in loads:
        rng = np.random.default_rng(w.seed)
        per_router = []
        for r in range(R):
            seq = []
            for wi in range(windows_per_router):
                src = pool[(r + wi) % 4]
                cuts = st.split_batches(W, rng, 4096, 4 << 20)
                seq += [src[a:b] for a, b in zip(cuts[:-1], cuts[1:])]
            per_router.append(seq)
        n_batches = sum(len(q) for q in per_router)
        total = R * windows_per_router * W
        rate = load * capacity_pps / (total / n_batches)     # batches per second over all routers
        times = np.cumsum(rng.exponential(1.0 / rate, size=n_batches))
        times -= times[0]
        cursor = [0] * R
        routers, tensors = [], []
        for i in range(n_batches):
            live = [r for r in range(R) if cursor[r] < len(per_router[r])]
            r = live[int(rng.integers(0, len(live)))]
            routers.append(r)
            tensors.append(per_router[r][cursor[r]])
            cursor[r] += 1
        srv = spd.Server(params, n_routers=R, window_pairs=W, hbm_budget_bytes=budget, max_slots=max_slots,
                         max_group_pairs=64 << 20, use_graphs=use_graphs, tuning=t, min_scan_pairs=min_scan_pairs)
        sched = srv.schedule(times, routers, tensors)   # the arrival array, built before the clock starts
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        srv.replay(sched)
        lat, rep = [], {}
        for _ in range(R * windows_per_router):
            got = srv.next(timeout_ms=120000)
            if got is None:
                raise RuntimeError("serving: a window did not finish")
            lat.append(got[0]["latency_ms"])
            rep[(got[0]["router"], got[0]["window"])] = got[1]
        el = time.perf_counter() - t0
        stats = srv.stats
        srv.close()
        log(f"serving load {load}: {total / el / 1e9:.1f} Gpairs/s, {len(lat)} windows, p50 {pct(lat, 50):.2f} ms, "
            f"p99 {pct(lat, 99):.2f} ms, {stats['slots']} slots")
        results.append({"offered_load": load, "offered_pairs_per_s": load * capacity_pps, "value": total / el,
                        "unit": "packets/s", "routers": R, "windows": len(lat), "pairs": total,
                        "batches": n_batches,
                        "window_latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99), "max": max(lat)},
                        "slots": stats["slots"], "max_open": stats["max_open"],
                        "admission_waits": stats["admission_waits"], "groups": stats["groups"],
                        "hbm_budget_bytes": budget})
        reports.append(rep)
    del pool
    return results, pool_np, reports


# ------------------------------------------------------------------------------ CPU baseline
def host_facts():
    model, mem = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem = int(line.split()[1]) / (1 << 20)
                    break
    except OSError:
        pass
    return model, mem


def oracle_threads(oracle, p, parts, P):
    """The oracle's sketch of the union of `parts`, scanned by P threads, each a contiguous share of
    the parts into a private sketch, then OR-merged (the result depends only on the set of pairs)."""
    import numpy as np
    pieces = []
    for part in parts:
        pieces += [q for q in np.array_split(part, max(1, P // max(1, len(parts)))) if len(q)]
    groups = [pieces[i::P] for i in range(min(P, len(pieces)))]
    sketches = [oracle.Sketch(p) for _ in groups]

    def work(k):
        for q in groups[k]:
            sketches[k].scan(q)

    th = [threading.Thread(target=work, args=(k,)) for k in range(len(groups))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    merged = sketches[0]
    for s in sketches[1:]:
        merged.merge(s)
    return merged


def cpu_baseline_and_checks(oracle, np, st, pairs, rec, extra):
    """The oracle on the host: the plain_64m window with one thread and with P threads (timed), then
    the oracle's reports for the other workloads, compared with the GPU's."""
    w = st.CONFIGS["plain_64m"]
    p = oracle.params(w.params)
    P = max(1, min(len(os.sched_getaffinity(0)), CPU_THREADS_MAX))
    model, mem = host_facts()
    log("CPU oracle: one full plain_64m window, single thread")
    c0 = time.perf_counter()
    ref1 = oracle.Sketch(p).scan(pairs).detect()
    t1 = time.perf_counter() - c0
    log(f"CPU oracle: the same window, {P} threads + OR merge")
    c0 = time.perf_counter()
    refP = oracle_threads(oracle, p, [pairs], P).detect()
    tP = time.perf_counter() - c0
    n = pairs.shape[0]
    base = {"value": n / tP, "unit": "packets/s", "cores": P, "kind": "oracle",
            "sample": f"the full 64Mi-pair plain_64m window once: {P} threads each scan a contiguous split into "
                      "a private sketch, OR merge, end of window on one thread",
            "seconds": tP,
            "single_thread": {"value": n / t1, "unit": "packets/s", "cores": 1, "seconds": t1},
            "cpu_model": model, "host_memory_gib": mem, "affinity_cores": len(os.sched_getaffinity(0))}
    match = {"plain_64m": bool(np.array_equal(ref1.astype(rec.dtype), rec)
                               and np.array_equal(refP.astype(rec.dtype), rec))}
    if "plain_1m" in extra:
        pm, rm = extra["plain_1m"]
        want = oracle.Sketch(oracle.params(st.CONFIGS["plain_1m"].params)).scan(pm).detect()
        match["plain_1m"] = bool(np.array_equal(want.astype(rm.dtype), rm))
    if "routers_8x16m" in extra:
        log("CPU oracle: routers_8x16m, merged sketch of the 8 routers")
        win, rr = extra["routers_8x16m"]
        want = oracle_threads(oracle, oracle.params(st.CONFIGS["routers_8x16m"].params), win.pairs, P).detect()
        match["routers_8x16m"] = bool(np.array_equal(want.astype(rr.dtype), rr))
    if "sliding_300x1m" in extra:
        slices, reps = extra["sliding_300x1m"]
        ws = st.CONFIGS["sliding_300x1m"]
        K = ws.params.window_slices
        ok, checked = True, []
        for t in (K - 1, (ws.n_slices + K) // 2, ws.n_slices - 1):
            log(f"CPU oracle: sliding window ending at slice {t}")
            want = oracle_threads(oracle, oracle.params(ws.params), slices[t - K + 1:t + 1], P).detect()
            ok = ok and bool(np.array_equal(want.astype(reps[t].dtype), reps[t]))
            checked.append(t)
        match["sliding_300x1m"] = {"windows_checked": checked, "match": ok}
    if "serving_16r" in extra:
        pool_np, reports = extra["serving_16r"]
        ps = oracle.params(st.CONFIGS["serving_16r"].params)
        ok, n_checked = True, 0
        for k, pw in enumerate(pool_np):
            log(f"CPU oracle: serving pool window {k}")
            want = oracle_threads(oracle, ps, [pw], P).detect()
            for rep in reports:
                for (r, wi), got in rep.items():
                    if (r + wi) % len(pool_np) == k:
                        ok = ok and bool(np.array_equal(want.astype(got.dtype), got))
                        n_checked += 1
        match["serving_16r"] = {"windows_checked": n_checked, "distinct_windows": len(pool_np), "match": ok}
    return base, match


# ------------------------------------------------------------------------------ ceilings
def ceilings(torch):
    """Hardware ceilings behind the design, from the microbenchmark kernels of libspd_ceilings.so."""
    from paper_1901_07306_amd import ceilings as cl
    return cl.run_all(torch, log)


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=5, help="steps for the plain per-batch kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-run", action="store_true",
                    help="short run for rocprofv3 counter collection: 2 windows + one 512 MiB copy for scaling")
    ap.add_argument("--pmc-workload", default="plain_64m", choices=["plain_64m", "sliding_300x1m"],
                    help="--pmc-run on the sliding workload: its first 64 slices, each scanned and reported")
    ap.add_argument("--configs", default="plain_1m,routers_8x16m,sliding_300x1m",
                    help="other workloads to measure (comma list; empty: none)")
    ap.add_argument("--serving-windows", type=int, default=8, help="windows per router in the serving run (0: skip)")
    ap.add_argument("--serving-loads", default="0.5,1.0", help="offered loads, fractions of the measured capacity")
    ap.add_argument("--serving-budget-gib", type=float, default=16.0, help="HBM budget of the serving loop")
    ap.add_argument("--no-autotune", action="store_true", help="time the library's default settings")
    ap.add_argument("--ceilings", action="store_true", help="print the hardware ceilings instead")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path.  Several GPUs would each "
              "scan their routers' pairs into their own sketches and OR-combine them once per window.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1901_07306_amd as spd
    import synth_traffic as st
    from paper_1901_07306_amd import autotune as at

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
    if args.ceilings:
        print(json.dumps(ceilings(torch)), flush=True)
        return 0
    if args.pmc_run and args.pmc_workload == "sliding_300x1m":
        ws = st.CONFIGS["sliding_300x1m"]
        tr = st.gen_sliding(ws)
        det = spd.Detector(spd.params_from(ws.params))
        for t in range(64):
            if t:
                det.slide()
            det.scan(0, torch.from_numpy(tr.slice(t).view(np.int32)).to("cuda"))
            det.close_window(0)
        torch.cuda.synchronize()
        det.close()
        log("pmc run done: 64 sliding slices")
        return 0
    w = st.CONFIGS["plain_64m"]
    log(f"generating {w.name}: {w.n_packets} pairs")
    g0 = time.perf_counter()
    win = st.gen_plain(w)
    pairs = win.pairs[0]
    log(f"generated in {time.perf_counter() - g0:.1f} s")
    x = torch.from_numpy(pairs.view(np.int32)).to("cuda")
    torch.cuda.synchronize()
    n = x.shape[0]
    params = spd.params_from(w.params)

    if args.pmc_run:
        det = spd.Detector(params)
        for _ in range(2):
            det.scan(0, x)
            det.close_window(0)
        y = x.clone()          # plain copy kernel of known size: reads and writes n * 8 bytes
        torch.cuda.synchronize()
        det.close()
        log(f"pmc run done: copy of {n * 8} bytes, checksum {int(y[-1, 0])}")
        return 0

    tuned = {}
    if not args.no_autotune:
        log("autotune: binned layouts, tiles and workgroups; direct-kernel shape; direct/binned crossover")
        probe = spd.Detector(params)
        tuned = at.autotune(probe, x, quick=True)
        tables = at.last_tables(at.cache_key(probe, x))
        probe.close()
        log(f"autotune chose {tuned}")

    # the library's binned scan with the tuned settings -- the headline value
    log(f"timing the scan: {args.warmup} warmup + {args.steps} steps")
    el, close_ms, window_ms, kinds, (dom, (dom_launches, dom_ms)), rec, stats, el_blocking = run_detector(
        spd, torch, params, x, args.steps, args.warmup, tuned)
    if dom_launches != args.steps:
        raise RuntimeError(f"unexpected dominant kernel {dom} ({dom_launches} launches)")
    value = n * args.steps / el
    ms_step = el / args.steps * 1e3
    log("device ms per step: " + ", ".join(f"{k} {v[1] / args.steps:.3f}" for k, v in kinds.items()))
    head = config_entry(n, args.steps, el, close_ms, window_ms, kinds, dom, dom_launches, dom_ms,
                        measured_traffic() if dom == "bin" else None)

    # the plain per-batch kernel: one thread per pair, global atomicOr into the sketches
    log(f"timing plain scan: 1 warmup + {args.plain_steps} steps")
    pel, pclose, pwin, _, _, prec, _, _ = run_detector(spd, torch, params, x, args.plain_steps, 1,
                                                       {"direct_max_pairs": 1 << 62})
    plain_value = n * args.plain_steps / pel
    assert np.array_equal(prec, rec), "plain and binned scans disagree"

    out = {
        "metric": "packets/s scanned (1 GPU, % HBM roofline); p99 window-close latency, batched vs plain",
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic (seeded; CAIDA-shaped core-network window)",
        "config": {
            "workload": "plain_64m: 1 router, 1 window of 64Mi (src,dst) uint32 pairs; 2M Zipf(1.1)<=500 "
                        "sources, 500 planted super points |OP| in [1024,20000], 30% duplicates, theta 1024",
            "method": {"r": w.params.r, "sr": w.params.sr, "a": w.params.a, "log2k": w.params.log2k,
                       "lr": w.params.lr, "log2lc": w.params.log2lc, "theta": w.params.theta},
            "step": "scan 64Mi pairs (binned LDS scan) + end of window (rebuild, filter, report, reset); "
                    "windows back to back, each report collected after the next window's scan is enqueued",
            "parallelism": "1 GPU",
        },
        "roofline": head["roofline"],
        "scan_ms_per_window": head["scan_ms_per_window"],
        "scan_roofline_frac": head["scan_roofline_frac"],
        "close_device_ms": kinds.get("close", (1, 0.0))[1] / max(1, kinds.get("close", (1, 0))[0]),
        "close_latency_ms": head["close_latency_ms"],
        "window_latency_ms": head["window_latency_ms"],
        "kernel_ms_per_step": head["kernel_ms_per_step"],
        "reported_super_points": int(len(rec)),
        "candidates": int(stats.candidates_last),
        "blocking_close": {"value": n * args.steps / el_blocking, "unit": "packets/s",
                           "ms_per_step": el_blocking / args.steps * 1e3,
                           "step": "scan, then spd_close_window (the host waits for each report before "
                                   "the next scan is enqueued)"},
        "tuning": {"autotuned": not args.no_autotune, "settings": tuned,
                   "candidates_ms": [[c, ms] for c, ms in tables["binned"]] if tuned else None},
        "plain": {
            "value": plain_value,
            "unit": "packets/s",
            "ms_per_step": pel / args.plain_steps * 1e3,
            "close_latency_ms": {"p50": pct(pclose, 50), "p99": pct(pclose, 99)},
            "window_latency_ms": {"p50": pct(pwin, 50), "p99": pct(pwin, 99)},
            "kernel": "direct (one thread per pair, global atomicOr)",
        },
        "batched_over_plain": value / plain_value,
        "gpu": torch.cuda.get_device_name(0),
    }

    log("both directions: one fused call, source- and destination-keyed")
    bpps, bms, bsizes = run_both_directions(spd, torch, params, x, args.plain_steps, 1, tuned)
    out["both_directions"] = {"value": bpps, "unit": "packets/s", "ms_per_step": bms,
                              "reported_super_points": {"source_keyed": bsizes[0], "destination_keyed": bsizes[1]},
                              "step": "scan of the window keyed both ways in one call + both ends of window"}

    log("host ingestion: page-locked host buffer, double-buffered copies overlapping the scan")
    hpps, hms = run_host_ingest(spd, torch, params, pairs, args.plain_steps, 1, tuned)
    out["host_ingest"] = {"value": hpps, "unit": "packets/s", "ms_per_step": hms, "bytes_per_pair": BYTES_PER_PAIR,
                          "host_link_GBps": hpps * BYTES_PER_PAIR / 1e9,
                          "step": "64Mi pairs from pinned host memory (16Mi-pair chunks) + end of window"}

    extra = {}
    configs = {}
    wanted = [c for c in args.configs.split(",") if c]
    if "plain_1m" in wanted:
        log("plain_1m: one 1,000,000-pair window")
        configs["plain_1m"], p1, r1 = bench_plain_1m(spd, torch, np, st, at, args.steps, args.warmup)
        extra["plain_1m"] = (p1, r1)
    if "routers_8x16m" in wanted:
        log("routers_8x16m: 8 routers fused, merged, global end of window")
        configs["routers_8x16m"], win8, r8 = bench_routers(spd, torch, np, st, at, max(5, args.steps // 4), 2)
        extra["routers_8x16m"] = (win8, r8)
    if "sliding_300x1m" in wanted:
        log("sliding_300x1m: 300 slices, window of 60")
        configs["sliding_300x1m"], slices, sreps = bench_sliding(spd, torch, np, st)
        extra["sliding_300x1m"] = (slices, sreps)
    torch.cuda.empty_cache()
    if configs:
        out["configs"] = configs

    if args.serving_windows > 0:
        log("serving loop: 16 routers")
        budget = int(args.serving_budget_gib * (1 << 30))
        loads = [float(v) for v in args.serving_loads.split(",")]
        out["serving"], pool_np, reports = bench_serving(spd, torch, np, st, value, args.serving_windows, loads,
                                                         tuned, budget, 48)
        extra["serving_16r"] = (pool_np, reports)

    if not args.no_cpu_baseline:
        import oracle
        out["cpu_baseline"], out["oracle_match"] = cpu_baseline_and_checks(oracle, np, st, pairs, rec, extra)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
