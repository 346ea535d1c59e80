#!/usr/bin/env python3
"""Benchmark of the super-point detection hot path on one MI355X.

One step = one window of the 64 Mi-pair workload (1 router): the scan of every pair into the
short estimator array vector and the long estimator array, then the end of window (candidate
rebuild from the SEAV, LDCA filter against theta, report, reset).  Inputs are seeded synthetic
traffic already resident in HBM when the timed region starts.

Prints ONE JSON line: throughput in packets (pairs) per second for the library's default
(binned) scan, the roofline of the dominant kernel (HIP events on the launch stream), p50/p99
end-of-window latency, the same figures for the plain per-batch kernel (one thread per pair,
global atomics), and the CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, public figure
BYTES_PER_PAIR = 8             # algorithmic HBM bytes per pair: one uint32 (hip, oip) record
PROFILE_TRAFFIC = os.path.join(ROOT, "profiles", "region_kernel_plain_64m_traffic.txt")


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


def run_detector(spd, torch, params, x, steps, warmup, tune):
    """Three passes of `steps` windows each (scan + end of window, the report on the host):
    1. every kernel kind timed with the library's HIP events: the per-kernel breakdown and the
       dominant kernel;
    2. the timed region: back-to-back windows, only the dominant kernel timed (two events per
       launch, so the timing hardly disturbs the run);
    3. untimed, a synchronisation after each scan: the end-of-window latency alone."""
    det = spd.Detector(params)
    t = det.tuning
    for k, v in tune.items():
        setattr(t, k, v)
    det.tuning = t
    for _ in range(warmup):
        det.scan(0, x)
        det.close_window(0)
    torch.cuda.synchronize()
    det.profile_enable(True)
    for _ in range(steps):
        det.scan(0, x)
        det.close_window(0)
    breakdown = {k: v for k, v in det.profile().items() if v[0]}
    dom = max(breakdown, key=lambda k: breakdown[k][1])
    det.profile_enable(True, kinds=[dom])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rec = None
    for _ in range(steps):
        det.scan(0, x)
        rec = det.close_window(0)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    timed = det.profile()[dom]
    det.profile_enable(False)
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
    return elapsed, close_ms, window_ms, breakdown, (dom, timed), rec, stats


def run_both_directions(spd, torch, params, x, steps, warmup):
    """Source- and destination-keyed super points of the same window: one fused scan call with the
    pairs as given (router 0) and swapped (router 1), then both ends of window.  Returns pairs/s
    (each pair counted once) and the two report sizes."""
    det = spd.Detector(params, n_routers=2)
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


def run_host_ingest(spd, torch, params, pairs_np, steps, warmup):
    """The window handed over in page-locked host memory: spd_scan_host copies it in 16 Mi-pair
    chunks on its own stream, each copy overlapping the scan of the previous chunk, then the end of
    window.  PCIe-inclusive pairs/s (the host link, not HBM, bounds this figure)."""
    import numpy as np
    host = torch.from_numpy(pairs_np.view(np.int32)).pin_memory()
    det = spd.Detector(params)
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


def bench_serving(spd, torch, np, st, capacity_pps, windows_per_router, load, log_fn):
    """The serving loop on the 16-router workload: batches of log-uniform size in [4Ki, 4Mi] pairs,
    Poisson arrivals at `load` x capacity_pps, a window closed every 64Mi pairs per router.  Router
    r's window w replays pool window (r + w) mod 4 of plain_64m-shaped traffic (1000 planted super
    points spread over the pool).  Returns throughput, window latencies and admission figures."""
    w = st.CONFIGS["serving_16r"]
    R, W = w.n_routers, w.n_packets
    pool = []
    for k in range(4):
        g = st.gen_plain(st.scaled(w, n_planted=w.n_planted // 4, seed=w.seed + k))
        pool.append(torch.from_numpy(g.pairs[0].view(np.int32)).to("cuda"))
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
    mean = total / n_batches
    rate = load * capacity_pps / mean          # batches per second over all routers
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
    srv = spd.Server(spd.params_from(w.params), n_routers=R, window_pairs=W, hbm_budget_bytes=2 << 30,
                     max_group_pairs=64 << 20, use_graphs=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    srv.replay(times, routers, tensors)
    lat = []
    for _ in range(R * windows_per_router):
        got = srv.next(timeout_ms=120000)
        if got is None:
            raise RuntimeError("serving: a window did not finish")
        lat.append(got[0]["latency_ms"])
    el = time.perf_counter() - t0
    stats = srv.stats
    srv.close()
    log_fn(f"serving load {load}: {total / el / 1e9:.1f} Gpairs/s, p50 {pct(lat, 50):.2f} ms, p99 {pct(lat, 99):.2f} ms")
    return {"offered_load": load, "offered_pairs_per_s": load * capacity_pps, "value": total / el,
            "unit": "packets/s", "routers": R, "windows": R * windows_per_router, "pairs": total,
            "batches": n_batches, "window_latency_ms": {"p50": pct(lat, 50), "p99": pct(lat, 99),
                                                        "max": max(lat)},
            "slots": stats["slots"], "admission_waits": stats["admission_waits"], "groups": stats["groups"]}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--plain-steps", type=int, default=5, help="steps for the plain per-batch kernel")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pmc-run", action="store_true",
                    help="short run for rocprofv3 counter collection: 2 windows + one 512 MiB copy for scaling")
    ap.add_argument("--serving-windows", type=int, default=1, help="windows per router in the serving run (0: skip)")
    ap.add_argument("--serving-loads", default="0.5,1.0", help="offered loads, fractions of the measured capacity")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path.  Several GPUs would each "
              "scan their routers' pairs into their own sketches and OR-combine them once per window.",
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1901_07306_amd as spd
    import synth_traffic as st

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 2
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

    # the library's default path (binned scan) -- the headline value
    log(f"timing default scan: {args.warmup} warmup + {args.steps} steps")
    el, close_ms, window_ms, kinds, (dom, (dom_launches, dom_ms)), rec, stats = run_detector(
        spd, torch, params, x, args.steps, args.warmup, {})
    value = n * args.steps / el
    ms_step = el / args.steps * 1e3
    avg_ms = dom_ms / dom_launches
    # every scan kernel launch covers all n pairs of the step: 8 B of algorithmic traffic per pair
    if dom not in ("bin", "transpose", "apply", "direct", "fill", "count", "offsets") or dom_launches != args.steps:
        raise RuntimeError(f"unexpected dominant kernel {dom} ({dom_launches} launches)")
    alg_bytes = BYTES_PER_PAIR * n
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    scan_kinds = ("bin", "transpose", "apply", "fill", "direct", "count", "offsets")
    scan_ms = sum(kinds.get(k, (0, 0.0))[1] for k in scan_kinds) / args.steps
    close_dev_ms = kinds.get("close", (0, 0.0))[1] / max(1, kinds.get("close", (1, 0))[0])
    traffic = measured_traffic()
    log("device ms per step: " + ", ".join(f"{k} {v[1] / args.steps:.3f}" for k, v in kinds.items()))

    # the plain per-batch kernel: one thread per pair, global atomicOr into the sketches
    log(f"timing plain scan: 1 warmup + {args.plain_steps} steps")
    pel, pclose, pwin, _, _, prec, _ = run_detector(spd, torch, params, x, args.plain_steps, 1,
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
            "step": "scan 64Mi pairs (binned LDS scan) + end of window (rebuild, filter, report, reset)",
            "parallelism": "1 GPU",
        },
        "roofline": {
            "kernel": dom,
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "alg_bytes_per_launch": alg_bytes,
            "avg_launch_ms": avg_ms,
            "launches": dom_launches,
        },
        "scan_ms_per_window": scan_ms,
        "scan_roofline_frac": (BYTES_PER_PAIR * n / (scan_ms * 1e-3) / 1e9) / HBM_PEAK_GBS,
        "close_device_ms": close_dev_ms,
        "close_latency_ms": {"p50": pct(close_ms, 50), "p99": pct(close_ms, 99)},
        "window_latency_ms": {"p50": pct(window_ms, 50), "p99": pct(window_ms, 99)},
        "kernel_ms_per_step": {k: v[1] / args.steps for k, v in kinds.items()},
        "reported_super_points": int(len(rec)),
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
    bpps, bms, bsizes = run_both_directions(spd, torch, params, x, args.plain_steps, 1)
    out["both_directions"] = {"value": bpps, "unit": "packets/s", "ms_per_step": bms,
                              "reported_super_points": {"source_keyed": bsizes[0], "destination_keyed": bsizes[1]},
                              "step": "scan of the window keyed both ways in one call + both ends of window"}

    log("host ingestion: page-locked host buffer, double-buffered copies overlapping the scan")
    hpps, hms = run_host_ingest(spd, torch, params, pairs, args.plain_steps, 1)
    out["host_ingest"] = {"value": hpps, "unit": "packets/s", "ms_per_step": hms, "bytes_per_pair": BYTES_PER_PAIR,
                          "host_link_GBps": hpps * BYTES_PER_PAIR / 1e9,
                          "step": "64Mi pairs from pinned host memory (16Mi-pair chunks) + end of window"}

    if args.serving_windows > 0:
        log("serving loop: 16 routers")
        out["serving"] = [bench_serving(spd, torch, np, st, value, args.serving_windows, float(ld), log)
                          for ld in args.serving_loads.split(",")]

    if not args.no_cpu_baseline:
        import oracle
        log("timing the CPU oracle on the host (one full window, single thread)")
        c0 = time.perf_counter()
        sk = oracle.Sketch(oracle.params(w.params)).scan(pairs)
        ref = sk.detect()
        cel = time.perf_counter() - c0
        out["cpu_baseline"] = {"value": n / cel, "unit": "packets/s", "cores": 1, "kind": "oracle",
                               "sample": "the full 64Mi-pair window once: scan + end of window, single thread",
                               "seconds": cel}
        out["oracle_match"] = bool(np.array_equal(ref.astype(rec.dtype), rec))
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
