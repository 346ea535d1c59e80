"""Autotuner for the scan launch settings of libspd.

Every setting gives identical sketch bits; only speed changes.  The tuner times the scan of a
representative device batch under each candidate setting (device time from the library's own
HIP-event profiler) and keeps the fastest.  It also finds the batch size above which the binned
scan beats the direct-atomic kernel, which decides the path per batch and the batch grouping of
the serving loop.  Results are cached in memory per (GPU name, method parameters, batch size).
"""
from __future__ import annotations

import itertools
from typing import Dict, List, Optional, Tuple

_CACHE: Dict[tuple, dict] = {}

SCAN_KINDS = ("direct", "bin", "transpose", "apply", "fill", "count", "offsets", "spill")
TUNED_FIELDS = ("bin_mode", "bucket_bits", "tile_pairs", "bin_block", "apply_block", "apply_unroll",
                "direct_block", "direct_grid_per_cu", "seav_lds", "direct_max_pairs")


def _scan_ms(det, x, reps: int, batches=None, merge: bool = False) -> float:
    """Device time of one scan of x into router 0, or of one fused call over `batches`
    ((router, tensor) pairs; with `merge`, the call that also ORs them into the global sketch, whose
    merge time then counts), averaged over reps; the routers are reset afterwards."""
    det.profile_enable(True)
    for _ in range(reps):
        if batches:
            det.scan_batches(batches, merge=merge)
        else:
            det.scan(0, x)
    prof = det.profile()
    det.profile_enable(False)
    if batches:
        for r in sorted({b[0] for b in batches}):
            det.reset(r)
    else:
        det.close_window(0)
    return sum(prof[k][1] for k in SCAN_KINDS + (("merge",) if merge else ())) / reps


def candidate_settings(quick: bool = False) -> List[dict]:
    """Binned-scan settings the tuner times: the layout (bin_mode), the LDS bucket size, the tile,
    the binning workgroup and the apply kernel's loads in flight per lane."""
    if quick:
        return [dict(bin_mode=2, bucket_bits=20, tile_pairs=8192, bin_block=1024, apply_block=1024, apply_unroll=16),
                dict(bin_mode=2, bucket_bits=20, tile_pairs=8192, bin_block=512, apply_block=1024, apply_unroll=16),
                dict(bin_mode=2, bucket_bits=20, tile_pairs=16384, bin_block=1024, apply_block=1024, apply_unroll=16),
                dict(bin_mode=2, bucket_bits=20, tile_pairs=8192, bin_block=1024, apply_block=1024, apply_unroll=32),
                dict(bin_mode=2, bucket_bits=20, tile_pairs=8192, bin_block=1024, apply_block=512, apply_unroll=16),
                dict(bin_mode=2, bucket_bits=20, tile_pairs=4096, bin_block=1024, apply_block=1024, apply_unroll=16),
                dict(bin_mode=2, bucket_bits=20, tile_pairs=4096, bin_block=512, apply_block=1024, apply_unroll=16),
                dict(bin_mode=1, bucket_bits=20, tile_pairs=8192, bin_block=1024, apply_block=1024, apply_unroll=16),
                dict(bin_mode=0, bucket_bits=20, tile_pairs=16384, bin_block=1024, apply_block=1024, apply_unroll=16),
                # small sketches: more, smaller buckets give the apply phase workgroups for every CU
                dict(bin_mode=2, bucket_bits=17, tile_pairs=4096, bin_block=1024, apply_block=256, apply_unroll=8),
                dict(bin_mode=2, bucket_bits=18, tile_pairs=4096, bin_block=1024, apply_block=512, apply_unroll=8)]
    out = []
    for mode, S, T, bb, u in itertools.product((0, 1, 2), (19, 20), (8192, 16384), (512, 1024), (8, 16)):
        out.append(dict(bin_mode=mode, bucket_bits=S, tile_pairs=T, bin_block=bb, apply_block=1024, apply_unroll=u))
    return out


def _apply(det, settings: dict) -> None:
    t = det.tuning
    for k, v in settings.items():
        setattr(t, k, v)
    det.tuning = t


def tune_binned(det, x, reps: int = 3, quick: bool = False, batches=None,
                merge: bool = False) -> Tuple[dict, List[Tuple[dict, float]]]:
    """Fastest binned-scan setting for batch x on detector det (router 0 is used and reset), or for
    the fused call over `batches` when given (the routers named there are reset)."""
    base = det.tuning
    table = []
    for cand in candidate_settings(quick):
        try:
            _apply(det, dict(cand, direct_max_pairs=0))
        except Exception:
            continue
        _scan_ms(det, x, 1, batches, merge)   # warm-up (scratch growth)
        table.append((cand, _scan_ms(det, x, reps, batches, merge)))
    det.tuning = base
    best = min(table, key=lambda e: e[1])[0]
    return best, table


def tune_direct(det, x, reps: int = 3) -> Tuple[dict, List[Tuple[dict, float]]]:
    base = det.tuning
    table = []
    for block, per_cu, lds in itertools.product((256, 512), (4, 8, 16), (0, 1)):
        cand = dict(direct_block=block, direct_grid_per_cu=per_cu, seav_lds=lds)
        _apply(det, dict(cand, direct_max_pairs=1 << 62))
        _scan_ms(det, x, 1)
        table.append((cand, _scan_ms(det, x, reps)))
    det.tuning = base
    return min(table, key=lambda e: e[1])[0], table


def crossover(det, x, sizes=(1 << 14, 1 << 16, 1 << 18, 1 << 20, 1 << 22), reps: int = 5) -> int:
    """Largest tested batch size at which the direct kernel is still at least as fast."""
    base = det.tuning
    best = 0
    for n in sizes:
        if n > x.shape[0]:
            break
        xs = x[:n]
        t = det.tuning
        t.direct_max_pairs = 1 << 62
        det.tuning = t
        _scan_ms(det, xs, 1)
        d = _scan_ms(det, xs, reps)
        t.direct_max_pairs = 0
        det.tuning = t
        _scan_ms(det, xs, 1)
        b = _scan_ms(det, xs, reps)
        if d <= b:
            best = n
    det.tuning = base
    return best


def autotune(det, x, key: Optional[tuple] = None, quick: bool = False, batches=None, merge: bool = False) -> dict:
    """Tune det for batches like x and apply the result.  With `batches` ((router, tensor) pairs of
    one fused call; `merge`: the call that also merges them into the global sketch), the binned
    settings are those of that fused call; the direct kernel's shape and
    the direct/binned crossover are still tuned on x.  Returns the chosen settings; the timing tables
    are kept in the cache entry (``last_tables(key)``)."""
    import torch
    key = key or cache_key(det, x, batches, merge)
    if key not in _CACHE:
        b, tb = tune_binned(det, x, quick=quick, batches=batches, merge=merge)
        d, td = tune_direct(det, x[: min(x.shape[0], 1 << 20)])
        cross = crossover(det, x)
        _CACHE[key] = dict(settings=dict(b, **d, direct_max_pairs=cross), binned=tb, direct=td,
                           gpu=torch.cuda.get_device_name(0))
    _apply(det, _CACHE[key]["settings"])
    return dict(_CACHE[key]["settings"])


def cache_key(det, x, batches=None, merge: bool = False) -> tuple:
    import torch
    p = det.params
    fused = tuple((int(r), int(t.shape[0])) for r, t in batches) if batches else ()
    return (torch.cuda.get_device_name(0), tuple(p.hash_mul[:3]), p.r, p.sr, p.log2k, p.lr, p.log2lc,
            int(x.shape[0]), fused, bool(merge))


def last_tables(key: tuple) -> dict:
    """The timing tables behind a cached choice: binned candidates and direct-kernel settings (ms)."""
    e = _CACHE[key]
    return {"binned": [(c, ms) for c, ms in e["binned"]], "direct": [(c, ms) for c, ms in e["direct"]]}


def tuning_of(det, settings: dict):
    """An spd_tuning structure: det's current tuning with the given settings applied."""
    t = det.tuning
    for k, v in settings.items():
        setattr(t, k, v)
    return t
