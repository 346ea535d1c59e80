"""Helpers for the GPU parity tests: move pairs to the device, run the HIP path, compare with the
oracle.  Imported only by tests."""
import sys

import numpy as np

import oracle
import synth_traffic as st


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def to_dev(pairs):
    import torch
    arr = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
    return torch.from_numpy(arr.view(np.int32)).to("cuda")


def set_tuning(det, **kw):
    t = det.tuning
    for k, v in kw.items():
        setattr(t, k, v)
    det.tuning = t


def oracle_sketch(mp, pairs, isb=None, ibn=None):
    return oracle.Sketch(oracle.params(mp, isb, ibn)).scan(pairs)


def assert_same_sketch(det, target, ref, what=""):
    seav, ldca = det.export(target)
    if not np.array_equal(seav, ref.seav):
        bad = np.flatnonzero(seav != ref.seav)
        raise AssertionError(f"{what}: SEAV differs at {bad.size} bytes, first {bad[:5]}")
    if not np.array_equal(ldca, ref.ldca):
        bad = np.flatnonzero(ldca != ref.ldca)
        raise AssertionError(f"{what}: LDCA differs at {bad.size} words, first {bad[:5]}")


def assert_same_report(got, want, what=""):
    want = want.astype(got.dtype)
    if not np.array_equal(got, want):
        g, w = set(got["ip"].tolist()), set(want["ip"].tolist())
        raise AssertionError(f"{what}: reports differ: gpu {len(got)} oracle {len(want)}; "
                             f"only gpu {sorted(g - w)[:5]} only oracle {sorted(w - g)[:5]}")


def random_pairs(rng, n, n_hosts=None):
    src = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    if n_hosts:
        hosts = rng.integers(0, 1 << 32, size=n_hosts, dtype=np.uint64).astype(np.uint32)
        src = hosts[rng.integers(0, n_hosts, size=n)]
    dst = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    return np.stack([src, dst], axis=1)


def heavy_hosts(rng, n_hosts, peers, noise=0):
    """n_hosts hosts with `peers` distinct peers each, plus `noise` random pairs, shuffled."""
    hosts = st.distinct_ips(rng, n_hosts)
    src = np.repeat(hosts, peers)
    dst = rng.integers(0, 1 << 32, size=src.size, dtype=np.uint64).astype(np.uint32)
    pairs = np.stack([src, dst], axis=1)
    if noise:
        pairs = np.concatenate([pairs, random_pairs(rng, noise)])
    return pairs[rng.permutation(len(pairs))], hosts


def oracle_sketch_threads(mp, parts, threads=8):
    """The oracle's sketch of the union of `parts`, each part scanned by its own thread into a private
    sketch, then OR-merged (the sketch depends only on the set of pairs)."""
    import threading
    p = oracle.params(mp)
    sks = [oracle.Sketch(p) for _ in parts]
    ths = [threading.Thread(target=s.scan, args=(np.ascontiguousarray(q),)) for s, q in zip(sks, parts)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    out = sks[0]
    for s in sks[1:]:
        out.merge(s)
    return out
