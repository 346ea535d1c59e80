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


def sampled_oips(mp, n, rng):
    """n distinct destinations that the sampling of Section 3.1 keeps for parameters mp: the low tau
    bits of H1(oip) zero (tau from Eq. 1), found with the oracle's hash."""
    mul, add = mp.hashes()
    mask = (1 << oracle.tau(mp.theta)) - 1
    out = set()
    while len(out) < n:
        for x in rng.integers(0, 1 << 32, size=2 * (n - len(out)) + 16, dtype=np.uint64).tolist():
            if oracle.hash32(x, mul[0], add[0], 32) & mask == 0:
                out.add(x)
    return np.array(sorted(out)[:n], np.uint32)


def overflow_traffic(mp, rng, n_hosts, peers, noise):
    """Pairs with a contiguous run of n_hosts * peers pairs whose destinations are all sampled
    (n_hosts hosts with `peers` distinct sampled peers each, shuffled within the run), between two
    halves of `noise` random pairs.  With tau >= 1 every binning tile inside the run has more
    sampled pairs than it stages (about half its pairs, plus a margin).  Returns (pairs, hosts)."""
    pool = sampled_oips(mp, max(4 * peers, 4096), rng)
    hosts = st.distinct_ips(rng, n_hosts)
    run = np.concatenate([np.stack([np.full(peers, h, np.uint32),
                                    pool[rng.choice(pool.size, size=peers, replace=False)]], axis=1)
                          for h in hosts])
    run = run[rng.permutation(len(run))]
    a = random_pairs(rng, noise // 2)
    b = random_pairs(rng, noise - noise // 2)
    return np.concatenate([a, run, b]), hosts
