"""GPU parity: the HIP path through the C ABI against the CPU oracle, bit-exact.

Sketch bits (SEAV bytes and LDCA words) and the reported super points (ip, z0, est, flags) must
be identical to the oracle's on the same seeded inputs.  The cases cover both scan kernels
(direct atomics and LDS-binned), tiny tiles that give many buckets and ragged tails, every row
count the binned kernel supports, router merges, window resets, import/export, edge inputs,
saturated SEAs (the brute-force branch of the end-of-window kernel), the sliding window, and the
full-size 1,000,000-pair and 64 Mi-pair windows.
"""
import zlib

import numpy as np
import pytest

import oracle
import synth_traffic as st
from gpu_util import (assert_same_report, assert_same_sketch, heavy_hosts, log, oracle_sketch, overflow_traffic,
                      random_pairs, set_tuning, to_dev)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402

DIRECT = dict(direct_max_pairs=1 << 62)
# bin_mode 0: per-tile item regions; the library default is the region layout (bin_mode 2)
BINNED_SMALL = dict(direct_max_pairs=0, bin_mode=0, tile_pairs=2048, bucket_bits=12, bin_block=512, apply_block=256,
                    apply_unroll=8)
BINNED_DEFAULT = dict(direct_max_pairs=0)
BINNED_TILES = dict(direct_max_pairs=0, bin_mode=0)
BINNED_CHUNKED = dict(direct_max_pairs=0, bin_mode=0, launch_pairs=50_000, tile_pairs=16384, apply_unroll=32)
BUCKET_MAJOR = dict(direct_max_pairs=0, bin_mode=1)
BUCKET_MAJOR_SMALL = dict(direct_max_pairs=0, bin_mode=1, tile_pairs=2048, bucket_bits=12, bin_block=512,
                          apply_block=256, launch_pairs=70_000)
BUCKET_MAJOR_WIDE = dict(direct_max_pairs=0, bin_mode=1, tile_pairs=8192, apply_unroll=32)
# bin_mode 2: fixed-capacity (chunk, bucket) regions; region_words forces words onto the spill list
REGION = dict(direct_max_pairs=0, bin_mode=2)
REGION_SMALL = dict(direct_max_pairs=0, bin_mode=2, tile_pairs=2048, bucket_bits=12, bin_block=512, apply_block=256,
                    launch_pairs=70_000)
REGION_SPILL = dict(direct_max_pairs=0, bin_mode=2, region_words=5, apply_unroll=8)
REGION_SPILL_ALL = dict(direct_max_pairs=0, bin_mode=2, region_words=1, tile_pairs=4096, bin_block=512,
                        apply_unroll=32)


def detector(mp, n_routers=1, isb=None, ibn=None, **tune):
    det = spd.Detector(spd.params_from(mp, isb, ibn), n_routers=n_routers)
    if tune:
        set_tuning(det, **tune)
    return det


PARAMS = {
    "tiny_r20_sr3": st.MethodParams(theta=256, r=20, sr=3, a=1, log2k=10, lr=2, log2lc=6, hash_seed=7),
    "plain_1m": st.CONFIGS["plain_1m"].params,
    "lr1_sr2": st.MethodParams(theta=1024, r=10, sr=2, a=3, log2k=12, lr=1, log2lc=10, hash_seed=11),
    "lr3_sr5": st.MethodParams(theta=512, r=12, sr=5, a=2, log2k=11, lr=3, log2lc=9, hash_seed=13),
    "lr4_sr4": st.MethodParams(theta=2048, r=8, sr=4, a=2, log2k=13, lr=4, log2lc=7, hash_seed=17),
    # a 32 KiB SEAV: small enough for the direct kernel's per-workgroup LDS copy
    "seav_32k": st.MethodParams(theta=1024, r=4, sr=4, a=2, log2k=12, lr=2, log2lc=10, hash_seed=19),
}


MODES = {"direct": DIRECT, "binned_small": BINNED_SMALL, "binned_default": BINNED_DEFAULT,
         "binned_chunked": BINNED_CHUNKED, "bucket_major": BUCKET_MAJOR, "bucket_major_small": BUCKET_MAJOR_SMALL,
         "bucket_major_wide": BUCKET_MAJOR_WIDE, "region": REGION, "region_small": REGION_SMALL,
         "region_spill": REGION_SPILL, "region_spill_all": REGION_SPILL_ALL,
         # the direct kernel's per-workgroup LDS copy of the SEAV (taken when the SEAV is at most 64 KiB)
         "direct_seav_lds": dict(DIRECT, seav_lds=1),
         # end-of-window workgroups of one and two wavefronts
         "direct_close64": dict(DIRECT, close_block=64),
         "region_close128": dict(REGION, close_block=128)}


def seed_of(*names) -> int:
    """A fixed seed per test case (CRC-32 of its name), the same in every process."""
    return zlib.crc32("/".join(names).encode())


@pytest.mark.parametrize("pname", list(PARAMS))
@pytest.mark.parametrize("mode", list(MODES))
def test_scan_and_close_parity(pname, mode):
    mp = PARAMS[pname]
    seed = seed_of(pname, mode)
    log(f"case params={pname} mode={mode} seed={seed}")
    tune = MODES[mode]
    rng = np.random.default_rng(seed)
    heavy, _ = heavy_hosts(rng, 8, 3000, noise=150_001)   # ragged: not a multiple of any tile
    det = detector(mp, **tune)
    try:
        # three uneven batches into one window
        cuts = [0, 1, 70_001, len(heavy)]
        for a, b in zip(cuts[:-1], cuts[1:]):
            det.scan(0, to_dev(heavy[a:b]))
        ref = oracle_sketch(mp, heavy)
        assert_same_sketch(det, 0, ref, f"{pname}/{mode}")
        got = det.close_window(0)
        assert_same_report(got, ref.detect(), f"{pname}/{mode}")
        # the window was reset: an empty window reports nothing and exports zeros
        seav, ldca = det.export(0)
        assert not seav.any() and not ldca.any()
        assert len(det.close_window(0)) == 0
    finally:
        det.close()


def test_empty_single_and_extreme_ips():
    mp = PARAMS["plain_1m"]
    log("case empty/single/extreme")
    det = detector(mp, **DIRECT)
    try:
        det.scan(0, to_dev(np.zeros((0, 2), np.uint32)))
        assert not det.export(0)[1].any()
        pairs = np.array([[0, 0], [0xFFFFFFFF, 0xFFFFFFFF], [0, 0xFFFFFFFF], [0xFFFFFFFF, 0]], np.uint32)
        det.scan(0, to_dev(pairs[:1]))
        det.scan(0, to_dev(pairs[1:]))
        assert_same_sketch(det, 0, oracle_sketch(mp, pairs), "extreme ips")
    finally:
        det.close()


def test_oip_whose_h1_is_zero_is_sampled():
    """lsb(0) = 32 >= tau: choose the H1 addend so that H1(x0) = 0 exactly and check parity."""
    base = PARAMS["tiny_r20_sr3"]
    x0 = 0x12345678
    mul, add = base.hashes()
    add[0] = (-(mul[0] * x0)) % (1 << 64)
    assert oracle.hash32(x0, mul[0], add[0], 32) == 0
    p = spd.make_params(base.theta, base.r, base.sr, base.a, base.log2k, base.lr, base.log2lc, mul, add)
    pairs = np.array([[0xCAFEBABE, x0]], np.uint32)
    for tune in (DIRECT, BINNED_SMALL):
        det = spd.Detector(p)
        set_tuning(det, **tune)
        try:
            det.scan(0, to_dev(pairs))
            op = oracle.params(base)
            for j in range(3 + base.lr):
                op.mul[j], op.add[j] = mul[j], add[j]
            ref = oracle.Sketch(op).scan(pairs)
            assert ref.seav.any()          # sampled
            assert_same_sketch(det, 0, ref, "h1=0")
        finally:
            det.close()


@pytest.mark.parametrize("mode", ["direct", "binned_small", "bucket_major_small", "region_small", "region_spill"])
def test_routers_fused_batches_and_merge(mode):
    mp = PARAMS["tiny_r20_sr3"].replace(theta=512)
    log(f"case routers mode={mode}")
    tune = MODES[mode]
    rng = np.random.default_rng(5)
    R = 5
    det = detector(mp, n_routers=R, **tune)
    try:
        heavy, _ = heavy_hosts(rng, 10, 2000, noise=60_000)
        owner = rng.integers(0, R, size=len(heavy))
        per = [heavy[owner == r] for r in range(R)]
        batches = []
        for r in range(R):
            cuts = np.sort(rng.integers(0, len(per[r]), size=3))
            cuts = [0, *cuts.tolist(), len(per[r])]
            for a, b in zip(cuts[:-1], cuts[1:]):
                batches.append((r, to_dev(per[r][a:b])))
        order = rng.permutation(len(batches))
        det.scan_batches([batches[i] for i in order])
        refs = [oracle_sketch(mp, per[r]) for r in range(R)]
        for r in range(R):
            assert_same_sketch(det, r, refs[r], f"router {r}")
        det.merge([3, 1, 4, 0, 2, 1])            # any order, duplicates ignored
        glob = oracle_sketch(mp, heavy)
        assert_same_sketch(det, spd.GLOBAL, glob, "merged")
        assert_same_report(det.close_window(spd.GLOBAL), glob.detect(), "global close")
        # merging a subset == the oracle on that subset (a router dropped at close)
        det.merge([0, 2])
        sub = oracle_sketch(mp, np.concatenate([per[0], per[2]]))
        assert_same_sketch(det, spd.GLOBAL, sub, "subset merge")
        # per-router close reports that router's own detection and resets only it
        assert_same_report(det.close_window(1), refs[1].detect(), "router close")
        assert not det.export(1)[1].any()
        assert_same_sketch(det, 2, refs[2], "router 2 untouched")
    finally:
        det.close()


def test_import_export_roundtrip_and_determinism():
    mp = PARAMS["plain_1m"]
    rng = np.random.default_rng(9)
    heavy, _ = heavy_hosts(rng, 12, 2500, noise=100_000)
    ref = oracle_sketch(mp, heavy)
    det = detector(mp, n_routers=2)
    try:
        det.import_(1, ref.seav, ref.ldca)
        assert_same_sketch(det, 1, ref, "imported")
        assert_same_report(det.close_window(1), ref.detect(), "close after import")
        for _ in range(2):   # same bits on repeated runs
            det.scan(0, to_dev(heavy))
            assert_same_sketch(det, 0, ref, "repeat")
            det.close_window(0)
    finally:
        det.close()


def test_saturated_sea_uses_brute_force_branch():
    """SEAs where every cell is hot: the tuple product exceeds 2^L, so the end-of-window kernel
    tests every LP of the SEA instead; the report must still equal the oracle's."""
    mp = st.MethodParams(theta=64, r=20, sr=4, a=1, log2k=9, lr=2, log2lc=8, hash_seed=23)
    rng = np.random.default_rng(31)
    rps = np.array([5, 77, 4000], np.uint32)
    n = 60_000
    lp = rng.integers(0, 1 << 12, size=n, dtype=np.uint64).astype(np.uint32)
    src = (lp << np.uint32(20)) | rps[rng.integers(0, len(rps), size=n)]
    dst = rng.integers(0, 1 << 32, size=n, dtype=np.uint64).astype(np.uint32)
    pairs = np.stack([src, dst], axis=1)
    ref = oracle_sketch(mp, pairs)
    cand = ref.candidates()
    assert len(cand) > 3 * 1000
    det = detector(mp, **DIRECT)
    try:
        det.scan(0, to_dev(pairs))
        assert_same_sketch(det, 0, ref, "saturated")
        got = det.close_window(0)
        assert_same_report(got, ref.detect(), "saturated close")
        assert det.stats.candidates_last == len(cand)
    finally:
        det.close()


def test_many_reports_grow_record_buffer():
    """More super points than the initial device record buffer (65536) holds."""
    mp = st.MethodParams(theta=8, r=16, sr=4, a=2, log2k=6, lr=2, log2lc=16, hash_seed=41)
    rng = np.random.default_rng(43)
    pairs, hosts = heavy_hosts(rng, 90_000, 24)
    ref = oracle_sketch(mp, pairs)
    want = ref.detect()
    assert len(want) > 65536
    det = detector(mp, direct_max_pairs=0)
    try:
        det.scan(0, to_dev(pairs))
        got = det.close_window(0, cap=200_000)
        assert_same_report(got, want, "many reports")
        with pytest.raises(spd.SpdError):
            det.scan(0, to_dev(pairs))
            det.close_window(0, cap=10)
    finally:
        det.close()


def test_error_paths():
    mp = PARAMS["plain_1m"]
    det = detector(mp, n_routers=2)
    try:
        x = to_dev(np.zeros((10, 2), np.uint32))
        with pytest.raises(spd.SpdError) as e:
            det.scan(2, x)
        assert e.value.status == spd.SPD_E_STATE
        with pytest.raises(spd.SpdError) as e:
            det.slide()
        assert e.value.status == spd.SPD_E_STATE
        with pytest.raises(spd.SpdError) as e:
            det.close_window(7)
        assert e.value.status == spd.SPD_E_STATE
        # misaligned pair pointer (4 bytes past an 8-byte boundary)
        lib = spd.lib()
        st_ = lib.spd_scan(det.ctx, 0, x.data_ptr() + 4, 1, None)
        assert st_ == spd.SPD_E_INVALID
        # tunings out of range are refused and leave the previous tuning in place
        before = det.tuning.bin_mode
        for bad in (dict(bin_mode=3), dict(region_words=(1 << 24) + 1), dict(apply_unroll=12)):
            with pytest.raises(spd.SpdError) as e:
                set_tuning(det, **bad)
            assert e.value.status == spd.SPD_E_INVALID
        assert det.tuning.bin_mode == before
    finally:
        det.close()
    # HBM budget: the sketches alone exceed it
    with pytest.raises(spd.SpdError) as e:
        spd.Detector(spd.params_from(st.CONFIGS["plain_64m"].params), n_routers=4, hbm_budget_bytes=100 << 20)
    assert e.value.status == spd.SPD_E_NOMEM


# ------------------------------------------------------------------------------ sliding window
@pytest.mark.parametrize("counter", ["at_pool", "stamps16"])
@pytest.mark.parametrize("mode", ["one_router", "merged"])
def test_sliding_window_parity(mode, counter):
    K = 4
    mp = st.MethodParams(theta=256, r=12, sr=4, a=2, log2k=10, lr=2, log2lc=8, window_slices=K, hash_seed=51,
                         sliding_counter=0 if counter == "at_pool" else 1)
    log(f"case sliding {mode} {counter}")
    rng = np.random.default_rng(53)
    R = 1 if mode == "one_router" else 3
    det = detector(mp, n_routers=R, direct_max_pairs=0)
    sl = [oracle.SlidingSketch(oracle.params(mp), K) for _ in range(R)]
    slices = []
    try:
        for t in range(11):
            if t:
                det.slide()
            pairs, _ = heavy_hosts(rng, 3, int(rng.integers(100, 400)), noise=20_000 + t)
            owner = rng.integers(0, R, size=len(pairs))
            for r in range(R):
                det.scan(r, to_dev(pairs[owner == r]))
                sl[r].scan_slice(pairs[owner == r], t)
            slices.append(pairs)
            assert spd.spd_current_slice(det.ctx) == t
            if mode == "one_router":
                ts_seav, ts_ldca = det.export_stamps(0)
                if counter == "stamps16":
                    np.testing.assert_array_equal(ts_seav, sl[0].seav_ts)
                    np.testing.assert_array_equal(ts_ldca, sl[0].ldca_ts)
                else:
                    # every counter left by maintenance holds the exact last slice, and every
                    # counter active in the window is left
                    for got_ts, want_ts in ((ts_seav, sl[0].seav_ts), (ts_ldca, sl[0].ldca_ts)):
                        kept = got_ts != 0
                        np.testing.assert_array_equal(got_ts[kept], want_ts[kept])
                        live = want_ts >= max(1, t - K + 2)
                        np.testing.assert_array_equal(got_ts[live], want_ts[live])
                view = sl[0].bit_view(t)
                assert_same_sketch(det, 0, view, f"slice {t}")
                assert_same_report(det.close_window(0), view.detect(), f"slice {t} close")
            else:
                det.merge(list(range(R)))
                union = oracle_sketch(mp, np.concatenate(slices[max(0, t - K + 1): t + 1]))
                assert_same_sketch(det, spd.GLOBAL, union, f"merged slice {t}")
                assert_same_report(det.close_window(spd.GLOBAL), union.detect(), f"merged close {t}")
    finally:
        det.close()


# ------------------------------------------------------------------------------ full size
def test_plain_1m_full_window():
    w = st.CONFIGS["plain_1m"]
    log("case plain_1m full")
    win = st.gen_plain(w)
    ref = oracle_sketch(w.params, win.pairs[0])
    for tune in (DIRECT, BINNED_DEFAULT):
        det = detector(w.params, **tune)
        try:
            det.scan(0, to_dev(win.pairs[0]))
            assert_same_sketch(det, 0, ref, "plain_1m")
            got = det.close_window(0)
            assert_same_report(got, ref.detect(), "plain_1m")
            assert sorted(got["ip"].tolist()) == sorted(win.planted_ips.tolist())
        finally:
            det.close()


def test_plain_64m_full_window():
    w = st.CONFIGS["plain_64m"]
    log("case plain_64m full: generating")
    win = st.gen_plain(w)
    log("case plain_64m full: oracle")
    ref = oracle_sketch(w.params, win.pairs[0])
    want = ref.detect()
    x = to_dev(win.pairs[0])
    # default tuning (the configuration the benchmark times), then the per-tile item layout
    for name, tune in (("default", {}), ("tiles", BINNED_TILES), ("bucket-major", BUCKET_MAJOR), ("regions", REGION)):
        log(f"case plain_64m full: gpu {name}")
        det = detector(w.params, **tune)
        try:
            det.scan(0, x)
            assert_same_sketch(det, 0, ref, f"plain_64m {name}")
            got = det.close_window(0)
            assert_same_report(got, want, f"plain_64m {name}")
            assert len(got) >= 490   # sanity: (nearly) all 500 planted hosts are reported
        finally:
            det.close()


def test_overflow_tiles_every_layout():
    """Tiles with more sampled pairs than they stage (a run of pairs whose destinations are all
    sampled, tau = 1): the per-tile and exact-count layouts record their SEAV bits directly (the
    counting pass must leave them out consistently), the region layout lists the tiles for its
    spill pass."""
    mp = st.CONFIGS["plain_64m"].params.replace(theta=16)   # tau = 1: about half the pairs sampled
    rng = np.random.default_rng(71)
    pairs, _ = overflow_traffic(mp, rng, 12, 2500, noise=30_000)
    for tune in (BUCKET_MAJOR, BUCKET_MAJOR_SMALL, BINNED_TILES, REGION, REGION_SMALL):
        det = detector(mp, **tune)
        try:
            det.scan(0, to_dev(pairs))
            ref = oracle_sketch(mp, pairs)
            assert_same_sketch(det, 0, ref, f"overflow {tune}")
            assert_same_report(det.close_window(0, cap=1 << 18), ref.detect(), "overflow report")
        finally:
            det.close()


def test_many_batches_one_call_binned():
    """More batches in one fused call than one launch takes: the call is split into launch groups
    and later groups must OR into the slots the earlier ones wrote."""
    mp = PARAMS["plain_1m"]
    rng = np.random.default_rng(61)
    pairs, _ = heavy_hosts(rng, 6, 2200, noise=90_000)
    cuts = np.sort(rng.choice(np.arange(1, len(pairs)), size=70, replace=False))
    parts = np.split(pairs, cuts)
    owner = [0 if i % 3 else 1 for i in range(len(parts))]
    for tune in (BINNED_SMALL, BUCKET_MAJOR_SMALL, REGION_SMALL, REGION_SPILL):
        det = detector(mp, n_routers=2, **tune)
        try:
            det.scan_batches([(o, to_dev(p)) for o, p in zip(owner, parts)])
            for r in range(2):
                mine = np.concatenate([p for o, p in zip(owner, parts) if o == r])
                assert_same_sketch(det, r, oracle_sketch(mp, mine), f"router {r}")
        finally:
            det.close()


@pytest.mark.parametrize("layout", [1, 2])
def test_thousands_of_batches_one_call(layout):
    """More batches in one fused call than the descriptor ring holds at first (1024): the ring grows,
    every tile finds its batch by binary search, and three routers' sketches equal the oracle's."""
    mp = PARAMS["plain_1m"]
    rng = np.random.default_rng(67)
    pairs, _ = heavy_hosts(rng, 5, 2500, noise=1_400_000)
    cuts = np.sort(rng.choice(np.arange(1, len(pairs)), size=1499, replace=False))
    parts = np.split(pairs, cuts)
    owner = rng.integers(0, 3, size=len(parts))
    log(f"case {len(parts)} batches in one call, bin_mode {layout}")
    det = detector(mp, n_routers=3, direct_max_pairs=0, bin_mode=layout)
    try:
        x = to_dev(pairs)
        starts = np.concatenate([[0], cuts])
        det.scan_batches([(int(o), x[a:a + len(p)]) for o, a, p in zip(owner, starts, parts)])
        for r in range(3):
            mine = np.concatenate([p for o, p in zip(owner, parts) if o == r])
            ref = oracle_sketch(mp, mine)
            assert_same_sketch(det, r, ref, f"router {r}")
            assert_same_report(det.close_window(r), ref.detect(), f"router {r}")
    finally:
        det.close()


@pytest.mark.parametrize("n_batches", [1, 8, 9, 40])
def test_batches_inline_and_from_device_memory(n_batches):
    """Up to 8 batches of a region launch travel in the kernel arguments, more in device memory:
    both sides of the boundary, batches of two routers interleaved, equal the oracle."""
    mp = PARAMS["plain_1m"]
    rng = np.random.default_rng(97 + n_batches)
    pairs, _ = heavy_hosts(rng, 4, 2500, noise=150_003)
    cuts = np.sort(rng.choice(np.arange(1, len(pairs)), size=n_batches - 1, replace=False))
    parts = np.split(pairs, cuts)
    owner = [i % 2 for i in range(len(parts))]
    log(f"case {n_batches} batches, region layout")
    det = detector(mp, n_routers=2, **REGION)
    try:
        x = to_dev(pairs)
        starts = np.concatenate([[0], cuts])
        det.scan_batches([(o, x[a:a + len(p)]) for o, a, p in zip(owner, starts, parts)])
        for r in range(2):
            mine = np.concatenate([p for o, p in zip(owner, parts) if o == r] or [np.zeros((0, 2), np.uint32)])
            ref = oracle_sketch(mp, mine)
            assert_same_sketch(det, r, ref, f"router {r}")
            assert_same_report(det.close_window(r), ref.detect(), f"router {r}")
    finally:
        det.close()


def test_scan_larger_than_one_launch():
    """A call over more pairs than one launch's 32-bit item offsets allow (about 1.79 Gi pairs at
    plain_64m sizes) is split into launches; the sketch is a function of the set of pairs, so it
    equals the sketch of the same pairs scanned in four calls (far too many pairs for the oracle)."""
    mp = st.CONFIGS["plain_64m"].params
    n = 2 << 30
    gen = torch.Generator(device="cuda").manual_seed(2024)
    x = torch.randint(-(1 << 31), (1 << 31) - 1, (n, 2), dtype=torch.int32, device="cuda", generator=gen)
    log(f"case {n} pairs in one call")
    one, four = detector(mp, **REGION), detector(mp, **REGION)
    try:
        one.scan(0, x)
        for k in range(4):
            four.scan(0, x[k * (n // 4):(k + 1) * (n // 4)])
        torch.cuda.synchronize()
        assert one.stats.binned_launches >= 2
        a, b = one.export(0), four.export(0)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        assert a[1].any()
    finally:
        one.close()
        four.close()
        del x
        torch.cuda.empty_cache()


# ------------------------------------------------------------------------------ both directions
@pytest.mark.parametrize("mode", ["direct", "binned_small", "binned_default", "bucket_major_small", "region_spill"])
def test_both_directions_one_call(mode):
    """Source-keyed and destination-keyed super points of the same pairs in one fused call: router 0
    reads records as (hip, oip), router 1 as (oip, hip); each equals the oracle on the pairs as
    given and on the swapped pairs."""
    mp = PARAMS["plain_1m"]
    rng = np.random.default_rng(83)
    src_heavy, _ = heavy_hosts(rng, 4, 2500, noise=120_000)
    dst_heavy, _ = heavy_hosts(rng, 4, 2500, noise=0)
    pairs = np.concatenate([src_heavy, dst_heavy[:, ::-1]])   # super points on both sides
    pairs = np.ascontiguousarray(pairs[rng.permutation(len(pairs))])
    log(f"case both directions mode={mode}")
    det = detector(mp, n_routers=2, **MODES[mode])
    try:
        x = to_dev(pairs)
        half = len(pairs) // 2
        det.scan_batches([(0, x[:half]), (1, x[:half], spd.BATCH_DST), (0, x[half:]), (1, x[half:], spd.BATCH_DST)])
        for r, view in ((0, pairs), (1, np.ascontiguousarray(pairs[:, ::-1]))):
            ref = oracle_sketch(mp, view)
            assert_same_sketch(det, r, ref, f"router {r}")
            got = det.close_window(r)
            assert_same_report(got, ref.detect(), f"router {r}")
            assert len(got) >= 4
    finally:
        det.close()


def test_both_directions_sliding():
    mp = st.CONFIGS["plain_1m"].params.replace(window_slices=3)
    rng = np.random.default_rng(89)
    p = oracle.params(mp)
    det = detector(mp, n_routers=2)
    sk = [oracle.SlidingSketch(p, 3), oracle.SlidingSketch(p, 3)]
    try:
        for t in range(4):
            if t:
                det.slide()
            pairs, _ = heavy_hosts(rng, 2, 1500, noise=40_000)
            x = to_dev(pairs)
            det.scan_batches([(0, x), (1, x, spd.BATCH_DST)])
            sk[0].scan_slice(pairs, t)
            sk[1].scan_slice(np.ascontiguousarray(pairs[:, ::-1]), t)
            for r in range(2):
                assert_same_report(det.close_window(r), sk[r].bit_view(t).detect(), f"slice {t} router {r}")
    finally:
        det.close()


# ------------------------------------------------------------------------------ host ingestion
@pytest.mark.parametrize("pinned", [False, True])
def test_scan_from_host_memory(pinned):
    """Pairs handed over in host memory, in chunks through the double-buffered staging (a ragged
    last chunk; small chunks take the direct kernel, large ones the binned scan), both keyings."""
    mp = PARAMS["plain_1m"]
    rng = np.random.default_rng(97)
    pairs, _ = heavy_hosts(rng, 5, 2500, noise=700_001)
    host = torch.from_numpy(pairs.view(np.int32)).pin_memory() if pinned else pairs
    log(f"case host ingestion pinned={pinned}")
    det = detector(mp, n_routers=2)
    try:
        det.scan_host(0, host, chunk_pairs=300_000)
        det.scan_host(1, host, flags=spd.BATCH_DST, chunk_pairs=100_000)
        for r, view in ((0, pairs), (1, np.ascontiguousarray(pairs[:, ::-1]))):
            ref = oracle_sketch(mp, view)
            assert_same_sketch(det, r, ref, f"router {r}")
            assert_same_report(det.close_window(r), ref.detect(), f"router {r}")
    finally:
        det.close()
