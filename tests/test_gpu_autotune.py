"""The autotuner's search space is exact: every candidate setting it may choose (binned layouts,
bucket sizes, tiles, workgroups, loads in flight; direct-kernel shapes and the per-workgroup SEAV
copy) gives the oracle's SEAV and LDCA bits and report, and the tuner's choice is applied."""
import numpy as np
import pytest

import synth_traffic as st
from gpu_util import assert_same_report, assert_same_sketch, heavy_hosts, log, oracle_sketch, set_tuning, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1901_07306_amd as spd  # noqa: E402
from paper_1901_07306_amd import autotune  # noqa: E402

PARAMS = {"plain_1m": st.CONFIGS["plain_1m"].params,
          "lr4_sr4": st.MethodParams(theta=2048, r=8, sr=4, a=2, log2k=13, lr=4, log2lc=7, hash_seed=17)}


@pytest.mark.parametrize("pname", list(PARAMS))
def test_every_candidate_setting_is_exact(pname):
    mp = PARAMS[pname]
    rng = np.random.default_rng(4001 + len(pname))
    pairs, _ = heavy_hosts(rng, 6, 2500, noise=400_001)
    ref = oracle_sketch(mp, pairs)
    want = ref.detect()
    x = to_dev(pairs)
    det = spd.Detector(spd.params_from(mp))
    try:
        cands = autotune.candidate_settings(quick=False) + autotune.candidate_settings(quick=True)
        log(f"case autotune candidates {pname}: {len(cands)} binned settings")
        for cand in cands:
            set_tuning(det, direct_max_pairs=0, **cand)
            det.scan(0, x)
            assert_same_sketch(det, 0, ref, f"{pname} {cand}")
            assert_same_report(det.close_window(0), want, f"{pname} {cand}")
        for block in (256, 512):
            for per_cu in (4, 8, 16):
                for lds in (0, 1):
                    set_tuning(det, direct_max_pairs=1 << 62, direct_block=block, direct_grid_per_cu=per_cu,
                               seav_lds=lds)
                    det.scan(0, x)
                    assert_same_sketch(det, 0, ref, f"{pname} direct {block}/{per_cu}/{lds}")
                    det.close_window(0)
    finally:
        det.close()


def test_autotune_choice_is_applied_and_exact():
    mp = PARAMS["plain_1m"]
    rng = np.random.default_rng(4011)
    pairs, _ = heavy_hosts(rng, 6, 2500, noise=1_500_000)
    x = to_dev(pairs)
    det = spd.Detector(spd.params_from(mp))
    try:
        log("case autotune: quick search on a 1.5 Mi-pair batch")
        chosen = autotune.autotune(det, x, quick=True)
        t = det.tuning
        for k, v in chosen.items():
            assert getattr(t, k) == v, k
        tables = autotune.last_tables(autotune.cache_key(det, x))
        assert len(tables["binned"]) == len(autotune.candidate_settings(quick=True))
        assert autotune.autotune(det, x, quick=True) == chosen          # cached
        ref = oracle_sketch(mp, pairs)
        det.scan(0, x)
        assert_same_sketch(det, 0, ref, "tuned")
        assert_same_report(det.close_window(0), ref.detect(), "tuned")
    finally:
        det.close()


def test_autotune_on_a_fused_call():
    """Tuning on the fused call of two routers' batches: the choice is applied and the sketches of
    both routers still equal the oracle's."""
    mp = PARAMS["plain_1m"]
    rng = np.random.default_rng(4021)
    p0, _ = heavy_hosts(rng, 4, 2500, noise=700_000)
    p1, _ = heavy_hosts(rng, 4, 2500, noise=500_000)
    x0, x1 = to_dev(p0), to_dev(p1)
    det = spd.Detector(spd.params_from(mp), n_routers=2)
    try:
        log("case autotune on a fused call of two routers")
        chosen = autotune.autotune(det, x0, quick=True, batches=[(0, x0), (1, x1)])
        t = det.tuning
        for k, v in chosen.items():
            assert getattr(t, k) == v, k
        det.scan_batches([(0, x0), (1, x1)])
        for r, p in ((0, p0), (1, p1)):
            ref = oracle_sketch(mp, p)
            assert_same_sketch(det, r, ref, f"router {r}")
            assert_same_report(det.close_window(r), ref.detect(), f"router {r}")
    finally:
        det.close()
