"""CPU checks of the C-ABI library: it loads, exports every entry point declared in include/spd.h,
and its host-side parameter logic (Eq. 1, Section 3.2 layout and constraints, Eq. 4 threshold)
agrees with the oracle.  No kernel is launched here."""
import os
import re

import numpy as np
import pytest

import oracle
import paper_1901_07306_amd as spd
import synth_traffic as st

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    with open(os.path.join(ROOT, "include", "spd.h")) as f:
        text = f.read()
    decl = r"^(?:spd_status|void|uint32_t|const char \*)\s*\*?\s*(spd_[a-z_]+)\s*\("
    return sorted(set(re.findall(decl, text, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = spd.lib(require_torch=False)
    names = header_symbols()
    assert len(names) >= 17
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(spd.EXPORTED)


def test_strerror_codes():
    assert spd.spd_strerror(0) == "ok"
    for code in (-1, -2, -3, -4, -5):
        assert spd.spd_strerror(code) != "unknown status"
    assert spd.spd_strerror(-99) == "unknown status"


@pytest.mark.parametrize("name", list(st.CONFIGS))
def test_derive_matches_oracle_for_configs(name):
    mp = st.CONFIGS[name].params
    d = spd.spd_derive(spd.params_from(mp))
    p = oracle.params(mp)
    assert d.tau == oracle.tau(mp.theta)
    assert d.z_theta == oracle.z_theta(mp.log2k, mp.theta)
    assert list(d.isb)[: mp.sr] == list(p.isb)[: mp.sr]
    assert list(d.ibn)[: mp.sr] == list(p.ibn)[: mp.sr]
    assert d.seav_bytes == oracle.seav_bytes(p)
    assert d.ldca_words == oracle.ldca_words(p)


def test_derive_grid_matches_oracle():
    rng = np.random.default_rng(0)
    for _ in range(300):
        mp = st.MethodParams(theta=int(rng.integers(1, 1 << 20)), r=int(rng.integers(0, 25)),
                             sr=int(rng.integers(1, 7)), a=int(rng.integers(1, 4)), log2k=int(rng.integers(5, 15)),
                             lr=int(rng.integers(1, 5)), log2lc=int(rng.integers(0, 12)))
        p = spd.params_from(mp)
        try:
            d = spd.spd_derive(p)
        except spd.SpdError:
            # the library refuses layouts the oracle also finds uncovered, rows wider than 16 bits,
            # and sketches of more than 2^32 bits (the SEAV is padded to 128 KiB)
            op = oracle.params(mp)
            padded = -(-oracle.seav_bytes(op) // (1 << 17)) * (1 << 17)
            too_big = oracle.ldca_words(op) * 32 + padded * 8 > 1 << 32
            assert (not oracle.covers_all(op)) or max(list(op.ibn)[: mp.sr]) > 16 or too_big
            continue
        assert d.tau == oracle.tau(mp.theta)
        assert d.z_theta == oracle.z_theta(mp.log2k, mp.theta)
        op = oracle.params(mp)
        assert list(d.isb)[: mp.sr] == list(op.isb)[: mp.sr]
        assert list(d.ibn)[: mp.sr] == list(op.ibn)[: mp.sr]


def test_derive_rejects_bad_parameters():
    base = st.CONFIGS["plain_1m"].params
    bad = [base.replace(theta=0), base.replace(sr=0), base.replace(sr=9), base.replace(lr=0),
           base.replace(log2k=4), base.replace(log2k=17), base.replace(r=25), base.replace(log2lc=25)]
    for mp in bad:
        with pytest.raises(spd.SpdError):
            spd.spd_derive(spd.params_from(mp))
    # even hash multiplier
    p = spd.params_from(base)
    p.hash_mul[0] = 2
    with pytest.raises(spd.SpdError):
        spd.spd_derive(p)
    # explicit layout that leaves an LP bit uncovered (constraint 1)
    p = spd.params_from(base.replace(r=20, sr=2), isb=[0, 5], ibn=[5, 6])
    with pytest.raises(spd.SpdError):
        spd.spd_derive(p)
    # explicit layout that covers every bit is accepted as given
    p = spd.params_from(base.replace(r=20, sr=2), isb=[0, 5], ibn=[6, 7])
    d = spd.spd_derive(p)
    assert list(d.isb)[:2] == [0, 5] and list(d.ibn)[:2] == [6, 7]


def test_ceilings_library_exports_its_declarations():
    """The microbenchmark library of the hardware ceilings exports every call its header declares."""
    import ctypes
    with open(os.path.join(ROOT, "include", "spd_ceilings.h")) as f:
        names = sorted(set(re.findall(r"^(?:int|uint32_t)\s+(spd_ceil_[a-z0-9_]+)\s*\(", f.read(), flags=re.M)))
    assert len(names) == 5
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_1901_07306_amd", "libspd_ceilings.so"))
    for n in names:
        assert hasattr(lib, n), n
