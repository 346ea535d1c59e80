"""Python access to the plain CPU oracle in ``spd_oracle.c``.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of the
benchmark use this module to check the GPU library; the product path never imports it.  It shares
no code with the GPU library; the only common module is ``synth_traffic``, which generates inputs
and holds none of the detection arithmetic.

The C source implements the method of Xu, Ding and Hu (arXiv 1901.07306) step by step: the short
estimator array vector (Section 3.1-3.2), the linear distinct counter array (Section 3.3), the OR
merge of routers (Section 4.2) and time-stamp counters for the sliding window (Section 5).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence, Tuple

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "spd_oracle.c")
LIB = os.path.join(HERE, "libspd_oracle.so")
MAX_ROWS = 8


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        subprocess.run(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"],
                       check=True)
    return LIB


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("theta", ctypes.c_uint32), ("r", ctypes.c_uint32), ("sr", ctypes.c_uint32),
        ("isb", ctypes.c_uint32 * MAX_ROWS), ("ibn", ctypes.c_uint32 * MAX_ROWS),
        ("log2k", ctypes.c_uint32), ("lr", ctypes.c_uint32), ("log2lc", ctypes.c_uint32),
        ("mul", ctypes.c_uint64 * (3 + MAX_ROWS)), ("add", ctypes.c_uint64 * (3 + MAX_ROWS)),
    ]


RECORD = np.dtype([("ip", "<u4"), ("z0", "<u4"), ("est", "<u4"), ("flags", "<u4")])

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        u32, u64, i64, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p
        P = ctypes.POINTER(OrcParams)
        sig = {
            "orc_tau": (u32, [u32]),
            "orc_est": (u32, [u32, u32]),
            "orc_z_theta": (u32, [u32, u32]),
            "orc_layout": (ctypes.c_int, [u32, u32, u32, vp, vp]),
            "orc_covers_all": (ctypes.c_int, [P]),
            "orc_hash": (u32, [u32, u64, u64, u32]),
            "orc_idx": (u32, [u32, u32, u32, u32]),
            "orc_lp_from_idx": (ctypes.c_int, [P, vp, vp]),
            "orc_sea_bytes": (u64, [P]),
            "orc_seav_bytes": (u64, [P]),
            "orc_ldca_words": (u64, [P]),
            "orc_scan": (None, [P, vp, vp, vp, u64]),
            "orc_merge": (None, [vp, vp, vp, vp, P]),
            "orc_candidates": (u64, [P, vp, vp, u64]),
            "orc_candidates_brute": (u64, [P, vp, u32, u32, vp, u64]),
            "orc_uldc_zeros": (u32, [P, vp, u32]),
            "orc_detect": (i64, [P, vp, vp, vp, u64]),
            "orc_scan_slice": (None, [P, vp, vp, vp, u64, u32]),
            "orc_bit_view": (None, [P, vp, vp, u32, u32, vp, vp]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


# ------------------------------------------------------------------------------ constants
def tau(theta: int) -> int:
    return lib().orc_tau(theta)


def est(log2k: int, z0: int) -> int:
    return lib().orc_est(log2k, z0)


def z_theta(log2k: int, theta: int) -> int:
    return lib().orc_z_theta(log2k, theta)


def layout(r: int, sr: int, a: int) -> Tuple[List[int], List[int]]:
    isb = np.zeros(MAX_ROWS, np.uint32)
    ibn = np.zeros(MAX_ROWS, np.uint32)
    if lib().orc_layout(r, sr, a, _ptr(isb), _ptr(ibn)) != 0:
        raise ValueError("invalid layout parameters")
    return [int(v) for v in isb[:sr]], [int(v) for v in ibn[:sr]]


def hash32(x: int, mul: int, add: int, m: int) -> int:
    return lib().orc_hash(x & 0xFFFFFFFF, mul & ((1 << 64) - 1), add & ((1 << 64) - 1), m)


def idx(lp: int, isb: int, ibn: int, L: int) -> int:
    return lib().orc_idx(lp, isb, ibn, L)


# ------------------------------------------------------------------------------ parameters
def params(mp, isb: Optional[Sequence[int]] = None, ibn: Optional[Sequence[int]] = None) -> OrcParams:
    """Oracle parameter block from a ``synth_traffic.MethodParams``; the row layout is derived
    by the oracle's own reading of Section 3.2 unless ``isb``/``ibn`` are given explicitly."""
    p = OrcParams()
    p.theta, p.r, p.sr = mp.theta, mp.r, mp.sr
    if isb is None:
        isb, ibn = layout(mp.r, mp.sr, mp.a)
    for i in range(mp.sr):
        p.isb[i], p.ibn[i] = isb[i], ibn[i]
    p.log2k, p.lr, p.log2lc = mp.log2k, mp.lr, mp.log2lc
    mul, add = mp.hashes()
    for j in range(3 + mp.lr):
        p.mul[j], p.add[j] = mul[j], add[j]
    return p


def covers_all(p: OrcParams) -> bool:
    return bool(lib().orc_covers_all(ctypes.byref(p)))


def lp_from_idx(p: OrcParams, idxs: Sequence[int]) -> Optional[int]:
    arr = np.zeros(MAX_ROWS, np.uint32)
    arr[: len(idxs)] = idxs
    out = np.zeros(1, np.uint32)
    ok = lib().orc_lp_from_idx(ctypes.byref(p), _ptr(arr), _ptr(out))
    return int(out[0]) if ok else None


def sea_bytes(p: OrcParams) -> int:
    return int(lib().orc_sea_bytes(ctypes.byref(p)))


def seav_bytes(p: OrcParams) -> int:
    return int(lib().orc_seav_bytes(ctypes.byref(p)))


def ldca_words(p: OrcParams) -> int:
    return int(lib().orc_ldca_words(ctypes.byref(p)))


# ------------------------------------------------------------------------------ sketches
class Sketch:
    """One router's (or the merged) SEAV bytes and LDCA words, canonical layouts:
    SEAV ``[2^r][row][2^IBN(row)]`` uint8, LDCA ``[LR][LC][k/32]`` uint32."""

    def __init__(self, p: OrcParams):
        self.p = p
        self.seav = np.zeros(seav_bytes(p), np.uint8)
        self.ldca = np.zeros(ldca_words(p), np.uint32)

    def scan(self, pairs: np.ndarray) -> "Sketch":
        pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
        lib().orc_scan(ctypes.byref(self.p), _ptr(self.seav), _ptr(self.ldca), _ptr(pairs), pairs.shape[0])
        return self

    def merge(self, other: "Sketch") -> "Sketch":
        lib().orc_merge(_ptr(self.seav), _ptr(other.seav), _ptr(self.ldca), _ptr(other.ldca), ctypes.byref(self.p))
        return self

    def copy(self) -> "Sketch":
        s = Sketch.__new__(Sketch)
        s.p, s.seav, s.ldca = self.p, self.seav.copy(), self.ldca.copy()
        return s

    def candidates(self) -> np.ndarray:
        n = lib().orc_candidates(ctypes.byref(self.p), _ptr(self.seav), None, 0)
        out = np.zeros(max(n, 1), np.uint32)
        lib().orc_candidates(ctypes.byref(self.p), _ptr(self.seav), _ptr(out), n)
        return out[:n]

    def candidates_brute(self, rp_lo: int, rp_hi: int) -> np.ndarray:
        n = lib().orc_candidates_brute(ctypes.byref(self.p), _ptr(self.seav), rp_lo, rp_hi, None, 0)
        out = np.zeros(max(n, 1), np.uint32)
        lib().orc_candidates_brute(ctypes.byref(self.p), _ptr(self.seav), rp_lo, rp_hi, _ptr(out), n)
        return out[:n]

    def uldc_zeros(self, h: int) -> int:
        return int(lib().orc_uldc_zeros(ctypes.byref(self.p), _ptr(self.ldca), h))

    def detect(self) -> np.ndarray:
        n = lib().orc_detect(ctypes.byref(self.p), _ptr(self.seav), _ptr(self.ldca), None, 0)
        if n < 0:
            raise MemoryError("oracle detect: allocation failed")
        out = np.zeros(max(n, 1), RECORD)
        lib().orc_detect(ctypes.byref(self.p), _ptr(self.seav), _ptr(self.ldca), _ptr(out), n)
        return out[:n]


class SlidingSketch:
    """Time-stamp counters for the sliding window: one uint16 per SEAV bit and per LDCA bit."""

    def __init__(self, p: OrcParams, K: int):
        self.p, self.K = p, K
        self.seav_ts = np.zeros(seav_bytes(p) * 8, np.uint16)
        self.ldca_ts = np.zeros(ldca_words(p) * 32, np.uint16)

    def scan_slice(self, pairs: np.ndarray, t: int) -> "SlidingSketch":
        pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
        lib().orc_scan_slice(ctypes.byref(self.p), _ptr(self.seav_ts), _ptr(self.ldca_ts), _ptr(pairs),
                             pairs.shape[0], t)
        return self

    def bit_view(self, t: int) -> Sketch:
        s = Sketch(self.p)
        lib().orc_bit_view(ctypes.byref(self.p), _ptr(self.seav_ts), _ptr(self.ldca_ts), t, self.K,
                           _ptr(s.seav), _ptr(s.ldca))
        return s
