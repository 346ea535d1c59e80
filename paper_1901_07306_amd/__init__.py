"""Python binding of libspd (include/spd.h): super-point detection on MI355X.

Argument marshalling only: every step of the detection path runs in the HIP kernels of
``libspd.so``.  The functions keep the C names (``spd_create``, ``spd_scan``, ...).  Pair buffers
are torch tensors on the GPU (``[n, 2]``, any 4-byte integer dtype holding the uint32 bits of
(hip, oip)); streams default to torch's current stream.  torch provides device memory and
streams only.

The library is loaded on first use; if ``libspd.so`` has not been built the call raises instead of
falling back to anything else.
"""
from __future__ import annotations

import ctypes
import threading
import os
from typing import Iterable, List, Optional, Sequence, Tuple

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libspd.so")
MAX_ROWS = 8
GLOBAL = -1

SPD_OK, SPD_E_INVALID, SPD_E_NOMEM, SPD_E_HIP, SPD_E_TRUNCATED, SPD_E_STATE = 0, -1, -2, -3, -4, -5

u32, u64, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int32


class SpdParams(ctypes.Structure):
    _fields_ = [("theta", u32), ("r", u32), ("sr", u32), ("a", u32), ("explicit_layout", u32),
                ("isb", u32 * MAX_ROWS), ("ibn", u32 * MAX_ROWS), ("log2k", u32), ("lr", u32),
                ("log2lc", u32), ("window_slices", u32), ("sliding_counter", u32),
                ("hash_mul", u64 * (3 + MAX_ROWS)), ("hash_add", u64 * (3 + MAX_ROWS))]


class SpdDerived(ctypes.Structure):
    _fields_ = [("tau", u32), ("z_theta", u32), ("isb", u32 * MAX_ROWS), ("ibn", u32 * MAX_ROWS),
                ("sea_bytes", u64), ("seav_bytes", u64), ("ldca_words", u64)]


class SpdSuperpoint(ctypes.Structure):
    _fields_ = [("ip", u32), ("z0", u32), ("est", u32), ("flags", u32)]


class SpdBatch(ctypes.Structure):
    _fields_ = [("router", u32), ("flags", u32), ("pairs_dev", ctypes.c_void_p), ("n_pairs", u64)]


class SpdTuning(ctypes.Structure):
    _fields_ = [("direct_max_pairs", u64), ("bucket_bits", u32), ("tile_pairs", u32), ("bin_block", u32),
                ("apply_block", u32), ("direct_block", u32), ("direct_grid_per_cu", u32), ("seav_lds", u32),
                ("close_block", u32), ("launch_pairs", u64), ("apply_unroll", u32), ("bin_mode", u32),
                ("region_words", u32)]


class SpdStats(ctypes.Structure):
    _fields_ = [("pairs_scanned", u64), ("direct_launches", u64), ("binned_launches", u64), ("closes", u64),
                ("candidates_last", u64), ("reported_last", u64), ("device_bytes", u64)]


K_KINDS = ["direct", "stamp", "bin", "transpose", "apply", "merge", "close", "fill", "count", "offsets", "spill"]


class SpdProfile(ctypes.Structure):
    _fields_ = [("launches", u64 * len(K_KINDS)), ("total_ms", ctypes.c_double * len(K_KINDS))]


class SpdServerConfig(ctypes.Structure):
    _fields_ = [("n_routers", u32), ("max_slots", u32), ("window_pairs", u64), ("hbm_budget_bytes", u64),
                ("max_group_pairs", u64), ("max_group_batches", u32), ("use_graphs", u32), ("min_scan_pairs", u64),
                ("tuning", ctypes.c_void_p)]


class SpdWindowResult(ctypes.Structure):
    _fields_ = [("router", u32), ("window", u32), ("pairs", u64), ("latency_ms", ctypes.c_double),
                ("n_super", u32), ("reserved", u32)]


class SpdArrival(ctypes.Structure):
    _fields_ = [("t_s", ctypes.c_double), ("router", u32), ("flags", u32), ("pairs_dev", ctypes.c_void_p),
                ("n_pairs", u64)]


class SpdServerStats(ctypes.Structure):
    _fields_ = [("batches", u64), ("pairs", u64), ("groups", u64), ("windows", u64), ("admission_waits", u64),
                ("slots", u32), ("max_open", u32)]


RECORD = np.dtype([("ip", "<u4"), ("z0", "<u4"), ("est", "<u4"), ("flags", "<u4")])

EXPORTED = ["spd_derive", "spd_create", "spd_destroy", "spd_scan", "spd_scan_noalloc", "spd_scan_host", "spd_scan_batches", "spd_scan_batches_merge", "spd_merge",
            "spd_close_window", "spd_close_begin", "spd_close_end", "spd_reset", "spd_slide", "spd_export", "spd_import", "spd_export_stamps",
            "spd_current_slice", "spd_get_tuning", "spd_set_tuning", "spd_get_stats", "spd_strerror",
            "spd_last_error", "spd_profile_enable", "spd_profile_select", "spd_get_profile", "spd_server_create", "spd_server_submit",
            "spd_server_next", "spd_server_drain", "spd_server_get_stats", "spd_server_set_tuning",
            "spd_server_last_error", "spd_server_destroy", "spd_server_replay"]

SPD_E_AGAIN = -6
SPD_SUBMIT_CLOSE = 1
SPD_SUBMIT_DST = 2


class SpdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def _hip_runtimes() -> List[str]:
    paths = set()
    try:
        with open("/proc/self/maps") as f:
            for line in f:
                if "libamdhip64" in line:
                    paths.add(os.path.realpath(line.split()[-1]))
    except OSError:
        pass
    return sorted(paths)


def lib(require_torch: bool = True) -> ctypes.CDLL:
    """Load libspd.so.  torch is imported first so that the library binds to the HIP runtime
    that torch's streams and allocations belong to."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    if require_torch:
        import torch  # noqa: F401  (loads torch's HIP runtime before libspd)
        if torch.cuda.is_available():
            torch.cuda.init()
    L = ctypes.CDLL(LIB_PATH)
    runtimes = _hip_runtimes()
    if len(runtimes) > 1:
        raise RuntimeError("two HIP runtimes are mapped in this process: " + ", ".join(runtimes))
    P, vp = ctypes.POINTER, ctypes.c_void_p
    sig = {
        "spd_derive": (i32, [P(SpdParams), P(SpdDerived)]),
        "spd_create": (i32, [P(SpdParams), u32, u64, P(vp)]),
        "spd_destroy": (None, [vp]),
        "spd_scan": (i32, [vp, u32, vp, u64, vp]),
        "spd_scan_host": (i32, [vp, u32, vp, u64, u32, u64, vp]),
        "spd_scan_noalloc": (i32, [vp, u32, vp, u64, u32, vp]),
        "spd_scan_batches": (i32, [vp, P(SpdBatch), u32, vp]),
        "spd_scan_batches_merge": (i32, [vp, P(SpdBatch), u32, vp]),
        "spd_merge": (i32, [vp, P(u32), u32, vp]),
        "spd_close_window": (i32, [vp, i32, P(SpdSuperpoint), u32, P(u32), vp]),
        "spd_close_begin": (i32, [vp, i32, vp, P(u32)]),
        "spd_close_end": (i32, [vp, u32, P(SpdSuperpoint), u32, P(u32)]),
        "spd_slide": (i32, [vp, vp]),
        "spd_reset": (i32, [vp, i32, vp]),
        "spd_export": (i32, [vp, i32, vp, vp]),
        "spd_import": (i32, [vp, i32, vp, vp]),
        "spd_export_stamps": (i32, [vp, i32, vp, vp]),
        "spd_current_slice": (u32, [vp]),
        "spd_get_tuning": (i32, [vp, P(SpdTuning)]),
        "spd_set_tuning": (i32, [vp, P(SpdTuning)]),
        "spd_get_stats": (i32, [vp, P(SpdStats)]),
        "spd_profile_enable": (i32, [vp, u32]),
        "spd_profile_select": (i32, [vp, u32]),
        "spd_get_profile": (i32, [vp, P(SpdProfile)]),
        "spd_server_create": (i32, [P(SpdParams), P(SpdServerConfig), P(vp)]),
        "spd_server_submit": (i32, [vp, u32, vp, u64, u32]),
        "spd_server_next": (i32, [vp, P(SpdWindowResult), P(SpdSuperpoint), u32, i32]),
        "spd_server_drain": (i32, [vp]),
        "spd_server_get_stats": (i32, [vp, P(SpdServerStats)]),
        "spd_server_set_tuning": (i32, [vp, P(SpdTuning)]),
        "spd_server_last_error": (ctypes.c_char_p, [vp]),
        "spd_server_destroy": (None, [vp]),
        "spd_server_replay": (i32, [vp, P(SpdArrival), u64, P(ctypes.c_double)]),
        "spd_strerror": (ctypes.c_char_p, [i32]),
        "spd_last_error": (ctypes.c_char_p, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype, f.argtypes = res, args
    _lib = L
    return L


def _check(status: int, ctx=None):
    if status != SPD_OK:
        L = lib()
        msg = L.spd_last_error(ctx).decode() if ctx else ""
        raise SpdError(status, (msg or L.spd_strerror(status).decode()))


# ------------------------------------------------------------------------------ parameters
SLIDING_AT, SLIDING_STAMPS = 0, 1   # spd_params.sliding_counter


def make_params(theta: int, r: int, sr: int, a: int, log2k: int, lr: int, log2lc: int,
                hash_mul: Sequence[int], hash_add: Sequence[int], window_slices: int = 0,
                isb: Optional[Sequence[int]] = None, ibn: Optional[Sequence[int]] = None,
                sliding_counter: int = SLIDING_AT) -> SpdParams:
    p = SpdParams()
    p.theta, p.r, p.sr, p.a = theta, r, sr, a
    p.log2k, p.lr, p.log2lc, p.window_slices = log2k, lr, log2lc, window_slices
    p.sliding_counter = sliding_counter
    if isb is not None:
        p.explicit_layout = 1
        for i in range(sr):
            p.isb[i], p.ibn[i] = isb[i], ibn[i]
    for j in range(3 + lr):
        p.hash_mul[j], p.hash_add[j] = hash_mul[j], hash_add[j]
    return p


def params_from(mp, isb=None, ibn=None) -> SpdParams:
    """From any object with theta, r, sr, a, log2k, lr, log2lc, window_slices, sliding_counter and
    hashes()."""
    mul, add = mp.hashes()
    return make_params(mp.theta, mp.r, mp.sr, mp.a, mp.log2k, mp.lr, mp.log2lc, mul, add,
                       getattr(mp, "window_slices", 0), isb, ibn, getattr(mp, "sliding_counter", SLIDING_AT))


def spd_derive(p: SpdParams) -> SpdDerived:
    d = SpdDerived()
    _check(lib(require_torch=False).spd_derive(ctypes.byref(p), ctypes.byref(d)))
    return d


# ------------------------------------------------------------------------------ contexts
def _stream_ptr(stream) -> Optional[int]:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _pairs_ptr(pairs) -> Tuple[int, int]:
    if pairs.numel() == 0:
        return 0, 0
    if not pairs.is_cuda or pairs.dim() != 2 or pairs.shape[1] != 2 or pairs.element_size() != 4:
        raise ValueError("pairs must be a CUDA tensor of shape [n, 2] with 4-byte elements")
    if not pairs.is_contiguous():
        raise ValueError("pairs must be contiguous")
    return pairs.data_ptr(), pairs.shape[0]


def spd_create(p: SpdParams, n_routers: int = 1, hbm_budget_bytes: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(lib().spd_create(ctypes.byref(p), n_routers, hbm_budget_bytes, ctypes.byref(h)))
    return h.value


def spd_destroy(ctx: int) -> None:
    lib().spd_destroy(ctx)


def spd_scan(ctx: int, router: int, pairs, stream=None) -> None:
    ptr, n = _pairs_ptr(pairs)
    _check(lib().spd_scan(ctx, router, ptr or None, n, _stream_ptr(stream)), ctx)


BATCH_DST = 1   # destination-keyed batch: records read as (oip, hip)
NOALLOC_SCRATCH_BYTES = 64 << 20   # SPD_NOALLOC_SCRATCH_BYTES


def spd_scan_noalloc(ctx: int, router: int, pairs, flags: int = 0, stream=None) -> None:
    """spd_scan that allocates nothing (scratch in the library's fixed per-GPU array)."""
    ptr, n = _pairs_ptr(pairs)
    _check(lib().spd_scan_noalloc(ctx, router, ptr or None, n, flags, _stream_ptr(stream)), ctx)


def _host_pairs_ptr(pairs) -> Tuple[int, int, object]:
    """(address, n, owner) of a host buffer of n (hip, oip) uint32 records: a numpy array or a CPU
    torch tensor (page-locked when made with pin_memory=True)."""
    if isinstance(pairs, np.ndarray):
        if pairs.ndim != 2 or pairs.shape[1] != 2 or pairs.dtype.itemsize != 4 or not pairs.flags.c_contiguous:
            raise ValueError("pairs must be a C-contiguous [n, 2] array of 4-byte elements")
        return pairs.ctypes.data if pairs.size else 0, pairs.shape[0], pairs
    if pairs.is_cuda or pairs.dim() != 2 or pairs.shape[1] != 2 or pairs.element_size() != 4 or not pairs.is_contiguous():
        raise ValueError("pairs must be a contiguous CPU tensor of shape [n, 2] with 4-byte elements")
    return (pairs.data_ptr() if pairs.numel() else 0), pairs.shape[0], pairs


def spd_scan_host(ctx: int, router: int, pairs, flags: int = 0, chunk_pairs: int = 0, stream=None) -> None:
    ptr, n, _owner = _host_pairs_ptr(pairs)
    _check(lib().spd_scan_host(ctx, router, ptr or None, n, flags, chunk_pairs, _stream_ptr(stream)), ctx)


def spd_scan_batches(ctx: int, batches: Iterable[Tuple], stream=None, merge: bool = False) -> None:
    """batches: (router, pairs) or (router, pairs, flags) with flags BATCH_DST for destination-keyed.
    merge: then the global sketch := OR of the routers named (spd_scan_batches_merge)."""
    items = []
    for b in batches:
        router, pairs = b[0], b[1]
        flags = b[2] if len(b) > 2 else 0
        ptr, n = _pairs_ptr(pairs)
        items.append(SpdBatch(router, flags, ptr or None, n))
    arr = (SpdBatch * max(1, len(items)))(*items)
    fn = lib().spd_scan_batches_merge if merge else lib().spd_scan_batches
    _check(fn(ctx, arr, len(items), _stream_ptr(stream)), ctx)


def spd_merge(ctx: int, routers: Sequence[int], stream=None) -> None:
    arr = (u32 * max(1, len(routers)))(*routers)
    _check(lib().spd_merge(ctx, arr, len(routers), _stream_ptr(stream)), ctx)


_out_bufs = threading.local()   # per thread: the last record buffer handed to spd_close_window


def _out_buffer(cap: int):
    """A reusable ctypes array of cap records (the result is copied out before the next call)."""
    cap = max(1, cap)
    b = getattr(_out_bufs, "buf", None)
    if b is None or len(b) != cap:
        b = (SpdSuperpoint * cap)()
        _out_bufs.buf = b
    return b


def spd_close_window(ctx: int, target: int, cap: int = 1 << 16, stream=None) -> np.ndarray:
    """Super points of the target, sorted by ip, as a structured array (ip, z0, est, flags)."""
    out = _out_buffer(cap)
    n = u32(0)
    st = lib().spd_close_window(ctx, target, out, cap, ctypes.byref(n), _stream_ptr(stream))
    if st == SPD_E_TRUNCATED:
        raise SpdError(st, f"{n.value} super points exceed cap {cap}")
    _check(st, ctx)
    return np.frombuffer(out, dtype=RECORD, count=len(out))[: n.value].copy()


MAX_PENDING_CLOSES = 4   # SPD_MAX_PENDING_CLOSES


def spd_close_begin(ctx: int, target: int, stream=None) -> int:
    """Enqueue the end of window of the target; returns the ticket that spd_close_end collects."""
    t = u32(0)
    _check(lib().spd_close_begin(ctx, target, _stream_ptr(stream), ctypes.byref(t)), ctx)
    return t.value


def spd_close_end(ctx: int, ticket: int, cap: int = 1 << 16) -> np.ndarray:
    """The report of a begun close (waits for it), as spd_close_window returns it."""
    out = _out_buffer(cap)
    n = u32(0)
    st = lib().spd_close_end(ctx, ticket, out, cap, ctypes.byref(n))
    if st == SPD_E_TRUNCATED:
        raise SpdError(st, f"{n.value} super points: {lib().spd_last_error(ctx).decode()}")
    _check(st, ctx)
    return np.frombuffer(out, dtype=RECORD, count=len(out))[: n.value].copy()


def spd_reset(ctx: int, target: int, stream=None) -> None:
    _check(lib().spd_reset(ctx, target, _stream_ptr(stream)), ctx)


def spd_slide(ctx: int, stream=None) -> None:
    _check(lib().spd_slide(ctx, _stream_ptr(stream)), ctx)


def spd_export(ctx: int, target: int, d: SpdDerived) -> Tuple[np.ndarray, np.ndarray]:
    seav = np.empty(d.seav_bytes, np.uint8)
    ldca = np.empty(d.ldca_words, np.uint32)
    _check(lib().spd_export(ctx, target, seav.ctypes.data, ldca.ctypes.data), ctx)
    return seav, ldca


def spd_import(ctx: int, target: int, seav: np.ndarray, ldca: np.ndarray) -> None:
    seav = np.ascontiguousarray(seav, np.uint8)
    ldca = np.ascontiguousarray(ldca, np.uint32)
    _check(lib().spd_import(ctx, target, seav.ctypes.data, ldca.ctypes.data), ctx)


def spd_export_stamps(ctx: int, target: int, d: SpdDerived) -> Tuple[np.ndarray, np.ndarray]:
    seav = np.empty(d.seav_bytes * 8, np.uint16)
    ldca = np.empty(d.ldca_words * 32, np.uint16)
    _check(lib().spd_export_stamps(ctx, target, seav.ctypes.data, ldca.ctypes.data), ctx)
    return seav, ldca


def spd_current_slice(ctx: int) -> int:
    return lib().spd_current_slice(ctx)


def spd_get_tuning(ctx: int) -> SpdTuning:
    t = SpdTuning()
    _check(lib().spd_get_tuning(ctx, ctypes.byref(t)), ctx)
    return t


def spd_set_tuning(ctx: int, t: SpdTuning) -> None:
    _check(lib().spd_set_tuning(ctx, ctypes.byref(t)), ctx)


def spd_get_stats(ctx: int) -> SpdStats:
    s = SpdStats()
    _check(lib().spd_get_stats(ctx, ctypes.byref(s)), ctx)
    return s


def spd_profile_enable(ctx: int, on: bool = True) -> None:
    _check(lib().spd_profile_enable(ctx, 1 if on else 0), ctx)


def spd_profile_select(ctx: int, kinds=None) -> None:
    """Time only the given kernel kinds (names from K_KINDS) while profiling is on; None: all."""
    mask = 0xFFFFFFFF if kinds is None else sum(1 << K_KINDS.index(k) for k in kinds)
    _check(lib().spd_profile_select(ctx, mask), ctx)


def spd_get_profile(ctx: int) -> dict:
    """{kind: (launches, total device ms)} since the last spd_profile_enable()."""
    p = SpdProfile()
    _check(lib().spd_get_profile(ctx, ctypes.byref(p)), ctx)
    return {k: (int(p.launches[i]), float(p.total_ms[i])) for i, k in enumerate(K_KINDS)}


def spd_strerror(status: int) -> str:
    return lib(require_torch=False).spd_strerror(status).decode()


class Detector:
    """A context with its derived sizes; closes the context when garbage collected."""

    def __init__(self, params: SpdParams, n_routers: int = 1, hbm_budget_bytes: int = 0):
        self.params = params
        self.derived = spd_derive(params)
        self.n_routers = n_routers
        self.ctx = spd_create(params, n_routers, hbm_budget_bytes)

    def close(self):
        if getattr(self, "ctx", None):
            spd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def scan(self, router, pairs, stream=None):
        spd_scan(self.ctx, router, pairs, stream)

    def scan_noalloc(self, router, pairs, flags=0, stream=None):
        spd_scan_noalloc(self.ctx, router, pairs, flags, stream)

    def scan_host(self, router, pairs, flags=0, chunk_pairs=0, stream=None):
        """Pairs in host memory (numpy array or CPU tensor), copied in chunks overlapping the scan."""
        spd_scan_host(self.ctx, router, pairs, flags, chunk_pairs, stream)

    def scan_batches(self, batches, stream=None, merge=False):
        spd_scan_batches(self.ctx, batches, stream, merge)

    def merge(self, routers, stream=None):
        spd_merge(self.ctx, routers, stream)

    def close_window(self, target=0, cap=1 << 16, stream=None):
        return spd_close_window(self.ctx, target, cap, stream)

    def close_begin(self, target=0, stream=None) -> int:
        return spd_close_begin(self.ctx, target, stream)

    def close_end(self, ticket: int, cap=1 << 16):
        return spd_close_end(self.ctx, ticket, cap)

    def reset(self, target=0, stream=None):
        spd_reset(self.ctx, target, stream)

    def slide(self, stream=None):
        spd_slide(self.ctx, stream)

    def export(self, target=0):
        return spd_export(self.ctx, target, self.derived)

    def export_stamps(self, target=0):
        return spd_export_stamps(self.ctx, target, self.derived)

    def import_(self, target, seav, ldca):
        spd_import(self.ctx, target, seav, ldca)

    @property
    def tuning(self) -> SpdTuning:
        return spd_get_tuning(self.ctx)

    @tuning.setter
    def tuning(self, t: SpdTuning):
        spd_set_tuning(self.ctx, t)

    def profile_enable(self, on=True, kinds=None):
        spd_profile_select(self.ctx, kinds)
        spd_profile_enable(self.ctx, on)

    def profile(self) -> dict:
        return spd_get_profile(self.ctx)

    @property
    def stats(self) -> SpdStats:
        return spd_get_stats(self.ctx)


# ------------------------------------------------------------------------------ serving loop
class Server:
    """The serving loop of libspd: submit batches per router as they arrive, collect finished
    windows with next()."""

    def __init__(self, params: SpdParams, n_routers: int, window_pairs: int = 0, hbm_budget_bytes: int = 0,
                 max_slots: int = 0, max_group_pairs: int = 0, max_group_batches: int = 0, use_graphs: bool = True,
                 min_scan_pairs: int = 0, tuning: Optional[SpdTuning] = None):
        self.params = params
        self._tuning = tuning
        cfg = SpdServerConfig(n_routers, max_slots, window_pairs, hbm_budget_bytes, max_group_pairs,
                              max_group_batches, 1 if use_graphs else 0, min_scan_pairs,
                              ctypes.cast(ctypes.pointer(tuning), ctypes.c_void_p) if tuning is not None else None)
        h = ctypes.c_void_p()
        st = lib().spd_server_create(ctypes.byref(params), ctypes.byref(cfg), ctypes.byref(h))
        if st != SPD_OK:
            raise SpdError(st, "spd_server_create failed")
        self.h = h.value
        self._keep = []   # device tensors handed over, kept alive until the server is closed

    def _check(self, st):
        if st != SPD_OK:
            raise SpdError(st, lib().spd_server_last_error(self.h).decode() or lib().spd_strerror(st).decode())

    def submit(self, router: int, pairs, close: bool = False, keep: bool = True, dst: bool = False):
        ptr, n = _pairs_ptr(pairs)
        if keep:
            self._keep.append(pairs)
        flags = (SPD_SUBMIT_CLOSE if close else 0) | (SPD_SUBMIT_DST if dst else 0)
        self._check(lib().spd_server_submit(self.h, router, ptr or None, n, flags))

    def next(self, timeout_ms: int = -1, cap: int = 1 << 16):
        """(header dict, structured array of super points) or None on timeout."""
        hdr = SpdWindowResult()
        out = _out_buffer(cap)
        st = lib().spd_server_next(self.h, ctypes.byref(hdr), out, cap, timeout_ms)
        if st == SPD_E_AGAIN:
            return None
        self._check(st)
        sp = np.frombuffer(out, dtype=RECORD, count=len(out))[: hdr.n_super].copy()
        return dict(router=hdr.router, window=hdr.window, pairs=hdr.pairs, latency_ms=hdr.latency_ms,
                    n_super=hdr.n_super), sp

    def schedule(self, times, routers, tensors, flags=None):
        """The arrival array of replay (built ahead, so that replaying it costs no Python time)."""
        n = len(times)
        arr = (SpdArrival * max(1, n))()
        for i in range(n):
            ptr, cnt = _pairs_ptr(tensors[i])
            arr[i] = SpdArrival(float(times[i]), int(routers[i]), int(flags[i]) if flags is not None else 0,
                                ptr or None, cnt)
            self._keep.append(tensors[i])
        return arr, n

    def replay(self, times, routers=None, tensors=None, flags=None) -> float:
        """Submit tensors[i] for routers[i] at times[i] seconds (sorted) from a native loop; `times`
        may instead be what schedule() returned."""
        arr, n = times if routers is None else self.schedule(times, routers, tensors, flags)
        el = ctypes.c_double(0.0)
        self._check(lib().spd_server_replay(self.h, arr, n, ctypes.byref(el)))
        return el.value

    def drain(self):
        self._check(lib().spd_server_drain(self.h))

    @property
    def stats(self) -> dict:
        s = SpdServerStats()
        self._check(lib().spd_server_get_stats(self.h, ctypes.byref(s)))
        return {k: getattr(s, k) for k, _ in SpdServerStats._fields_}

    def set_tuning(self, t: SpdTuning):
        self._check(lib().spd_server_set_tuning(self.h, ctypes.byref(t)))

    def close(self):
        if getattr(self, "h", None):
            lib().spd_server_destroy(self.h)
            self.h = None
            self._keep = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
