"""Hardware ceilings behind the scan's design, measured by the kernels of libspd_ceilings.so
(include/spd_ceilings.h): streaming read bandwidth, device-wide random atomicOr rate against the
table footprint, random 16-bit store rate, and LDS atomicOr rate.  Timed with HIP events on
torch's current stream; each figure is the median of a few repetitions."""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libspd_ceilings.so")

_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        import torch  # noqa: F401  (torch's HIP runtime first)
        L = ctypes.CDLL(LIB_PATH)
        u32, u64, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
        for name, args in {"spd_ceil_stream_read": [vp, u64, vp, vp],
                           "spd_ceil_atomic_or": [vp, u64, u64, u64, vp],
                           "spd_ceil_store16": [vp, u64, u64, u64, vp],
                           "spd_ceil_lds_atomic_or": [u32, u32, vp, vp]}.items():
            f = getattr(L, name)
            f.restype, f.argtypes = ctypes.c_int, args
        L.spd_ceil_block.restype, L.spd_ceil_block.argtypes = u32, []
        _lib = L
    return _lib


def _time_ms(torch, fn, reps=5):
    s = torch.cuda.current_stream()
    fn()                                  # warm-up
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(s)
        fn()
        b.record(s)
        b.synchronize()
        out.append(a.elapsed_time(b))
    out.sort()
    return out[len(out) // 2]


def run_all(torch, log=print) -> dict:
    L = lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    res = {"gpu": torch.cuda.get_device_name(0)}

    def ok(rc):
        if rc != 0:
            raise RuntimeError(f"ceiling kernel refused its arguments ({rc})")

    nbytes = 4 << 30
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    buf.fill_(1)
    ms = _time_ms(torch, lambda: ok(L.spd_ceil_stream_read(buf.data_ptr(), nbytes, sink.data_ptr(), st)))
    res["stream_read_GBps"] = nbytes / (ms * 1e-3) / 1e9
    half = buf[: nbytes // 2]
    dst = torch.empty_like(half)
    ms = _time_ms(torch, lambda: dst.copy_(half))
    res["copy_GBps_read_plus_write"] = 2 * half.numel() / (ms * 1e-3) / 1e9
    log(f"ceilings: stream read {res['stream_read_GBps']:.0f} GB/s, copy {res['copy_GBps_read_plus_write']:.0f} GB/s")
    del dst, half

    n_ops = 1 << 28
    atom = {}
    for mib in (1, 4, 16, 64, 256, 1024):
        words = (mib << 20) // 4
        t = buf[: mib << 20].view(torch.int32)
        ms = _time_ms(torch, lambda: ok(L.spd_ceil_atomic_or(t.data_ptr(), words, n_ops, 12345, st)), reps=3)
        atom[f"{mib}MiB"] = n_ops / (ms * 1e-3)
    res["random_atomic_or_per_s"] = atom
    log("ceilings: random atomicOr/s " + ", ".join(f"{k} {v / 1e9:.1f}G" for k, v in atom.items()))

    stores = {}
    for mib in (16, 128, 1024, 2048):
        elems = (mib << 20) // 2
        t = buf[: mib << 20].view(torch.int16)
        ms = _time_ms(torch, lambda: ok(L.spd_ceil_store16(t.data_ptr(), elems, n_ops, 777, st)), reps=3)
        stores[f"{mib}MiB"] = n_ops / (ms * 1e-3)
    res["random_store16_per_s"] = stores
    log("ceilings: random 16-bit stores/s " + ", ".join(f"{k} {v / 1e9:.1f}G" for k, v in stores.items()))

    blocks, n_iter = 1024, 4096
    ms = _time_ms(torch, lambda: ok(L.spd_ceil_lds_atomic_or(blocks, n_iter, sink.data_ptr(), st)), reps=3)
    res["lds_atomic_or_per_s"] = blocks * L.spd_ceil_block() * n_iter / (ms * 1e-3)
    log(f"ceilings: LDS atomicOr {res['lds_atomic_or_per_s'] / 1e12:.2f} T/s")
    res["ops_per_measurement"] = n_ops
    del buf
    torch.cuda.empty_cache()
    return res
