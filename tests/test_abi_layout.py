"""The ctypes structures of the Python binding have the same layout as the C declarations in
include/spd.h: a C program built here with gcc prints sizeof and offsetof of every field."""
import ctypes
import os
import subprocess

import pytest

import paper_1901_07306_amd as spd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

STRUCTS = {
    "spd_params": spd.SpdParams,
    "spd_derived": spd.SpdDerived,
    "spd_superpoint": spd.SpdSuperpoint,
    "spd_batch": spd.SpdBatch,
    "spd_tuning": spd.SpdTuning,
    "spd_stats": spd.SpdStats,
    "spd_profile": spd.SpdProfile,
    "spd_server_config": spd.SpdServerConfig,
    "spd_window_result": spd.SpdWindowResult,
    "spd_server_stats": spd.SpdServerStats,
    "spd_arrival": spd.SpdArrival,
}


def c_layout(tmp_path):
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "spd.h"', 'int main(void) {']
    for cname, cls in STRUCTS.items():
        lines.append(f'printf("{cname} sizeof %zu\\n", sizeof({cname}));')
        for f in cls._fields_:
            lines.append(f'printf("{cname} {f[0]} %zu\\n", offsetof({cname}, {f[0]}));')
    lines += ['return 0;', '}']
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    return {tuple(l.split()[:2]): int(l.split()[2]) for l in out.splitlines()}


def test_ctypes_layout_matches_header(tmp_path):
    got = c_layout(tmp_path)
    for cname, cls in STRUCTS.items():
        assert got[(cname, "sizeof")] == ctypes.sizeof(cls), cname
        for f in cls._fields_:
            assert got[(cname, f[0])] == getattr(cls, f[0]).offset, (cname, f[0])
