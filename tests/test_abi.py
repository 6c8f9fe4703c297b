"""The C-ABI library: it loads, exports every function include/sky.h declares, and rejects bad
arguments synchronously (paths that return before any device work, so no GPU is needed)."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2412_02274_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sky.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libsky.so is not built (run __graft_entry__.build())")
    return _lib.load()


def test_header_declarations_exported(lib):
    declared = _declared_functions()
    assert set(declared) == set(_lib.EXPORTS), declared
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    for name in declared:
        assert name in exported, name
        assert hasattr(lib, name)


def test_struct_layouts_match_header(tmp_path):
    # the ctypes mirrors of the header's structs: size and every field's offset, as a C
    # compiler lays them out from include/sky.h
    structs = {"sky_params": _lib.SkyParams, "sky_info": _lib.SkyInfo,
               "sky_gres_opts": _lib.GresOpts, "sky_tune": _lib.SkyTune}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "sky.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)],
                   check=True)
    got = {}
    for line in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.splitlines():
        cname, field, val = line.split()
        got[(cname, field)] = int(val)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)


def test_status_strings(lib):
    for code in range(8):
        s = lib.sky_status_string(code).decode()
        assert s.startswith("SKY_")
    assert lib.sky_version() >= 10000


def test_workspace_sizes(lib):
    prm = _lib.SkyParams(_lib.SKY_GRID, 64, 0, 0)
    assert lib.sky_build_workspace_bytes(10000, 4, C.byref(prm)) > 10000 * 4 * 4
    assert lib.sky_build_workspace_bytes(0, 4, C.byref(prm)) == 0
    assert lib.sky_build_workspace_bytes(100, 0, C.byref(prm)) == 0
    assert lib.sky_build_workspace_bytes(100, 17, C.byref(prm)) == 0
    bad = _lib.SkyParams(9, 64, 0, 0)
    assert lib.sky_build_workspace_bytes(100, 4, C.byref(bad)) == 0
    for reps in (-1, _lib.SKY_MAX_REPS + 1):  # Representative Filtering: 0..SKY_MAX_REPS
        bad_reps = _lib.SkyParams(_lib.SKY_NONE, 1, 0, reps)
        assert lib.sky_build_workspace_bytes(100, 4, C.byref(bad_reps)) == 0
    ok_reps = _lib.SkyParams(_lib.SKY_NONE, 1, 0, _lib.SKY_MAX_REPS)
    assert lib.sky_build_workspace_bytes(100, 4, C.byref(ok_reps)) > 0
    ang1 = _lib.SkyParams(_lib.SKY_ANGULAR, 16, 0, 0)
    assert lib.sky_build_workspace_bytes(100, 1, C.byref(ang1)) == 0  # Angular needs d >= 2
    big = _lib.SkyParams(_lib.SKY_GRID, 1 << 20, 0, 0)
    assert lib.sky_build_workspace_bytes(100, 8, C.byref(big)) == 0  # m^d above the cell limit
    assert lib.gres_workspace_bytes(1000, 6, 25) > 1000 * 6 * 4
    assert lib.gres_workspace_bytes(1000, 6, 1) == 0
    assert lib.gres_workspace_bytes(-1, 6, 25) == 0
    assert lib.gres_workspace_bytes(0, 6, 25) > 0


def test_argument_errors_return_synchronously(lib):
    fake = C.c_void_p(0x1000)  # never dereferenced: every call below fails its checks first
    prm = _lib.SkyParams(_lib.SKY_NONE, 1, 0, 0)
    h = C.c_void_p()
    E = _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_build(None, 10, 2, 10, C.byref(prm), fake, 1 << 20, fake, None, C.byref(h)) == E
    assert lib.sky_build(fake, 0, 2, 10, C.byref(prm), fake, 1 << 20, fake, None, C.byref(h)) == E
    assert lib.sky_build(fake, 10, 2, 5, C.byref(prm), fake, 1 << 20, fake, None, C.byref(h)) == E
    assert lib.sky_build(fake, 10, 2, 10, C.byref(prm), fake, 1 << 20, None, None, C.byref(h)) == E
    assert lib.sky_build(fake, 10, 2, 10, C.byref(prm), fake, 1, fake, None,
                         C.byref(h)) == _lib.SKY_ERR_WORKSPACE
    sl = _lib.SkyParams(_lib.SKY_SLICED, 4, 3, 0)  # slice_dim outside [0, d)
    assert lib.sky_build(fake, 10, 2, 10, C.byref(sl), fake, 1 << 20, fake, None, C.byref(h)) == E
    assert h.value is None
    assert lib.sky_local_skylines(None, None) == E
    assert lib.sky_merge(None, fake, 1, fake, None, None) == E
    assert lib.sky_plan_info(None, None) == E
    assert lib.sky_plan_partitions(None, fake, None) == E
    assert lib.sky_plan_local(None, fake, None) == E
    assert lib.sky_plan_partition_tests(None, fake, None) == E
    lib.sky_plan_destroy(None)
    assert lib.sky_ingest(fake, -1, 2, fake, 10, fake, None) == E
    assert lib.sky_ingest(fake, 10, 2, fake, 9, fake, None) == E
    assert lib.sky_ingest(None, 10, 2, fake, 10, fake, None) == E
    assert lib.sky_ingest(None, 0, 2, None, 0, None, None) == _lib.SKY_OK  # nothing to do
    o = _lib.GresOpts(0)
    assert lib.gres_compute(fake, 10, 2, 10, fake, 5, 1, fake, fake, fake, 1 << 20, fake,
                            C.byref(o), None) == E  # g_max < 2
    assert lib.gres_compute(fake, 10, 2, 10, fake, 5, 25, fake, fake, fake, 1 << 20, None,
                            C.byref(o), None) == E  # no status word
    assert lib.gres_compute(fake, 10, 2, 10, fake, 5, _lib.SKY_MAX_G + 1, fake, fake, fake, 1 << 20,
                            fake, C.byref(o), None) == E  # g_max above the limit
    assert lib.gres_compute(fake, 10, 2, 10, fake, 5, 25, fake, fake, fake, 16, fake,
                            C.byref(o), None) == _lib.SKY_ERR_WORKSPACE
    bad = _lib.GresOpts(9)
    assert lib.gres_compute(fake, 10, 2, 10, fake, 5, 25, fake, fake, fake, 1 << 20, fake,
                            C.byref(bad), None) == E
    assert lib.gres_compute(None, 0, 2, 0, None, 0, 25, None, None, None, 0, fake, None,
                            None) == _lib.SKY_OK  # s = 0: nothing to do


def test_gres_search_target_cap(lib):
    # target values are addressed with 32-bit byte offsets per attribute column: the target
    # count is capped like the rows of a plan (targets may repeat rows, so n does not bound it)
    cap = (1 << 30) - (1 << 20)
    assert lib.gres_search_bytes(cap, 6) > 0
    assert lib.gres_search_bytes(cap + 1, 6) == 0
    assert lib.gres_search_bytes(1 << 30, 1) == 0
    fake = C.c_void_p(0x1000)  # never dereferenced: the size check comes first
    assert lib.gres_search(fake, 10, 2, fake, 10, 10, fake, cap + 1, 25, fake, fake, fake, 1 << 40,
                           fake, None, None) == _lib.SKY_ERR_INVALID_ARG


def test_gres_noalloc_limits(lib):
    # the allocation-free gres_compute refuses work beyond its fixed workspace before any
    # device call, and checks its arguments like gres_compute
    fake = C.c_void_p(0x1000)  # never dereferenced: the checks come first
    assert _lib.SKY_NOALLOC_SCRATCH_BYTES == 64 << 20
    # the limit is the workspace without the packed key table (none above g_max 64)
    assert lib.gres_workspace_bytes(1000, 6, 25) > lib.gres_workspace_bytes(1000, 6, 65)
    assert lib.gres_workspace_bytes(1000, 6, 65) == lib.gres_workspace_bytes(1000, 6, 1 << 20)
    s_fit, s_over = 1, 1
    while lib.gres_workspace_bytes(s_over, 6, 65) <= _lib.SKY_NOALLOC_SCRATCH_BYTES:
        s_fit, s_over = s_over, s_over * 2
    while s_over - s_fit > 1:
        mid = (s_fit + s_over) // 2
        if lib.gres_workspace_bytes(mid, 6, 65) <= _lib.SKY_NOALLOC_SCRATCH_BYTES:
            s_fit = mid
        else:
            s_over = mid
    assert s_fit > 500_000  # the documented order of magnitude at d = 6
    assert lib.gres_compute_noalloc(fake, s_over, 6, s_over, fake, s_over, 25, fake, fake, fake,
                                    None, None) == _lib.SKY_ERR_UNSUPPORTED
    assert lib.gres_compute_noalloc(fake, 10, 6, 10, fake, 10, 1, fake, fake, fake, None,
                                    None) == _lib.SKY_ERR_INVALID_ARG  # g_max < 2
    assert lib.gres_compute_noalloc(fake, 10, 0, 10, fake, 10, 25, fake, fake, fake, None,
                                    None) == _lib.SKY_ERR_INVALID_ARG  # d < 1
    assert lib.gres_compute_noalloc(fake, 10, 6, 10, fake, 10, 25, fake, fake, None, None,
                                    None) == _lib.SKY_ERR_INVALID_ARG  # no status word


def test_literal_level_arguments(lib):
    fake = C.c_void_p(0x1000)  # never dereferenced: the checks come first
    assert lib.sky_literal_level(fake, -1, 5, fake, None, None) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_literal_level(fake, 10, 0, fake, None, None) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_literal_level(fake, 10, _lib.SKY_MAX_G + 1, fake, None, None) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_literal_level(None, 10, 5, fake, None, None) == _lib.SKY_ERR_INVALID_ARG  # member needed
    assert lib.sky_literal_level(fake, 10, 5, None, None, None) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_literal_level(None, 0, 5, None, None, None) == _lib.SKY_OK  # nothing to do


def test_sliced_workspace_holds_partition_histogram(lib):
    # Sliced partitions go through the same stable counting sort by partition as Grid/Angular,
    # so for equal p its workspace must hold the same histogram table (regression: it used to
    # reserve 64 entries and the table overran into the scan scratch).
    for n in (5003, 1_000_000, 10_000_000):
        ang = _lib.SkyParams(_lib.SKY_ANGULAR, 64, 0, 0)   # d = 4 -> m = 4, p = 64
        sli = _lib.SkyParams(_lib.SKY_SLICED, 64, 0, 0)
        assert lib.sky_build_workspace_bytes(n, 4, C.byref(sli)) >= \
            lib.sky_build_workspace_bytes(n, 4, C.byref(ang))
    too_many = _lib.SkyParams(_lib.SKY_SLICED, 5000, 0, 0)
    assert lib.sky_build_workspace_bytes(100000, 4, C.byref(too_many)) == 0


def test_batch_arguments(lib):
    I64 = C.c_int64
    off = (I64 * 4)(0, 10, 10, 25)
    assert lib.sky_batch_workspace_bytes(off, 3, 4) > 25 * 4 * 4
    assert lib.sky_batch_workspace_bytes(off, 3, 0) == 0
    assert lib.sky_batch_workspace_bytes(off, 3, 17) == 0
    assert lib.sky_batch_workspace_bytes(None, 3, 4) == 0
    assert lib.sky_batch_workspace_bytes(off, 0, 4) == 0
    bad = (I64 * 4)(0, 10, 9, 25)      # decreasing
    assert lib.sky_batch_workspace_bytes(bad, 3, 4) == 0
    bad0 = (I64 * 4)(1, 10, 10, 25)    # must start at 0
    assert lib.sky_batch_workspace_bytes(bad0, 3, 4) == 0
    empty = (I64 * 3)(0, 0, 0)         # no rows at all
    assert lib.sky_batch_workspace_bytes(empty, 2, 4) == 0
    many = (I64 * 4098)(*range(4098))  # more relations than SKY_MAX_CELLS
    assert lib.sky_batch_workspace_bytes(many, 4097, 2) == 0
    fake = C.c_void_p(0x1000)
    h = C.c_void_p()
    E = _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_batch_create(fake, 4, 25, off, 3, fake, 1 << 30, fake, None, None) == E
    assert lib.sky_batch_create(fake, 4, 24, off, 3, fake, 1 << 30, fake, None, C.byref(h)) == E
    assert lib.sky_batch_create(fake, 4, 25, bad, 3, fake, 1 << 30, fake, None, C.byref(h)) == E
    assert lib.sky_batch_create(fake, 4, 25, off, 3, fake, 16, fake, None,
                                C.byref(h)) == _lib.SKY_ERR_WORKSPACE
    assert h.value is None
    assert lib.sky_batch_skylines(None, fake, 1, fake, None) == E
    assert lib.sky_batch_tune(None, None, None) == E
    assert lib.sky_batch_gres(None, 25, None, None, None, None, None) == E
    assert lib.sky_batch_keys_bytes(None, 100, 25) == 0
    assert lib.sky_batch_set_keys(None, fake, 1 << 20, 100, 25) == E
    assert lib.sky_batch_info(None, None) == E
    lib.sky_batch_destroy(None)


def test_serving_arena_first_fit():
    from paper_2412_02274_amd.serve import Arena
    a = Arena(4096, "cpu")
    r1 = a.alloc(100)      # 256
    r2 = a.alloc(1000)     # 1024
    r3 = a.alloc(2000)     # 2048
    assert r1 == (0, 256) and r2 == (256, 1024) and r3 == (1280, 2048)
    assert a.alloc(1024) is None          # 768 left
    a.release(r2)
    assert a.alloc(1024) == (256, 1024)   # the freed range is reused
    a.release(r1)
    a.release((256, 1024))
    a.release(r3)
    assert a.free == [(0, 4096)] and a.used == 0  # neighbours merge back


def test_project_arguments(lib):
    fake = C.c_void_p(0x1000)
    E = _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_project(fake, 10, 2, 10, fake, 5, 0, fake, 5, fake, None) == E   # g < 1
    assert lib.sky_project(fake, 10, 2, 10, fake, 5, _lib.SKY_MAX_G + 1, fake, 5, fake, None) == E
    assert lib.sky_project(fake, 10, 2, 10, fake, 5, 25, fake, 4, fake, None) == E  # ld_out < s
    assert lib.sky_project(None, 10, 2, 10, fake, 5, 25, fake, 5, fake, None) == E
    assert lib.sky_project(fake, 10, 0, 10, fake, 5, 25, fake, 5, fake, None) == E
    assert lib.sky_project(None, 0, 2, 0, None, 0, 25, None, 0, None, None) == _lib.SKY_OK


def test_gbar_arguments(lib):
    fake = C.c_void_p(0x1000)
    E = _lib.SKY_ERR_INVALID_ARG
    ws = lib.gres_gbar_workspace_bytes(1000)
    assert ws > 4 * 4 * 1000 and lib.gres_gbar_workspace_bytes(-1) == 0
    assert lib.gres_gbar_workspace_bytes(0) > 0
    assert lib.gres_gbar(fake, 10, 2, 10, fake, fake, fake, ws, None, None) == E   # no status word
    assert lib.gres_gbar(fake, 10, 2, 10, None, None, fake, ws, fake, None) == E   # no output
    assert lib.gres_gbar(fake, 10, 0, 10, fake, fake, fake, ws, fake, None) == E   # d < 1
    assert lib.gres_gbar(fake, 10, 2, 9, fake, fake, fake, ws, fake, None) == E    # ld < n
    assert lib.gres_gbar(None, 10, 2, 10, fake, fake, fake, ws, fake, None) == E
    assert lib.gres_gbar(fake, -1, 2, 10, fake, fake, fake, ws, fake, None) == E
    assert lib.gres_gbar(fake, 1000, 2, 1000, fake, fake, fake, 16, fake,
                         None) == _lib.SKY_ERR_WORKSPACE
    assert lib.gres_gbar(fake, 1000, 2, 1000, fake, fake, None, ws, fake,
                         None) == _lib.SKY_ERR_WORKSPACE


def test_probe_arguments(lib):
    # the measurement probes check their arguments before any device call
    fake = C.c_void_p(0x1000)  # never dereferenced
    ops = C.c_int64()
    assert lib.sky_probe_valu(0, 64, fake, None, None, None, C.byref(ops)) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_probe_valu(10, 0, fake, None, None, None, C.byref(ops)) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_probe_valu(10, 64, None, None, None, None, C.byref(ops)) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_probe_valu(10, 64, fake, fake, None, None, C.byref(ops)) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_probe_copy(fake, fake, 0, None, None, None) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_probe_copy(fake, fake, 24, None, None, None) == _lib.SKY_ERR_INVALID_ARG  # not 16k
    assert lib.sky_probe_copy(C.c_void_p(0x1004), fake, 32, None, None, None) == _lib.SKY_ERR_INVALID_ARG
    assert lib.sky_probe_copy(None, fake, 32, None, None, None) == _lib.SKY_ERR_INVALID_ARG
