"""The oracle -- TEST INFRASTRUCTURE ONLY.

Plain CPU implementations of the skyline and grid-resistance computations, written from the
paper's definitions (Def. 1, Def. 2, Def. 3, Eq. (1), Alg. 1 of arXiv 2412.02274). Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import this package; the GPU
library never does, and the two share no code.

``sky_oracle.c`` (compiled by ``oracle/build.py`` with gcc, IEEE semantics, no FMA) holds the
nested-loop definitions; ``brute.py`` holds a literal, set-based Python reading of Def. 2 for
tiny inputs (FP32 and exact rationals). This module marshals numpy arrays for the C library:
inputs are row-major ``float32 [N, d]``; they are transposed to the structure-of-arrays
layout ``x[k*N + i]`` the C code reads.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_f32p = C.POINTER(C.c_float)
_i64p = C.POINTER(C.c_int64)
_i32p = C.POINTER(C.c_int32)
_u8p = C.POINTER(C.c_uint8)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    sig = {
        "orc_count_invalid": (C.c_int64, [_f32p, C.c_int64, C.c_int32, C.c_int64]),
        "orc_skyline": (None, [_f32p, C.c_int64, C.c_int32, C.c_int64, _u8p]),
        "orc_skyline_sfs": (C.c_int64, [_f32p, C.c_int64, C.c_int32, C.c_int64, _u8p]),
        "orc_local_skylines": (None, [_f32p, C.c_int64, C.c_int32, C.c_int64, _i32p, _u8p, _u8p]),
        "orc_grid_part": (None, [_f32p, C.c_int64, C.c_int32, C.c_int64, C.c_int32, _i32p]),
        "orc_grid_pruned": (None, [_u8p, C.c_int32, C.c_int32, _u8p]),
        "orc_angular_part": (None, [_f32p, C.c_int64, C.c_int32, C.c_int64, C.c_int32, _i32p, _i32p]),
        "orc_sliced_part": (None, [_f32p, C.c_int64, C.c_int32, C.c_int64, C.c_int32, C.c_int32, _i32p]),
        "orc_closest_m": (C.c_int32, [C.c_int64, C.c_int32]),
        "orc_gres": (None, [_f32p, C.c_int64, C.c_int32, C.c_int64, _i64p, C.c_int64, C.c_int32,
                            _i32p, _i64p]),
        "orc_gres_rows": (None, [_f32p, C.c_int64, C.c_int32, C.c_int64, _i64p, C.c_int64, _i64p,
                                 C.c_int64, C.c_int32, _i32p]),
        "orc_skyline_rows": (None, [_f32p, C.c_int64, C.c_int32, C.c_int64, _i64p, C.c_int64, _u8p]),
        "orc_key": (C.c_int32, [C.c_float, C.c_int32]),
        "orc_ell": (C.c_double, [_f32p, C.c_int64, C.c_int32, C.c_int64]),
        "orc_ell_sorted": (C.c_double, [_f32p, C.c_int64, C.c_int32, C.c_int64]),
        "orc_gbar": (C.c_double, [C.c_double]),
        "orc_representatives": (C.c_int64, [_f32p, C.c_int64, C.c_int32, C.c_int64, C.c_int64, _i64p,
                                            _u8p]),
        "orc_dominated_by": (None, [_f32p, C.c_int64, C.c_int32, C.c_int64, _i64p, C.c_int64, _u8p]),
        "orc_num_threads": (C.c_int32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _p(a, t):
    return a.ctypes.data_as(t)


def _soa(x: np.ndarray):
    x = np.asarray(x, dtype=np.float32)
    if x.ndim != 2:
        raise ValueError("expected a [N, d] array")
    n, d = x.shape
    return np.ascontiguousarray(x.T), n, d


def num_threads() -> int:
    return int(_load().orc_num_threads())


def count_invalid(x) -> int:
    xs, n, d = _soa(x)
    return int(_load().orc_count_invalid(_p(xs, _f32p), n, d, n))


def skyline(x) -> np.ndarray:
    """Def. 1 by nested loops: boolean membership per row."""
    xs, n, d = _soa(x)
    m = np.zeros(n, dtype=np.uint8)
    _load().orc_skyline(_p(xs, _f32p), n, d, n, _p(m, _u8p))
    return m.astype(bool)


def skyline_sfs(x):
    """SFS (presort by FP32 attribute sum, window scan): (membership, dominance tests)."""
    xs, n, d = _soa(x)
    m = np.zeros(n, dtype=np.uint8)
    tests = _load().orc_skyline_sfs(_p(xs, _f32p), n, d, n, _p(m, _u8p))
    return m.astype(bool), int(tests)


def skyline_rows(x, rows) -> np.ndarray:
    xs, n, d = _soa(x)
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    m = np.zeros(len(rows), dtype=np.uint8)
    _load().orc_skyline_rows(_p(xs, _f32p), n, d, n, _p(rows, _i64p), len(rows), _p(m, _u8p))
    return m.astype(bool)


def local_skylines(x, part, skip=None) -> np.ndarray:
    xs, n, d = _soa(x)
    part = np.ascontiguousarray(part, dtype=np.int32)
    out = np.zeros(n, dtype=np.uint8)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.uint8)
    _load().orc_local_skylines(_p(xs, _f32p), n, d, n, _p(part, _i32p),
                               None if sk is None else _p(sk, _u8p), _p(out, _u8p))
    return out.astype(bool)


def grid_part(x, m: int) -> np.ndarray:
    xs, n, d = _soa(x)
    part = np.zeros(n, dtype=np.int32)
    _load().orc_grid_part(_p(xs, _f32p), n, d, n, m, _p(part, _i32p))
    return part


def grid_pruned(nonempty, m: int, d: int) -> np.ndarray:
    ne = np.ascontiguousarray(nonempty, dtype=np.uint8)
    if ne.size != m ** d:
        raise ValueError("nonempty must have m**d entries")
    out = np.zeros(m ** d, dtype=np.uint8)
    _load().orc_grid_pruned(_p(ne, _u8p), m, d, _p(out, _u8p))
    return out.astype(bool)


def angular_part(x, m: int):
    """Eq. (1): (partition ids, near-boundary masks). Bit a of mask[i] is set when angle a of
    row i lies within 1e-9 of a bucket boundary (there an equally faithful evaluation may give
    the neighbouring bucket of that angle); 0 for every other row."""
    xs, n, d = _soa(x)
    part = np.zeros(n, dtype=np.int32)
    near = np.zeros(n, dtype=np.int32)
    _load().orc_angular_part(_p(xs, _f32p), n, d, n, m, _p(part, _i32p), _p(near, _i32p))
    return part, near


def sliced_part(x, p: int, dim: int = 0) -> np.ndarray:
    xs, n, d = _soa(x)
    part = np.zeros(n, dtype=np.int32)
    _load().orc_sliced_part(_p(xs, _f32p), n, d, n, dim, p, _p(part, _i32p))
    return part


def closest_m(target: int, e: int) -> int:
    return int(_load().orc_closest_m(target, e))


def key(v: float, g: int) -> int:
    return int(_load().orc_key(C.c_float(v), g))


def gres(x, cand, g_max: int):
    """Def. 2 over candidate rows ``cand`` (normally Sky(r)), levels 2..g_max as in Alg. 1:
    (g_exit[len(cand)], tests).
    gres = 1 / g_exit; g_exit == 1 means the tuple never left the skyline."""
    xs, n, d = _soa(x)
    cand = np.ascontiguousarray(cand, dtype=np.int64)
    ge = np.zeros(len(cand), dtype=np.int32)
    tests = C.c_int64(0)
    _load().orc_gres(_p(xs, _f32p), n, d, n, _p(cand, _i64p), len(cand), g_max, _p(ge, _i32p),
                     C.byref(tests))
    return ge, int(tests.value)


def gres_rows(x, cand, targets, g_max: int) -> np.ndarray:
    xs, n, d = _soa(x)
    cand = np.ascontiguousarray(cand, dtype=np.int64)
    targets = np.ascontiguousarray(targets, dtype=np.int64)
    ge = np.zeros(len(targets), dtype=np.int32)
    _load().orc_gres_rows(_p(xs, _f32p), n, d, n, _p(cand, _i64p), len(cand), _p(targets, _i64p),
                          len(targets), g_max, _p(ge, _i32p))
    return ge


def ell(x, sorted_: bool = False) -> float:
    """Sec. 3.2's ell: the smallest non-zero difference between two values of one attribute
    (FP64 differences), +inf when there is none. ``sorted_`` uses the sort-based form."""
    xs, n, d = _soa(x)
    fn = _load().orc_ell_sorted if sorted_ else _load().orc_ell
    return float(fn(_p(xs, _f32p), n, d, n))


def gbar(x, sorted_: bool = True):
    """(ell, g_bar) with g_bar = floor(1/ell) as a Python int (1 when ell is +inf)."""
    e = ell(x, sorted_)
    return e, int(_load().orc_gbar(e))


def representatives(x, k: int):
    """Representative Filtering (Sec. 3.1): (rows of the k smallest FP32 attribute sums, ties in
    row order; kept flags = not dominated by another representative)."""
    xs, n, d = _soa(x)
    k = min(int(k), n)
    rows = np.zeros(max(k, 1), dtype=np.int64)
    kept = np.zeros(max(k, 1), dtype=np.uint8)
    _load().orc_representatives(_p(xs, _f32p), n, d, n, k, _p(rows, _i64p), _p(kept, _u8p))
    return rows[:k], kept[:k].astype(bool)


def dominated_by(x, by) -> np.ndarray:
    """Rows of x dominated by some row listed in ``by`` (Def. 1)."""
    xs, n, d = _soa(x)
    by = np.ascontiguousarray(by, dtype=np.int64)
    out = np.zeros(n, dtype=np.uint8)
    _load().orc_dominated_by(_p(xs, _f32p), n, d, n, _p(by, _i64p), len(by), _p(out, _u8p))
    return out.astype(bool)


def local_skylines_reps(x, part, skip, k: int):
    """Local skylines with Representative Filtering: rows of each partition's skyline that no
    kept representative dominates."""
    rows, kept = representatives(x, k)
    return local_skylines(x, part, skip) & ~dominated_by(x, rows[kept])


def gres_values(g_exit) -> np.ndarray:
    """gres = 1/g_exit in FP32 (Def. 2; 1 when the tuple never exits)."""
    return (np.float32(1.0) / np.asarray(g_exit).astype(np.float32)).astype(np.float32)


def grid_p(target: int, d: int):
    """(m, p) for Grid partitioning at the target number of partitions."""
    m = closest_m(target, d)
    return m, m ** d


def angular_p(target: int, d: int):
    if d < 2:
        raise ValueError("angular partitioning needs d >= 2")
    m = closest_m(target, d - 1)
    return m, m ** (d - 1)
