"""ctypes binding of libsky.so (the C ABI in include/sky.h). Argument marshalling only.

The library is loaded from this package directory; there is no fallback: if it is missing the
import of the compute entry points fails loudly (build it with ``python -m
paper_2412_02274_amd.build`` or ``__graft_entry__.build()``).
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsky.so")

SKY_OK = 0
SKY_ERR_INVALID_ARG = 1
SKY_ERR_DOMAIN = 2
SKY_ERR_WORKSPACE = 3
SKY_ERR_CAPACITY = 4
SKY_ERR_HIP = 5
SKY_ERR_STATE = 6
SKY_ERR_UNSUPPORTED = 7

SKY_NONE, SKY_GRID, SKY_ANGULAR, SKY_SLICED = 0, 1, 2, 3
SCHEMES = {"none": SKY_NONE, "grid": SKY_GRID, "angular": SKY_ANGULAR, "sliced": SKY_SLICED}

SKY_GRES_AUTO, SKY_GRES_TILES, SKY_GRES_LEVELS = 0, 1, 2
MAPPINGS = {"auto": SKY_GRES_AUTO, "tiles": SKY_GRES_TILES, "levels": SKY_GRES_LEVELS}

SKY_MAX_D = 16
SKY_MAX_CELLS = 4096
SKY_MAX_G = 16777216
SKY_MAX_REPS = 1024
SKY_KILLERS = 8
SKY_NOALLOC_SCRATCH_BYTES = 64 << 20

# every function the header declares (checked against the header by the tests)
EXPORTS = ("sky_status_string", "sky_version", "sky_ingest", "sky_build_workspace_bytes",
           "sky_build", "sky_local_skylines", "sky_merge", "sky_plan_partitions", "sky_plan_local",
           "sky_plan_partition_tests", "sky_plan_set_events",
           "sky_plan_info", "sky_plan_destroy",
           "gres_workspace_bytes", "gres_compute", "gres_prepare_bytes", "gres_prepare",
           "gres_search_bytes", "gres_search",
           "sky_batch_workspace_bytes", "sky_batch_create", "sky_batch_skylines", "sky_batch_tune",
           "sky_batch_gres", "sky_batch_keys_bytes", "sky_batch_set_keys", "sky_batch_info",
           "sky_batch_destroy", "sky_project",
           "gres_gbar_workspace_bytes", "gres_gbar", "sky_gres",
           "gres_compute_noalloc", "sky_literal_level", "sky_probe_valu", "sky_probe_copy")


class SkyParams(C.Structure):
    _fields_ = [("scheme", C.c_int32), ("target_p", C.c_int32), ("slice_dim", C.c_int32),
                ("reps", C.c_int32), ("prefilter_off", C.c_int32)]


class SkyInfo(C.Structure):
    _fields_ = [("n", C.c_int64), ("d", C.c_int32), ("scheme", C.c_int32), ("p", C.c_int32),
                ("m", C.c_int32), ("pruned_cells", C.c_int32), ("rounds_local", C.c_int32),
                ("rounds_merge", C.c_int32), ("state", C.c_int32), ("pruned_rows", C.c_int64),
                ("local_count", C.c_int64), ("sky_count", C.c_int64), ("tests_local", C.c_int64),
                ("tests_merge", C.c_int64), ("max_partition", C.c_int64),
                ("events_used", C.c_int32), ("reps_kept", C.c_int32),
                ("tests_local_max", C.c_int64), ("rows_kept", C.c_int64),
                ("tests_prefilter", C.c_int64), ("tests_gres", C.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class GresOpts(C.Structure):
    _fields_ = [("mapping", C.c_int32), ("reserved", C.c_int32), ("ev_begin", C.c_void_p),
                ("ev_end", C.c_void_p), ("dev_tests", C.c_void_p)]


class SkyTune(C.Structure):
    _fields_ = [("mapping", C.c_int32), ("near_first", C.c_int32), ("lpt", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class SkyError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = int(code)
        super().__init__(f"{where}: {status_string(code)}")


_lib = None


def load():
    """Load libsky.so and declare the signatures. Raises if the library was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsky.so not found at {LIB_PATH}; build it first "
                          "(python -m paper_2412_02274_amd.build)")
    lib = C.CDLL(LIB_PATH)
    vp, i64, i32, sz = C.c_void_p, C.c_int64, C.c_int32, C.c_size_t
    sig = {
        "sky_status_string": (C.c_char_p, [i32]),
        "sky_version": (i32, []),
        "sky_ingest": (i32, [vp, i64, i32, vp, i64, vp, vp]),
        "sky_build_workspace_bytes": (sz, [i64, i32, C.POINTER(SkyParams)]),
        "sky_build": (i32, [vp, i64, i32, i64, C.POINTER(SkyParams), vp, sz, vp, vp,
                            C.POINTER(vp)]),
        "sky_local_skylines": (i32, [vp, vp]),
        "sky_merge": (i32, [vp, vp, i64, vp, vp, vp]),
        "sky_plan_partitions": (i32, [vp, vp, vp]),
        "sky_plan_local": (i32, [vp, vp, vp]),
        "sky_plan_partition_tests": (i32, [vp, vp, vp]),
        "sky_plan_set_events": (i32, [vp, vp, vp, i32]),
        "sky_plan_info": (i32, [vp, C.POINTER(SkyInfo)]),
        "sky_plan_destroy": (None, [vp]),
        "gres_workspace_bytes": (sz, [i64, i32, i32]),
        "gres_compute": (i32, [vp, i64, i32, i64, vp, i64, i32, vp, vp, vp, sz, vp,
                               C.POINTER(GresOpts), vp]),
        "gres_prepare_bytes": (sz, [i64, i32]),
        "gres_prepare": (i32, [vp, i64, i32, i64, vp, i64, vp, sz, vp, vp]),
        "gres_search_bytes": (sz, [i64, i32]),
        "gres_search": (i32, [vp, i64, i32, vp, i64, i64, vp, i64, i32, vp, vp, vp, sz, vp,
                              C.POINTER(GresOpts), vp]),
        "sky_batch_workspace_bytes": (sz, [C.POINTER(i64), i32, i32]),
        "sky_batch_create": (i32, [vp, i32, i64, C.POINTER(i64), i32, vp, sz, vp, vp, C.POINTER(vp)]),
        "sky_batch_skylines": (i32, [vp, vp, i64, vp, vp]),
        "sky_batch_tune": (i32, [vp, C.POINTER(SkyTune), vp]),
        "sky_batch_gres": (i32, [vp, i32, vp, vp, vp, vp, vp]),
        "sky_batch_keys_bytes": (sz, [vp, i64, i32]),
        "sky_batch_set_keys": (i32, [vp, vp, sz, i64, i32]),
        "sky_batch_info": (i32, [vp, C.POINTER(SkyInfo)]),
        "sky_batch_destroy": (None, [vp]),
        "sky_project": (i32, [vp, i64, i32, i64, vp, i64, i32, vp, i64, vp, vp]),
        "gres_gbar_workspace_bytes": (sz, [i64]),
        "gres_gbar": (i32, [vp, i64, i32, i64, vp, vp, vp, sz, vp, vp]),
        "sky_gres": (i32, [vp, i32, vp, vp, vp, sz, vp, C.POINTER(GresOpts), vp]),
        "sky_literal_level": (i32, [vp, i64, i32, vp, vp, vp]),
        "gres_compute_noalloc": (i32, [vp, i64, i32, i64, vp, i64, i32, vp, vp, vp,
                                       C.POINTER(GresOpts), vp]),
        "sky_probe_valu": (i32, [i64, i32, vp, vp, vp, vp, C.POINTER(i64)]),
        "sky_probe_copy": (i32, [vp, vp, i64, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def status_string(code: int) -> str:
    try:
        return load().sky_status_string(int(code)).decode()
    except ImportError:
        return f"status {code}"


def check(code: int, where: str):
    if code != SKY_OK:
        raise SkyError(code, where)
