"""Python entry points over libsky, with torch owning device memory and streams.

Every step of the path runs in libsky's HIP kernels; this module only allocates tensors,
marshals pointers and reads back counts. Names follow the C ABI in include/sky.h:

    x_soa  = ingest(x_rows)                                   # validate + [N, d] -> SoA [d, N]
    plan   = build(x_soa, scheme="grid", target_p=64)         # partitions (Sec. 3.1)
    plan.local_skylines()                                     # Sec. 3, phase 1
    sky    = plan.merge()                                     # Sec. 3, phase 2 -> Sky(r) rows
    g_exit, gres_v = gres(x_soa, sky, g_max=25)               # Def. 2 via Alg. 1

Data-dependent errors are raised after the stream is synchronised (``check_status``).
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import SkyError

__all__ = ["ingest", "build", "Plan", "Pipeline", "PreparedCandidates", "gres", "skyline",
           "project", "gres_literal", "gres_noalloc",
           "gres_workspace_bytes",
           "build_workspace_bytes", "check_status", "SkyError"]


def _stream_ptr(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def new_status(device="cuda") -> torch.Tensor:
    return torch.zeros(1, dtype=torch.int32, device=device)


def check_status(status: torch.Tensor, where: str = "device"):
    code = int(status.item())
    if code != _lib.SKY_OK:
        raise SkyError(code, where)


def ingest(x_rows: torch.Tensor, status: torch.Tensor | None = None, stream=None,
           out: torch.Tensor | None = None) -> torch.Tensor:
    """Validate a row-major float32 [N, d] device tensor and return its SoA copy [d, N]."""
    lib = _lib.load()
    if x_rows.dtype != torch.float32 or x_rows.dim() != 2 or not x_rows.is_cuda:
        raise ValueError("x_rows must be a float32 [N, d] CUDA tensor")
    x_rows = x_rows.contiguous()
    n, d = x_rows.shape
    if out is None:
        out = torch.empty((d, n), dtype=torch.float32, device=x_rows.device)
    st = status if status is not None else new_status(x_rows.device)
    _lib.check(lib.sky_ingest(_ptr(x_rows), n, d, _ptr(out), n, _ptr(st), _stream_ptr(stream)),
               "sky_ingest")
    if status is None:
        check_status(st, "sky_ingest")
    return out


def _params(scheme, target_p, slice_dim, reps=0, prefilter=True):
    code = _lib.SCHEMES[scheme] if isinstance(scheme, str) else int(scheme)
    return _lib.SkyParams(code, int(target_p), int(slice_dim), int(reps), 0 if prefilter else 1)


def build_workspace_bytes(n: int, d: int, scheme="none", target_p: int = 16,
                          slice_dim: int = 0, reps: int = 0) -> int:
    prm = _params(scheme, target_p, slice_dim, reps)
    return int(_lib.load().sky_build_workspace_bytes(n, d, C.byref(prm)))


class Plan:
    """A built partitioning of one relation (owns its workspace tensor)."""

    def __init__(self, handle, ws, status, x_soa, stream):
        self._h = handle
        self.ws = ws
        self.status = status
        self.x_soa = x_soa
        self.stream = stream
        self.sky_idx = None
        self.count = None
        self.cap = 0

    def local_skylines(self):
        _lib.check(_lib.load().sky_local_skylines(self._h, _stream_ptr(self.stream)),
                   "sky_local_skylines")
        return self

    def merge(self, member: bool = False, cap: int | None = None):
        """sky_merge, then the count is read back: the skyline's rows (ascending), and with
        member=True also the uint8[n] membership flags."""
        lib = _lib.load()
        n = self.x_soa.shape[1]
        cap = n if cap is None else cap
        self.cap = cap
        dev = self.x_soa.device
        self.sky_idx = torch.empty(max(cap, 1), dtype=torch.int64, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)
        mem = torch.empty(n, dtype=torch.uint8, device=dev) if member else None
        _lib.check(lib.sky_merge(self._h, _ptr(self.sky_idx), cap, _ptr(self.count), _ptr(mem),
                                 _stream_ptr(self.stream)), "sky_merge")
        s = int(self.count.item())  # synchronises
        check_status(self.status, "sky_merge")
        out = self.sky_idx[:s]
        return (out, mem) if member else out

    def gres(self, g_max: int = 25, mapping="auto"):
        """sky_gres after merge(): (g_exit int32[s], gres float32[s]) aligned with the skyline
        merge() returned (the plan's own skyline as candidates and tuples)."""
        lib = _lib.load()
        inf = self.info()
        s, d = int(inf["sky_count"]), self.x_soa.shape[0]
        dev = self.x_soa.device
        # sky_gres reads the skyline size on the device; its workspace holds sky_merge's cap
        c = max(1, min(self.cap, self.x_soa.shape[1]))
        need = int(lib.gres_workspace_bytes(c, d, g_max))
        if need == 0:
            raise SkyError(_lib.SKY_ERR_INVALID_ARG, "gres_workspace_bytes")
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
        ge = torch.empty(max(s, 1), dtype=torch.int32, device=dev)
        gr = torch.empty(max(s, 1), dtype=torch.float32, device=dev)
        opts = _lib.GresOpts(_lib.MAPPINGS[mapping] if isinstance(mapping, str) else int(mapping))
        _lib.check(lib.sky_gres(self._h, g_max, _ptr(ge), _ptr(gr), _ptr(ws), need, _ptr(self.status),
                                C.byref(opts), _stream_ptr(self.stream)), "sky_gres")
        torch.cuda.current_stream().synchronize() if self.stream is None else self.stream.synchronize()
        check_status(self.status, "sky_gres")
        return ge[:s], gr[:s]

    def partitions(self) -> torch.Tensor:
        """Partition of every original row (int32[n])."""
        part = torch.empty(self.x_soa.shape[1], dtype=torch.int32, device=self.x_soa.device)
        _lib.check(_lib.load().sky_plan_partitions(self._h, _ptr(part), _stream_ptr(self.stream)),
                   "sky_plan_partitions")
        return part

    def local_members(self) -> torch.Tensor:
        """1 for rows in the skyline of their own (non-pruned) partition (uint8[n])."""
        loc = torch.empty(self.x_soa.shape[1], dtype=torch.uint8, device=self.x_soa.device)
        _lib.check(_lib.load().sky_plan_local(self._h, _ptr(loc), _stream_ptr(self.stream)),
                   "sky_plan_local")
        return loc

    def partition_tests(self) -> torch.Tensor:
        """Local-phase dominance tests per partition (int64[p]); their maximum is the parallel
        phase's cost as Sec. 4 counts it."""
        p = int(self.info()["p"])
        out = torch.zeros(p, dtype=torch.int64, device=self.x_soa.device)
        if p == 0:  # Sliced over no rows
            return out
        _lib.check(_lib.load().sky_plan_partition_tests(self._h, _ptr(out), _stream_ptr(self.stream)),
                   "sky_plan_partition_tests")
        return out

    def info(self) -> dict:
        inf = _lib.SkyInfo()
        _lib.check(_lib.load().sky_plan_info(self._h, C.byref(inf)), "sky_plan_info")
        return inf.as_dict()

    def close(self):
        if self._h:
            _lib.load().sky_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def build(x_soa: torch.Tensor, scheme="none", target_p: int = 16, slice_dim: int = 0,
          status: torch.Tensor | None = None, stream=None, ws: torch.Tensor | None = None,
          reps: int = 0, prefilter: bool = True) -> Plan:
    """Partition assignment + partition-contiguous copy (sky_build). reps: Representative
    Filtering (Sec. 3.1), the number of representatives (0 = off). prefilter: drop the rows
    that a killer row of their own partition dominates before sorting (no effect on any
    result; sky_params.prefilter_off)."""
    lib = _lib.load()
    if x_soa.dtype != torch.float32 or x_soa.dim() != 2 or not x_soa.is_cuda:
        raise ValueError("x_soa must be a float32 [d, N] CUDA tensor")
    d, n = x_soa.shape
    ld = x_soa.stride(0)
    if x_soa.stride(1) != 1:
        raise ValueError("x_soa rows must be contiguous")
    prm = _params(scheme, target_p, slice_dim, reps, prefilter)
    need = int(lib.sky_build_workspace_bytes(n, d, C.byref(prm)))
    if need == 0:
        raise SkyError(_lib.SKY_ERR_INVALID_ARG, "sky_build_workspace_bytes")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=x_soa.device)
    st = status if status is not None else new_status(x_soa.device)
    h = C.c_void_p()
    _lib.check(lib.sky_build(_ptr(x_soa), n, d, ld, C.byref(prm), _ptr(ws), need, _ptr(st),
                             _stream_ptr(stream), C.byref(h)), "sky_build")
    return Plan(h, ws, st, x_soa, stream)


def gres_workspace_bytes(s: int, d: int, g_max: int) -> int:
    return int(_lib.load().gres_workspace_bytes(s, d, g_max))


def gres(x_soa: torch.Tensor, sky_idx: torch.Tensor, g_max: int = 25, mapping="auto",
         status: torch.Tensor | None = None, stream=None, ws: torch.Tensor | None = None,
         g_exit: torch.Tensor | None = None, gres_out: torch.Tensor | None = None):
    """gres_compute: (g_exit int32[s], gres float32[s]) for the rows sky_idx of x_soa."""
    lib = _lib.load()
    d, n = x_soa.shape
    s = sky_idx.numel()
    dev = x_soa.device
    if sky_idx.dtype != torch.int64:
        raise ValueError("sky_idx must be int64")
    sky_idx = sky_idx.contiguous()
    need = int(lib.gres_workspace_bytes(s, d, g_max))
    if need == 0:
        raise SkyError(_lib.SKY_ERR_INVALID_ARG, "gres_workspace_bytes")
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    if g_exit is None:
        g_exit = torch.empty(s, dtype=torch.int32, device=dev)
    if gres_out is None:
        gres_out = torch.empty(s, dtype=torch.float32, device=dev)
    st = status if status is not None else new_status(dev)
    opts = _lib.GresOpts(_lib.MAPPINGS[mapping] if isinstance(mapping, str) else int(mapping))
    _lib.check(lib.gres_compute(_ptr(x_soa), n, d, x_soa.stride(0), _ptr(sky_idx), s, g_max,
                                _ptr(g_exit), _ptr(gres_out), _ptr(ws), need, _ptr(st),
                                C.byref(opts), _stream_ptr(stream)), "gres_compute")
    if status is None:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        check_status(st, "gres_compute")
    return g_exit, gres_out


def gres_noalloc(x_soa: torch.Tensor, sky_idx: torch.Tensor, g_max: int = 25, mapping="auto",
                 status: torch.Tensor | None = None, stream=None,
                 g_exit: torch.Tensor | None = None, gres_out: torch.Tensor | None = None):
    """gres_compute_noalloc: gres_compute with the library's fixed per-device workspace (no
    workspace tensor); (g_exit int32[s], gres float32[s]) for the rows sky_idx of x_soa."""
    lib = _lib.load()
    d, n = x_soa.shape
    s = sky_idx.numel()
    dev = x_soa.device
    if sky_idx.dtype != torch.int64:
        raise ValueError("sky_idx must be int64")
    sky_idx = sky_idx.contiguous()
    if g_exit is None:
        g_exit = torch.empty(s, dtype=torch.int32, device=dev)
    if gres_out is None:
        gres_out = torch.empty(s, dtype=torch.float32, device=dev)
    st = status if status is not None else new_status(dev)
    opts = _lib.GresOpts(_lib.MAPPINGS[mapping] if isinstance(mapping, str) else int(mapping))
    _lib.check(lib.gres_compute_noalloc(_ptr(x_soa), n, d, x_soa.stride(0), _ptr(sky_idx), s, g_max,
                                        _ptr(g_exit), _ptr(gres_out), _ptr(st), C.byref(opts),
                                        _stream_ptr(stream)), "gres_compute_noalloc")
    if status is None:
        torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
        check_status(st, "gres_compute_noalloc")
    return g_exit, gres_out


def gbar(x_soa: torch.Tensor, status: torch.Tensor | None = None, stream=None):
    """gres_gbar: (ell, g_bar) of Alg. 1's level range (Sec. 3.2) for the relation x_soa, read
    back to the host: ell as a float (+inf when no attribute holds two different values), g_bar
    = floor(1/ell) as an int (saturated at 2^62; 1 when ell is +inf)."""
    lib = _lib.load()
    d, n = x_soa.shape
    dev = x_soa.device
    need = int(lib.gres_gbar_workspace_bytes(n))
    if need == 0:
        raise SkyError(_lib.SKY_ERR_INVALID_ARG, "gres_gbar_workspace_bytes")
    ws = torch.empty(need, dtype=torch.uint8, device=dev)
    ell = torch.empty(1, dtype=torch.float64, device=dev)
    gb = torch.empty(1, dtype=torch.int64, device=dev)
    st = status if status is not None else new_status(dev)
    _lib.check(lib.gres_gbar(_ptr(x_soa), n, d, x_soa.stride(0), _ptr(ell), _ptr(gb), _ptr(ws), need,
                             _ptr(st), _stream_ptr(stream)), "gres_gbar")
    torch.cuda.current_stream().synchronize() if stream is None else stream.synchronize()
    check_status(st, "gres_gbar")
    return float(ell.item()), int(gb.item())


def gres_exact(x_soa: torch.Tensor, sky_idx: torch.Tensor, mapping="auto", status=None, stream=None):
    """Def. 2 over Alg. 1's whole level range: g_max = g_bar = floor(1/ell) from gres_gbar, capped
    at SKY_MAX_G (the largest level at which the key contract's (float)g is exact). Returns
    (g_exit, gres, info) with info = {"ell", "g_bar", "g_max", "capped"}; when capped is True,
    levels above SKY_MAX_G were not searched."""
    ell, gb = gbar(x_soa, status=status, stream=stream)
    # g_bar = 1 leaves no level to search; level 2 is then above g_bar and cannot hold an exit
    # (and gres_compute needs g_max >= 2), so searching it gives the same all-ones answer
    g_max = max(2, min(gb, _lib.SKY_MAX_G))
    info = {"ell": ell, "g_bar": gb, "g_max": g_max, "capped": gb > _lib.SKY_MAX_G}
    ge, gr = gres(x_soa, sky_idx, g_max, mapping=mapping, status=status, stream=stream)
    return ge, gr, info


class PreparedCandidates:
    """A candidate set (normally a skyline) prepared once for many gres searches."""

    def __init__(self, x_soa: torch.Tensor, cand_idx: torch.Tensor, status=None, stream=None):
        lib = _lib.load()
        self.x_soa = x_soa
        self.d, self.n = x_soa.shape
        self.s = int(cand_idx.numel())
        self.cand_idx = cand_idx.contiguous()
        nb = int(lib.gres_prepare_bytes(self.s, self.d))
        if nb == 0:
            raise SkyError(_lib.SKY_ERR_INVALID_ARG, "gres_prepare_bytes")
        self.prep = torch.empty(nb, dtype=torch.uint8, device=x_soa.device)
        self.status = status if status is not None else new_status(x_soa.device)
        _lib.check(lib.gres_prepare(_ptr(x_soa), self.n, self.d, x_soa.stride(0),
                                    _ptr(self.cand_idx), self.s, _ptr(self.prep), nb,
                                    _ptr(self.status), _stream_ptr(stream)), "gres_prepare")

    def search(self, targets: torch.Tensor | None = None, g_max: int = 25, mapping="auto",
               stream=None, status=None, ws=None, g_exit=None, gres_out=None, check=True):
        """(g_exit, gres) for `targets` (row indices of x), or for every candidate if None."""
        lib = _lib.load()
        nt = self.s if targets is None else int(targets.numel())
        dev = self.x_soa.device
        need = int(lib.gres_search_bytes(nt, self.d))
        if ws is None or ws.numel() < need:
            ws = torch.empty(max(need, 1), dtype=torch.uint8, device=dev)
        if g_exit is None:
            g_exit = torch.empty(nt, dtype=torch.int32, device=dev)
        if gres_out is None:
            gres_out = torch.empty(nt, dtype=torch.float32, device=dev)
        st = status if status is not None else self.status
        opts = _lib.GresOpts(_lib.MAPPINGS[mapping] if isinstance(mapping, str) else int(mapping))
        tptr = None if targets is None else _ptr(targets)
        _lib.check(lib.gres_search(_ptr(self.prep), self.s, self.d, _ptr(self.x_soa), self.n,
                                   self.x_soa.stride(0), tptr, nt, g_max, _ptr(g_exit),
                                   _ptr(gres_out), _ptr(ws), need, _ptr(st), C.byref(opts),
                                   _stream_ptr(stream)), "gres_search")
        if check:
            (stream or torch.cuda.current_stream()).synchronize()
            check_status(st, "gres_search")
        return g_exit, gres_out


def project(x_soa: torch.Tensor, rows: torch.Tensor, g: int, out: torch.Tensor | None = None,
            status: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Grid projection (Def. 2) of rows of x at level g as an SoA relation [d, s] of scaled keys
    (``sky_project``)."""
    lib = _lib.load()
    d, n = x_soa.shape
    s = int(rows.numel())
    if out is None:
        out = torch.empty((d, max(s, 1)), dtype=torch.float32, device=x_soa.device)
    st = status if status is not None else new_status(x_soa.device)
    _lib.check(lib.sky_project(_ptr(x_soa), n, d, x_soa.stride(0), _ptr(rows), s, int(g), _ptr(out),
                               out.stride(0), _ptr(st), _stream_ptr(stream)), "sky_project")
    if status is None:
        check_status(st, "sky_project")
    return out


def gres_literal(x_soa: torch.Tensor, sky_idx: torch.Tensor, g_max: int = 25, scheme="none",
                 target_p: int = 16, slice_dim: int = 0, reps: int = 0, prefilter: bool = True):
    """Alg. 1 as written: for g = g_max .. 2, the skyline of the grid projection of the candidate
    set (Sky(r)) is computed through the two-phase partitioned scheme (build, local skylines,
    merge on the projected relation); every candidate not in it that has no value yet gets
    g_exit = g, on the device (sky_literal_level); the host only reads how many are left, to stop
    once none is. Returns (g_exit int32[s] on the host, per-level statistics). Equal to
    ``gres()`` for every input (gres is stable and dominance between projections is the per-tuple
    test); kept to run the paper's own formulation and count its work. reps > 0 applies
    Representative Filtering (Sec. 3.1) inside every level's skyline; prefilter as in
    ``build``."""
    lib = _lib.load()
    s = int(sky_idx.numel())
    d = x_soa.shape[0]
    dev = x_soa.device
    if s == 0:
        return torch.ones(0, dtype=torch.int32).numpy(), []
    ge = torch.zeros(s, dtype=torch.int32, device=dev)  # 0: no level yet (Alg. 1's empty map)
    nil_left = torch.zeros(1, dtype=torch.int32, device=dev)
    proj = torch.empty((d, s), dtype=torch.float32, device=dev)
    status = new_status(dev)
    levels = []
    sp = _stream_ptr()
    for g in range(int(g_max), 1, -1):
        project(x_soa, sky_idx, g, out=proj, status=status)
        plan = build(proj, scheme, target_p, slice_dim, status=status, reps=reps, prefilter=prefilter)
        plan.local_skylines()
        sky_g, member = plan.merge(member=True)
        inf = plan.info()
        plan.close()
        check_status(status, "gres_literal")
        # the level's exits, assigned on the device (sky_literal_level)
        nil_left.zero_()
        _lib.check(lib.sky_literal_level(_ptr(member), s, g, _ptr(ge), _ptr(nil_left), sp),
                   "sky_literal_level")
        left = int(nil_left.item())
        levels.append({"g": g, "sky": int(inf["sky_count"]), "nil_left": left,
                       "p": int(inf["p"]), "tests_local": int(inf["tests_local"]),
                       "tests_local_max": int(inf["tests_local_max"]),
                       "tests_merge": int(inf["tests_merge"]),
                       # Sec. 4's count: the heaviest partition plus the final phase
                       "tests_paper": int(inf["tests_local_max"]) + int(inf["tests_merge"])})
        if left == 0:
            break
    _lib.check(lib.sky_literal_level(None, s, 1, _ptr(ge), None, sp), "sky_literal_level")
    for i, lv in enumerate(levels):  # tuples that left at each level
        before = s if i == 0 else levels[i - 1]["nil_left"]
        lv["exits"] = before - lv["nil_left"]
    return ge.cpu().numpy(), levels


def skyline(x_rows: torch.Tensor, scheme="none", target_p: int = 16, slice_dim: int = 0):
    """Whole skyline path on a row-major [N, d] device tensor: (sky_idx, plan info)."""
    x_soa = ingest(x_rows)
    plan = build(x_soa, scheme, target_p, slice_dim)
    plan.local_skylines()
    idx = plan.merge()
    info = plan.info()
    plan.close()
    return idx, info


class Pipeline:
    """The whole hot path on one relation shape with every buffer allocated once:

        ingest (validate, SoA) -> build (partitions) -> local skylines -> merge -> gres

    ``run(x_rows)`` queues one pass on torch's current stream and returns without waiting: no
    call of the pass reads anything back, so a pass can also be captured in a HIP graph
    (``capture``) and replayed. ``result()`` waits and returns ``(sky_idx, g_exit, gres)`` views
    of the last pass (valid until the next one); ``info()`` its plan counters."""

    def __init__(self, n: int, d: int, scheme="none", target_p: int = 16, slice_dim: int = 0,
                 g_max: int = 25, mapping="auto", device="cuda", reps: int = 0, prefilter: bool = True):
        lib = _lib.load()
        self.n, self.d, self.g_max = int(n), int(d), int(g_max)
        self.scheme, self.target_p, self.slice_dim, self.mapping = scheme, target_p, slice_dim, mapping
        self.reps = int(reps)
        self.prefilter = bool(prefilter)
        dev = torch.device(device)
        self.device = dev
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        self.x_soa = torch.empty((d, n), dtype=torch.float32, device=dev)
        prm = _params(scheme, target_p, slice_dim, reps)
        self.build_bytes = int(lib.sky_build_workspace_bytes(n, d, C.byref(prm)))
        if self.build_bytes == 0:
            raise SkyError(_lib.SKY_ERR_INVALID_ARG, "sky_build_workspace_bytes")
        self.build_ws = torch.empty(self.build_bytes, dtype=torch.uint8, device=dev)
        self.gres_bytes = int(lib.gres_workspace_bytes(n, d, g_max))  # any skyline size up to n
        self.gres_ws = torch.empty(self.gres_bytes, dtype=torch.uint8, device=dev)
        self.sky_buf = torch.empty(n, dtype=torch.int64, device=dev)
        self.count = torch.zeros(1, dtype=torch.int64, device=dev)
        self.g_exit = torch.empty(n, dtype=torch.int32, device=dev)
        self.gres_v = torch.empty(n, dtype=torch.float32, device=dev)
        self.events = None
        self._h = None
        self._ev_keep = None

    def _close_plan(self):
        if self._h is not None:
            _lib.load().sky_plan_destroy(self._h)
            self._h = None

    def run(self, x_rows: torch.Tensor, timing: bool = False, test_events=None, gres_events=None,
            gres_counter: torch.Tensor | None = None, stream=None):
        """Queue one pass. test_events: optional (begin[], end[]) lists of hipEvent_t handles
        recorded around the dominance-test launches; gres_events: optional (begin, end) around
        the gres search; gres_counter: optional int64 device tensor to which the gres search
        adds the candidate tests it evaluates; timing: torch events between the phases
        (``phase_ms``)."""
        lib = _lib.load()
        st = stream if stream is not None else torch.cuda.current_stream()
        sp = C.c_void_p(st.cuda_stream)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)] if timing else None
        self._close_plan()
        self.status.zero_()
        if ev:
            ev[0].record(st)
        _lib.check(lib.sky_ingest(_ptr(x_rows), self.n, self.d, _ptr(self.x_soa), self.n,
                                  _ptr(self.status), sp), "sky_ingest")
        if ev:
            ev[1].record(st)
        prm = _params(self.scheme, self.target_p, self.slice_dim, self.reps, self.prefilter)
        h = C.c_void_p()
        _lib.check(lib.sky_build(_ptr(self.x_soa), self.n, self.d, self.n, C.byref(prm),
                                 _ptr(self.build_ws), self.build_bytes, _ptr(self.status), sp,
                                 C.byref(h)), "sky_build")
        self._h = h
        if test_events is not None:
            nb = len(test_events[0])
            arr_b = (C.c_void_p * nb)(*test_events[0])
            arr_e = (C.c_void_p * nb)(*test_events[1])
            self._ev_keep = (arr_b, arr_e)
            _lib.check(lib.sky_plan_set_events(h, arr_b, arr_e, nb), "sky_plan_set_events")
        if ev:
            ev[2].record(st)
        _lib.check(lib.sky_local_skylines(h, sp), "sky_local_skylines")
        if ev:
            ev[3].record(st)
        _lib.check(lib.sky_merge(h, _ptr(self.sky_buf), self.n, _ptr(self.count), None, sp),
                   "sky_merge")
        if ev:
            ev[4].record(st)
        opts = _lib.GresOpts(_lib.MAPPINGS[self.mapping] if isinstance(self.mapping, str)
                             else int(self.mapping))
        if gres_events is not None:
            opts.ev_begin, opts.ev_end = gres_events
        if gres_counter is not None:
            opts.dev_tests = gres_counter.data_ptr()
        # gres of the plan's own skyline: candidates straight from the curve-ordered copy
        _lib.check(lib.sky_gres(h, self.g_max, _ptr(self.g_exit), _ptr(self.gres_v),
                                _ptr(self.gres_ws), self.gres_bytes, _ptr(self.status),
                                C.byref(opts), sp), "sky_gres")
        if ev:
            ev[5].record(st)
            self.events = ev
        return self

    def capture(self, x_rows: torch.Tensor, stream=None):
        """Capture one pass over x_rows (a tensor that stays allocated) in a CUDA/HIP graph;
        graph.replay() then reruns the whole pass. The plan of the captured pass stays open."""
        graph = torch.cuda.CUDAGraph()
        side = stream if stream is not None else torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(graph, stream=side):
            self.run(x_rows, stream=side)
        torch.cuda.current_stream().wait_stream(side)
        return graph

    def result(self, check: bool = True):
        """Waits for the last pass: (sky_idx, g_exit, gres) views, after the status check."""
        s = int(self.count.item())  # synchronises
        if check:
            check_status(self.status, "pipeline")
        return self.sky_buf[:s], self.g_exit[:s], self.gres_v[:s]

    def info(self) -> dict:
        """The plan counters of the last pass (sky_plan_info; waits for it)."""
        inf = _lib.SkyInfo()
        _lib.check(_lib.load().sky_plan_info(self._h, C.byref(inf)), "sky_plan_info")
        return inf.as_dict()

    def phase_ms(self):
        """Per-phase milliseconds of the last timed run: ingest, build, local, merge, gres."""
        ev = self.events
        ev[5].synchronize()
        names = ("ingest", "build", "local", "merge", "gres")
        return {names[i]: ev[i].elapsed_time(ev[i + 1]) for i in range(5)}

    def close(self):
        self._close_plan()

    def __del__(self):
        try:
            self._close_plan()
        except Exception:
            pass
