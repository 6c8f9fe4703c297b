"""Many independent relations at once, over the batched C ABI (``sky_batch_*`` in
include/sky.h); argument marshalling, packing and scheduling only.

    runner = BatchRunner(datasets, g_max=25)   # host [n_i, d_i] float32 arrays
    runner.run()                               # skyline + gres of every relation
    rows, g_exit, gres = runner.result(i)      # relation i: its skyline rows (local indices)

Relations are grouped by d. Each group is one ``sky_batch``: its rows packed one relation after
the other in one device buffer, every relation's skyline computed by the same rounds of the
segmented engine, then the gres of every skyline tuple (Def. 2 via Alg. 1, with the relation's
own skyline as candidates) in one persistent search launch per group. After the first step
each group gets packed key tables sized by its skyline total (``sky_batch_set_keys``; a later
skyline that outgrows them is searched on the values, with the same results). A step --
ingest, skylines and gres of every group -- reads nothing back, so it is captured once in a HIP
graph and replayed. ``GresTuner`` picks each group's search choices (mapping, tile order, relation
order) by timing them on the group itself; results never depend on the choice.

``PlainRunner`` is the one-relation-at-a-time path over the plain entry points (ingest, build,
local skylines, merge, gres_compute), the reference for the batched path's throughput.
"""
from __future__ import annotations

import ctypes as C
import json
import os

import numpy as np
import torch

from . import _lib
from ._lib import SkyError
from .api import _ptr, check_status

__all__ = ["BatchGroup", "BatchRunner", "GresTuner", "PlainRunner", "pack_by_d"]


def pack_by_d(datasets):
    """Group relation indices by d: {d: [i, ...]} in ascending d, indices ascending."""
    groups = {}
    for i, x in enumerate(datasets):
        groups.setdefault(int(x.shape[1]), []).append(i)
    return dict(sorted(groups.items()))


class BatchGroup:
    """One sky_batch: relations of equal d packed into one row-major device buffer."""

    def __init__(self, datasets, members, device, g_max):
        lib = _lib.load()
        self.members = list(members)
        self.d = int(datasets[self.members[0]].shape[1])
        sizes = [int(datasets[i].shape[0]) for i in self.members]
        self.offsets = np.zeros(len(sizes) + 1, dtype=np.int64)
        self.offsets[1:] = np.cumsum(sizes)
        self.n = int(self.offsets[-1])
        self.nb = len(self.members)
        self.g_max = int(g_max)
        host = np.concatenate([np.ascontiguousarray(datasets[i], dtype=np.float32)
                               for i in self.members]) if self.n else np.zeros((0, self.d), np.float32)
        self.x_rows = torch.from_numpy(host).to(device)
        self.x_soa = torch.empty((self.d, self.n), dtype=torch.float32, device=device)
        self._off_c = (C.c_int64 * (self.nb + 1))(*self.offsets.tolist())
        self.ws_bytes = 0
        if self.n > 0:  # a group of empty relations only has nothing to compute
            self.ws_bytes = int(lib.sky_batch_workspace_bytes(self._off_c, self.nb, self.d))
            if self.ws_bytes == 0:
                raise SkyError(_lib.SKY_ERR_INVALID_ARG, "sky_batch_workspace_bytes")
        self.ws = torch.empty(max(self.ws_bytes, 1), dtype=torch.uint8, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.sky_idx = torch.empty(max(self.n, 1), dtype=torch.int64, device=device)
        self.sky_off = torch.zeros(self.nb + 1, dtype=torch.int64, device=device)
        self.g_exit = torch.empty(max(self.n, 1), dtype=torch.int32, device=device)
        self.gres = torch.empty(max(self.n, 1), dtype=torch.float32, device=device)
        self.h = None
        self.tune = _lib.SkyTune(_lib.SKY_GRES_AUTO, 1, 1)

    def create(self, stream):
        """sky_batch_create (once; waits for the copy of the offsets)."""
        if self.h is not None or self.n == 0:
            return
        h = C.c_void_p()
        _lib.check(_lib.load().sky_batch_create(_ptr(self.x_soa), self.d, self.n, self._off_c, self.nb,
                                                _ptr(self.ws), self.ws_bytes, _ptr(self.status),
                                                C.c_void_p(stream.cuda_stream), C.byref(h)),
                   "sky_batch_create")
        self.h = h
        self.set_tune(self.tune)

    def skylines(self, stream):
        """Queue ingest and sky_batch_skylines (no synchronisation)."""
        if self.h is None:
            return
        lib = _lib.load()
        sp = C.c_void_p(stream.cuda_stream)
        _lib.check(lib.sky_ingest(_ptr(self.x_rows), self.n, self.d, _ptr(self.x_soa), self.n,
                                  _ptr(self.status), sp), "sky_ingest")
        _lib.check(lib.sky_batch_skylines(self.h, _ptr(self.sky_idx), self.n, _ptr(self.sky_off),
                                          sp), "sky_batch_skylines")

    def set_tune(self, tune):
        self.tune = tune
        if self.h is not None:
            _lib.check(_lib.load().sky_batch_tune(self.h, C.byref(tune), None), "sky_batch_tune")

    def attach_keys(self, sky_total=None):
        """Packed key tables for the gres search (sky_batch_set_keys), sized for a skyline total
        of sky_total tuples (default: the last pass's, read back); nothing when they do not
        apply to this group's d and g_max."""
        if self.h is None:
            return
        lib = _lib.load()
        total = self.sky_count if sky_total is None else int(sky_total)
        nb = int(lib.sky_batch_keys_bytes(self.h, total, self.g_max))
        if nb == 0:
            return
        self.keys_ws = torch.empty(nb, dtype=torch.uint8, device=self.x_soa.device)
        _lib.check(lib.sky_batch_set_keys(self.h, _ptr(self.keys_ws), nb, total, self.g_max),
                   "sky_batch_set_keys")

    def launch_gres(self, stream, ev_begin=None, ev_end=None):
        if self.h is None:
            return
        _lib.check(_lib.load().sky_batch_gres(self.h, self.g_max, _ptr(self.g_exit), _ptr(self.gres),
                                              ev_begin, ev_end, C.c_void_p(stream.cuda_stream)),
                   "sky_batch_gres")

    @property
    def sky_count(self):
        """Total skyline size of the last pass (reads the offsets back)."""
        return int(self.sky_off[-1].item()) if self.nb else 0

    def info(self):
        if self.h is None:
            return {"n": 0, "d": self.d, "p": self.nb, "sky_count": 0}
        inf = _lib.SkyInfo()
        _lib.check(_lib.load().sky_batch_info(self.h, C.byref(inf)), "sky_batch_info")
        return inf.as_dict()

    def close(self):
        if self.h is not None:
            _lib.load().sky_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GresTuner:
    """Per-group choice of the gres search by measurement: coordinate descent over the mapping,
    the tile order and the relation order, each candidate timed on the group's own prepared
    candidates (torch events on the launch stream). Choices are cached per (d, skyline size,
    largest relation's skyline, g_max) in memory and, if `path` is given, in a JSON file."""

    LEVELS_MAX_CANDIDATES = 8192

    def __init__(self, path=None, repeats=2):
        self.path = path
        self.repeats = repeats
        self.cache = {}
        if path and os.path.exists(path):
            with open(path) as f:
                self.cache = json.load(f)
        self.trials = []

    @staticmethod
    def key(group):
        cnt = np.diff(group.sky_off.cpu().numpy())
        return f"d{group.d}_s{int(cnt.sum())}_m{int(cnt.max()) if cnt.size else 0}_g{group.g_max}"

    def _time(self, group, tune, stream):
        group.set_tune(tune)
        best = None
        for _ in range(self.repeats):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            group.launch_gres(stream)
            b.record(stream)
            b.synchronize()
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
        self.trials.append((group.d, tune.as_dict(), best))
        return best

    def choose(self, group, stream):
        if group.sky_count == 0:
            return _lib.SkyTune(_lib.SKY_GRES_AUTO, 1, 1)
        k = self.key(group)
        if k in self.cache:
            return _lib.SkyTune(**self.cache[k])
        cur = dict(mapping=_lib.SKY_GRES_TILES, near_first=1, lpt=1)
        best_ms = None
        # lanes over levels only pays off for small candidate sets (every lane walks all of them)
        cnt = np.diff(group.sky_off.cpu().numpy())
        mappings = (_lib.SKY_GRES_TILES,) if cnt.max() > self.LEVELS_MAX_CANDIDATES else (
            _lib.SKY_GRES_TILES, _lib.SKY_GRES_LEVELS)
        for field, values in (("mapping", mappings), ("near_first", (1, 0)), ("lpt", (1, 0))):
            best_v = cur[field]
            for v in values:
                trial = dict(cur, **{field: v})
                ms = self._time(group, _lib.SkyTune(**trial), stream)
                if best_ms is None or ms < best_ms:
                    best_ms, best_v = ms, v
            cur[field] = best_v
        self.cache[k] = cur
        if self.path:
            with open(self.path, "w") as f:
                json.dump(self.cache, f, indent=1, sort_keys=True)
        return _lib.SkyTune(**cur)


class BatchRunner:
    """Skyline and gres of many relations of mixed d (see the module docstring). The first run
    is eager (and tunes the groups when a tuner is given); with use_graph, that step is then
    captured once and every later run replays it."""

    def __init__(self, datasets, g_max=25, device="cuda", tuner=None, use_graph=True, keys=True):
        self.device = torch.device(device)
        self.g_max = int(g_max)
        self.keys = keys
        self.sizes = [(int(x.shape[0]), int(x.shape[1])) for x in datasets]
        self.groups = [BatchGroup(datasets, mem, self.device, g_max)
                       for mem in pack_by_d(datasets).values()]
        self.where = {}
        for gi, g in enumerate(self.groups):
            for j, i in enumerate(g.members):
                self.where[i] = (gi, j)
        self.tuner = tuner
        self.use_graph = use_graph
        self.graph = None
        self.stream = torch.cuda.Stream(self.device)
        self._ev = None
        for g in self.groups:
            g.create(self.stream)
        self.stream.synchronize()

    def _step(self, st, ev=None):
        for g in self.groups:
            g.status.zero_()
            g.skylines(st)
        if ev is not None:
            ev.record(st)
        for g in self.groups:
            g.launch_gres(st)

    def run(self, check=True, tune=True, timing=False):
        st = self.stream
        cur = torch.cuda.current_stream(self.device)
        st.wait_stream(cur)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e2 = torch.cuda.Event(enable_timing=True)
        with torch.cuda.stream(st):
            e0.record(st)
            if self.graph is not None and not timing:
                self.graph.replay()
                e1 = None
            else:
                self._step(st, e1)
            e2.record(st)
            again = False
            if self.graph is None and self.keys:
                st.synchronize()
                for g in self.groups:  # key tables sized by the skylines just computed
                    g.attach_keys()
                again = True
            if self.graph is None and tune and self.tuner is not None:
                for g in self.groups:
                    if g.h is not None and g.sky_count:
                        g.set_tune(self.tuner.choose(g, st))
                again = True
            if again:
                for g in self.groups:  # the results of the search every later step runs
                    g.launch_gres(st)
            if self.graph is None and self.use_graph:
                self._capture()
        cur.wait_stream(st)
        if check:
            st.synchronize()
            for g in self.groups:
                check_status(g.status, "batch")
        self._ev = (e0, e1, e2)
        return self

    def _capture(self):
        st = self.stream
        st.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph, stream=st):
            self._step(torch.cuda.current_stream())

    def phase_ms(self):
        """Milliseconds of the last run: its total, and with timing=True (an eager step) the
        skylines and gres phases."""
        e0, e1, e2 = self._ev
        e2.synchronize()
        out = {"step": e0.elapsed_time(e2)}
        if e1 is not None:
            out["skylines"] = e0.elapsed_time(e1)
            out["gres"] = e1.elapsed_time(e2)
        return out

    def sky_total(self):
        return sum(g.sky_count for g in self.groups)

    def result(self, i):
        """(skyline rows of relation i as local row indices, g_exit, gres) on the host."""
        gi, j = self.where[i]
        g = self.groups[gi]
        off = g.sky_off.cpu().numpy()
        a, b = int(off[j]), int(off[j + 1])
        rows = g.sky_idx[a:b].cpu().numpy() - int(g.offsets[j])
        return rows, g.g_exit[a:b].cpu().numpy(), g.gres[a:b].cpu().numpy()

    def info(self):
        return [dict(g.info(), tune=g.tune.as_dict()) for g in self.groups]

    def close(self):
        self.graph = None
        for g in self.groups:
            g.close()


class PlainRunner:
    """One relation at a time through the plain entry points (ingest -> build -> local
    skylines -> merge -> gres_compute), buffers sized once for the largest relation of each d."""

    def __init__(self, datasets, g_max=25, device="cuda"):
        lib = _lib.load()
        self.device = torch.device(device)
        self.g_max = int(g_max)
        self.x = [torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).to(self.device)
                  for x in datasets]
        self.bufs = {}
        for x in datasets:
            n, d = int(x.shape[0]), int(x.shape[1])
            nmax = max(n, self.bufs.get(d, 0))
            self.bufs[d] = nmax
        prm = _lib.SkyParams(_lib.SKY_NONE, 1, 0, 0)
        for d, nmax in list(self.bufs.items()):
            bb = int(lib.sky_build_workspace_bytes(nmax, d, C.byref(prm)))
            gb = int(lib.gres_workspace_bytes(nmax, d, self.g_max))
            self.bufs[d] = dict(
                nmax=nmax, bb=bb, gb=gb,
                bws=torch.empty(bb, dtype=torch.uint8, device=self.device),
                gws=torch.empty(gb, dtype=torch.uint8, device=self.device),
                soa=torch.empty(d * nmax, dtype=torch.float32, device=self.device),
                sky=torch.empty(nmax, dtype=torch.int64, device=self.device),
                cnt=torch.zeros(1, dtype=torch.int64, device=self.device),
                ge=torch.empty(nmax, dtype=torch.int32, device=self.device),
                gr=torch.empty(nmax, dtype=torch.float32, device=self.device))
        self.status = torch.zeros(1, dtype=torch.int32, device=self.device)
        self.counts = [0] * len(datasets)
        self.keep = None

    def run_one(self, i, keep=False):
        lib = _lib.load()
        st = torch.cuda.current_stream(self.device)
        sp = C.c_void_p(st.cuda_stream)
        x = self.x[i]
        n, d = int(x.shape[0]), int(x.shape[1])
        b = self.bufs[d]
        _lib.check(lib.sky_ingest(_ptr(x), n, d, _ptr(b["soa"]), n, _ptr(self.status), sp), "sky_ingest")
        prm = _lib.SkyParams(_lib.SKY_NONE, 1, 0, 0)
        h = C.c_void_p()
        _lib.check(lib.sky_build(_ptr(b["soa"]), n, d, n, C.byref(prm), _ptr(b["bws"]), b["bb"],
                                 _ptr(self.status), sp, C.byref(h)), "sky_build")
        try:
            _lib.check(lib.sky_local_skylines(h, sp), "sky_local_skylines")
            _lib.check(lib.sky_merge(h, _ptr(b["sky"]), n, _ptr(b["cnt"]), None, sp), "sky_merge")
            s = int(b["cnt"].item())
        finally:
            lib.sky_plan_destroy(h)
        opts = _lib.GresOpts(_lib.SKY_GRES_AUTO)
        _lib.check(lib.gres_compute(_ptr(b["soa"]), n, d, n, _ptr(b["sky"]), s, self.g_max,
                                    _ptr(b["ge"]), _ptr(b["gr"]), _ptr(b["gws"]), b["gb"],
                                    _ptr(self.status), C.byref(opts), sp), "gres_compute")
        self.counts[i] = s
        if keep:
            return (b["sky"][:s].cpu().numpy(), b["ge"][:s].cpu().numpy(), b["gr"][:s].cpu().numpy())
        return None

    def run(self, check=True):
        self.status.zero_()
        for i in range(len(self.x)):
            self.run_one(i)
        if check:
            torch.cuda.current_stream(self.device).synchronize()
            check_status(self.status, "plain")
        return self
