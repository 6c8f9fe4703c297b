"""Benchmark: one step = the whole hot path on one synthetic relation already resident in HBM:
ingest (validate, SoA) -> partition assignment -> local skylines -> merge (final skyline) ->
gres of every skyline tuple.

Default workload: anticorrelated 1,000,000 x 6 FP32 (seed 0), plain method (one partition),
g_max = 25. Prints ONE JSON line.

value = dominance tests per second, counting the tests of the plain sequential method the
paper measures (SFS for the skyline, Alg. 1's per-tuple descending scan for gres; recorded by
the oracle in tests/golden/workload_counts.json) over the measured step time.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "dominance tests/s + skyline tuples' gres/s at 1 GPU; p50/p99 query latency"


# MI355X published peaks used for the roofline
PEAK_HBM_GBS = 8000.0
PEAK_ALU_TOPS = 256 * 64 * 2.4e9 / 1e12  # 256 CUs x 64 lanes x 2.4 GHz: 32-bit lane-ops


class HipEvents:
    """A pool of hipEvent_t handles (libamdhip64 through ctypes) for kernel-level timing on the
    stream the library launches on."""

    def __init__(self, count):
        self.lib = C.CDLL("libamdhip64.so")
        self.lib.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
        self.lib.hipEventSynchronize.argtypes = [C.c_void_p]
        self.lib.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
        self.lib.hipEventDestroy.argtypes = [C.c_void_p]
        self.ev = []
        for _ in range(count):
            e = C.c_void_p()
            if self.lib.hipEventCreate(C.byref(e)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.ev.append(e.value)

    def elapsed_ms(self, a, b):
        self.lib.hipEventSynchronize(b)
        ms = C.c_float()
        if self.lib.hipEventElapsedTime(C.byref(ms), a, b) != 0:
            raise RuntimeError("hipEventElapsedTime failed")
        return float(ms.value)

    def close(self):
        for e in self.ev:
            self.lib.hipEventDestroy(e)
        self.ev = []


def source_sha(name):
    """First 16 hex digits of the SHA-256 of a kernel source file followed by the headers every
    kernel includes (csrc/sky_internal.hpp, include/sky.h): the key under which the committed
    profiles store a kernel's counters."""
    import hashlib
    h = hashlib.sha256()
    for path in (os.path.join(ROOT, "paper_2412_02274_amd", "csrc", name),
                 os.path.join(ROOT, "paper_2412_02274_amd", "csrc", "sky_internal.hpp"),
                 os.path.join(ROOT, "include", "sky.h")):
        h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(workload):
    """HBM bytes per step of the dominance-test kernel and per launch of the gres search kernel
    from the committed PMC summary (profiles/traffic_<workload>.txt); each is None when its
    kernel source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    out = {"dominance_test": None, "gres_search": None}
    if not os.path.exists(path):
        return out
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    sha = source_sha
    if kv.get("src_sha256_16") == sha("sky_skyline.hip"):
        out["dominance_test"] = int(kv["fetch_bytes_per_step"]) + int(kv["write_bytes_per_step"])
    if "gres_search_fetch_bytes" in kv and kv.get("gres_search_src_sha256_16") == sha("sky_gres.hip"):
        out["gres_search"] = int(kv["gres_search_fetch_bytes"]) + int(kv["gres_search_write_bytes"])
    return out


def stored_valu(workload):
    """VALU figures of the dominance-test and gres-search kernels from the committed PMC summary
    (profiles/valu_<workload>.txt): per kernel, the VALU instructions issued per launch and the
    share of the chip's VALU issue slots they fill over the kernel's traced duration; None for a
    kernel whose source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"valu_{workload}.txt")
    out = {"dominance_test": None, "gres_search": None}
    if not os.path.exists(path):
        return out
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    sha = source_sha
    for name, src in (("dominance_test", "sky_skyline.hip"), ("gres_search", "sky_gres.hip")):
        if kv.get(f"{name}.src_sha256_16") == sha(src):
            out[name] = {"valu_insts_per_launch": float(kv[f"{name}.valu_insts_per_launch"]),
                         "valu_issue_frac": float(kv[f"{name}.valu_issue_frac"]),
                         "valu_active_frac": float(kv[f"{name}.valu_active_frac"])}
    return out


def cpu_baseline(x, g_max, rows):
    """The oracle as it stands on the first `rows` rows of the workload (all of them by
    default): SFS on one thread, then Alg. 1's per-tuple search of every skyline tuple on every
    host core (OpenMP); each leg timed and counted on its own."""
    import numpy as np
    import oracle
    sub = np.ascontiguousarray(x[:rows])
    t0 = time.perf_counter()
    mem, t_sfs = oracle.skyline_sfs(sub)
    t1 = time.perf_counter()
    sky = np.flatnonzero(mem)
    _, t_gres = oracle.gres(sub, sky, g_max)
    t2 = time.perf_counter()
    cpu_model = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    dt = t2 - t0
    part = "the whole workload" if rows >= x.shape[0] else f"the first {rows} rows of the workload"
    return {"value": (t_sfs + t_gres) / dt, "unit": "dominance tests/s",
            "cores": oracle.num_threads(), "kind": "oracle", "cpu_model": cpu_model,
            "host_cpus": os.cpu_count(),
            "legs": {"skyline_sfs": {"tests": int(t_sfs), "seconds": t1 - t0, "threads": 1,
                                     "tests_per_s": t_sfs / (t1 - t0)},
                     "gres_alg1": {"tests": int(t_gres), "seconds": t2 - t1,
                                   "threads": oracle.num_threads(), "tuples": int(len(sky)),
                                   "tests_per_s": t_gres / (t2 - t1)}},
            "seconds_per_pass": dt,
            "sample": f"{part}: SFS skyline ({t_sfs} tests, 1 thread) + Alg. 1 gres of its "
                      f"{len(sky)} skyline tuples ({t_gres} tests, OpenMP); {dt:.1f} s"}


def measured_peaks():
    """The two rates the rooflines are priced against, measured on this device with the
    library's probes: VALU lane-ops/s of 32-bit integer add/xor/max/min (the dominance test's
    mix; best of 3 launches of 2048 workgroups) and HBM bytes/s of a streaming 1 GiB copy
    (read + written bytes; best of 5)."""
    import torch
    from paper_2412_02274_amd import _lib
    lib = _lib.load()
    ev = HipEvents(2)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    grid = 2048
    sink = torch.empty(grid, dtype=torch.int32, device="cuda:0")
    ops = C.c_int64()
    best = 0.0
    for it in (2000, 200000, 200000, 200000):
        _lib.check(lib.sky_probe_valu(it, grid, C.c_void_p(sink.data_ptr()), ev.ev[0], ev.ev[1], st,
                                      C.byref(ops)), "sky_probe_valu")
        ms = ev.elapsed_ms(ev.ev[0], ev.ev[1])
        if it > 2000:
            best = max(best, ops.value / (ms * 1e-3) / 1e12)
    nbytes = 1 << 30
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    src.fill_(1)
    cbest = 0.0
    for k in range(6):
        _lib.check(lib.sky_probe_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                                      ev.ev[0], ev.ev[1], st), "sky_probe_copy")
        ms = ev.elapsed_ms(ev.ev[0], ev.ev[1])
        if k:
            cbest = max(cbest, 2 * nbytes / (ms * 1e-3) / 1e9)
    del src, dst
    torch.cuda.empty_cache()
    ev.close()
    return {"valu_TOPs": best, "valu_frac_of_published": best / PEAK_ALU_TOPS,
            "copy_GBs": cbest, "copy_frac_of_published": cbest / PEAK_HBM_GBS,
            "note": "sky_probe_valu (4 independent chains of 32-bit add/xor/max/min per lane) and "
                    "sky_probe_copy (16-byte streaming copy of 1 GiB; read + written bytes)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ant_1m_d6")
    ap.add_argument("--scheme", default="none", choices=["none", "grid", "angular", "sliced"])
    ap.add_argument("--p", type=int, default=16)
    ap.add_argument("--mapping", default="auto", choices=["auto", "tiles", "levels"])
    ap.add_argument("--cpu-rows", type=int, default=0, help="oracle baseline rows (0: all)")
    ap.add_argument("--no-sub", action="store_true", help="default line without the partitioned "
                    "and serving sub-results")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-prefilter", action="store_true",
                    help="every row through the local phase (sky_params.prefilter_off)")
    ap.add_argument("--rate", type=float, default=500.0, help="serve_ties: queries per second")
    ap.add_argument("--serve-seconds", type=float, default=60.0, help="serve_ties: trace length")
    ap.add_argument("--sub-serve-seconds", type=float, default=10.0,
                    help="default line: trace length of the serving sub-result")
    ap.add_argument("--budget-mb", type=int, default=256, help="serve_ties: HBM budget of queries")
    ap.add_argument("--slots", type=int, default=4, help="serve_ties: concurrent query streams")
    ap.add_argument("--no-plain", action="store_true", help="batch/serve: skip the plain path")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch_4096":
        return bench_batch(args)
    if args.workload == "serve_ties":
        return bench_serve(args)

    import numpy as np
    import torch
    from paper_2412_02274_amd import api
    from tests.golden import workloads as W

    counts = W.load_counts()[args.workload]
    kind, n, d, seed, g_max = W.WORKLOADS[args.workload]
    x = W.make(args.workload)
    dev = torch.device("cuda:0")
    xr = torch.from_numpy(x).to(dev)
    pipe = api.Pipeline(n, d, args.scheme, args.p, 0, g_max, args.mapping, dev,
                        prefilter=not args.no_prefilter)
    peaks = measured_peaks()
    for _ in range(args.warmup):
        pipe.run(xr)
    pipe.result()
    # kernel-level events for every timed step: dominance-test launches and the gres search
    max_pairs = 64
    pool = HipEvents(args.steps * (2 * max_pairs + 2))
    per_step = []
    for k in range(args.steps):
        base = k * (2 * max_pairs + 2)
        tb = pool.ev[base: base + max_pairs]
        te = pool.ev[base + max_pairs: base + 2 * max_pairs]
        gb, ge_ = pool.ev[base + 2 * max_pairs], pool.ev[base + 2 * max_pairs + 1]
        per_step.append((tb, te, gb, ge_))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        tb, te, gb, ge_ = per_step[k]
        pipe.run(xr, test_events=(tb, te), gres_events=(gb, ge_))
    torch.cuda.synchronize()
    dt_eager = (time.perf_counter() - t0) / args.steps
    sky, ge, gr = pipe.result()
    used = pipe.info()["events_used"]  # the same launch sequence every pass
    test_ms = sum(sum(pool.elapsed_ms(per_step[k][0][i], per_step[k][1][i]) for i in range(used))
                  for k in range(args.steps)) / args.steps
    gres_ms = sum(pool.elapsed_ms(per_step[k][2], per_step[k][3]) for k in range(args.steps)) / args.steps
    launches = used
    s = int(sky.numel())
    if s != counts["sky_size"]:
        raise SystemExit(f"skyline size {s} differs from the oracle's {counts['sky_size']}")
    hist = np.bincount(ge.cpu().numpy(), minlength=g_max + 1).tolist()  # index = g_exit
    if counts.get("g_exit_hist") is not None and hist != counts["g_exit_hist"]:
        raise SystemExit("g_exit histogram differs from the oracle's")
    # the same pass captured once in a HIP graph and replayed (no host work per step)
    graph = pipe.capture(xr)
    graph.replay()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    dt_graph = (time.perf_counter() - t1) / args.steps
    sky_g, ge_g, _ = pipe.result()
    if not (torch.equal(sky_g, sky) and torch.equal(ge_g, ge)):
        raise SystemExit("graph replay differs from the eager pass")
    del graph
    dt = min(dt_eager, dt_graph)
    # per-phase breakdown (one more, separately timed run)
    gres_counter = torch.zeros(1, dtype=torch.int64, device=dev)
    pipe.run(xr, timing=True, gres_counter=gres_counter)
    phases = pipe.phase_ms()
    gres_executed = int(gres_counter.item())
    info = pipe.info()
    tests = counts["sfs_tests"] + counts["gres_tests"]
    executed = info["tests_local"] + info["tests_merge"]
    # of which the dominance-test kernel's own (the build's prefilter runs in another kernel)
    executed_kernel = executed - info["tests_prefilter"]
    ops_per_test = 2 * d  # the kernel's one <= and one < comparison per attribute (Def. 1)
    test_tops = executed_kernel * ops_per_test / (test_ms * 1e-3) / 1e12
    # rooflines: algorithmic work per launch over the kernel's average launch time.
    # Dominance tests: oracle-order SFS test count x d element compares; gres search: Alg. 1's
    # per-tuple descending-scan test count x d key compares. Reported for both kernels; the
    # `roofline` field is the one of the kernel that takes the most time per step.
    traffic = stored_traffic(args.workload)
    kernels = {
        "dominance_test": {"ms_per_step": test_ms, "launches_per_step": launches,
                           "executed_tests_per_step": executed_kernel, "ops_per_executed_test": ops_per_test,
                           "executed_TOPs": test_tops},
        "gres_search": {"ms_per_step": gres_ms, "launches_per_step": 1,
                        "executed_tests_per_step": gres_executed,
                        "ops_per_executed_test": 3 * d},
    }

    valu = stored_valu(args.workload)

    def roof(name, alg_tests, ms, nl, traffic_step, executed_ops, valu_k):
        # achieved: the element ops of the tests the kernel evaluates (device counters x ops per
        # test) per launch over its average launch time; the plain method's test count (far more
        # tests than the pruned kernel evaluates) only as an upper-bound credit
        exe = executed_ops / (ms * 1e-3) / 1e12
        alg = alg_tests * d / (ms * 1e-3) / 1e12
        r = {"kernel": name, "bound": "alu", "achieved": exe, "peak": PEAK_ALU_TOPS,
             "unit": "TOP/s", "frac": exe / PEAK_ALU_TOPS,
             "traffic": None if traffic_step is None else traffic_step / nl,
             "launches_per_step": nl, "avg_launch_us": ms * 1e3 / nl,
             "executed_ops_per_launch": executed_ops / nl,
             "algorithmic_credit": {"ops_per_launch": alg_tests * d / nl, "TOPs": alg,
                                    "frac_upper_bound": min(alg / PEAK_ALU_TOPS, 1.0),
                                    "upper_bound": True}}
        if valu_k is not None:
            r["valu_pmc"] = valu_k
        r["frac_of_measured_peak"] = exe / peaks["valu_TOPs"]
        return r

    # executed ops: a dominance test compares 2d values (<= and <); a gres candidate test
    # multiplies d values by g and compares each product with two thresholds
    roofs = {"dominance_test": roof("dominance_test", counts["sfs_tests"], test_ms, launches,
                                    traffic["dominance_test"], executed_kernel * ops_per_test,
                                    valu["dominance_test"]),
             "gres_search": roof("gres_search", counts["gres_tests"], gres_ms, 1,
                                 traffic["gres_search"], gres_executed * 3 * d, valu["gres_search"])}
    # the HBM-bound ingest (validate + transpose): 4 N d bytes read and 4 N d bytes written, over
    # the event-timed ingest phase of the separately timed pass (one kernel)
    ingest_bytes = 8 * n * d
    ingest_gbs = ingest_bytes / (phases["ingest"] * 1e-3) / 1e9
    roofs["ingest"] = {"kernel": "ingest", "bound": "hbm", "achieved": ingest_gbs, "peak": PEAK_HBM_GBS,
                       "unit": "GB/s", "frac": ingest_gbs / PEAK_HBM_GBS, "traffic": None,
                       "frac_of_measured_peak": ingest_gbs / peaks["copy_GBs"],
                       "launches_per_step": 1, "avg_launch_us": phases["ingest"] * 1e3,
                       "alg_bytes_per_launch": ingest_bytes}
    dominant = max(kernels, key=lambda k: kernels[k]["ms_per_step"])
    roofline = dict(roofs[dominant])
    roofline["note"] = ("achieved = element ops of the tests the kernel evaluates (device counters: "
                        "2d compares per dominance test, d multiplies + 2d compares per gres "
                        "candidate test) per launch / the kernel's average HIP-event launch time; "
                        "peak = 256 CUs x 64 lanes x 2.4 GHz 32-bit VALU lane-ops; valu_pmc = "
                        "SQ_INSTS_VALU and SQ_ACTIVE_INST_VALU from rocprofv3 against the issue "
                        "slots of the traced duration; algorithmic_credit = the plain method's "
                        "test count (SFS, Alg. 1) x d, an upper bound the pruned kernel does not "
                        "execute; traffic = PMC FETCH_SIZE+WRITE_SIZE bytes per launch "
                        "(calibrated), null when the kernel changed since")
    line = {
        "metric": METRIC,
        "value": tests / dt,
        "unit": "dominance tests/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "ms_per_step_eager": dt_eager * 1e3,
        "ms_per_step_graph": dt_graph * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "generator": kind, "n": n, "d": d, "seed": seed,
                   "g_max": g_max, "scheme": args.scheme,
                   "target_p": args.p if args.scheme != "none" else 1,
                   "launch": "hip_graph" if dt_graph <= dt_eager else "stream"},
        "sky_size": s,
        "gres_tuples_per_s": s / dt,
        "algorithmic_tests": {"skyline_sfs": counts["sfs_tests"], "gres_alg1": counts["gres_tests"]},
        "executed_skyline_tests": executed,
        "executed_prefilter_tests": info["tests_prefilter"],
        "executed_gres_tests": gres_executed,
        "executed_tests_per_s": (executed + gres_executed) / dt,
        # the paper's own count of the partitioned method (Sec. 4): the heaviest partition's
        # local-phase tests plus the final phase's
        "paper_skyline_tests": info["tests_local_max"] + info["tests_merge"],
        "phase_ms": phases,
        "roofline": roofline,
        "roofline_kernels": roofs,
        "measured_peaks": peaks,
        "kernels": kernels,
        "plan": {k: info[k] for k in ("p", "m", "rounds_local", "rounds_merge", "local_count",
                                      "pruned_cells", "pruned_rows", "max_partition", "rows_kept")},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(x, g_max, n if args.cpu_rows <= 0 else min(args.cpu_rows, n))
    pool.close()
    if args.workload == "ant_1m_d6" and args.scheme == "none" and not args.no_sub:
        # the other single-GPU workloads, compact: partitioned (three schemes), serving, the
        # small relation at a large g_max, and the 4096-relation batch
        pipe.close()
        del pipe, xr
        torch.cuda.empty_cache()
        line["sub_results"] = {"partitioned": sub_partitioned()}
        m = serve_measure(dev, args.rate, args.sub_serve_seconds, args.budget_mb, args.slots)
        line["sub_results"]["serving"] = {k: m[k] for k in (
            "rate_per_s", "seconds", "latency", "plain_latency", "saturation", "plain_saturation",
            "same_results_as_plain", "max_in_flight", "sky_sizes")}
        torch.cuda.empty_cache()
        line["sub_results"]["small"] = sub_small()
        line["sub_results"]["batch"] = sub_batch()
    print(json.dumps(line), flush=True)


def _base_line(args, value, unit, ms, dtype, config, higher=True):
    return {"metric": METRIC, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": higher,
            "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": "synthetic",
            "config": config}


def batch_measure(steps, warmup):
    """The 4096-relation batch through the batched path: the relations, the runner (open), the
    graph-replayed step time in seconds, the skyline total (checked against the oracle's
    stored total), the phases of one eager step and the stored oracle counts."""
    import torch
    from paper_2412_02274_amd import datagen as G
    from paper_2412_02274_amd.api import check_status
    from paper_2412_02274_amd.batch import BatchRunner, GresTuner
    from tests.golden import workloads as W

    specs = G.batch_specs()
    data = [G.batch_dataset(sp) for sp in specs]
    run = BatchRunner(data, g_max=25, device=torch.device("cuda:0"), tuner=GresTuner())
    for _ in range(max(warmup, 1)):  # the first run tunes and captures the step
        run.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        run.run(check=False)  # graph replay of the whole step
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    for g in run.groups:
        check_status(g.status, "batch")
    s_total = run.sky_total()
    run.run(timing=True)  # one eager step with an event between the phases
    phases = run.phase_ms()
    counts = None
    if os.path.exists(W.BATCH_COUNTS):
        with open(W.BATCH_COUNTS) as f:
            counts = json.load(f)
        if counts["sky_total"] != s_total:
            raise SystemExit(f"skyline total {s_total} differs from the oracle's {counts['sky_total']}")
    return specs, data, run, dt, s_total, phases, counts


def sub_batch(steps=5):
    """The 4096-relation batch, compact: graph-replayed step time, skyline tuples per second and
    the phases of one eager step (the full line: --workload batch_4096)."""
    specs, data, run, dt, s_total, phases, counts = batch_measure(steps, 1)
    run.close()
    return {"workload": "batch_4096", "relations": len(data), "rows": sum(x.shape[0] for x in data),
            "ms_per_step": dt * 1e3, "sky_total": s_total, "tuples_per_s": s_total / dt,
            "phase_ms": phases, "sky_total_matches_oracle": counts is not None}


def sub_small(steps=20):
    """The small relation at a large level range (uniform 10,000 x 4, seed 0, g_max 10^4),
    compact: graph-replayed step time and the skyline size checked against the oracle's."""
    import torch
    from paper_2412_02274_amd import api
    from tests.golden import workloads as W
    counts = W.load_counts()["uni_10k_d4"]
    kind, n, d, seed, g_max = W.WORKLOADS["uni_10k_d4"]
    x = torch.from_numpy(W.make("uni_10k_d4")).to("cuda:0")
    pipe = api.Pipeline(n, d, "none", 1, 0, g_max, "auto", "cuda:0")
    pipe.run(x)
    sky, ge, _ = pipe.result()
    if int(sky.numel()) != counts["sky_size"]:
        raise SystemExit(f"small: skyline size {int(sky.numel())} differs from the oracle's")
    graph = pipe.capture(x)
    graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        graph.replay()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    del graph
    pipe.close()
    return {"workload": "uni_10k_d4", "n": n, "d": d, "g_max": g_max, "ms_per_step": dt * 1e3,
            "sky_size": int(sky.numel())}


def bench_batch(args):
    """Many-dataset workload: 4096 relations (log-normal N in [1k, 200k], d in 2..8, uniform and
    anticorrelated alternating, seed 0); one step = skyline and gres of every relation through
    the batched path (groups by d, tuned work tables, graph-replayed gres launches)."""
    import numpy as np
    import torch
    from paper_2412_02274_amd.batch import PlainRunner

    dev = torch.device("cuda:0")
    specs, data, run, dt, s_total, phases, counts = batch_measure(args.steps, args.warmup)
    rows = sum(x.shape[0] for x in data)
    line = _base_line(args, s_total / dt, "skyline tuples/s", dt * 1e3, "f32",
                      {"workload": "batch_4096", "relations": len(data), "rows": rows,
                       "d": "2..8", "kinds": "uni/ant alternating", "seed": 0, "g_max": 25})
    line["rows_per_s"] = rows / dt
    line["sky_total"] = s_total
    line["phase_ms"] = phases
    line["groups"] = [{"d": g.d, "relations": g.nb, "rows": g.n, "sky": g.sky_count,
                       "rounds": g.info().get("rounds_local"), "tune": g.tune.as_dict()}
                      for g in run.groups]
    line["launch"] = "one HIP graph per step (ingest, skylines and gres of every group)"
    # the gres phase (one persistent search launch per group) dominates the step: its executed
    # work = the candidate tests the searches evaluated (device counters) x 3d lane-ops (d
    # multiplies, 2d compares), over the event-timed gres phase of the eager step
    infos = [g.info() for g in run.groups]
    gres_ops = sum(inf["tests_gres"] * 3 * g.d for inf, g in zip(infos, run.groups))
    sky_ops = sum((inf["tests_local"] - inf["tests_prefilter"]) * 2 * g.d for inf, g in zip(infos, run.groups))
    gres_tops = gres_ops / (phases["gres"] * 1e-3) / 1e12
    line["executed_gres_tests"] = sum(inf["tests_gres"] for inf in infos)
    line["executed_skyline_tests"] = sum(inf["tests_local"] for inf in infos)
    line["roofline"] = {"kernel": "gres search (one persistent launch per group)", "bound": "alu",
                        "achieved": gres_tops, "peak": PEAK_ALU_TOPS, "unit": "TOP/s",
                        "frac": gres_tops / PEAK_ALU_TOPS, "traffic": None,
                        "launches_per_step": len(run.groups),
                        "executed_ops_per_step": gres_ops,
                        "note": "executed candidate tests (device counters) x 3d lane-ops over the "
                                "event-timed gres phase of an eager step; peak = 256 CUs x 64 lanes "
                                "x 2.4 GHz 32-bit VALU lane-ops"}
    sky_tops = sky_ops / (phases["skylines"] * 1e-3) / 1e12
    line["skyline_phase"] = {"executed_TOPs": sky_tops, "executed_frac": sky_tops / PEAK_ALU_TOPS,
                             "note": "dominance tests of the skyline rounds (device counters) x 2d "
                                     "over the whole skyline phase (build included)"}
    if counts is not None:
        alg = sum(t * sp[1] for t, sp in zip(counts["sfs_tests"], specs))
        ach = alg / (phases["skylines"] * 1e-3) / 1e12
        line["algorithmic_sfs_tests"] = counts["sfs_total"]
        line["skyline_phase"]["algorithmic_credit"] = {
            "TOPs": ach, "frac_upper_bound": min(ach / PEAK_ALU_TOPS, 1.0), "upper_bound": True,
            "note": "oracle SFS tests x d per relation over the skyline phase: the plain method's "
                    "work, which the pruned kernels do not execute"}
    if not args.no_plain:
        plain = PlainRunner(data, g_max=25, device=dev)
        for i in range(64):
            plain.run_one(i)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        plain.run()
        pt = time.perf_counter() - t1
        if sum(plain.counts) != s_total:
            raise SystemExit("plain path skyline total differs")
        line["plain"] = {"s_per_pass": pt, "tuples_per_s": s_total / pt,
                         "note": "one launch sequence per relation, serialized (ingest, build, "
                                 "local skylines, merge, gres_compute)"}
        line["speedup_vs_plain"] = pt / dt
    if not args.no_cpu_baseline:
        import oracle
        t2 = time.perf_counter()
        tup, k = 0, 0
        while time.perf_counter() - t2 < 15.0 and k < len(data):
            mem, _ = oracle.skyline_sfs(data[k])
            sky = np.flatnonzero(mem)
            oracle.gres(data[k], sky, 25)
            tup += len(sky)
            k += 1
        ct = time.perf_counter() - t2
        line["cpu_baseline"] = {"value": tup / ct, "unit": "skyline tuples/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": f"the first {k} relations (SFS 1 thread + Alg. 1 gres "
                                          f"OpenMP), {ct:.1f} s"}
    run.close()
    print(json.dumps(line), flush=True)


def serve_measure(dev, rate, seconds, budget_mb, slots, plain=True):
    """The served relations (9 resident tie-heavy relations, N in {20k, 130k, 2M} x d in
    {5, 6, 7}, seeds 0..8) under Poisson arrivals of gres queries (a relation, a random subset
    of its skyline, g_max 25): continuous batching under an HBM budget, then (plain) the
    serialized one-query-at-a-time path on the same arrivals, and both at saturation."""
    from paper_2412_02274_amd import datagen as G
    from paper_2412_02274_amd.serve import (PlainServer, Resident, Server, latency_stats,
                                            poisson_trace)
    residents = [Resident(x, dev) for x in G.serve_relations()]
    srv = Server(residents, budget_bytes=budget_mb << 20, slots=slots, device=dev)
    warm = poisson_trace(residents, rate=rate, duration=2.0, seed=1, start=10_000_000)
    srv.run_trace(warm)
    trace = poisson_trace(residents, rate=rate, duration=seconds, seed=0)
    done = srv.run_trace(trace)
    out = {"relations": [f"{n}x{d}" for n, d, _ in G.SERVE_SPECS], "rate_per_s": rate,
           "seconds": seconds, "g_max": 25, "budget_mb": budget_mb, "slots": slots,
           "latency": latency_stats(done)}
    burst = poisson_trace(residents, rate=1e9, duration=1e-9 * 2000, seed=2)  # all at once
    out["saturation"] = latency_stats(Server(residents, budget_bytes=budget_mb << 20, slots=slots,
                                             device=dev).run_trace(burst))
    out["resident_mb"] = sum(r.resident_bytes() for r in residents) / 2**20
    out["sky_sizes"] = [r.s for r in residents]
    out["max_in_flight"] = srv.max_in_flight
    if plain:
        pl = PlainServer(residents, device=dev)
        pl.run_trace(poisson_trace(residents, rate=rate, duration=1.0, seed=1))
        pdone = pl.run_trace(poisson_trace(residents, rate=rate, duration=seconds, seed=0))
        out["plain_latency"] = latency_stats(pdone)
        out["plain_saturation"] = latency_stats(PlainServer(residents, device=dev).run_trace(
            poisson_trace(residents, rate=1e9, duration=1e-9 * 2000, seed=2)))
        mix = {q.qid: q.g_exit for q in done}
        out["same_results_as_plain"] = all((q.g_exit == mix[q.qid]).all() for q in pdone)
    return out


def bench_serve(args):
    """Serving workload (serve_measure) as the line's own workload."""
    import torch
    dev = torch.device("cuda:0")
    m = serve_measure(dev, args.rate, args.serve_seconds, args.budget_mb, args.slots, not args.no_plain)
    st = m["latency"]
    cfg = {"workload": "serve_ties"}
    cfg.update({k: m[k] for k in ("relations", "rate_per_s", "seconds", "g_max", "budget_mb", "slots")})
    line = _base_line(args, st["tuples_per_s"], "skyline tuples' gres/s", st["mean_ms"], "f32", cfg)
    line["steps"] = st["requests"]
    line.update({k: v for k, v in m.items() if k not in cfg})
    print(json.dumps(line), flush=True)


def sub_partitioned(steps=10):
    """The partitioned workload (uniform 10,000,000 x 4, seed 0, g_max 25) under Grid, Angular
    and Sliced partitioning (target 64 partitions) through the captured pipeline: step time,
    phases, and the HBM-bound phases against the 8 TB/s roof -- build (partition ids, curve
    order and the partition-contiguous copy: 12d + 8 bytes per row algorithmically: read d
    values, write d values plus row id and partition id, read and write the staged row) and the
    local skylines (uniform data: the rows are read once, 4d bytes per row)."""
    import numpy as np
    import torch
    from paper_2412_02274_amd import api
    from tests.golden import workloads as W
    counts = W.load_counts()["uni_10m_d4"]
    kind, n, d, seed, g_max = W.WORKLOADS["uni_10m_d4"]
    x = torch.from_numpy(W.make("uni_10m_d4")).to("cuda:0")
    out = {"workload": "uni_10m_d4", "n": n, "d": d, "g_max": g_max, "target_p": 64}
    for scheme in ("grid", "angular", "sliced"):
        pipe = api.Pipeline(n, d, scheme, 64, 0, g_max, "auto", "cuda:0")
        pipe.run(x)
        sky, ge, _ = pipe.result()
        if int(sky.numel()) != counts["sky_size"]:
            raise SystemExit(f"{scheme}: skyline size {int(sky.numel())} differs from the oracle's")
        hist = np.bincount(ge.cpu().numpy(), minlength=g_max + 1).tolist()
        if counts.get("g_exit_hist") is not None and hist != counts["g_exit_hist"]:
            raise SystemExit(f"{scheme}: g_exit histogram differs from the oracle's")
        graph = pipe.capture(x)
        graph.replay()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            graph.replay()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        del graph
        pipe.run(x, timing=True)
        ph = pipe.phase_ms()
        inf = pipe.info()
        build_bytes = n * (12 * d + 8)
        local_bytes = n * 4 * d
        hbm = lambda b, ms: {"achieved": b / (ms * 1e-3) / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "frac": b / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, "alg_bytes": b}
        out[scheme] = {"ms_per_step": dt * 1e3, "phase_ms": ph, "sky_size": int(sky.numel()),
                       "p": inf["p"], "pruned_rows": inf["pruned_rows"], "rows_kept": inf["rows_kept"],
                       "rounds": [inf["rounds_local"], inf["rounds_merge"]],
                       "paper_skyline_tests": inf["tests_local_max"] + inf["tests_merge"],
                       "build_hbm": hbm(build_bytes, ph["build"]),
                       "local_hbm": hbm(local_bytes, ph["local"])}
        pipe.close()
        del pipe
        torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
