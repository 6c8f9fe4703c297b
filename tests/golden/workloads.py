"""The benchmark workloads (seeded synthetic inputs standing in for the paper's UNI/ANT data
and real datasets) and the script that records, from the oracle only, their reference
dominance-test counts into workload_counts.json.

Counts are those of the oracle's plain sequential method: SFS for the skyline (Sec. 4 uses
SFS for its sequential timings) and Alg. 1's per-tuple descending scan for gres, candidates
in ascending row order, each search stopping at the first dominator. They depend on the scan
order, so they are reported as the algorithmic work of a workload, never compared.

Run:  python tests/golden/workloads.py [name ...]
      python tests/golden/workloads.py batch      (the many-dataset workload: skyline sizes and
                                                   SFS counts per relation, batch_counts.json)
"""
from __future__ import annotations

import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

COUNTS = os.path.join(HERE, "workload_counts.json")

# name -> (generator, n, d, seed, g_max)
WORKLOADS = {
    "uni_10k_d4": ("uni", 10_000, 4, 0, 10_000),
    "ant_1m_d6": ("ant", 1_000_000, 6, 0, 25),
    "uni_10m_d4": ("uni", 10_000_000, 4, 0, 25),
}


def make(name):
    from paper_2412_02274_amd import datagen
    kind, n, d, seed, _ = WORKLOADS[name]
    return datagen.make(kind, n, d, seed)


def load_counts():
    with open(COUNTS) as f:
        return json.load(f)


def record(names):
    import numpy as np
    import oracle
    out = load_counts() if os.path.exists(COUNTS) else {}
    for name in names:
        kind, n, d, seed, g_max = WORKLOADS[name]
        x = make(name)
        t0 = time.time()
        mem, sfs_tests = oracle.skyline_sfs(x)
        sky = np.flatnonzero(mem)
        ge, gres_tests = oracle.gres(x, sky, g_max)
        out[name] = {"kind": kind, "n": n, "d": d, "seed": seed, "g_max": g_max,
                     "sky_size": int(len(sky)), "sfs_tests": int(sfs_tests),
                     "gres_tests": int(gres_tests),
                     "g_exit_hist": np.bincount(ge, minlength=g_max + 1).tolist()
                     if g_max <= 100 else None,
                     "oracle_seconds": round(time.time() - t0, 1),
                     "oracle_threads": oracle.num_threads()}
        print(name, {k: v for k, v in out[name].items() if k != "g_exit_hist"}, flush=True)
        with open(COUNTS, "w") as f:
            json.dump(out, f, indent=1, sort_keys=True)


BATCH_COUNTS = os.path.join(HERE, "batch_counts.json")


def _batch_one(spec):
    import oracle
    from paper_2412_02274_amd import datagen
    x = datagen.batch_dataset(spec)
    mem, tests = oracle.skyline_sfs(x)
    return int(mem.sum()), int(tests)


def record_batch(seed=0, workers=8):
    """Skyline size and oracle SFS test count of every relation of the many-dataset workload
    (relations in parallel processes, each single-threaded)."""
    from multiprocessing import Pool
    from paper_2412_02274_amd import datagen
    specs = datagen.batch_specs(seed=seed)
    order = sorted(range(len(specs)), key=lambda i: -specs[i][0] * specs[i][1])
    t0 = time.time()
    with Pool(workers) as pool:
        res = pool.map(_batch_one, [specs[i] for i in order], chunksize=1)
    sky = [0] * len(specs)
    sfs = [0] * len(specs)
    for i, (s, t) in zip(order, res):
        sky[i], sfs[i] = s, t
    out = {"seed": seed, "count": len(specs), "sky_size": sky, "sfs_tests": sfs,
           "sky_total": int(sum(sky)), "sfs_total": int(sum(sfs)),
           "oracle_seconds": round(time.time() - t0, 1), "processes": workers}
    with open(BATCH_COUNTS, "w") as f:
        json.dump(out, f)
    print("batch", {k: v for k, v in out.items() if k not in ("sky_size", "sfs_tests")}, flush=True)


if __name__ == "__main__":
    if sys.argv[1:] == ["batch"]:
        record_batch()
    else:
        record(sys.argv[1:] or list(WORKLOADS))
