"""The benchmark workloads (seeded synthetic inputs standing in for the paper's UNI/ANT data
and real datasets) and the script that records, from the oracle only, their reference
dominance-test counts into workload_counts.json.

Counts are those of the oracle's plain sequential method: SFS for the skyline (Sec. 4 uses
SFS for its sequential timings) and Alg. 1's per-tuple descending scan for gres, candidates
in ascending row order, each search stopping at the first dominator. They depend on the scan
order, so they are reported as the algorithmic work of a workload, never compared.

Run:  python tests/golden/workloads.py [name ...]
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


if __name__ == "__main__":
    record(sys.argv[1:] or list(WORKLOADS))
