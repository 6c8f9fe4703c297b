"""The efficiency experiments of Sec. 4 (Figs. 2-5) re-run on this implementation's synthetic data.

Every point computes Sky(r) of one generated relation with a partitioning scheme, then gres with
Alg. 1 as written (``api.gres_literal``: for g = g_max .. 2 the skyline of the projected skyline
through the same scheme's two-phase computation) and checks the result against the per-tuple
search (``api.gres``). Dominance tests are counted the way Sec. 4 counts them: per skyline
computation, the heaviest partition's local-phase tests plus the final phase's; for gres, that
sum over the levels. The plain method (scheme "none") runs one partition, so its count is all
of its tests.

The counts are the row-against-row tests the device evaluates, with the build's killer
prefilter off (it is this implementation's addition, not the paper's, and it would count its
own tests in the local phase). Tile-box pruning removes many tests the paper's sequential filter
would make, so absolute numbers are this implementation's;
what carries over is how they move with the scheme, the size, the dimensions, the partitions
and the representatives. Data come from ``datagen`` (uniform, and the anticorrelated generator
around the plane sum(x) = d/2), not the paper's generator.

    python -m paper_2412_02274_amd.experiments --sweep all --seeds 5 --out results.jsonl
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np
import torch

from . import api, datagen as G

SCHEMES = ("none", "grid", "angular", "sliced")
# operating parameters of Sec. 4 (defaults: N = 1M, d = 3, p = 16, no representatives)
DEFAULTS = {"n": 1_000_000, "d": 3, "p": 16, "reps": 0}
SWEEPS = {
    "size": ("n", [100_000, 500_000, 1_000_000, 5_000_000, 10_000_000]),
    "dims": ("d", [2, 3, 4, 5, 6, 7]),
    "parts": ("p", [16, 32, 64, 128]),
    "reps": ("reps", [0, 1, 10, 100, 1000]),
}


def _skyline(xs, scheme, p, reps):
    plan = api.build(xs, scheme, p, reps=reps, prefilter=False)
    plan.local_skylines()
    sky = plan.merge().clone()
    inf = plan.info()
    plan.close()
    return sky, inf


def point(xs: torch.Tensor, p: int, reps: int, scheme: str, g_max: int = 25) -> dict:
    """One relation (SoA on the device), one scheme: Sky(r) and gres by Alg. 1 as written, with
    the paper's counts."""
    t0 = time.perf_counter()
    sky, inf = _skyline(xs, scheme, p, reps)
    torch.cuda.synchronize()
    t_sky = time.perf_counter() - t0
    t0 = time.perf_counter()
    ge_lit, levels = api.gres_literal(xs, sky, g_max, scheme=scheme, target_p=p, reps=reps, prefilter=False)
    torch.cuda.synchronize()
    t_gres = time.perf_counter() - t0
    ge, _ = api.gres(xs, sky, g_max)
    if not np.array_equal(ge_lit, ge.cpu().numpy()):
        raise RuntimeError(f"Alg. 1 as written differs from the per-tuple search: {scheme} "
                           f"p={p} reps={reps}")
    return {
        "target_p": p, "reps": reps, "scheme": scheme, "g_max": g_max, "p": int(inf["p"]),
        "sky": int(sky.numel()),
        "sky_local_max": int(inf["tests_local_max"]), "sky_final": int(inf["tests_merge"]),
        "gres_local_max": sum(lv["tests_local_max"] for lv in levels),
        "gres_final": sum(lv["tests_merge"] for lv in levels),
        "gres_levels": len(levels), "exits": int((ge_lit > 1).sum()),
        "sky_s": t_sky, "gres_s": t_gres,
    }


def _mean(rows, key):
    return float(np.mean([r[key] for r in rows]))


def sweep(name: str, kinds, seeds: int, out=None, log=sys.stderr):
    """All points of one figure: both distributions, every scheme, every value of the varied
    parameter, averaged over `seeds` generated instances. Returns the averaged rows."""
    param, values = SWEEPS[name]
    schemes = SCHEMES if name != "reps" else SCHEMES[1:]
    table = []
    for kind in kinds:
        for v in values:
            cfg = dict(DEFAULTS, **{param: v})
            per_scheme = {s: [] for s in schemes}
            for seed in range(seeds):
                x = G.make(kind, cfg["n"], cfg["d"], seed)
                xs = api.ingest(torch.from_numpy(x).to("cuda"))
                del x
                for scheme in schemes:
                    r = point(xs, cfg["p"], cfg["reps"], scheme)
                    r.update(kind=kind, n=cfg["n"], d=cfg["d"], seed=seed, sweep=name)
                    per_scheme[scheme].append(r)
                    if out is not None:
                        out.write(json.dumps(r) + "\n")
                        out.flush()
                del xs
            for scheme in schemes:
                rows = per_scheme[scheme]
                # "p" is the partition count the scheme reached (Grid and Angular take the
                # closest achievable one), "value" the varied parameter's setting
                avg = {"sweep": name, "kind": kind, "param": param, "value": v, "scheme": scheme,
                       "p": rows[0]["p"], "seeds": seeds}
                for key in ("sky", "sky_local_max", "sky_final", "gres_local_max", "gres_final",
                            "exits", "sky_s", "gres_s"):
                    avg[key] = _mean(rows, key)
                avg["gres_paper"] = avg["gres_local_max"] + avg["gres_final"]
                table.append(avg)
                print(f"{name} {kind} {param}={v} {scheme:8s} p={avg['p']:4d} |Sky|={avg['sky']:9.1f} "
                      f"gres tests: max-part {avg['gres_local_max']:.4g} + final {avg['gres_final']:.4g}"
                      f" = {avg['gres_paper']:.4g}", file=log, flush=True)
    return table


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--sweep", default="all", choices=list(SWEEPS) + ["all"])
    ap.add_argument("--kinds", default="ant,uni")
    ap.add_argument("--seeds", type=int, default=5)
    ap.add_argument("--out", default=None, help="JSON lines, one per point and seed")
    args = ap.parse_args(argv)
    if not torch.cuda.is_available():
        raise SystemExit("experiments need a GPU")
    names = list(SWEEPS) if args.sweep == "all" else [args.sweep]
    out = open(args.out, "w") if args.out else None
    table = []
    for name in names:
        table += sweep(name, args.kinds.split(","), args.seeds, out)
    if out is not None:
        for r in table:
            out.write(json.dumps(dict(r, average=True)) + "\n")
        out.close()
    print(json.dumps({"points": table}))


if __name__ == "__main__":
    main()
