"""GPU tests of Alg. 1 as written: at every level the skyline of the grid-projected candidate
set is recomputed through the partitioned two-phase scheme (sky_project + sky_build /
sky_local_skylines / sky_merge). Bit-exact against the per-tuple search (gres_compute) and the
oracle, for every partitioning scheme; the projection itself against the oracle's keys."""
from __future__ import annotations

import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2412_02274_amd import api, datagen as G  # noqa: E402


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _data(kind, n, d, seed):
    if kind == "ties":
        return G.ties(n, d, seed, levels=12)
    if kind == "dyadic":
        return G.dyadic(n, d, seed, bits=5)
    return G.make(kind, n, d, seed)


@pytest.mark.parametrize("g", [1, 2, 7, 25, 1000, 1 << 20, (1 << 20) + 3, 1 << 24])
def test_project_is_the_scaled_key(dev, g):
    x = G.uni(3001, 5, 11)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    rows = torch.from_numpy(np.arange(0, 3001, 3, dtype=np.int64)).to(dev)
    out = api.project(xs, rows, g).cpu().numpy()
    b = max(0, math.ceil(math.log2(g)))
    sub = x[::3]
    want = np.array([[oracle.key(float(v), g) for v in sub[:, k]] for k in range(5)], dtype=np.float64)
    assert np.array_equal(out.astype(np.float64), want * 2.0 ** -b)
    assert (out < 1.0).all() and (out >= 0.0).all()


@pytest.mark.parametrize("scheme", ["none", "grid", "angular", "sliced"])
@pytest.mark.parametrize("kind,n,d", [("uni", 2000, 3), ("ant", 3000, 4), ("ties", 4000, 5),
                                      ("dyadic", 1500, 3)])
@pytest.mark.parametrize("g_max", [25, 130])
def test_literal_equals_per_tuple(dev, scheme, kind, n, d, g_max):
    x = _data(kind, n, d, 5)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    plan = api.build(xs)
    plan.local_skylines()
    sky = plan.merge().clone()
    plan.close()
    ge_lit, levels = api.gres_literal(xs, sky, g_max, scheme=scheme, target_p=16)
    ge, _ = api.gres(xs, sky, g_max)
    assert np.array_equal(ge_lit, ge.cpu().numpy())
    want, _ = oracle.gres(x, sky.cpu().numpy(), g_max)
    assert np.array_equal(ge_lit, want)
    # every candidate exits at most once, and the counts add up
    assert sum(lv["exits"] for lv in levels) == int((ge_lit > 1).sum())
    # the paper's count per level: the heaviest partition plus the final phase
    for lv in levels:
        assert lv["tests_local_max"] <= lv["tests_local"]
        assert lv["tests_paper"] == lv["tests_local_max"] + lv["tests_merge"]
        if scheme == "none":
            assert lv["tests_local_max"] == lv["tests_local"]


def test_literal_anticorrelated_partitioned(dev):
    x = G.ant(20000, 4, 3)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    plan = api.build(xs)
    plan.local_skylines()
    sky = plan.merge().clone()
    plan.close()
    ge, _ = api.gres(xs, sky, 25)
    for scheme in ("grid", "angular", "sliced"):
        ge_lit, levels = api.gres_literal(xs, sky, 25, scheme=scheme, target_p=64)
        assert np.array_equal(ge_lit, ge.cpu().numpy()), scheme
        assert all(lv["p"] > 1 for lv in levels)
        # partitioning spreads the local phase: its heaviest partition holds a part of it
        assert all(lv["tests_local_max"] < lv["tests_local"] for lv in levels), scheme


def test_experiment_point_counts(dev):
    # one point of the Sec. 4 sweeps: the same skyline and exits under every scheme, and the
    # paper's counts (heaviest partition + final phase) add up from the per-level records
    from paper_2412_02274_amd import experiments
    x = G.ant(30000, 3, 4)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    rows = {s: experiments.point(xs, 16, 0, s) for s in experiments.SCHEMES}
    base = rows["none"]
    assert base["p"] == 1 and base["gres_levels"] >= 1 and base["gres_local_max"] > 0
    for s, r in rows.items():
        assert r["sky"] == base["sky"] and r["exits"] == base["exits"], s
        if s != "none":
            assert r["p"] > 1
            assert r["sky_local_max"] < base["sky_local_max"], s
    r = experiments.point(xs, 16, 10, "sliced")  # with representatives
    assert r["sky"] == base["sky"] and r["exits"] == base["exits"]
