"""GPU tests of the serving loop: every query's answer is the same alone (the plain one-at-a-
time path) and in the mix (continuous batching on several streams under a tight HBM budget),
and equal to the oracle's gres of those tuples in their relation. Bit-exact."""
from __future__ import annotations

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2412_02274_amd import datagen as G  # noqa: E402
from paper_2412_02274_amd.serve import (PlainServer, Resident, Server, _query_bytes,  # noqa: E402
                                        latency_stats, poisson_trace)


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


@pytest.fixture(scope="module")
def relations():
    return [G.ties(5000, 5, 0), G.ties(20000, 6, 1), G.ties(60000, 7, 2), G.ant(3000, 3, 3)]


@pytest.fixture(scope="module")
def residents(dev, relations):
    return [Resident(x, dev) for x in relations]


def test_resident_skylines_match_oracle(residents, relations):
    for r, x in zip(residents, relations):
        mem, _ = oracle.skyline_sfs(x)
        assert np.array_equal(r.sky_host, np.flatnonzero(mem))


def test_mix_equals_alone_equals_oracle(dev, residents, relations):
    # a burst far above what one stream keeps up with, so queries overlap on the device
    trace = poisson_trace(residents, rate=20000.0, duration=0.03, seed=5)
    assert len(trace) > 100
    largest = max(sum(-(-p // 256) * 256 for p in _query_bytes(r.s, r.d)[1]) for r in residents)
    srv = Server(residents, budget_bytes=2 * largest, slots=4, device=dev)
    done = srv.run_trace(trace)
    assert len(done) == len(trace)
    _say("mix:", latency_stats(done), "max in flight", srv.max_in_flight, "peak bytes", srv.peak_used)
    assert srv.max_in_flight >= 2          # work really overlapped
    assert max(len(b) for _, b in srv.batch_log) >= 2  # queries really shared launches
    assert srv.peak_used <= 2 * largest    # the budget held
    mix = {q.qid: q.g_exit for q in done}
    alone = PlainServer(residents, device=dev)
    rng = np.random.default_rng(0)
    for q in poisson_trace(residents, rate=20000.0, duration=0.03, seed=5):
        alone.run_one(q)
        assert np.array_equal(q.g_exit, mix[q.qid]), q.qid
        if rng.random() < 0.15:
            x = relations[q.rel]
            want = oracle.gres_rows(x, residents[q.rel].sky_host, q.targets, q.g_max)
            assert np.array_equal(q.g_exit, want), q.qid


def test_budget_below_largest_query_rejected(dev, residents):
    with pytest.raises(ValueError):
        Server(residents, budget_bytes=1024, slots=2, device=dev)


def test_fifo_admission_under_budget(dev, residents):
    # budget for exactly one of the largest queries: batches shrink to fit, the oldest query
    # is never overtaken
    big = max(range(len(residents)), key=lambda i: residents[i].s)
    r = residents[big]
    largest = sum(-(-p // 256) * 256 for p in _query_bytes(r.s, r.d)[1])
    trace = poisson_trace(residents, rate=50000.0, duration=0.004, seed=9)
    srv = Server(residents, budget_bytes=largest, slots=4, device=dev)
    done = srv.run_trace(trace)
    assert len(done) == len(trace)
    assert sorted(srv.admit_order) == [q.qid for q in trace]
    # every batch starts with the oldest query still queued, and holds one relation
    admitted = set()
    rel = {q.qid: q.rel for q in trace}
    for oldest, qids in srv.batch_log:
        assert qids[0] == oldest
        assert oldest == min(q.qid for q in trace if q.qid not in admitted)
        assert len({rel[x] for x in qids}) == 1
        admitted.update(qids)
    assert srv.peak_used <= largest


# ------------------------------------------- the served workload itself: its nine relations

@pytest.fixture(scope="module")
def spec_relations():
    _say("generating the nine served relations ...")
    return G.serve_relations()


@pytest.fixture(scope="module")
def spec_residents(dev, spec_relations):
    return [Resident(x, dev) for x in spec_relations]


@pytest.fixture(scope="module")
def spec_oracle(spec_relations):
    """Per relation: the oracle's skyline (SFS) and the g_exit of every skyline tuple (Def. 2
    search, g_max 25)."""
    out = []
    for (n, d, seed), x in zip(G.SERVE_SPECS, spec_relations):
        mem, _ = oracle.skyline_sfs(x)
        sky = np.flatnonzero(mem)
        ge, _ = oracle.gres(x, sky, 25)
        _say(f"oracle ties {n}x{d} seed {seed}: |Sky| = {len(sky)}")
        out.append((sky, ge))
    return out


def test_served_relations_skylines_and_gres_match_oracle(dev, spec_residents, spec_oracle):
    """Each of the nine tie-heavy relations (N in {20k, 130k, 2M} x d in {5, 6, 7}): the resident
    skyline and the gres of every skyline tuple of its prepared candidates equal the oracle's,
    g_exit and gres bits."""
    for (n, d, seed), r, (sky, want) in zip(G.SERVE_SPECS, spec_residents, spec_oracle):
        assert np.array_equal(r.sky_host, sky), (n, d)
        ge, gr = r.prep.search(None, 25)
        assert np.array_equal(ge.cpu().numpy(), want), (n, d)
        assert np.array_equal(gr.cpu().numpy().view(np.uint32),
                              oracle.gres_values(want).view(np.uint32)), (n, d)


def test_served_queries_match_oracle(dev, spec_residents, spec_oracle):
    """Queries of the served workload (Poisson arrivals, a relation, a random subset of its
    skyline) through continuous batching under a tight budget: every answer equals the oracle's
    g_exit of those tuples in their relation (a tuple's gres does not depend on which other
    tuples a query names)."""
    largest = max(sum(-(-p // 256) * 256 for p in _query_bytes(r.s, r.d)[1]) for r in spec_residents)
    trace = poisson_trace(spec_residents, rate=5000.0, duration=0.1, seed=3)
    srv = Server(spec_residents, budget_bytes=2 * largest, slots=4, device=dev)
    done = srv.run_trace(trace)
    assert len(done) == len(trace) > 100
    assert srv.max_in_flight >= 2
    for q in done:
        sky, want = spec_oracle[q.rel]
        pos = np.searchsorted(sky, q.targets)
        assert np.array_equal(sky[pos], q.targets)
        assert np.array_equal(q.g_exit, want[pos]), q.qid
