"""GPU parity: the HIP path (through the C ABI) against the oracle, element by element.

Bar: bit-exact. Skyline membership and partition ids are integer/index results; g_exit is an
integer decided by FP32 products taken the same way on both sides (one RNE multiply, then
floor), so every value must match exactly; gres = 1/g_exit in FP32 must match bitwise.
Angular partition ids are compared exactly except in the angles the oracle flags as lying
within 1e-9 of a bucket boundary, where two faithful evaluations of Eq. (1) may round to either
side: there the GPU's bucket of that angle may be the oracle's or its neighbour across the
boundary, and every other angle's bucket must still be equal.
"""
from __future__ import annotations

import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2412_02274_amd import _lib, api, datagen as G  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _rows(kind, n, d, seed):
    if kind == "ties":
        return G.ties(n, d, seed, levels=12)
    if kind == "dyadic":
        return G.dyadic(n, d, seed, bits=5)
    return G.make(kind, n, d, seed)


def run_skyline(dev, x, scheme="none", p=16, slice_dim=0, prefilter=True):
    xs = api.ingest(torch.from_numpy(x).to(dev))
    plan = api.build(xs, scheme, p, slice_dim, prefilter=prefilter)
    plan.local_skylines()
    part = plan.partitions().cpu().numpy()
    loc = plan.local_members().cpu().numpy().astype(bool)
    info = plan.info()
    info["partition_tests"] = plan.partition_tests().cpu().numpy()
    idx = plan.merge().cpu().numpy()
    info.update({k: v for k, v in plan.info().items() if k != "partition_tests"})
    plan.close()
    return xs, idx, part, loc, info


def oracle_partition(x, scheme, p, slice_dim=0):
    n, d = x.shape
    if scheme == "none":
        return np.zeros(n, np.int32), None, 1, None
    if scheme == "grid":
        m, pp = oracle.grid_p(p, d)
        part = oracle.grid_part(x, m)
        ne = np.zeros(pp, np.uint8)
        ne[np.unique(part)] = 1
        return part, None, pp, oracle.grid_pruned(ne, m, d).astype(np.uint8)
    if scheme == "angular":
        m, pp = oracle.angular_p(p, d)
        part, near = oracle.angular_part(x, m)
        return part, near, pp, None
    pp = min(p, n)
    return oracle.sliced_part(x, pp, slice_dim), None, pp, None


def check_partition_tests(info, part, pp, skip, reps_kept=0):
    """The local phase's per-partition test counts (Sec. 4 counts the parallel phase by their
    maximum): they add up to tests_local, their maximum is tests_local_max, a partition without
    live rows has none, one with two or more has some, and no partition exceeds one test per
    (row, row of the partition) pair plus one per (row, kept representative) pair plus one per
    (row, killer row) pair of the build's prefilter (at most SKY_KILLERS per row; a pair can
    be tested there and again by the local phase). Counts depend on the order of the work, so
    they are checked by these properties only."""
    pt = np.asarray(info["partition_tests"], np.int64)
    assert len(pt) == pp
    assert int(pt.sum()) == info["tests_local"]
    assert int(pt.max(initial=0)) == info["tests_local_max"]
    live = np.bincount(part, minlength=pp).astype(np.int64)
    if skip is not None:
        live[skip.astype(bool)] = 0
    assert (pt[live == 0] == 0).all()
    if reps_kept == 0:
        assert (pt[live >= 2] > 0).all()
    bound = live * live + live * (reps_kept + _lib.SKY_KILLERS)
    assert (pt <= bound).all(), np.flatnonzero(pt > bound)


def angular_ids_agree(part, opart, near, pp, d):
    """Per row: every angle's bucket (a base-m digit of the id, Eq. (1)) equals the oracle's,
    except that an angle the oracle flags as lying on a bucket boundary may take the
    neighbouring bucket (one step away)."""
    m = int(round(pp ** (1.0 / (d - 1))))
    assert m ** (d - 1) == pp
    ok = np.ones(len(part), bool)
    w = 1
    for a in range(d - 1):
        dg, do = (part // w) % m, (opart // w) % m
        flagged = ((near >> a) & 1).astype(bool)
        ok &= (dg == do) | (flagged & (np.abs(dg - do) == 1))
        w *= m
    return ok


def check_partitioned(x, scheme, p, part, loc, info, slice_dim=0):
    opart, near, pp, skip = oracle_partition(x, scheme, p, slice_dim)
    assert info["p"] == pp
    check_partition_tests(info, part, pp, skip)
    if near is None:
        assert (part == opart).all()
    else:
        ok = angular_ids_agree(part, opart, near, pp, x.shape[1])
        assert ok.all(), np.flatnonzero(~ok)[:10]
        opart = np.where(near != 0, part, opart)  # boundary rows: take the GPU's (valid) bucket
    want_local = oracle.local_skylines(x, opart, skip)
    assert (loc == want_local).all(), np.flatnonzero(loc != want_local)[:10]


# ------------------------------------------------------------------------------------- ingest

def test_ingest_transpose_canonical(dev):
    x = G.uni(1000, 5, 1)
    x[3, 2] = -0.0
    x[7, 0] = np.float32(1e-40)  # subnormal stays
    xs = api.ingest(torch.from_numpy(x).to(dev)).cpu().numpy()
    want = x.T.copy()
    want[2, 3] = 0.0
    assert (xs.view(np.uint32) == want.view(np.uint32)).all()


@pytest.mark.parametrize("bad", [np.nan, 1.0, -0.25, np.inf])
def test_ingest_domain_error(dev, bad):
    x = G.uni(300, 3, 2)
    x[123, 1] = bad
    with pytest.raises(api.SkyError) as e:
        api.ingest(torch.from_numpy(x).to(dev))
    assert e.value.code == 2


# ------------------------------------------------------------------------------------- skyline

@pytest.mark.parametrize("kind", ["uni", "ant", "ties", "dyadic"])
@pytest.mark.parametrize("d", [1, 3, 8])
def test_skyline_none_no_prefilter(dev, kind, d):
    x = _rows(kind, 3001, d, 11 * d)
    want = np.flatnonzero(oracle.skyline(x))
    _, idx, part, loc, info = run_skyline(dev, x, "none", prefilter=False)
    assert (idx == want).all() and len(idx) == len(want)
    assert info["rows_kept"] == len(x)
    check_partition_tests(info, part, 1, None)


@pytest.mark.parametrize("kind", ["uni", "ant", "ties", "dyadic"])
@pytest.mark.parametrize("d", [1, 2, 3, 5, 8])
@pytest.mark.parametrize("n", [1, 2, 37, 3001])
def test_skyline_none(dev, kind, d, n):
    _say("skyline none", kind, d, n)
    x = _rows(kind, n, d, 3 * d + n)
    want = np.flatnonzero(oracle.skyline(x))
    _, idx, part, loc, info = run_skyline(dev, x, "none")
    assert (idx == want).all() and len(idx) == len(want)
    assert info["sky_count"] == len(want)
    check_partition_tests(info, part, 1, None)
    assert info["tests_local_max"] == info["tests_local"]


@pytest.mark.parametrize("scheme,p", [("grid", 16), ("grid", 64), ("angular", 16),
                                      ("angular", 64), ("sliced", 16), ("sliced", 64)])
@pytest.mark.parametrize("kind", ["uni", "ant", "ties"])
@pytest.mark.parametrize("d", [2, 3, 4, 6])
@pytest.mark.parametrize("prefilter", [True, False])
def test_skyline_partitioned(dev, scheme, p, kind, d, prefilter):
    _say("skyline", scheme, p, kind, d, prefilter)
    n = 5003
    x = _rows(kind, n, d, 7 * d + p)
    want = np.flatnonzero(oracle.skyline(x))
    _, idx, part, loc, info = run_skyline(dev, x, scheme, p, slice_dim=d - 1, prefilter=prefilter)
    assert (idx == want).all() and len(idx) == len(want)
    check_partitioned(x, scheme, p, part, loc, info, slice_dim=d - 1)
    check_rows_kept(x, scheme, p, loc, info, prefilter, slice_dim=d - 1)


def check_rows_kept(x, scheme, p, loc, info, prefilter, slice_dim=0):
    """Without the prefilter every row goes through the local phase. With it, the kept rows
    are those of unpruned partitions that no killer row dominates: never fewer than the
    local skylines' rows (a killer never dominates a row of its partition's skyline)."""
    n = len(x)
    if not prefilter:
        assert info["rows_kept"] == n
        return
    assert int(loc.sum()) <= info["rows_kept"] <= n


def test_skyline_duplicates_and_small_p(dev):
    base = G.uni(50, 3, 4)
    x = np.concatenate([base] * 20)  # every row 20 times
    want = np.flatnonzero(oracle.skyline(x))
    for scheme, p in (("none", 1), ("grid", 8), ("angular", 4), ("sliced", 2000)):
        _, idx, part, loc, info = run_skyline(dev, x, scheme, p)
        assert (idx == want).all()
        check_partitioned(x, scheme, p, part, loc, info)


@pytest.mark.parametrize("case", ["ties5", "signed_zeros", "p_eq_n", "adjacent_floats", "p4096",
                                  "slice_dim2"])
def test_sliced_boundaries(dev, case):
    """Sliced ids (Sec. 3.1: the (value, row) order of the slicing attribute cut into p equal
    runs) where the boundary keys are hard to find: ties across every boundary, -0 and +0 mixed,
    one row per partition, values a few ulps apart, more boundary prefixes than the selection
    keeps in LDS, another slicing attribute. Ids against the oracle's, and the skyline."""
    rng = np.random.default_rng(71)
    dim = 0
    if case == "ties5":
        x, p = (rng.integers(0, 5, (50000, 3)) / 5).astype(np.float32), 64
    elif case == "signed_zeros":
        x, p = rng.random((3000, 2), dtype=np.float32), 16
        x[::3, 0] = 0.0
        x[1::3, 0] = -0.0
    elif case == "p_eq_n":
        x, p = rng.random((200, 3), dtype=np.float32), 200
    elif case == "adjacent_floats":
        x, p = rng.random((30000, 3), dtype=np.float32), 32
        bits = np.float32(0.7).view(np.uint32) + rng.integers(0, 40, 30000).astype(np.uint32)
        x[:, 0] = bits.view(np.float32)
    elif case == "p4096":
        x, p = rng.random((20000, 2), dtype=np.float32), 4096
    else:
        x, p, dim = G.ties(40000, 4, 5, levels=30), 64, 2
    _, idx, part, loc, info = run_skyline(dev, x, "sliced", p, slice_dim=dim)
    check_partitioned(x, "sliced", p, part, loc, info, slice_dim=dim)
    assert np.array_equal(idx, np.flatnonzero(oracle.skyline(x)))


def test_skyline_all_equal(dev):
    x = np.full((4000, 4), 0.25, np.float32)
    _, idx, _, _, _ = run_skyline(dev, x, "none")
    assert (idx == np.arange(4000)).all()


@pytest.mark.parametrize("n", [4095, 4096, 4097, 12289])
@pytest.mark.parametrize("scheme,p", [("none", 1), ("sliced", 3)])
def test_selection_block_edges(dev, n, scheme, p):
    # every row in the skyline (all equal) and every second row (a staircase) at sizes around
    # the selection's 4096-position blocks: ascending ids, member bytes, per-row indices (the
    # gres store reads them) and the count
    for kind in ("equal", "stair"):
        if kind == "equal":
            x = np.full((n, 2), 0.25, np.float32)
            want = np.arange(n)
        else:
            t = (np.arange(n) // 2).astype(np.float64) / n
            x = np.stack([t, 1.0 - 1.0 / n - t], 1).astype(np.float32)
            x[1::2] += np.float32(0.5 / n)  # odd rows: dominated by the row before
            want = np.flatnonzero(oracle.skyline(x))
        xs = api.ingest(torch.from_numpy(x).to(dev))
        plan = api.build(xs, scheme, p)
        plan.local_skylines()
        idx, mem = plan.merge(member=True)
        ge, _ = plan.gres(25)
        plan.close()
        assert np.array_equal(idx.cpu().numpy(), want), (kind, n)
        assert np.array_equal(np.flatnonzero(mem.cpu().numpy()), want)
        if kind == "equal":  # equal rows never dominate one another: no exit at any level
            assert (ge.cpu().numpy() == 1).all()
        else:
            want_ge, _ = oracle.gres(x, want, 25)
            assert np.array_equal(ge.cpu().numpy(), want_ge)


def test_merge_capacity_error(dev):
    x = G.ant(2000, 4, 1)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    plan = api.build(xs, "sliced", 8)
    plan.local_skylines()
    with pytest.raises(api.SkyError) as e:
        plan.merge(cap=3)
    assert e.value.code == 4
    assert int(plan.count.item()) == int(oracle.skyline(x).sum())
    plan.close()


def test_plan_state_errors(dev):
    x = G.uni(100, 2, 1)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    plan = api.build(xs, "none")
    with pytest.raises(api.SkyError) as e:
        plan.merge()
    assert e.value.code == 6
    plan.local_skylines()
    with pytest.raises(api.SkyError) as e:
        plan.local_skylines()
    assert e.value.code == 6
    with pytest.raises(api.SkyError) as e:
        plan.gres(25)  # sky_gres needs the merged skyline
    assert e.value.code == 6
    plan.merge()
    plan.close()


# ---------------------------------------------------------------------------------------- gres

@pytest.mark.parametrize("mapping", ["tiles", "levels"])
@pytest.mark.parametrize("kind", ["uni", "ant", "ties", "dyadic"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 6])
@pytest.mark.parametrize("g_max", [2, 3, 25, 130, 1000])
def test_gres_small(dev, mapping, kind, d, g_max):
    _say("gres", mapping, kind, d, g_max)
    x = _rows(kind, 2000, d, 11 * d + g_max)
    sky = np.flatnonzero(oracle.skyline(x))
    want, _ = oracle.gres(x, sky, g_max)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    ge, gr = api.gres(xs, torch.from_numpy(sky).to(dev), g_max, mapping)
    ge = ge.cpu().numpy()
    assert (ge == want).all(), (np.flatnonzero(ge != want)[:10], ge[ge != want][:10],
                                want[ge != want][:10])
    assert (gr.cpu().numpy().view(np.uint32) == oracle.gres_values(want).view(np.uint32)).all()


@pytest.mark.parametrize("mapping", ["tiles", "levels"])
def test_gres_worked_pair(dev, mapping):
    x = np.array([[0.0625, 0.875], [0.125, 0.5625]], np.float32)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    ge, _ = api.gres(xs, torch.tensor([0, 1], device=dev), 25, mapping)
    assert ge.cpu().tolist() == [7, 1]


@pytest.mark.parametrize("mapping", ["tiles", "levels"])
def test_gres_all_rows_as_candidates(dev, mapping):
    # stability: candidates = every row gives the oracle's result over Sky(r)
    x = G.ant(1500, 3, 9)
    sky = np.flatnonzero(oracle.skyline(x))
    want, _ = oracle.gres(x, np.arange(1500), 25)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    ge, _ = api.gres(xs, torch.arange(1500, device=dev), 25, mapping)
    assert (ge.cpu().numpy() == want).all()
    ws, _ = oracle.gres(x, sky, 25)
    assert (want[sky] == ws).all()


def test_gres_bad_index(dev):
    x = G.uni(100, 2, 1)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    with pytest.raises(api.SkyError) as e:
        api.gres(xs, torch.tensor([0, 5, 100], device=dev), 25)
    assert e.value.code == 1


def test_gres_empty(dev):
    x = G.uni(100, 2, 1)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    ge, gr = api.gres(xs, torch.zeros(0, dtype=torch.int64, device=dev), 25)
    assert ge.numel() == 0 and gr.numel() == 0


# ------------------------------------------------------------------------ configurations (full)

def test_config_uni_10k_d4_gmax_1e4(dev):
    """Plain method, small: UNI 10,000 x 4, seed 0, g_max = 10^4 -- everything compared."""
    x = G.uni(10_000, 4, 0)
    want_sky = np.flatnonzero(oracle.skyline(x))
    want_ge, _ = oracle.gres(x, want_sky, 10_000)
    xs, idx, _, _, _ = run_skyline(dev, x, "none")
    assert (idx == want_sky).all()
    for mapping in ("auto", "tiles", "levels"):
        ge, gr = api.gres(xs, torch.from_numpy(idx).to(dev), 10_000, mapping)
        assert (ge.cpu().numpy() == want_ge).all(), mapping


def test_config_ant_1m_d6(dev):
    """Plain method, anticorrelated: ANT 1,000,000 x 6, g_max = 25, everything compared: the
    skyline (oracle SFS), then g_exit and the bits of gres of all 44,336 skyline tuples (oracle
    Def. 2 search), through gres_compute and through the plan's own sky_gres. The oracle's
    g_exit histogram must also be the one recorded in tests/golden/workload_counts.json."""
    from tests.golden.workloads import load_counts
    x = G.ant(1_000_000, 6, 0)
    _say("oracle sfs ...")
    want_mem, _ = oracle.skyline_sfs(x)
    want_sky = np.flatnonzero(want_mem)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    plan = api.build(xs, "none")
    plan.local_skylines()
    idx = plan.merge().clone()
    ge_plan, gr_plan = plan.gres(25)
    ge, gr = api.gres(xs, idx, 25)
    idx = idx.cpu().numpy()
    plan.close()
    assert len(idx) == len(want_sky) and (idx == want_sky).all()
    _say("oracle gres of", len(want_sky), "tuples ...")
    want_ge, _ = oracle.gres(x, want_sky, 25)
    rec = load_counts()["ant_1m_d6"]["g_exit_hist"]
    assert np.bincount(want_ge, minlength=26).tolist() == rec
    want_bits = oracle.gres_values(want_ge).view(np.uint32)
    for g_exit, g_val in ((ge, gr), (ge_plan, gr_plan)):
        g_exit = g_exit.cpu().numpy()
        bad = np.flatnonzero(g_exit != want_ge)
        assert len(bad) == 0, (len(bad), bad[:10], g_exit[bad[:10]], want_ge[bad[:10]])
        assert np.array_equal(g_val.cpu().numpy().view(np.uint32), want_bits)


@pytest.mark.parametrize("scheme", ["grid", "angular", "sliced"])
def test_config_uni_10m_d4_partitioned(dev, scheme):
    """Partitioned plain method: UNI 10,000,000 x 4, target 64 partitions per scheme. Partition
    ids, local skylines (per partition, by definition) and the final skyline in full; gres of
    every skyline tuple at g_max = 25."""
    x = _cached_uni_10m()
    want_sky = _cached_uni_10m_sky()
    _say("10m", scheme)
    xs, idx, part, loc, info = run_skyline(dev, x, scheme, 64, slice_dim=0)
    assert len(idx) == len(want_sky) and (idx == want_sky).all()
    check_partitioned(x, scheme, 64, part, loc, info, slice_dim=0)
    check_rows_kept(x, scheme, 64, loc, info, True, slice_dim=0)
    _say("10m", scheme, "rows kept", info["rows_kept"])
    assert info["rows_kept"] < len(x) // 5  # uniform data: the killer rows take most rows
    ge, _ = api.gres(xs, torch.from_numpy(idx).to(dev), 25)
    want_ge, _ = oracle.gres(x, want_sky, 25)
    assert (ge.cpu().numpy() == want_ge).all()


@pytest.mark.parametrize("scheme,p", [("none", 1), ("grid", 16), ("angular", 16), ("sliced", 64)])
@pytest.mark.parametrize("kind,n,d", [("uni", 3001, 3), ("ant", 4000, 5), ("ties", 5000, 4),
                                      ("dyadic", 2000, 6), ("uni", 1, 2), ("ant", 70, 1)])
@pytest.mark.parametrize("g_max", [25, 300])
def test_plan_gres(dev, scheme, p, kind, n, d, g_max):
    """sky_gres (the plan's own skyline, candidates read from its curve-ordered copy) against
    gres_compute on the skyline merge() returned, and against the oracle."""
    x = _rows(kind, n, d, 4)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    if d == 1 and scheme == "angular":  # Eq. (1) has no angle for one attribute
        with pytest.raises(api.SkyError) as e:
            api.build(xs, scheme, p)
        assert e.value.code == 1
        return
    plan = api.build(xs, scheme, p)
    plan.local_skylines()
    sky = plan.merge().clone()
    ge, gr = plan.gres(g_max)
    ge2, _ = plan.gres(g_max, mapping="levels")  # the plan's skyline state is only read
    plan.close()
    ref, ref_gr = api.gres(xs, sky, g_max)
    want, _ = oracle.gres(x, sky.cpu().numpy(), g_max)
    assert np.array_equal(ge.cpu().numpy(), want)
    assert np.array_equal(ge2.cpu().numpy(), want)
    assert np.array_equal(ref.cpu().numpy(), want)
    assert np.array_equal(gr.cpu().numpy(), ref_gr.cpu().numpy())


def test_plan_gres_all_equal_and_full_size(dev):
    # every row equal: the skyline is all of them, and nobody exits
    x = np.full((500, 3), 0.375, np.float32)
    xs = api.ingest(torch.from_numpy(x).to(dev))
    plan = api.build(xs)
    plan.local_skylines()
    sky = plan.merge()
    ge, _ = plan.gres(25)
    plan.close()
    assert len(sky) == 500 and (ge.cpu().numpy() == 1).all()
    # the anticorrelated 1,000,000 x 6 workload through the pipeline (which uses sky_gres):
    # every tuple equal to gres_compute on the same skyline
    x = G.ant(1_000_000, 6, 0)
    pipe = api.Pipeline(1_000_000, 6, g_max=25, device=dev)
    sky, ge, _ = pipe.run(torch.from_numpy(x).to(dev)).result()
    ref, _ = api.gres(pipe.x_soa, sky.clone(), 25)
    assert len(sky) == 44336
    assert np.array_equal(ge.cpu().numpy(), ref.cpu().numpy())


@pytest.mark.parametrize("kind,n,d,p", [("uni", 600000, 3, 4), ("ant", 300000, 4, 2),
                                        ("ties", 400000, 5, 3)])
def test_multi_round_segments(dev, kind, n, d, p):
    """Sliced partitions of more than 65,536 rows each: every segment runs several
    head-and-filter rounds (the all-pairs shortcut only ends them), side by side in the same
    launches. Local skylines and the final skyline against the oracle. The build's prefilter
    is off, so that every row reaches the rounds (on uniform data it leaves too few)."""
    x = _rows(kind, n, d, 33)
    xs, idx, part, loc, info = run_skyline(dev, x, "sliced", p, prefilter=False)
    _say(f"multi-round {kind} {n}x{d} p={p}: rounds {info['rounds_local']}+{info['rounds_merge']}")
    if kind != "ties":  # tied scores can put a whole segment into the first head
        assert info["rounds_local"] >= 2
    check_partitioned(x, "sliced", p, part, loc, info)
    mem, _ = oracle.skyline_sfs(x)
    assert np.array_equal(idx, np.flatnonzero(mem))


def _check_reps(dev, x, scheme, p, reps):
    xs = api.ingest(torch.from_numpy(x).to(dev))
    plan = api.build(xs, scheme, p, reps=reps)
    plan.local_skylines()
    part = plan.partitions().cpu().numpy()
    loc = plan.local_members().cpu().numpy().astype(bool)
    ptests = plan.partition_tests().cpu().numpy()
    idx = plan.merge().cpu().numpy()
    info = plan.info()
    info["partition_tests"] = ptests
    plan.close()
    opart, near, pp, skip = oracle_partition(x, scheme, p)
    check_partition_tests(info, part, pp, skip, info["reps_kept"])
    if near is not None:
        assert angular_ids_agree(part, opart, near, pp, x.shape[1]).all()
        opart = np.where(near != 0, part, opart)  # boundary rows: the GPU's (valid) bucket
    want = oracle.local_skylines_reps(x, opart, skip, reps)
    _, kept = oracle.representatives(x, reps)
    assert info["reps_kept"] == int(kept.sum())
    assert np.array_equal(loc, want), np.flatnonzero(loc != want)[:10]
    assert np.array_equal(idx, np.flatnonzero(oracle.skyline_sfs(x)[0]))
    return info


@pytest.mark.parametrize("scheme,p", [("none", 1), ("grid", 16), ("angular", 16), ("sliced", 16)])
@pytest.mark.parametrize("kind,n,d", [("uni", 5000, 3), ("ant", 8000, 4), ("ties", 6000, 5),
                                      ("dyadic", 3000, 2)])
@pytest.mark.parametrize("reps", [1, 10, 100, 1000])
def test_representative_filtering(dev, scheme, p, kind, n, d, reps):
    """Sec. 3.1: the kept representatives' dominated rows leave every local skyline; the local
    skylines equal the oracle's (the same representatives: smallest FP32 sums, ties in row
    order), and the final skyline is unchanged."""
    _check_reps(dev, _rows(kind, n, d, 8), scheme, p, reps)


def test_representative_filtering_large(dev):
    # more rows than one all-pairs round takes, and more representatives than one LDS chunk
    x = _rows("ant", 200_000, 5, 9)
    for scheme, p in (("none", 1), ("sliced", 16)):
        info = _check_reps(dev, x, scheme, p, 1000)
        _say("reps", scheme, info["reps_kept"], info["local_count"], info["rounds_local"])


_C10M = {}


def _cached_uni_10m():
    if "x" not in _C10M:
        _C10M["x"] = G.uni(10_000_000, 4, 0)
    return _C10M["x"]


def _cached_uni_10m_sky():
    if "sky" not in _C10M:
        _C10M["sky"] = np.flatnonzero(oracle.skyline_sfs(_cached_uni_10m())[0])
    return _C10M["sky"]


@pytest.mark.parametrize("mapping", ["tiles", "levels"])
@pytest.mark.parametrize("kind,d,g_max", [("ant", 4, 25), ("uni", 3, 300), ("ties", 5, 25)])
def test_gres_prepare_search_targets(dev, mapping, kind, d, g_max):
    """Prepared candidates (the skyline) searched for arbitrary target rows: skyline subsets in
    any order with repeats, and dominated rows."""
    x = _rows(kind, 20000, d, 5 * d)
    sky = np.flatnonzero(oracle.skyline(x)) if len(x) <= 5000 else \
        np.flatnonzero(oracle.skyline_sfs(x)[0])
    xs = api.ingest(torch.from_numpy(x).to(dev))
    prep = api.PreparedCandidates(xs, torch.from_numpy(sky).to(dev))
    rng = np.random.default_rng(d)
    targets = np.concatenate([rng.choice(sky, min(len(sky), 300)), sky[:5], rng.integers(0, 20000, 100)])
    ge, gr = prep.search(torch.from_numpy(targets).to(dev), g_max, mapping)
    want = oracle.gres_rows(x, sky, targets, g_max)
    assert (ge.cpu().numpy() == want).all()
    assert (gr.cpu().numpy().view(np.uint32) == oracle.gres_values(want).view(np.uint32)).all()
    # every candidate, twice on one prepared set (the set is not consumed)
    for _ in range(2):
        ge_all, _ = prep.search(None, g_max, mapping)
        want_all, _ = oracle.gres(x, sky, g_max)
        assert (ge_all.cpu().numpy() == want_all).all()


def test_gres_search_concurrent_streams(dev):
    """Searches of one prepared set on several streams at once give the results they give alone."""
    x = G.ant(50000, 5, 2)
    sky = np.flatnonzero(oracle.skyline_sfs(x)[0])
    xs = api.ingest(torch.from_numpy(x).to(dev))
    prep = api.PreparedCandidates(xs, torch.from_numpy(sky).to(dev))
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    reqs = [np.sort(rng.choice(sky, int(rng.integers(1, len(sky))), replace=False)) for _ in range(6)]
    alone = [prep.search(torch.from_numpy(r).to(dev), 25)[0].cpu().numpy() for r in reqs]
    streams = [torch.cuda.Stream() for _ in reqs]
    outs = []
    for r, st in zip(reqs, streams):
        with torch.cuda.stream(st):
            t = torch.from_numpy(r).to(dev, non_blocking=False)
            outs.append(prep.search(t, 25, stream=st, status=api.new_status(dev), check=False))
    torch.cuda.synchronize()
    for a, (ge, _), r in zip(alone, outs, reqs):
        assert (ge.cpu().numpy() == a).all()
        assert (a == oracle.gres_rows(x, sky, r, 25)).all()


@pytest.mark.parametrize("scheme,p", [("none", 1), ("grid", 16), ("angular", 16), ("sliced", 64)])
def test_pipeline_graph_replay(dev, scheme, p):
    """The whole pass (ingest, build, local skylines, merge, gres) captured once in a HIP graph:
    no call reads anything back, so every replay recomputes the pass on whatever the captured
    input buffer holds. Replays, with the program's own work between them, equal the eager pass
    and the oracle; a new relation copied into the input gives that relation's results."""
    n, d = 60000, 5
    x = _rows("ant", n, d, 21)
    xr = torch.from_numpy(x).to(dev)
    pipe = api.Pipeline(n, d, scheme, p, 0, g_max=25, device=dev)
    sky0, ge0, gr0 = [t.clone() for t in pipe.run(xr).result()]
    mem, _ = oracle.skyline_sfs(x)
    want_sky = np.flatnonzero(mem)
    want_ge, _ = oracle.gres(x, want_sky, 25)
    assert np.array_equal(sky0.cpu().numpy(), want_sky)
    assert np.array_equal(ge0.cpu().numpy(), want_ge)
    eager_info = pipe.info()
    graph = pipe.capture(xr)
    for rep in range(3):
        pipe.count.fill_(-1)  # eager work between the replays
        pipe.g_exit.fill_(-7)
        pipe.sky_buf.fill_(-3)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        sky, ge, gr = pipe.result()
        assert np.array_equal(sky.cpu().numpy(), want_sky), rep
        assert torch.equal(ge, ge0) and torch.equal(gr, gr0), rep
    info = pipe.info()
    for k in ("sky_count", "local_count", "rounds_local", "rounds_merge", "pruned_rows", "max_partition"):
        assert info[k] == eager_info[k], k
    # another relation of the same shape through the same graph
    x2 = _rows("uni", n, d, 5)
    xr.copy_(torch.from_numpy(x2))
    torch.cuda.synchronize()
    graph.replay()
    torch.cuda.synchronize()
    sky, ge, _ = pipe.result()
    mem2, _ = oracle.skyline_sfs(x2)
    want2 = np.flatnonzero(mem2)
    assert np.array_equal(sky.cpu().numpy(), want2)
    assert np.array_equal(ge.cpu().numpy(), oracle.gres(x2, want2, 25)[0])
    pipe.close()
    _say(f"graph {scheme}: |Sky| {len(want_sky)} and {len(want2)}, rounds "
         f"{info['rounds_local']}+{info['rounds_merge']}")


@pytest.mark.parametrize("g_max,mapping", [(10_000, "auto"), (10_000, "tiles"), (130, "levels")])
def test_pipeline_device_side_mapping(dev, g_max, mapping):
    """sky_gres picks the mapping and the work split on the device from the real skyline size
    (the pipeline sizes its buffers for n): the small uniform workload's shape at g_max 10^4
    (AUTO picks lanes over levels for its small skyline) against the oracle."""
    x = G.uni(10_000, 4, 0)
    pipe = api.Pipeline(10_000, 4, g_max=g_max, mapping=mapping, device=dev)
    sky, ge, gr = pipe.run(torch.from_numpy(x).to(dev)).result()
    mem, _ = oracle.skyline_sfs(x)
    want = np.flatnonzero(mem)
    assert np.array_equal(sky.cpu().numpy(), want)
    assert np.array_equal(ge.cpu().numpy(), oracle.gres(x, want, g_max)[0])
    assert np.array_equal(gr.cpu().numpy(), (1.0 / ge.cpu().numpy().astype(np.float32)))
    pipe.close()


def test_probes(dev):
    """The measurement probes: the copy moves every byte, the VALU probe reports the lane-ops
    of its launch (grid x 256 threads x iterations x 24) and writes its sink."""
    import ctypes as C
    lib = _lib.load()
    src = torch.randint(0, 255, (1 << 20,), dtype=torch.uint8, device=dev)
    dst = torch.zeros_like(src)
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    _lib.check(lib.sky_probe_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), src.numel(),
                                  None, None, st), "sky_probe_copy")
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    sink = torch.zeros(64, dtype=torch.int32, device=dev)
    ops = C.c_int64()
    _lib.check(lib.sky_probe_valu(1000, 64, C.c_void_p(sink.data_ptr()), None, None, st, C.byref(ops)),
               "sky_probe_valu")
    torch.cuda.synchronize()
    assert ops.value == 64 * 256 * 1000 * 24
    assert int((sink != 0).sum()) > 0
