"""GPU parity of the batched path (sky_batch_* through the C ABI) against the oracle, relation by
relation, and against the plain one-relation-at-a-time path.

Bar: bit-exact skyline membership of every relation, g_exit of every skyline tuple, and the
bits of gres = 1/g_exit (the same FP32 contract as the plain path). Tuning choices, graph
replays and the order of relations in the batch never change a result.
"""
from __future__ import annotations

import ctypes as C
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2412_02274_amd import _lib, datagen as G  # noqa: E402
from paper_2412_02274_amd.batch import BatchRunner, GresTuner, PlainRunner  # noqa: E402


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _mixed_batch(seed=0):
    """Relations of uneven size and d, every kind of data, and the degenerate cases."""
    rng = np.random.default_rng(seed)
    out = []
    sizes = (1, 2, 17, 63, 64, 65, 300, 2000)
    kinds = ("uni", "ant", "ties", "dyadic")
    k = 0
    for d in (1, 2, 3, 5, 8):
        for n in sizes:
            kind = kinds[k % 4]
            k += 1
            if kind == "ties":
                x = G.ties(n, d, seed + k, levels=12)
            elif kind == "dyadic":
                x = G.dyadic(n, d, seed + k, bits=5)
            else:
                x = G.make(kind, n, d, seed + k)
            out.append(x)
    out.append(np.zeros((0, 3), dtype=np.float32))                     # empty relation
    out.append(np.full((100, 3), 0.25, dtype=np.float32))              # all rows equal
    dup = G.uni(40, 3, seed + 99)
    out.append(np.concatenate([dup, dup, dup[:7]]))                    # duplicates
    out.append(np.zeros((0, 3), dtype=np.float32))                     # empty, last of its group
    rng.shuffle(out)
    return out


def _check_relation(x, rows, ge, gr, g_max, where):
    mem, _ = oracle.skyline_sfs(x) if x.shape[0] else (np.zeros(0, bool), 0)
    want = np.flatnonzero(mem)
    assert np.array_equal(rows, want), f"{where}: skyline rows differ"
    if len(want):
        wge, _ = oracle.gres(x, want, g_max)
        assert np.array_equal(ge, wge), f"{where}: g_exit differs at {np.flatnonzero(ge != wge)[:5]}"
        assert np.array_equal(gr.view(np.uint32), oracle.gres_values(wge).view(np.uint32)), where


@pytest.mark.parametrize("g_max", [25, 130])
def test_batch_mixed_vs_oracle(dev, g_max):
    data = _mixed_batch()
    _say(f"batch mixed: {len(data)} relations, g_max {g_max}")
    run = BatchRunner(data, g_max=g_max, device=dev, use_graph=False).run()
    for i, x in enumerate(data):
        rows, ge, gr = run.result(i)
        _check_relation(x, rows, ge, gr, g_max, f"relation {i} n={x.shape[0]} d={x.shape[1]}")
    run.close()


def test_batch_tunes_agree(dev):
    data = [G.ant(3000, 4, 1), G.uni(500, 4, 2), G.ant(9000, 4, 3), G.ties(4000, 4, 4, levels=20)]
    run = BatchRunner(data, g_max=25, device=dev, use_graph=False).run()
    g = run.groups[0]
    st = run.stream
    ref = None
    for mapping in (_lib.SKY_GRES_AUTO, _lib.SKY_GRES_TILES, _lib.SKY_GRES_LEVELS):
        for near in (1, 0):
            for lpt in (1, 0):
                with torch.cuda.stream(st):
                    g.set_tune(_lib.SkyTune(mapping, near, lpt))
                    g.g_exit.fill_(-7)
                    g.launch_gres(st)
                st.synchronize()
                got = g.g_exit[:g.sky_count].cpu().numpy().copy()
                if ref is None:
                    ref = got
                    for i in range(len(data)):
                        rows, ge, gr = run.result(i)
                        _check_relation(data[i], rows, ge, gr, 25, f"relation {i}")
                assert np.array_equal(got, ref), (mapping, near, lpt)
    run.close()


def test_batch_graph_replays(dev):
    data = [G.ant(2500, 6, 5), G.uni(7000, 6, 6), G.ant(400, 3, 7), G.ties(3000, 3, 8, levels=15)]
    eager = BatchRunner(data, g_max=25, device=dev, use_graph=False).run()
    want = [eager.result(i) for i in range(len(data))]
    eager.close()
    run = BatchRunner(data, g_max=25, device=dev, use_graph=True, tuner=GresTuner())
    for rep in range(4):
        run.run()
        # the program's own eager work between replays
        junk = torch.randn(1 << 20, device=dev).sum().item()
        assert np.isfinite(junk)
        for i in range(len(data)):
            got = run.result(i)
            for a, b in zip(got, want[i]):
                assert np.array_equal(a, b), f"replay {rep} relation {i}"
    run.close()


def test_batch_matches_plain_path(dev):
    data = [x for x in _mixed_batch(seed=3) if x.shape[0] > 0]
    run = BatchRunner(data, g_max=25, device=dev).run()
    plain = PlainRunner(data, g_max=25, device=dev)
    plain.status.zero_()
    for i in range(len(data)):
        rows, ge, gr = plain.run_one(i, keep=True)
        got = run.result(i)
        assert np.array_equal(got[0], rows), i
        assert np.array_equal(got[1], ge), i
        assert np.array_equal(got[2].view(np.uint32), gr.view(np.uint32)), i
    run.close()


def test_batch_keys_and_values_agree(dev):
    # the gres search on packed key tables, on the values (no tables) and on tables too small
    # for the skyline total (the device falls back to the values): identical results, and the
    # oracle's
    data = [G.ant(3000, 6, 21), G.uni(800, 6, 22), G.ant(12000, 6, 23), G.ties(5000, 6, 24, levels=9),
            G.dyadic(700, 6, 25, bits=4)]
    _say("batch keys vs values")
    ref = BatchRunner(data, g_max=25, device=dev, use_graph=False, keys=False).run()
    want = [ref.result(i) for i in range(len(data))]
    ref.close()
    run = BatchRunner(data, g_max=25, device=dev, use_graph=False).run()
    g = run.groups[0]
    assert getattr(g, "keys_ws", None) is not None  # d = 6 at g_max 25: tables attached
    for i, x in enumerate(data):
        got = run.result(i)
        for a, b in zip(got, want[i]):
            assert np.array_equal(a, b), f"relation {i}"
        _check_relation(x, *got, 25, f"relation {i}")
    st = run.stream
    lib = _lib.load()
    for total in (g.sky_count - 1, 0):  # too small: searched on the values
        with torch.cuda.stream(st):
            g.attach_keys(sky_total=total)
            g.g_exit.fill_(-7)
            g.launch_gres(st)
        st.synchronize()
        for i in range(len(data)):
            got = run.result(i)
            assert np.array_equal(got[1], want[i][1]), (total, i)
    # argument checks: g_max above the table's levels, no tables for d > 10 at g_max 25
    assert lib.sky_batch_keys_bytes(g.h, 100, 65) == 0
    assert lib.sky_batch_keys_bytes(g.h, 100, 25) > 0
    assert lib.sky_batch_set_keys(g.h, None, 0, 0, 25) == _lib.SKY_OK  # detach
    with torch.cuda.stream(st):
        g.g_exit.fill_(-7)
        g.launch_gres(st)
    st.synchronize()
    assert np.array_equal(run.result(2)[1], want[2][1])
    run.close()


def test_batch_capacity_and_state_errors(dev):
    lib = _lib.load()
    x = G.uni(1000, 3, 1)
    run = BatchRunner([x, x], g_max=25, device=dev, use_graph=False)
    g = run.groups[0]
    st = torch.cuda.current_stream()
    sp = C.c_void_p(st.cuda_stream)
    h = C.c_void_p()
    g.status.zero_()
    assert lib.sky_ingest(g.x_rows.data_ptr(), g.n, g.d, g.x_soa.data_ptr(), g.n,
                          g.status.data_ptr(), sp) == 0
    assert lib.sky_batch_create(g.x_soa.data_ptr(), g.d, g.n, g._off_c, g.nb, g.ws.data_ptr(),
                                g.ws_bytes, g.status.data_ptr(), sp, C.byref(h)) == 0
    assert lib.sky_batch_gres(h, 25, None, None, None, None, sp) == _lib.SKY_ERR_STATE
    assert lib.sky_batch_tune(h, None, sp) == 0  # choices may be set any time
    bad = _lib.SkyTune(7, 1, 1)
    assert lib.sky_batch_tune(h, C.byref(bad), sp) == _lib.SKY_ERR_INVALID_ARG
    # capacity 1 is below the two relations' skylines: reported on the device
    assert lib.sky_batch_skylines(h, g.sky_idx.data_ptr(), 1, g.sky_off.data_ptr(), sp) == 0
    torch.cuda.synchronize()
    assert int(g.status.item()) == _lib.SKY_ERR_CAPACITY
    inf = _lib.SkyInfo()
    assert lib.sky_batch_info(h, C.byref(inf)) == 0
    mem, _ = oracle.skyline_sfs(x)
    assert inf.sky_count == 2 * int(mem.sum())
    # the costliest relation's local tests: at most all of them, at least their mean
    assert 0 < inf.tests_local_max <= inf.tests_local <= 2 * inf.tests_local_max
    # with room for every row the same batch gives the oracle's skylines
    g.status.zero_()
    assert lib.sky_batch_skylines(h, g.sky_idx.data_ptr(), g.n, g.sky_off.data_ptr(), sp) == 0
    assert lib.sky_batch_gres(h, 25, g.g_exit.data_ptr(), None, None, None, sp) == 0
    torch.cuda.synchronize()
    assert int(g.status.item()) == 0
    off = g.sky_off.cpu().numpy()
    want = np.flatnonzero(mem)
    assert np.array_equal(g.sky_idx[off[0]:off[1]].cpu().numpy(), want)
    assert np.array_equal(g.sky_idx[off[1]:off[2]].cpu().numpy() - 1000, want)
    wge, _ = oracle.gres(x, want, 25)
    assert np.array_equal(g.g_exit[:off[2]].cpu().numpy(), np.concatenate([wge, wge]))
    lib.sky_batch_destroy(h)
    run.close()


def test_batch_specs_sample_vs_oracle(dev):
    # the first relations of the many-dataset workload, sizes capped for the oracle
    specs = [(min(n, 30000), d, kind, s) for (n, d, kind, s) in G.batch_specs()[:48]]
    data = [G.batch_dataset(s) for s in specs]
    run = BatchRunner(data, g_max=25, device=dev, tuner=GresTuner()).run()
    rng = np.random.default_rng(0)
    for i, x in enumerate(data):
        rows, ge, gr = run.result(i)
        mem, _ = oracle.skyline_sfs(x)
        want = np.flatnonzero(mem)
        assert np.array_equal(rows, want), i
        pick = np.arange(len(want)) if len(want) <= 400 else np.sort(rng.choice(len(want), 400, False))
        wge = oracle.gres_rows(x, want, want[pick], 25)
        assert np.array_equal(ge[pick], wge), i
        assert np.array_equal(gr.view(np.uint32), oracle.gres_values(ge).view(np.uint32))
    run.close()


def test_batch_full_workload_sampled(dev):
    """All 4096 relations of the many-dataset workload in the configuration the benchmark times
    (groups by d, tuned work tables, graph replay); the oracle checks sampled relations in full
    and sampled tuples of the largest ones, and properties hold for every relation."""
    specs = G.batch_specs()
    data = [G.batch_dataset(s) for s in specs]
    _say(f"full batch: {sum(x.shape[0] for x in data)} rows")
    run = BatchRunner(data, g_max=25, device=dev, tuner=GresTuner())
    run.run()
    run.run()  # second pass: graph replay
    _say("full batch: ran", run.phase_ms(), "skyline total", run.sky_total())
    rng = np.random.default_rng(1)
    by_size = np.argsort([x.shape[0] for x in data])
    sample = list(by_size[:8]) + list(rng.choice(len(data), 12, replace=False)) + list(by_size[-2:])
    for i in sample:
        x = data[i]
        rows, ge, gr = run.result(int(i))
        n = x.shape[0]
        if n <= 60000:
            mem, _ = oracle.skyline_sfs(x)
            want = np.flatnonzero(mem)
            assert np.array_equal(rows, want), i
        else:
            # membership of sampled rows, and of sampled reported skyline rows, by Def. 1
            want = rows
            probe = rng.choice(n, 300, replace=False)
            expect = oracle.skyline_rows(x, probe)
            assert np.array_equal(np.isin(probe, rows), expect), i
            mine = rng.choice(rows, min(300, len(rows)), replace=False)
            assert oracle.skyline_rows(x, mine).all(), i
        pick = np.arange(len(want)) if len(want) <= 200 else rng.choice(len(want), 200, False)
        wge = oracle.gres_rows(x, want, want[pick], 25)
        assert np.array_equal(ge[pick], wge), i
    # every relation's skyline size against the oracle's (recorded by tests/golden/workloads.py)
    import json
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "batch_counts.json")
    with open(path) as f:
        want_sizes = json.load(f)["sky_size"]
    for g in run.groups:
        got = np.diff(g.sky_off.cpu().numpy())
        assert np.array_equal(got, [want_sizes[i] for i in g.members]), g.d
    for g in run.groups:
        s = g.sky_count
        ge = g.g_exit[:s].cpu().numpy()
        gr = g.gres[:s].cpu().numpy()
        assert ((ge == 1) | ((ge >= 2) & (ge <= 25))).all()
        assert np.array_equal(gr.view(np.uint32), oracle.gres_values(ge).view(np.uint32))
        off = g.sky_off.cpu().numpy()
        assert off[0] == 0 and off[-1] == s and (np.diff(off) >= 0).all()
        assert (np.diff(off) >= np.minimum(np.diff(g.offsets), 1)).all()  # non-empty -> non-empty
    run.close()
