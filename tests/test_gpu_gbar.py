"""GPU parity for Alg. 1's whole level range (Sec. 3.2): ell and g_bar = floor(1/ell) from
gres_gbar against the oracle, and gres searched up to large g_max (up to 2^24, where the
per-target start levels prune the scan) against the oracle's plain descending scan.

Bar: bit-exact. ell is the minimum of FP64 differences of the same FP32 pairs on both sides
(compared as doubles, bit for bit); g_bar and g_exit are integers.
"""
from __future__ import annotations

import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import oracle  # noqa: E402
from paper_2412_02274_amd import _lib, api, datagen as G  # noqa: E402

SAT = 1 << 62  # the device's g_bar saturates here


def _say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda:0")


def _check_gbar(dev, x, tag):
    _say("gbar", tag, x.shape)
    xs = api.ingest(torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev)) if len(x) else \
        torch.zeros((x.shape[1], 0), dtype=torch.float32, device=dev)
    ell, gb = api.gbar(xs)
    o_ell, o_gb = oracle.gbar(x)
    if math.isinf(o_ell):
        assert math.isinf(ell) and gb == 1
    else:
        assert np.float64(ell).tobytes() == np.float64(o_ell).tobytes(), (ell, o_ell)
        assert gb == min(o_gb, SAT)
    return ell, gb


@pytest.mark.parametrize("kind,n,d", [("uni", 5000, 4), ("ant", 20000, 6), ("ties", 30000, 5),
                                      ("dyadic", 4000, 3), ("uni", 1000, 1), ("ant", 70001, 8)])
def test_gbar_matches_oracle(dev, kind, n, d):
    if kind == "ties":
        x = G.ties(n, d, 3, levels=100)
    elif kind == "dyadic":
        x = G.dyadic(n, d, 3, bits=10)
    else:
        x = G.make(kind, n, d, 3)
    _check_gbar(dev, x, kind)


def test_gbar_full_size(dev):
    # 1,000,000 x 6 anticorrelated rows: the sort-based oracle against the device at full size
    x = G.make("ant", 1_000_000, 6, 0)
    _check_gbar(dev, x, "ant_1m_d6")


def test_gbar_edge_cases(dev):
    _check_gbar(dev, np.zeros((0, 3), np.float32), "empty")
    _check_gbar(dev, np.full((1, 2), 0.3, np.float32), "one row")
    _check_gbar(dev, np.full((7, 2), 0.3, np.float32), "constant")
    _check_gbar(dev, np.array([[0.0], [-0.0], [0.0]], np.float32), "signed zeros")
    x = np.array([[0.5, 0.25], [0.5, 0.375], [0.5, 0.875]], np.float32)
    assert _check_gbar(dev, x, "one constant attribute") == (0.125, 8)
    x = np.array([[0.0], [np.float32(1e-40)], [0.5]], np.float32)        # subnormal step
    ell, gb = _check_gbar(dev, x, "subnormal")
    assert ell == float(np.float32(1e-40)) and gb == SAT
    x = np.array([[0.0], [0.75]], np.float32)                            # ell > 1/2: g_bar = 1
    assert _check_gbar(dev, x, "wide") == (0.75, 1)
    # the smallest gap in the last attribute and between the last two rows (a ragged tail)
    x = G.dyadic(1025, 3, 9, bits=6)
    x[-1, 2] = np.float32(x[-2, 2] + np.float32(2.0 ** -20)) if x[-2, 2] < 0.5 else x[-1, 2]
    _check_gbar(dev, x, "ragged tail")


def test_gbar_domain_error(dev):
    x = torch.tensor([[0.5, 0.25], [0.25, 0.5]], dtype=torch.float32, device=dev).t().contiguous()
    bad = x.clone()
    bad[1, 0] = 1.0
    with pytest.raises(_lib.SkyError) as e:
        api.gbar(bad)
    assert e.value.code == _lib.SKY_ERR_DOMAIN
    bad[1, 0] = float("nan")
    with pytest.raises(_lib.SkyError):
        api.gbar(bad)
    assert api.gbar(x) == (0.25, 4)


def _sky(dev, x):
    xs = api.ingest(torch.from_numpy(x).to(dev))
    plan = api.build(xs)
    plan.local_skylines()
    sky = plan.merge().clone()
    plan.close()
    return xs, sky


@pytest.mark.parametrize("mapping", ["auto", "tiles", "levels"])
@pytest.mark.parametrize("kind,n,d,seed", [("ties", 3000, 4, 1), ("dyadic", 2000, 3, 2),
                                           ("dyadic", 1500, 5, 4)])
def test_gres_exact_matches_oracle(dev, mapping, kind, n, d, seed):
    # data whose g_bar the oracle can scan in full: 100 value levels (g_bar near 100) and the
    # 2^-10 lattice (g_bar <= 1024)
    x = G.ties(n, d, seed, levels=100) if kind == "ties" else G.dyadic(n, d, seed, bits=10)
    xs, sky = _sky(dev, x)
    ge, gr, info = api.gres_exact(xs, sky, mapping=mapping)
    _, o_gb = oracle.gbar(x)
    assert info["g_bar"] == o_gb and info["g_max"] == max(2, o_gb) and not info["capped"]
    cand = sky.cpu().numpy()
    want, _ = oracle.gres(x, cand, info["g_max"])
    _say("exact", kind, n, d, "g_bar", o_gb, "S", len(cand), "exits", int((want > 1).sum()))
    assert np.array_equal(ge.cpu().numpy(), want)
    assert np.array_equal(gr.cpu().numpy(), oracle.gres_values(want))
    if kind == "dyadic":
        # Sec. 3.2: nothing exits above g_bar (FP32 products are exact on the lattice)
        more, _ = api.gres(xs, sky, min(4 * o_gb, _lib.SKY_MAX_G), mapping=mapping)
        assert np.array_equal(more.cpu().numpy(), want)


_ORACLE = {}


def _oracle_rows(key, x, cand, targets, g_max):
    # the oracle's answer does not depend on the mapping under test: computed once per case
    if key not in _ORACLE:
        _ORACLE[key] = oracle.gres_rows(x, cand, targets, g_max)
    return _ORACLE[key]


@pytest.mark.parametrize("mapping", ["tiles", "levels"])
@pytest.mark.parametrize("n,d,g_max,exact_leg", [(300, 2, 1 << 24, True), (400, 3, (1 << 22) + 5, True),
                                                 (1000, 3, 1 << 20, True), (5000, 4, 10_000, False)])
def test_gres_large_gmax(dev, mapping, n, d, g_max, exact_leg):
    # levels far above 64 start at each target's bound; the oracle scans every level per target
    x = G.uni(n, d, 17)
    xs, sky = _sky(dev, x)
    cand = sky.cpu().numpy()
    _say("large g_max", n, d, g_max, mapping, "S", len(cand))
    ge, _ = api.gres(xs, sky, g_max, mapping=mapping)
    want = _oracle_rows((n, d, g_max), x, cand, cand, g_max)
    assert np.array_equal(ge.cpu().numpy(), want)
    # the whole level range of Sec. 3.2, up to the oracle's own g_bar (skipped where the
    # oracle's scan of 2^24 levels over a larger skyline would take minutes)
    ge_exact, _, info = api.gres_exact(xs, sky, mapping=mapping)
    _, o_gb = oracle.gbar(x)
    assert info["g_bar"] == o_gb and info["capped"] == (o_gb > _lib.SKY_MAX_G)
    if exact_leg:
        g_top = max(2, min(o_gb, _lib.SKY_MAX_G))
        _say("  g_bar", o_gb)
        want_exact = want if g_top == g_max else _oracle_rows((n, d, g_top), x, cand, cand, g_top)
        assert np.array_equal(ge_exact.cpu().numpy(), want_exact)


@pytest.mark.parametrize("mapping", ["tiles", "levels"])
def test_gres_large_gmax_sampled_full_size(dev, mapping):
    # 20,000 x 6 anticorrelated rows (a skyline of a few thousand), g_max = 5000: sampled targets
    x = G.make("ant", 20_000, 6, 5)
    xs, sky = _sky(dev, x)
    cand = sky.cpu().numpy()
    g_max = 5000
    ge, _ = api.gres(xs, sky, g_max, mapping=mapping)
    rng = np.random.default_rng(0)
    pick = np.sort(rng.choice(len(cand), size=min(48, len(cand)), replace=False))
    _say("sampled", len(cand), g_max, mapping)
    want = _oracle_rows(("ant", g_max), x, cand, cand[pick], g_max)
    assert np.array_equal(ge.cpu().numpy()[pick], want)
