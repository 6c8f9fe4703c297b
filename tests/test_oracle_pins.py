"""Pins for the oracle: values and properties fixed by the paper and by mathematics, not by
re-typing the oracle's own formulas. CPU only.

What pins what:
* Def. 1 skyline        -- literal brute force (sets of Python tuples); d = 1 closed form;
                           d = 2 textbook staircase sweep; SFS == definition; UNI size statistics.
* Def. 2 / Alg. 1 gres  -- literal set-based brute force over every g (FP32 and exact
                           rationals); the worked non-monotone pair (tests/golden); invariants:
                           non-increasing in g_max, lattice data never exits at g = 2^b,
                           duplicates, stability (candidates r vs Sky(r)), bounds, d = 1.
* quantisation          -- dyadic data: floor(x*g) equals integer (k*g) >> bits.
* Grid / Def. 3         -- the paper's 3x3 example (tests/golden); cell bounds in exact rationals.
* Angular / Eq. (1)     -- special directions with known angles; an arccos-based evaluation.
* Sliced                -- part sizes floor/ceil(N/p); order on the slicing attribute; ties by row.
* two-phase skyline     -- union of local skylines -> final skyline == Sky(r) for every scheme;
                           no skyline row inside a pruned Grid cell.
"""
from __future__ import annotations

import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import brute
from paper_2412_02274_amd import datagen as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(kind, n, d, seed):
    if kind == "ties":
        return G.ties(n, d, seed, levels=6)
    if kind == "dyadic":
        return G.dyadic(n, d, seed, bits=3)
    return G.make(kind, n, d, seed)


# ----------------------------------------------------------------------------- worked examples

def _read_golden_pair():
    rows, levels = [], None
    with open(os.path.join(GOLDEN, "nonmonotone_pair.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("levels"):
                levels = [int(v) for v in line.split()[1:]]
            else:
                a, b, g = line.split()
                rows.append((float(a), float(b), int(g)))
    return rows, levels


def test_golden_nonmonotone_pair(orc):
    rows, levels = _read_golden_pair()
    x = np.array([[a, b] for a, b, _ in rows], dtype=np.float32)
    ge, _ = orc.gres(x, [0, 1], 25)
    assert list(ge) == [g for _, _, g in rows]
    # the per-level picture: g_exit with g_max = G is the largest exit level <= G
    for gmax in range(2, 41):
        ge, _ = orc.gres(x, [0, 1], gmax)
        below = [lv for lv in levels if lv <= gmax]
        assert ge[0] == (max(below) if below else 1), gmax
        assert ge[1] == 1
    # and the literal set-based reading of Def. 2 agrees, exactly and in FP32
    assert brute.gres_g_exit(x, 25, "exact") == {0: 7, 1: 1}
    assert brute.gres_g_exit(x, 25, "fp32") == {0: 7, 1: 1}


def _read_grid_golden():
    out, cur = [], {}
    with open(os.path.join(GOLDEN, "grid_example.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *vals = line.split()
            vals = [int(v) for v in vals]
            if key in ("m", "d"):
                cur[key] = vals[0]
            elif key == "dominator":
                cur["dom"] = vals[0]
            elif key == "pruned":
                out.append((cur["m"], cur["d"], cur["dom"], sorted(vals)))
    return out


def test_golden_grid_example(orc):
    for m, d, dom, pruned in _read_grid_golden():
        ne = np.zeros(m ** d, dtype=np.uint8)
        ne[dom] = 1
        got = np.flatnonzero(orc.grid_pruned(ne, m, d)).tolist()
        assert got == pruned
    # numbering: a tuple in the middle of cell (1, 0) is in partition 1, (2, 1) -> 5, (2, 2) -> 8
    x = np.array([[0.5, 0.1], [0.9, 0.5], [0.9, 0.9], [0.1, 0.9]], dtype=np.float32)
    assert orc.grid_part(x, 3).tolist() == [1, 5, 8, 6]


# ------------------------------------------------------------------------------ quantisation

@pytest.mark.parametrize("g", [2, 3, 7, 25, 100, 1000, 4096])
def test_key_dyadic_exact(orc, g):
    bits = 12
    ks = np.arange(0, 1 << bits)
    for k in ks[:: max(1, len(ks) // 512)]:
        v = float(k) / (1 << bits)
        assert orc.key(v, g) == (int(k) * g) >> bits


def test_key_is_single_fp32_multiply_floor(orc):
    # a value where the exact-real floor and the FP32 rule differ: v = 0.35999998... (the
    # float just below 0.36) times 25 is 8.9999996... exactly, but the FP32 product rounds to
    # 9.0, so the FP32 key is 9 while the exact key is 8. The FP32 rule is the contract.
    v = 0.35999998450279236
    assert float(np.float32(v)) == v
    assert Fraction(v) * 25 < 9
    assert orc.key(v, 25) == 9
    assert orc.key(0.0, 25) == 0 and orc.key(-0.0, 25) == 0
    assert orc.key(float(np.nextafter(np.float32(1), np.float32(0))), 25) == 24


# --------------------------------------------------------------------------------- skyline

@pytest.mark.parametrize("kind", ["uni", "ant", "ties", "dyadic"])
@pytest.mark.parametrize("d", [1, 2, 3, 4])
def test_skyline_vs_brute(orc, kind, d):
    for seed in range(4):
        x = _rows(kind, 40, d, seed)
        assert (orc.skyline(x) == brute.skyline_rows(x)).all()


def test_skyline_d1_closed_form(orc):
    for seed in range(5):
        x = G.ties(300, 1, seed, levels=7)
        want = x[:, 0] == x[:, 0].min()
        assert (orc.skyline(x) == want).all()
        ge, _ = orc.gres(x, np.flatnonzero(want), 50)
        assert (ge == 1).all()  # d = 1: equal values never dominate each other


def _staircase(x):
    """Textbook 2-d skyline: sweep by the first attribute, keep the running minimum of the second."""
    n = len(x)
    order = sorted(range(n), key=lambda i: (float(x[i, 0]), float(x[i, 1])))
    member = np.zeros(n, dtype=bool)
    best = math.inf  # min second attribute over strictly smaller first attribute
    i = 0
    while i < n:
        j = i
        while j < n and x[order[j], 0] == x[order[i], 0]:
            j += 1
        grp_min = min(float(x[order[q], 1]) for q in range(i, j))
        for q in range(i, j):
            v = float(x[order[q], 1])
            member[order[q]] = v == grp_min and v < best
        best = min(best, grp_min)
        i = j
    return member


@pytest.mark.parametrize("kind", ["uni", "ant", "ties"])
def test_skyline_d2_staircase(orc, kind):
    for seed in range(3):
        x = _rows(kind, 3000, 2, seed)
        assert (orc.skyline(x) == _staircase(x)).all()


@pytest.mark.parametrize("kind", ["uni", "ant", "ties", "dyadic"])
@pytest.mark.parametrize("d", [2, 3, 5, 7])
def test_sfs_equals_definition(orc, kind, d):
    x = _rows(kind, 1500, d, d)
    want = orc.skyline(x)
    got, tests = orc.skyline_sfs(x)
    assert (got == want).all()
    assert tests >= 0


def _expected_uni_skyline(n, d):
    # E|Sky| of n i.i.d. continuous points in d dims: A(n,1)=1, A(n,d)=sum_{i<=n} A(i,d-1)/i
    a = np.ones(n + 1)
    a[0] = 0
    for _ in range(d - 1):
        b = np.zeros(n + 1)
        b[1:] = np.cumsum(a[1:] / np.arange(1, n + 1))
        a = b
    return a[n]


def test_uni_skyline_size_statistics(orc):
    n, d, reps = 4000, 3, 12
    sizes = [orc.skyline_sfs(G.uni(n, d, 100 + s))[0].sum() for s in range(reps)]
    mean = float(np.mean(sizes))
    want = _expected_uni_skyline(n, d)
    assert abs(mean - want) < 0.2 * want, (mean, want)


# ------------------------------------------------------------------------------------ gres

@pytest.mark.parametrize("kind", ["uni", "ant", "ties", "dyadic"])
@pytest.mark.parametrize("d", [2, 3, 4])
def test_gres_vs_brute_fp32(orc, kind, d):
    for seed in range(3):
        x = _rows(kind, 14, d, seed)
        cand = np.flatnonzero(orc.skyline(x))
        ge, _ = orc.gres(x, cand, 24)
        want = brute.gres_g_exit(x, 24, "fp32")
        assert [want[int(c)] for c in cand] == ge.tolist()


def test_gres_dyadic_exact_rationals(orc):
    for seed in range(4):
        x = G.dyadic(12, 3, seed, bits=6)
        cand = np.flatnonzero(orc.skyline(x))
        ge, _ = orc.gres(x, cand, 40)
        exact = brute.gres_g_exit(x, 40, "exact")
        assert [exact[int(c)] for c in cand] == ge.tolist()


def test_gres_nonincreasing_in_gmax(orc):
    x = G.uni(400, 3, 7)
    cand = np.flatnonzero(orc.skyline(x))
    prev = None
    for gmax in [2, 3, 5, 8, 13, 25, 60, 200]:
        ge, _ = orc.gres(x, cand, gmax)
        assert ((ge == 1) | ((ge >= 2) & (ge <= gmax))).all()  # 1/g_max <= gres <= 1
        if prev is not None:
            assert (ge >= prev).all()
            # g_exit(g_max) = max exit level <= g_max: whatever exited below the old bound stays
            keep = prev > 1
            assert (ge[keep] >= prev[keep]).all()
        prev = ge


def test_gres_lattice_never_exits_at_power_of_two(orc):
    # data on the 2^-b lattice: at g = 2^b (and multiples) the projection keeps every order and
    # every equality, so no skyline tuple can leave the skyline there
    b = 5
    for seed in range(3):
        x = G.dyadic(500, 3, seed, bits=b)
        cand = np.flatnonzero(orc.skyline(x))
        for g in (1 << b, 2 << b, 3 << b):
            ge, _ = orc.gres(x, cand, g)
            assert (ge != g).all()


def test_gres_duplicates(orc):
    base = G.uni(60, 3, 3)
    x = np.concatenate([base, base[:20]])  # rows 60..79 duplicate rows 0..19
    sky = orc.skyline(x)
    assert (sky[60:] == sky[:20]).all()
    cand = np.flatnonzero(sky)
    ge, _ = orc.gres(x, cand, 30)
    g = dict(zip(cand.tolist(), ge.tolist()))
    for i in range(20):
        if sky[i]:
            assert g[i] == g[60 + i]


def test_gres_stable_under_dominated_candidates(orc):
    for kind in ("uni", "ant", "ties"):
        x = _rows(kind, 300, 3, 11)
        cand = np.flatnonzero(orc.skyline(x))
        ge, _ = orc.gres(x, cand, 25)
        allrows, _ = orc.gres(x, np.arange(len(x)), 25)
        assert (allrows[cand] == ge).all()


def test_gres_rows_and_skyline_rows_match_full(orc):
    x = G.ant(3000, 4, 5)
    sky = orc.skyline(x)
    cand = np.flatnonzero(sky)
    ge, _ = orc.gres(x, cand, 25)
    pick = cand[::7]
    assert (orc.gres_rows(x, cand, pick, 25) == ge[::7]).all()
    rows = np.arange(0, 3000, 13)
    assert (orc.skyline_rows(x, rows) == sky[rows]).all()


# ----------------------------------------------------------------------------- partitioning

def test_closest_m():
    import oracle
    assert oracle.grid_p(64, 4) == (3, 81)
    assert oracle.angular_p(64, 4) == (4, 64)
    assert oracle.grid_p(16, 2) == (4, 16)
    assert oracle.grid_p(16, 3) == (2, 8)  # |8-16| = 8 < |27-16| = 11


def test_grid_cells_exact_bounds(orc):
    x = G.uni(20000, 3, 1)
    m = 3
    part = orc.grid_part(x, m)
    for i in range(0, 20000, 17):
        c = part[i]
        for k in range(3):
            ck = c % m
            c //= m
            v = Fraction(float(x[i, k])) * m
            # the FP32 product decides; away from integers it agrees with the exact floor
            if abs(v - round(v)) > Fraction(1, 1 << 20):
                assert ck == math.floor(v)


def test_angular_special_directions(orc):
    m = 3
    # axis directions and the diagonal of the plane: phi = 0 -> bucket 0; phi = pi/2 -> m-1;
    # phi = pi/4 -> floor(m/2)
    x = np.array([[0.5, 0.0, 0.0], [0.0, 0.5, 0.0], [0.0, 0.0, 0.5], [0.3, 0.3, 0.0],
                  [0.0, 0.3, 0.3], [0.0, 0.0, 0.0]], dtype=np.float32)
    part, near = orc.angular_part(x, m)
    # (b1, b2) -> b1 + m*b2
    assert part.tolist() == [0 + m * 0, (m - 1) + m * 0, (m - 1) + m * (m - 1), 1 + 0,
                             (m - 1) + m * 1, 0]
    assert not near.any()


def test_angular_matches_arccos(orc):
    for d, m in ((2, 16), (3, 4), (4, 4), (6, 2)):
        x = G.uni(5000, d, d) * np.float32(0.999)
        part, near = orc.angular_part(x, m)
        xs = x.astype(np.float64)
        for i in range(0, 5000, 7):
            if near[i]:
                continue
            want, w = 0, 1
            for a in range(d - 1):
                nrm = math.sqrt(sum(xs[i, j] ** 2 for j in range(a, d)))
                phi = math.acos(xs[i, a] / nrm) if nrm > 0 else 0.0
                b = min(m - 1, int(math.floor(2 * phi * m / math.pi)))
                want += b * w
                w *= m
            assert part[i] == want


@pytest.mark.parametrize("kind", ["uni", "ties"])
def test_sliced_sizes_and_order(orc, kind):
    x = _rows(kind, 1003, 3, 4)
    p = 16
    part = orc.sliced_part(x, p, dim=1)
    sizes = np.bincount(part, minlength=p)
    assert sizes.sum() == 1003 and set(sizes.tolist()) <= {1003 // p, 1003 // p + 1}
    col = x[:, 1]
    for j in range(p - 1):
        a, b = np.flatnonzero(part == j), np.flatnonzero(part == j + 1)
        assert col[a].max() <= col[b].min()
        # equal values straddling a boundary are split by row index
        tie = col[a].max() == col[b].min()
        if tie:
            v = col[a].max()
            assert a[col[a] == v].max() < b[col[b] == v].min()


@pytest.mark.parametrize("kind", ["uni", "ant", "ties"])
@pytest.mark.parametrize("d", [2, 3, 4])
def test_two_phase_equals_skyline(orc, kind, d):
    x = _rows(kind, 2500, d, 21 + d)
    want = orc.skyline(x)
    m, p = orc.grid_p(16, d)
    schemes = {"grid": orc.grid_part(x, m), "sliced": orc.sliced_part(x, 16, 0)}
    if d >= 2:
        schemes["angular"] = orc.angular_part(x, orc.angular_p(16, d)[0])[0]
    for name, part in schemes.items():
        skip = None
        if name == "grid":
            ne = np.zeros(p, dtype=np.uint8)
            ne[np.unique(part)] = 1
            skip = orc.grid_pruned(ne, m, d).astype(np.uint8)
            # I6: no skyline row lies in a pruned cell
            assert not skip[part[want]].any()
        local = orc.local_skylines(x, part, skip)
        assert (local | ~want).all()  # every skyline row survives its partition
        union = np.flatnonzero(local)
        final = np.zeros(len(x), dtype=bool)
        final[union] = orc.skyline(x[union])
        assert (final == want).all(), name


def _partition_ids(orc, x, scheme, target):
    """(ids, pruned-cell flags or None) of the oracle's Grid / Angular / Sliced partitioning."""
    d = x.shape[1]
    if scheme == "grid":
        m, p = orc.grid_p(target, d)
        part = orc.grid_part(x, m)
        ne = np.zeros(p, np.uint8)
        ne[np.unique(part)] = 1
        return part, orc.grid_pruned(ne, m, d).astype(np.uint8)
    if scheme == "angular":
        return orc.angular_part(x, orc.angular_p(target, d)[0])[0], None
    return orc.sliced_part(x, target, d - 1), None


@pytest.mark.parametrize("scheme,target", [("grid", 9), ("grid", 16), ("angular", 4),
                                           ("angular", 9), ("sliced", 5), ("sliced", 12)])
@pytest.mark.parametrize("kind,d", [("ties", 2), ("ties", 3), ("dyadic", 2), ("dyadic", 3)])
def test_local_skylines_per_partition_brute(orc, scheme, target, kind, d):
    """Sec. 3, phase 1: a local skyline is Def. 1 over the rows of ONE partition. Each partition
    is checked on its own against the Python brute force of Def. 1 over just its rows; rows of
    pruned Grid cells (Def. 3) are in no local skyline. Duplicated rows are added. At least one
    partition must hold a row that its partition keeps although another partition dominates it
    (so reading the local skyline as Sky(r) restricted to the partition fails here)."""
    x = _rows(kind, 240, d, 17 * d + target)
    x = np.concatenate([x, x[::7]])  # exact duplicates, in other positions
    part, skip = _partition_ids(orc, x, scheme, target)
    local = orc.local_skylines(x, part, skip)
    glob = orc.skyline(x)
    if scheme == "grid":
        assert skip[np.unique(part)].any(), "the data must put rows in a pruned cell"
    differs = 0
    for j in np.unique(part):
        rows = np.flatnonzero(part == j)
        if skip is not None and skip[j]:
            assert not local[rows].any(), j
            continue
        want = brute.skyline_rows(x[rows])
        assert np.array_equal(local[rows], want), (j, rows[local[rows] != want][:5])
        differs += int((want & ~glob[rows]).any())
    assert differs >= 1


def test_local_skylines_ignore_other_partitions(orc):
    """Hand-made: row 1 dominates row 0, but they lie in different partitions, so both are in
    their local skylines; row 2 (same partition as row 0, dominated by it) is not."""
    x = np.array([[0.5, 0.5], [0.25, 0.25], [0.75, 0.75]], np.float32)
    part = np.array([0, 1, 0], np.int32)
    assert orc.local_skylines(x, part).tolist() == [True, True, False]
    assert orc.local_skylines(x, part, np.array([0, 1], np.uint8)).tolist() == [True, False, False]


def test_count_invalid(orc):
    x = np.array([[0.0, 0.5], [-0.0, 0.999], [1.0, 0.2], [np.nan, 0.1], [0.3, -1e-30],
                  [np.inf, 0.0]], dtype=np.float32)
    assert orc.count_invalid(x) == 4


# ----------------------------------------------------------------------------- ell and g_bar

def test_ell_worked_lattice_example(orc):
    # attribute 0 holds 1/4, 1/2, 3/4 (gaps 1/4); attribute 1 holds 1/8, 1/8, 5/16 (gaps 0 and
    # 3/16): ell = 3/16 comes from the second attribute and g_bar = floor(16/3) = 5
    x = np.array([[0.25, 0.125], [0.5, 0.125], [0.75, 0.3125]], np.float32)
    assert brute.ell_exact(x) == Fraction(3, 16)
    assert orc.ell(x) == 0.1875 and orc.ell(x, sorted_=True) == 0.1875
    assert orc.gbar(x) == (0.1875, 5)


def test_ell_degenerate(orc):
    # no attribute holds two different values (-0 and +0 are one value): no ell, g_bar = 1
    for x in (np.zeros((0, 3), np.float32), np.full((1, 2), 0.3, np.float32),
              np.full((5, 2), 0.3, np.float32), np.array([[0.0], [-0.0]], np.float32)):
        assert orc.ell(x) == math.inf and orc.ell(x, sorted_=True) == math.inf
        assert orc.gbar(x)[1] == 1
        assert brute.ell_exact(x) is None and brute.gbar_exact(x) == 1
    # a constant attribute beside one with gaps 1/8 and 1/2
    x = np.array([[0.5, 0.25], [0.5, 0.375], [0.5, 0.875]], np.float32)
    assert orc.gbar(x) == (0.125, 8)
    # the smallest step above 0 is a subnormal: ell is that value, g_bar far beyond 2^62
    tiny = np.float32(1e-40)
    x = np.array([[0.0], [tiny], [0.5]], np.float32)
    assert orc.ell(x) == float(tiny) and orc.ell(x, sorted_=True) == float(tiny)
    assert orc.gbar(x)[1] > 2 ** 62


@pytest.mark.parametrize("kind", ["uni", "ties", "dyadic", "ant"])
def test_ell_vs_exact_pairs(orc, kind):
    for seed in range(6):
        d = 1 + seed % 4
        x = _rows(kind, 24, d, seed)
        x = np.concatenate([x, x[:3]])       # whole-row duplicates
        x[1, 0] = -0.0 if seed % 2 else x[1, 0]
        e = brute.ell_exact(x)
        assert e is not None
        assert orc.ell(x) == float(e)        # every difference here is exact in FP64
        assert orc.ell(x, sorted_=True) == orc.ell(x)
        assert orc.gbar(x)[1] == brute.gbar_exact(x)


def test_no_exit_beyond_gbar(orc):
    # Sec. 3.2: at g > g_bar every difference within an attribute spans more than one grid
    # interval, so projections keep every order and no new dominance appears. On dyadic data
    # (exact in FP32) the exact brute force over levels up to 3 g_bar + 2 finds no exit above
    # g_bar, and the oracle's search up to g_bar gives the same answer.
    for seed in range(5):
        x = G.dyadic(10, 2 + seed % 2, seed, bits=4)
        gb = brute.gbar_exact(x)
        assert orc.gbar(x)[1] == gb and 2 <= gb <= 16
        far = brute.gres_g_exit(x, 3 * gb + 2, "exact")
        assert far == brute.gres_g_exit(x, gb, "exact")
        cand = np.flatnonzero(orc.skyline(x))
        ge, _ = orc.gres(x, cand, gb)
        assert [far[int(c)] for c in cand] == ge.tolist()


# ------------------------------------------------------------------ Representative Filtering

def _fp32_scores(x):
    f = np.zeros(len(x), np.float32)
    for k in range(x.shape[1]):
        f = (f + x[:, k]).astype(np.float32)  # one IEEE FP32 addition per attribute, in order
    return f


@pytest.mark.parametrize("kind", ["uni", "ant", "ties"])
def test_representatives_selection(orc, kind):
    # Sec. 3.1: the k tuples with the smallest monotone score (FP32 attribute sum), equal scores
    # in row order; the kept ones are those no other representative dominates (Def. 1)
    for seed, k in ((0, 1), (1, 10), (2, 60)):
        x = _rows(kind, 400, 3 + seed % 3, seed)
        rows, kept = orc.representatives(x, k)
        f = _fp32_scores(x)
        assert rows.tolist() == np.lexsort((np.arange(len(x)), f))[:k].tolist()
        pts = [tuple(float(v) for v in x[r]) for r in rows]
        want = [not any(brute.dominates(pts[q], pts[j]) for q in range(k) if q != j)
                for j in range(k)]
        assert kept.tolist() == want
        assert kept[0]  # the smallest score is never dominated (f is monotone)


def test_dominated_by_brute(orc):
    for seed in range(3):
        x = _rows("ties", 60, 3, seed)
        by = np.array([0, 7, 19, 33])
        got = orc.dominated_by(x, by)
        pts = [tuple(float(v) for v in r) for r in x]
        want = [any(brute.dominates(pts[b], pts[i]) for b in by) for i in range(len(x))]
        assert got.tolist() == want


@pytest.mark.parametrize("kind", ["uni", "ant", "ties"])
def test_representatives_keep_the_skyline(orc, kind):
    # representatives are tuples of r, so removing what they dominate never touches Sky(r):
    # the final skyline of the reduced union is Sky(r), and each local skyline only shrinks
    x = _rows(kind, 3000, 4, 5)
    sky = orc.skyline(x)
    part = orc.sliced_part(x, 8, 0)
    plain = orc.local_skylines(x, part)
    for k in (1, 10, 100):
        loc = orc.local_skylines_reps(x, part, None, k)
        assert not (loc & ~plain).any()
        rows, kept = orc.representatives(x, k)
        assert (plain & ~loc == plain & orc.dominated_by(x, rows[kept])).all()
        u = np.flatnonzero(loc)
        final = np.zeros(len(x), bool)
        final[u[orc.skyline(x[u])]] = True
        assert (final == sky).all()
