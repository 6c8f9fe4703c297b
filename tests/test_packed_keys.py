"""The packed-key dominance test of the gres search, as arithmetic (no GPU): d keys in fields of
w bits with the top bit of each field clear, T the target's keys, S a candidate's, G the top bits.
For keys of at most 2^(w-1) - 2 in T and at most 2^(w-1) - 1 in S (the clamp value of padding),
((T | G) - S) & G == G exactly when every candidate key is <= the target's, and S != T then
decides strictness (Def. 2's dominance between projections, on integer keys). Checked
exhaustively for small widths and against the field-wise definition on random keys for the
widths the library uses."""
from __future__ import annotations

import itertools

import numpy as np


def _pack(keys, w):
    v = 0
    for k, x in enumerate(keys):
        v |= int(x) << (k * w)
    return v


def _guard(d, w):
    return sum(1 << (k * w + w - 1) for k in range(d))


def _packed_le(t, s, d, w):
    g = _guard(d, w)
    return (((_pack(t, w) | g) - _pack(s, w)) & g) == g


def test_exhaustive_small_fields():
    for d, w in ((1, 3), (2, 3), (3, 3), (2, 4)):
        tmax, smax = (1 << (w - 1)) - 2, (1 << (w - 1)) - 1
        for t in itertools.product(range(tmax + 1), repeat=d):
            for s in itertools.product(range(smax + 1), repeat=d):
                want = all(a <= b for a, b in zip(s, t))
                assert _packed_le(t, s, d, w) == want, (d, w, t, s)


def test_random_library_widths():
    rng = np.random.default_rng(5)
    # (d, g_max) pairs the key table takes: w = bit length of g_max + 1, plus one; d * w <= 64
    for d, g_max in ((2, 25), (6, 25), (8, 25), (10, 25), (6, 64), (9, 62), (16, 2)):
        b = int(g_max + 1).bit_length()
        w = b + 1
        assert d * w <= 64
        kmax = (1 << b) - 1
        assert g_max <= kmax - 1  # target keys stay below the clamp value
        for _ in range(3000):
            t = rng.integers(0, g_max + 1, d)
            s = np.minimum(t + rng.integers(-2, 3, d), kmax)
            s = np.maximum(s, 0)
            if rng.random() < 0.1:
                s[:] = kmax  # padding
            want_le = bool((s <= t).all())
            assert _packed_le(t, s, d, w) == want_le
            dominated = want_le and _pack(s, w) != _pack(t, w)
            assert dominated == (want_le and bool((s < t).any()))
