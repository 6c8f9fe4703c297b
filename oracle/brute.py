"""Literal brute force of Def. 1 and Def. 2 for tiny inputs -- TEST INFRASTRUCTURE ONLY.

Relations are treated as *sets* (Sec. 2): ``gproj(r, g)`` is built as a set of projected
tuples, its skyline is taken by Def. 1 over that set, and the grid resistance of a skyline
tuple t is ``min { 1/g : gproj(t, g) not in Sky(gproj(r, g)) }`` over g = 1..g_max (Def. 2,
restricted to the searched range), or 1 if t never leaves the skyline. The whole relation r
is used (not only Sky(r)), so agreement with the oracle also checks that gres is stable.

Two arithmetic modes for the projection ``floor(t[i] * g) / g``:
* ``"fp32"``  -- the product rounded once to FP32 (numpy float32 multiply), then floored;
* ``"exact"`` -- exact rationals (``fractions.Fraction``), for inputs whose FP32 product is
                 exact anyway (dyadic data) so that both modes must agree.
Projections are compared through their numerators floor(t[i]*g) (division by the same g > 0
keeps every order relation).
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def dominates(s, t) -> bool:
    """Def. 1: s <= t everywhere and s < t somewhere."""
    return all(a <= b for a, b in zip(s, t)) and any(a < b for a, b in zip(s, t))


def skyline_set(points):
    """Def. 1 over a set of tuples: the tuples no other tuple dominates."""
    pts = list(points)
    return {t for t in pts if not any(dominates(s, t) for s in pts)}


def skyline_rows(x) -> np.ndarray:
    """Membership of every row of x (multiset of rows) in Sky(r) by Def. 1."""
    rows = [tuple(float(v) for v in r) for r in np.asarray(x, dtype=np.float32)]
    return np.array([not any(dominates(s, t) for s in rows) for t in rows], dtype=bool)


def _project(row, g: int, mode: str):
    if mode == "fp32":
        return tuple(int(np.floor(np.float32(v) * np.float32(g))) for v in row)
    if mode == "exact":
        return tuple((Fraction(float(v)) * g).__floor__() for v in row)
    raise ValueError(mode)


def gres_g_exit(x, g_max: int, mode: str = "fp32") -> dict:
    """Def. 2 for every skyline row: {row index: g_exit}, with gres = 1/g_exit and g_exit = 1
    meaning the tuple never exits the skyline for g in 1..g_max."""
    x = np.asarray(x, dtype=np.float32)
    member = skyline_rows(x)
    out = {}
    proj_sky = {}
    for g in range(1, g_max + 1):
        proj = {i: _project(x[i], g, mode) for i in range(len(x))}
        proj_sky[g] = skyline_set(set(proj.values()))
        for i in np.flatnonzero(member):
            i = int(i)
            if proj[i] not in proj_sky[g]:
                out[i] = max(out.get(i, 1), g)  # min 1/g over exit levels = 1/(max g)
    return {int(i): out.get(int(i), 1) for i in np.flatnonzero(member)}


def ell_exact(x):
    """Sec. 3.2's ell in exact rationals, over every pair of rows and every attribute: the
    smallest non-zero |a - b| between two values of one attribute, or None if there is none."""
    x = np.asarray(x, dtype=np.float32)
    best = None
    n = len(x)
    for k in range(x.shape[1] if x.ndim == 2 else 0):
        col = [Fraction(float(v)) for v in x[:, k]]
        for i in range(n):
            for j in range(i + 1, n):
                e = abs(col[i] - col[j])
                if e != 0 and (best is None or e < best):
                    best = e
    return best


def gbar_exact(x) -> int:
    """g_bar = floor(1/ell) in exact rationals (1 when ell does not exist)."""
    e = ell_exact(x)
    return 1 if e is None else (1 / e).__floor__()
