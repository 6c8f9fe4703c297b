"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle checks.

This module only draws numbers: it holds none of the method's arithmetic (no dominance, no
projection, no partitioning). Every generator returns a C-contiguous ``float32`` array of
shape ``[N, d]`` (row-major, one tuple per row) with every value in ``[0, 1)``, the domain the
paper assumes for its synthetic data (Sec. 4) and for Grid partition numbering (Sec. 3.1).

Generators (numpy PCG64 via ``default_rng``):

* ``uni``     -- i.i.d. uniform, values ``k * 2**-24`` (stands in for the paper's UNI data).
* ``ant``     -- anticorrelated: points scattered around the hyperplane ``sum(x) = d * c`` with
                 ``c ~ 0.5 + N(0, sigma)`` per row and an in-plane spread from a uniform cube,
                 clipped into ``[0, 1)`` (stands in for the paper's ANT data, whose generator is
                 not available here).
* ``ties``    -- small-integer attributes ``v in 0..99`` with a Zipf(s) rank law, a Gaussian
                 copula with equicorrelation ``rho`` and a seeded per-attribute permutation from
                 rank to value, stored as ``float32(v / 100)``; heavy ties and duplicates (stands
                 in for the paper's real datasets, which are not available here).
* ``dyadic``  -- values ``k * 2**-bits``; with ``bits <= 12`` and ``g <= 4096`` every product
                 ``x * g`` is exact in FP32, so integer-only code can check quantisation.
* ``batch_specs`` / ``batch_dataset`` -- the heterogeneous many-dataset workload: log-normal
                 sizes, mixed dimensionality, alternating uniform / anticorrelated.
"""
from __future__ import annotations

import math

import numpy as np

_ONE_MINUS = np.float32(np.nextafter(np.float32(1.0), np.float32(0.0)))  # largest float32 < 1


def uni(n: int, d: int, seed: int) -> np.ndarray:
    """i.i.d. uniform FP32 in [0, 1)."""
    rng = np.random.default_rng(seed)
    return np.ascontiguousarray(rng.random((n, d), dtype=np.float32))


def ant(n: int, d: int, seed: int, sigma: float = 0.05) -> np.ndarray:
    """Anticorrelated FP32 data around the plane sum(x) = d * c, c ~ 0.5 + N(0, sigma)."""
    rng = np.random.default_rng(seed)
    u = rng.random((n, d))
    c = 0.5 + rng.normal(0.0, sigma, (n, 1))
    x = u - u.mean(axis=1, keepdims=True) + c
    np.clip(x, 0.0, float(_ONE_MINUS), out=x)
    return np.ascontiguousarray(x.astype(np.float32))


def _zipf_cdf(levels: int, s: float) -> np.ndarray:
    w = 1.0 / np.arange(1, levels + 1, dtype=np.float64) ** s
    c = np.cumsum(w)
    return c / c[-1]


def ties(n: int, d: int, seed: int, levels: int = 100, zipf_s: float = 1.1,
         rho: float = 0.3, chunk: int = 1 << 20) -> np.ndarray:
    """Tie-heavy data: integers 0..levels-1 (Zipf ranks, correlated by a Gaussian copula),
    mapped through a seeded per-attribute permutation and stored as float32(v / levels)."""
    from scipy.special import ndtr  # standard normal CDF

    rng = np.random.default_rng(seed)
    perms = np.stack([rng.permutation(levels) for _ in range(d)])  # [d, levels]
    cdf = _zipf_cdf(levels, zipf_s)
    out = np.empty((n, d), dtype=np.float32)
    a, b = math.sqrt(rho), math.sqrt(1.0 - rho)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        z0 = rng.standard_normal((hi - lo, 1))
        z = a * z0 + b * rng.standard_normal((hi - lo, d))
        u = ndtr(z)
        rank = np.minimum(np.searchsorted(cdf, u, side="right"), levels - 1)
        v = perms[np.arange(d)[None, :], rank]  # v[r, k] = perms[k, rank[r, k]]
        out[lo:hi] = (v.astype(np.float64) / levels).astype(np.float32)
    return out


# The served relations: tie-heavy data of N in {20k, 130k, 2M} rows x d in {5, 6, 7}
# attributes, seeds 0..8 in that order (stand-ins for the paper's real datasets of about 130k x 6
# and 2M x 7 rows, which are not available).
SERVE_SPECS = [(n, d, i) for i, (n, d) in
               enumerate((n, d) for n in (20_000, 130_000, 2_000_000) for d in (5, 6, 7))]


def serve_relations():
    """The nine served relations, as row-major float32 arrays, in SERVE_SPECS order."""
    return [ties(n, d, seed) for n, d, seed in SERVE_SPECS]


def dyadic(n: int, d: int, seed: int, bits: int = 12) -> np.ndarray:
    """Values k * 2**-bits, k uniform in [0, 2**bits)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(0, 1 << bits, size=(n, d))
    return np.ascontiguousarray((k.astype(np.float64) / float(1 << bits)).astype(np.float32))


def batch_specs(count: int = 4096, seed: int = 0, median: int = 20000, log_sd: float = 1.0,
                n_min: int = 1000, n_max: int = 200000, d_min: int = 2, d_max: int = 8):
    """Sizes, dimensionalities, kinds and seeds of the many-dataset workload.

    Returns a list of ``(n, d, kind, seed)`` with ``kind`` in {"uni", "ant"}: uniform for even
    positions, anticorrelated for odd ones; ``n`` log-normal around ``median`` clipped to
    ``[n_min, n_max]``; ``d`` uniform in ``d_min..d_max``.
    """
    rng = np.random.default_rng(seed)
    ns = np.clip(np.rint(np.exp(rng.normal(math.log(median), log_sd, count))), n_min, n_max)
    ds = rng.integers(d_min, d_max + 1, count)
    return [(int(ns[i]), int(ds[i]), "uni" if i % 2 == 0 else "ant", seed * 1_000_000 + i)
            for i in range(count)]


def batch_dataset(spec) -> np.ndarray:
    n, d, kind, s = spec
    return uni(n, d, s) if kind == "uni" else ant(n, d, s)


GENERATORS = {"uni": uni, "ant": ant, "ties": ties, "dyadic": dyadic}


def make(kind: str, n: int, d: int, seed: int) -> np.ndarray:
    return GENERATORS[kind](n, d, seed)
