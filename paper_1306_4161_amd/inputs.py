"""Seeded synthetic operands shared by the GPU path, its tests and the oracle.

This module holds no arithmetic of the method: it only draws numbers and
picks indices.  The paper names no data set or value distribution (it gives
matrix sizes only), so square FP64 matrices with i.i.d. entries stand in for
its workloads:

  uniform(m, n, seed)           U[-1, 1]
  exponent_spread(m, n, seed, sigma)
                                u * 2^e, u ~ U[-1, 1], e = rint(N(0, sigma^2))
                                (round half to even), a wide exponent range
  integer_valued(m, n, seed, r) integers in [-2^r, 2^r]
  sample_entries(...)           (row, col) pairs: uniform plus tile edges
  rademacher(n, seed)           x in {-1, +1}^n for Freivalds' check

Seeds used throughout: A = 2013, B = 4161, sampling = 1306.
"""
from __future__ import annotations

import numpy as np

SEED_A = 2013
SEED_B = 4161
SEED_SAMPLE = 1306


def uniform(m: int, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(m, n))


def exponent_spread(m: int, n: int, seed: int, sigma: float = 2.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    u = rng.uniform(-1.0, 1.0, size=(m, n))
    e = np.rint(rng.normal(0.0, sigma, size=(m, n))).astype(np.int64)
    return np.ldexp(u, e)


def integer_valued(m: int, n: int, seed: int, r: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    lim = 1 << r
    return rng.integers(-lim, lim + 1, size=(m, n)).astype(np.float64)


def rademacher(n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.integers(0, 2, size=n).astype(np.float64) * 2.0 - 1.0


def sample_entries(m: int, n: int, count_uniform: int, seed: int,
                   row_edges=(), col_edges=(), per_edge: int = 8):
    """Uniform (row, col) samples plus samples on the first/last row and
    column of every tile (row_edges / col_edges are tile start offsets)."""
    rng = np.random.default_rng(seed)
    r = list(rng.integers(0, m, size=count_uniform))
    c = list(rng.integers(0, n, size=count_uniform))
    row_edges = sorted(set(int(x) for x in row_edges) | {0, m})
    col_edges = sorted(set(int(x) for x in col_edges) | {0, n})
    for a, b in zip(row_edges[:-1], row_edges[1:]):
        if b <= a:
            continue
        for rr in (a, b - 1):
            r.extend([rr] * per_edge)
            c.extend(rng.integers(0, n, size=per_edge))
    for a, b in zip(col_edges[:-1], col_edges[1:]):
        if b <= a:
            continue
        for cc in (a, b - 1):
            c.extend([cc] * per_edge)
            r.extend(rng.integers(0, m, size=per_edge))
    return np.asarray(r, dtype=np.int64), np.asarray(c, dtype=np.int64)
