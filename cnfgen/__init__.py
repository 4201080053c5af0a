"""Seeded synthetic CNF workloads and relaxed-assignment inputs.

This module only draws random data: it holds none of the solver's arithmetic
(no scores, masks, losses, gradients or steps).  Both the CPU oracle and the
HIP library consume what it produces, so it lives apart from either.

Every CNF is returned DIMACS-style as a flat ``int32`` array: literals are
signed 1-based variable indices and every clause ends with a ``0``.

Workload recipes (the paper's own PySAT instances are not available, so these
stand in for them at the same or larger scale; see the paper's Table 2 for the
sizes it used):

* :func:`uniform_kcnf`  -- k distinct variables per clause drawn uniformly
  without replacement, each sign Bernoulli(0.5).
* :func:`structured_cnf` -- clause length ``min(2 + G, kmax)`` with ``G``
  Geometric(p) counting failures, variables from a finite Zipf(s) over ranks
  ``1..n`` mapped through a seeded permutation, distinct within a clause
  (a clause with a repeat is redrawn whole), sign Bernoulli(0.5).
* :func:`mixed_kcnf`    -- clause length uniform over a set (default 2/3/4),
  otherwise as :func:`uniform_kcnf`.
* :func:`serving_stream` -- request sizes and Poisson arrival times of the
  serving workload; each request's CNF is drawn on demand.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "uniform_kcnf",
    "structured_cnf",
    "mixed_kcnf",
    "planted_kcnf",
    "random_x",
    "to_clauses",
    "from_clauses",
    "ServingRequest",
    "serving_stream",
    "CONFIGS",
]


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def _distinct_rows(rng: np.random.Generator, rows: int, k: int, n: int) -> np.ndarray:
    """``rows`` x ``k`` matrix of variables in [0, n), distinct within a row."""
    if k > n:
        raise ValueError(f"cannot draw {k} distinct variables out of {n}")
    out = rng.integers(0, n, size=(rows, k), dtype=np.int64)
    while True:
        s = np.sort(out, axis=1)
        bad = np.nonzero((s[:, 1:] == s[:, :-1]).any(axis=1))[0] if k > 1 else np.zeros(0, np.int64)
        if bad.size == 0:
            return out
        out[bad] = rng.integers(0, n, size=(bad.size, k), dtype=np.int64)


def _pack(var_rows: np.ndarray, neg: np.ndarray, lengths: np.ndarray | None = None) -> np.ndarray:
    """Pack a (rows x kmax) variable matrix (0-based) into a DIMACS flat array."""
    rows, kmax = var_rows.shape
    lits = (var_rows + 1) * np.where(neg, -1, 1)
    if lengths is None:
        out = np.zeros((rows, kmax + 1), dtype=np.int32)
        out[:, :kmax] = lits
        return out.reshape(-1)
    lengths = np.asarray(lengths, dtype=np.int64)
    total = int(lengths.sum()) + rows
    out = np.zeros(total, dtype=np.int32)
    ends = np.cumsum(lengths + 1)
    starts = ends - lengths - 1
    col = np.arange(kmax)[None, :]
    keep = col < lengths[:, None]
    pos = (starts[:, None] + col)[keep]
    out[pos] = lits[keep]
    return out


def uniform_kcnf(n: int, m: int, k: int, seed: int) -> np.ndarray:
    """Uniform random k-CNF: m clauses of k distinct variables, fair signs."""
    rng = _rng(seed)
    if m == 0:
        return np.zeros(0, dtype=np.int32)
    v = _distinct_rows(rng, m, k, n)
    neg = rng.random((m, k)) < 0.5
    return _pack(v, neg)


def mixed_kcnf(n: int, m: int, seed: int, ks=(2, 3, 4)) -> np.ndarray:
    """Clause length uniform over ``ks``; variables distinct within a clause."""
    rng = _rng(seed)
    ks = np.asarray(ks, dtype=np.int64)
    lengths = ks[rng.integers(0, len(ks), size=m)]
    kmax = int(ks.max())
    v = _distinct_rows(rng, m, kmax, n)
    neg = rng.random((m, kmax)) < 0.5
    return _pack(v, neg, lengths)


def planted_kcnf(n: int, m: int, k: int, seed: int):
    """Random k-CNF satisfied by a hidden assignment (returned alongside).

    Each clause is drawn as in :func:`uniform_kcnf` and its signs are redrawn
    until the planted assignment makes at least one literal true.
    """
    rng = _rng(seed)
    plant = (rng.random(n) < 0.5).astype(np.uint8)
    v = _distinct_rows(rng, m, k, n)
    neg = rng.random((m, k)) < 0.5
    while True:
        truth = np.where(neg, plant[v] == 0, plant[v] == 1)
        bad = np.nonzero(~truth.any(axis=1))[0]
        if bad.size == 0:
            break
        neg[bad] = rng.random((bad.size, k)) < 0.5
    return _pack(v, neg), plant


def _finite_zipf_cdf(n: int, s: float) -> np.ndarray:
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def structured_cnf(n: int, m: int, seed: int, p_geom: float = 0.4, kmax: int = 12,
                   zipf_s: float = 1.1) -> np.ndarray:
    """Skewed-degree instance: geometric clause lengths, Zipf variable occurrence."""
    rng = _rng(seed)
    lengths = np.minimum(2 + (rng.geometric(p_geom, size=m) - 1), kmax).astype(np.int64)
    lengths = np.minimum(lengths, n)
    cdf = _finite_zipf_cdf(n, zipf_s)
    perm = rng.permutation(n)
    width = int(lengths.max()) if m else 0
    col = np.arange(width)[None, :]
    used = col < lengths[:, None]

    def draw(rows: int) -> np.ndarray:
        ranks = np.searchsorted(cdf, rng.random((rows, width)), side="right")
        return perm[np.minimum(ranks, n - 1)]

    v = draw(m)
    todo = np.arange(m)
    while todo.size:
        sub = np.where(used[todo], v[todo], -1 - np.arange(width)[None, :])
        s = np.sort(sub, axis=1)
        bad = todo[(s[:, 1:] == s[:, :-1]).any(axis=1)]
        if bad.size == 0:
            break
        v[bad] = draw(bad.size)
        todo = bad
    neg = rng.random((m, width)) < 0.5
    return _pack(v, neg, lengths)


def random_x(n: int, R: int, seed: int, lo: float = -1.0, hi: float = 1.0,
             specials: bool = False, nan: int = 0) -> np.ndarray:
    """Relaxed assignment ``[n][R]`` float32, U(lo, hi).

    With ``specials`` a few entries are replaced by rounding edge cases:
    +0.0, -0.0, the smallest subnormal of either sign, large magnitudes and
    +-infinity.  ``nan`` entries (after those) are set to NaN.
    """
    rng = _rng(seed)
    x = rng.uniform(lo, hi, size=(n, R)).astype(np.float32)
    if specials and x.size:
        vals = np.array([0.0, -0.0, 1e-45, -1e-45, 1e-30, -1e-30, 12.0, -12.0, 30.0, -30.0,
                         np.inf, -np.inf], dtype=np.float32)
        idx = rng.choice(x.size, size=min(x.size, 2 * len(vals)), replace=False)
        x.reshape(-1)[idx] = np.resize(vals, idx.size)
    if nan and x.size:
        idx = rng.choice(x.size, size=min(x.size, int(nan)), replace=False)
        x.reshape(-1)[idx] = np.float32(np.nan)
    return x


def to_clauses(lits: np.ndarray) -> list[list[int]]:
    """Split a DIMACS flat array into a list of clauses (no 0 terminators)."""
    out, cur = [], []
    for v in np.asarray(lits).tolist():
        if v == 0:
            out.append(cur)
            cur = []
        else:
            cur.append(int(v))
    if cur:
        raise ValueError("last clause is not 0-terminated")
    return out


def from_clauses(clauses) -> np.ndarray:
    flat = []
    for c in clauses:
        flat.extend(int(v) for v in c)
        flat.append(0)
    return np.asarray(flat, dtype=np.int32)


@dataclass
class ServingRequest:
    index: int
    arrival_s: float
    n: int
    m: int
    k: int
    seed: int

    def cnf(self) -> np.ndarray:
        return uniform_kcnf(self.n, self.m, self.k, self.seed)


def serving_stream(n_req: int = 512, seed: int = 5, rate: float = 200.0,
                   n_lo: int = 100, n_hi: int = 200000) -> list[ServingRequest]:
    """Requests: k ~ U{3,4,5}; n log-uniform in [n_lo, n_hi];
    m = round(n * U(3.5, 5) * 2^k / 8); Poisson arrivals at ``rate`` per second."""
    rng = _rng(seed)
    reqs = []
    t = 0.0
    for i in range(n_req):
        t += rng.exponential(1.0 / rate)
        k = int(rng.integers(3, 6))
        n = int(math.floor(math.exp(rng.uniform(math.log(n_lo), math.log(n_hi)))))
        ratio = rng.uniform(3.5, 5.0) * (2 ** k) / 8.0
        m = int(round(n * ratio))
        reqs.append(ServingRequest(i, t, n, m, k, int(seed) * 1_000_003 + i))
    return reqs


# The five workload configurations (sizes and schedules).
CONFIGS = {
    "cfg1": dict(kind="uniform", n=50, m=215, k=3, R=1, steps=1000, eval_every=1),
    "cfg2": dict(kind="uniform", n=20000, m=86000, k=3, R=64, steps=2000, eval_every=50),
    "cfg3": dict(kind="structured", n=500000, m=2500000, R=1, steps=200, eval_every=50),
    "cfg4": dict(kind="mixed", n=1000, m=4200, R=16, steps=1000, eval_every=1),
    "cfg5": dict(kind="serving", n_req=512, rate=200.0, steps=1000, eval_every=50),
}
