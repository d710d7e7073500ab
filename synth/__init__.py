"""Seeded synthetic inputs for the sparse Tucker workloads.

This module is shared by the FP64 oracle tests and by the GPU path. It only
draws random numbers and lays them out: observed index sets (COO, 0-based,
structure-of-arrays ``idx[N][nnz]``), observed values, and initial models. It
holds none of the row-wise ALS arithmetic (no delta vectors, Gram matrices,
solves, errors or QR).

The observed values of the planted workloads are "planted Tucker + Gaussian
noise": a random core and random factors are drawn, the model they define is
evaluated at the observed cells and noise is added. That evaluation is part of
the input recipe (a dense chunked product in numpy), not part of either side
under test; both sides receive the same float32 values.

Recipes (the workloads of the paper's synthetic experiments, Sec. 4.2, and the
shapes of the rating tensors of Table 3):

* ``c1``: 100^3, 10^4 distinct uniform cells, J=(5,5,5), planted core and
  factors N(0,1), noise variance 0.01, seed 0.
* ``c2``: order 4, 10^5 per mode, 10^7 distinct cells, per-mode truncated
  Zipf(1.1) index skew through a seeded permutation, J=10, planted rank 10,
  noise variance 0.1, seed 1.
* ``c3``: 480000 x 18000 x 2000 rating-shaped tensor, 10^8 distinct cells,
  users Zipf(0.6), items Zipf(0.9), days uniform, ratings 1..5 from a planted
  rank-8 score cut at fixed quantiles (5/10/25/35/25 %), J=16, seed 2.
* ``c4``: order 5, 10^4 per mode, 5*10^7 distinct cells, per-mode row weights
  lognormal(3, 2) scaled so that the clipped weights sum to nnz (clip [1,1e5]),
  planted rank 4, noise variance 0.1, J=8, seed 3.
* ``small``: any shape, uniform distinct cells, used by the parity tests.

Initial models follow Alg. 2's initialisation: core and factors i.i.d.
uniform on [0, 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "uniform_distinct", "zipf_distinct", "weighted_distinct",
    "planted_model", "planted_values", "init_model", "make", "CONFIGS",
    "make_random", "SWEEPS",
]


@dataclass
class Problem:
    """One synthetic workload: observed COO set, values, initial model."""
    name: str
    dims: tuple
    ranks: tuple
    idx: np.ndarray          # int32 [N][nnz], 0-based
    val: np.ndarray          # float32 [nnz]
    core: np.ndarray         # float32, shape ranks, C order (last mode fastest)
    factors: list            # float32 [I_n][J_n] row-major, one per mode
    lam: float = 0.01
    iters: int = 1
    meta: dict = field(default_factory=dict)

    @property
    def N(self):
        return len(self.dims)

    @property
    def nnz(self):
        return int(self.idx.shape[1])


# ----------------------------------------------------------------------------
# index sets
# ----------------------------------------------------------------------------
def _keys(idx: np.ndarray, dims) -> np.ndarray:
    """Row-major linear cell id, wrapping modulo 2^64.

    Equal tuples always map to equal keys, so every true duplicate is found;
    a rare wrap-around collision only causes an unnecessary redraw.
    """
    k = np.zeros(idx.shape[1], dtype=np.uint64)
    with np.errstate(over="ignore"):
        for n, I in enumerate(dims):
            k = k * np.uint64(I) + idx[n].astype(np.uint64)
    return k


def _dedup(idx: np.ndarray, dims, redraw, max_rounds: int = 200) -> np.ndarray:
    """Redraw every tuple that repeats an earlier one until all are distinct.

    The first pass keeps the first occurrence of every cell; later passes
    only test the redrawn tuples against the sorted set of kept cells.
    """
    keys = _keys(idx, dims)
    kept, first = np.unique(keys, return_index=True)
    dup = np.ones(idx.shape[1], dtype=bool)
    dup[first] = False
    todo = np.flatnonzero(dup)
    for _ in range(max_rounds):
        if todo.size == 0:
            return idx
        new = redraw(todo.size)
        nk = _keys(new, dims)
        pos = np.searchsorted(kept, nk)
        hit = (pos < kept.size) & (kept[np.minimum(pos, kept.size - 1)] == nk)
        _, f2 = np.unique(nk, return_index=True)
        fresh = np.zeros(todo.size, dtype=bool)
        fresh[f2] = True
        ok = fresh & ~hit
        idx[:, todo[ok]] = new[:, ok]
        add = np.sort(nk[ok])
        kept = np.insert(kept, np.searchsorted(kept, add), add)
        todo = todo[~ok]
    raise RuntimeError("could not draw a set of distinct cells")


def uniform_distinct(rng: np.random.Generator, dims, nnz: int) -> np.ndarray:
    """nnz distinct cells drawn uniformly at random."""
    total = math.prod(int(d) for d in dims)
    if nnz > total:
        raise ValueError("more cells requested than the tensor has")
    if nnz > total // 4:
        # dense regime: sample without replacement from all linear ids
        lin = rng.choice(total, size=nnz, replace=False)
        out = np.empty((len(dims), nnz), dtype=np.int32)
        for n in range(len(dims) - 1, -1, -1):
            out[n] = lin % dims[n]
            lin //= dims[n]
        return out

    def draw(m):
        return np.stack([rng.integers(0, d, size=m, dtype=np.int64)
                         for d in dims]).astype(np.int32)
    return _dedup(draw(nnz), dims, draw)


def _zipf_sampler(rng, I: int, s: float):
    """Truncated Zipf(s) over I items, ranks mapped through a seeded permutation."""
    w = np.arange(1, I + 1, dtype=np.float64) ** (-s)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    perm = rng.permutation(I).astype(np.int32)

    def draw(m):
        r = np.searchsorted(cdf, rng.random(m), side="right")
        np.minimum(r, I - 1, out=r)
        return perm[r]
    return draw


def _categorical_sampler(rng, weights: np.ndarray):
    cdf = np.cumsum(weights.astype(np.float64))
    cdf /= cdf[-1]
    I = len(weights)

    def draw(m):
        r = np.searchsorted(cdf, rng.random(m), side="right")
        np.minimum(r, I - 1, out=r)
        return r.astype(np.int32)
    return draw


def _from_samplers(dims, nnz, samplers):
    def draw(m):
        return np.stack([samplers[n](m) for n in range(len(dims))]).astype(np.int32)
    return _dedup(draw(nnz), dims, draw)


def zipf_distinct(rng, dims, nnz: int, s) -> np.ndarray:
    """Distinct cells with an independent truncated Zipf(s_n) skew per mode."""
    if np.isscalar(s):
        s = [s] * len(dims)
    samplers = [(_zipf_sampler(rng, d, sn) if sn > 0 else
                 (lambda m, d=d: rng.integers(0, d, size=m).astype(np.int32)))
                for d, sn in zip(dims, s)]
    return _from_samplers(dims, nnz, samplers)


def lognormal_row_weights(rng, I: int, nnz: int, mu=3.0, sigma=2.0,
                          lo=1.0, hi=1e5) -> np.ndarray:
    """Per-row target nnz: lognormal weights scaled so the clipped sum is nnz."""
    w = rng.lognormal(mu, sigma, size=I)
    a, b = 1e-6, 1e6
    for _ in range(200):                       # bisection on the scale c
        c = math.sqrt(a * b)
        t = np.clip(c * w, lo, hi).sum()
        if t > nnz:
            b = c
        else:
            a = c
    return np.clip(math.sqrt(a * b) * w, lo, hi)


def weighted_distinct(rng, dims, nnz: int, weights) -> np.ndarray:
    """Distinct cells, mode-n index drawn from a categorical over weights[n]."""
    samplers = [_categorical_sampler(rng, w) for w in weights]
    return _from_samplers(dims, nnz, samplers)


# ----------------------------------------------------------------------------
# models and values
# ----------------------------------------------------------------------------
def planted_model(rng, dims, ranks):
    """Planted core and factors, i.i.d. N(0, 1), float64."""
    G = rng.standard_normal(tuple(ranks))
    A = [rng.standard_normal((d, r)) for d, r in zip(dims, ranks)]
    return G, A


def init_model(rng, dims, ranks):
    """Alg. 2 initialisation: core and factors i.i.d. U[0, 1), float32."""
    G = rng.random(tuple(ranks), dtype=np.float64).astype(np.float32)
    A = [rng.random((d, r), dtype=np.float64).astype(np.float32)
         for d, r in zip(dims, ranks)]
    return G, A


def _kron_rows(rows):
    """Row-wise Kronecker product in C order (last factor fastest)."""
    K = rows[0]
    for R in rows[1:]:
        K = (K[:, :, None] * R[:, None, :]).reshape(K.shape[0], -1)
    return K


def planted_values(idx, G, A, chunk: int = 1 << 13) -> np.ndarray:
    """Evaluate a planted Tucker model at the given cells (input recipe only).

    The modes are split into a left and a right group; per chunk of cells the
    model value is <kron(left rows), G_mat @ kron(right rows)> with G_mat the
    core reshaped to (left cells, right cells). Chunks run on a thread pool
    and each writes its own slice, so the result does not depend on timing.
    """
    import concurrent.futures as cf
    import os
    N = len(A)
    ranks = G.shape
    h = max(1, N // 2)
    JL = math.prod(ranks[:h])
    Gm = np.ascontiguousarray(G.reshape(JL, -1))
    nnz = idx.shape[1]
    out = np.empty(nnz, dtype=np.float64)

    def work(s):
        e = min(nnz, s + chunk)
        KL = _kron_rows([A[n][idx[n, s:e]] for n in range(h)])
        KR = _kron_rows([A[n][idx[n, s:e]] for n in range(h, N)])
        M = KR @ Gm.T
        out[s:e] = np.einsum("bi,bi->b", KL, M)

    starts = range(0, nnz, chunk)
    workers = min(16, os.cpu_count() or 1)
    if nnz <= 4 * chunk or workers == 1:
        for s in starts:
            work(s)
    else:
        with cf.ThreadPoolExecutor(workers) as ex:
            list(ex.map(work, starts))
    return out


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
def _planted_problem(name, rng, dims, ranks, idx, noise_var, lam, iters,
                     planted_ranks=None, meta=None):
    pr = planted_ranks or ranks
    Gs, As = planted_model(rng, dims, pr)
    x = planted_values(idx, Gs, As)
    x += math.sqrt(noise_var) * rng.standard_normal(x.shape[0])
    G0, A0 = init_model(rng, dims, ranks)
    m = dict(meta or {})
    m.update(noise_var=noise_var, planted_ranks=tuple(pr))
    return Problem(name, tuple(dims), tuple(ranks), idx,
                   x.astype(np.float32), G0, A0, lam, iters, m)


def make_small(dims, ranks, nnz, seed=0, noise_var=0.01, lam=0.01, iters=1,
               skew=None):
    """A small planted workload with uniform (or Zipf-skewed) distinct cells."""
    rng = np.random.default_rng(seed)
    if skew:
        idx = zipf_distinct(rng, dims, nnz, skew)
    else:
        idx = uniform_distinct(rng, dims, nnz)
    return _planted_problem("small", rng, dims, ranks, idx, noise_var, lam, iters)


def make_c1(seed=0):
    rng = np.random.default_rng(seed)
    dims, ranks = (100, 100, 100), (5, 5, 5)
    idx = uniform_distinct(rng, dims, 10_000)
    return _planted_problem("c1", rng, dims, ranks, idx, 0.01, 0.01, 5)


def make_c2(seed=1, nnz=10_000_000, I=100_000):
    rng = np.random.default_rng(seed)
    dims, ranks = (I,) * 4, (10,) * 4
    idx = zipf_distinct(rng, dims, nnz, 1.1)
    return _planted_problem("c2", rng, dims, ranks, idx, 0.1, 0.01, 10)


def make_c3(seed=2, nnz=100_000_000, dims=(480_000, 18_000, 2_000)):
    rng = np.random.default_rng(seed)
    ranks = (16, 16, 16)
    idx = zipf_distinct(rng, dims, nnz, [0.6, 0.9, 0.0])
    Gs, As = planted_model(rng, dims, (8, 8, 8))
    score = planted_values(idx, Gs, As)
    cuts = np.quantile(score, [0.05, 0.15, 0.40, 0.75])
    val = (1 + np.searchsorted(cuts, score, side="right")).astype(np.float32)
    del score
    G0, A0 = init_model(rng, dims, ranks)
    return Problem("c3", tuple(dims), ranks, idx, val, G0, A0, 0.01, 1,
                   dict(planted_ranks=(8, 8, 8), ratings="1..5 by quantiles"))


def make_c4(seed=3, nnz=50_000_000, I=10_000):
    rng = np.random.default_rng(seed)
    dims, ranks = (I,) * 5, (8,) * 5
    weights = [lognormal_row_weights(rng, I, nnz) for _ in dims]
    idx = weighted_distinct(rng, dims, nnz, weights)
    return _planted_problem("c4", rng, dims, ranks, idx, 0.1, 0.01, 1,
                            planted_ranks=(4,) * 5)


def make_c5(seed=4, n_foldin=100_000, pred_every=20, dims=(100_000, 50_000, 1_000),
            J=16):
    """Serving workload: a planted order-3 model and a request stream.

    Fold-in requests (new rows of mode 0): k ~ lognormal(ln 50, 1.2) clipped
    to [5, 5000], entries at uniform (i_2, i_3), values of the planted model
    with a fresh N(0,1) row + N(0, 0.1) noise. After every `pred_every`
    fold-ins one prediction batch of log-uniform size in [1e3, 1e5] uniform
    cells. Returns (core, factors, requests); a request is
    ("f", mode, idx [N][k] int32, val float32) or ("p", None, idx [N][m], None).
    """
    rng = np.random.default_rng(seed)
    ranks = (J,) * 3
    G, A = planted_model(rng, dims, ranks)
    k = np.clip(np.rint(rng.lognormal(math.log(50.0), 1.2, n_foldin)), 5, 5000).astype(np.int64)
    tot = int(k.sum())
    owner = np.repeat(np.arange(n_foldin, dtype=np.int32), k)
    i2 = rng.integers(0, dims[1], tot, dtype=np.int64).astype(np.int32)
    i3 = rng.integers(0, dims[2], tot, dtype=np.int64).astype(np.int32)
    Anew = rng.standard_normal((n_foldin, J))
    x = planted_values(np.stack([owner, i2, i3]), G, [Anew, A[1], A[2]])
    x += math.sqrt(0.1) * rng.standard_normal(tot)
    x = x.astype(np.float32)
    reqs = []
    off = np.concatenate([[0], np.cumsum(k)])
    for r in range(n_foldin):
        a, b = off[r], off[r + 1]
        idx = np.stack([np.zeros(b - a, np.int32), i2[a:b], i3[a:b]])
        reqs.append(("f", 0, idx, x[a:b]))
        if (r + 1) % pred_every == 0:
            m = int(round(10 ** rng.uniform(3, 5)))
            pidx = np.stack([rng.integers(0, d, m, dtype=np.int64).astype(np.int32)
                             for d in dims])
            reqs.append(("p", None, pidx, None))
    return (G.astype(np.float32), [a.astype(np.float32) for a in A], reqs)


def make_random(dims, J, nnz, seed=0, lam=0.01):
    """The paper's synthetic scalability tensors (Sec. 4.2): equal ranks J,
    nnz distinct cells at uniform random positions, values U[0, 1); initial
    model U[0, 1) as in Alg. 2."""
    rng = np.random.default_rng(seed)
    idx = uniform_distinct(rng, dims, nnz)
    val = rng.random(nnz, dtype=np.float64).astype(np.float32)
    ranks = (J,) * len(dims)
    G0, A0 = init_model(rng, dims, ranks)
    return Problem("random", tuple(dims), ranks, idx, val, G0, A0, lam, 1,
                   {"values": "U[0,1)"})


# the four sweeps of Sec. 4.2 (order, dimensionality, observed entries, rank)
SWEEPS = {
    "order": [((100,) * N, 3, 1_000) for N in range(3, 11)],
    "dimensionality": [((I,) * 3, 10, 10 * I) for I in (10**2, 10**3, 10**4, 10**5,
                                                      10**6, 10**7)],
    "nnz": [((10**7,) * 3, 10, m) for m in (10**3, 10**4, 10**5, 10**6, 10**7)],
    "rank": [((10**6,) * 3, J, 10**7) for J in (3, 5, 7, 9, 11)],
    # the Cache-variant comparison of Sec. 4.3 (orders 6-10)
    "cache": [((100,) * N, 3, 1_000) for N in range(6, 11)],
}


CONFIGS = {"c1": make_c1, "c2": make_c2, "c3": make_c3, "c4": make_c4}


def make(name: str, **kw) -> Problem:
    return CONFIGS[name](**kw)
