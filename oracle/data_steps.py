"""FP64 numpy oracle for the steps either side of the fit.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: written from the
definitions below, shares no code with the GPU library.

* ``splitmix64``  -- the SplitMix64 generator (Steele, Lea and Flood,
  "Fast splittable pseudorandom number generators", OOPSLA 2014): state
  advanced by the golden-ratio increment, output = the mixing function of
  the state. ``splitmix64(seed, k)`` is output k (1-based) of the generator
  seeded with ``seed``.
* ``held_out``    -- the train/test rule: entry e goes to the test side when
  the top 53 bits of output e + 1, over 2^53, are below the test fraction
  (Sec. 4.1 holds out 10 % of the observed entries).
* ``normalize``   -- min-max scaling of the values to [0, 1] (Sec. 4.1).
* ``kmeans``      -- Lloyd's iterations over the rows of a factor matrix
  (concept discovery, Sec. 5): assign each row to the nearest centroid
  (squared Euclidean distance, lowest index on ties), move each centroid to
  the mean of its rows (a centroid without rows stays), repeat; then one
  last assignment.
"""
from __future__ import annotations

import numpy as np

_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


def _mix(z):
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def splitmix64_sequence(seed, count):
    """The first ``count`` outputs of the generator, advanced one by one."""
    state, out = seed & _M64, []
    for _ in range(count):
        state = (state + _GAMMA) & _M64
        out.append(_mix(state))
    return out


def splitmix64(seed, k):
    """Output k (k >= 1) of the generator seeded with ``seed`` (numpy uint64
    arithmetic, wrapping modulo 2^64)."""
    k = np.asarray(k, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + k * np.uint64(_GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def held_out(nnz, frac, seed):
    """Boolean mask of the held-out entries among nnz."""
    u = splitmix64(seed, np.arange(1, nnz + 1, dtype=np.uint64)) >> np.uint64(11)
    return u.astype(np.float64) * 2.0 ** -53 < frac


def normalize(val):
    """(v - min) / (max - min) in float64, rounded to float32; 0 if max = min."""
    v = np.asarray(val, dtype=np.float64)
    if v.size == 0:
        return v.astype(np.float32), (0.0, 0.0)
    lo, hi = float(v.min()), float(v.max())
    if hi > lo:
        out = (v - lo) / (hi - lo)
    else:
        out = np.zeros_like(v)
    return out.astype(np.float32), (lo, hi)


def assign_rows(X, C):
    """Nearest centroid per row and its squared distance (argmin takes the
    lowest index among equal distances)."""
    X = np.asarray(X, dtype=np.float64)
    d = ((X[:, None, :] - C[None, :, :]) ** 2).sum(axis=2)
    a = np.argmin(d, axis=1)
    return a.astype(np.int32), d[np.arange(len(X)), a], d


def kmeans(X, C0, iters):
    """Lloyd's iterations from C0; returns (C, assignment, inertia, changed
    rows in the last assignment, inertia after each assignment)."""
    X = np.asarray(X, dtype=np.float64)
    C = np.array(C0, dtype=np.float64)
    K = len(C)
    prev = np.full(len(X), -1, dtype=np.int32)
    hist = []
    for t in range(iters + 1):
        a, dmin, _ = assign_rows(X, C)
        changed = int((a != prev).sum())
        prev = a
        hist.append(float(dmin.sum()))
        if t == iters:
            break
        for k in range(K):
            rows = X[a == k]
            if len(rows):
                C[k] = rows.sum(axis=0) / len(rows)
    return C, prev, hist[-1], changed, hist
