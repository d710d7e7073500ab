"""Pins of the data-step oracle (oracle/data_steps.py) against facts that do
not come from the oracle itself: the published SplitMix64 outputs, the
bounds and invariances of min-max scaling, and k-means cases whose answer is
known by hand or in closed form. Mistakes planted in copies of the oracle
must fail them.
"""
import numpy as np
import pytest

from oracle import data_steps as ds


# Outputs of SplitMix64 seeded with 0 and with 1234567, as published with the
# generator's reference implementations.
SEED0 = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
SEED1234567 = [6457827717110365317, 3203168211198807973, 9817491932198370423]


def test_splitmix64_published_outputs():
    assert ds.splitmix64_sequence(0, 3) == SEED0
    assert ds.splitmix64_sequence(1234567, 3) == SEED1234567
    assert [int(x) for x in ds.splitmix64(0, [1, 2, 3])] == SEED0
    assert [int(x) for x in ds.splitmix64(1234567, [1, 2, 3])] == SEED1234567


def test_counter_form_matches_the_sequence():
    seq = ds.splitmix64_sequence(987654321, 1000)
    assert [int(x) for x in ds.splitmix64(987654321, np.arange(1, 1001))] == seq


def test_held_out_share_edges_and_nesting():
    n = 1_000_000
    m = ds.held_out(n, 0.1, 7)
    share = m.mean()
    assert abs(share - 0.1) < 5 * np.sqrt(0.1 * 0.9 / n)
    assert not ds.held_out(1000, 0.0, 7).any()
    assert ds.held_out(1000, 1.0, 7).all()
    small, big = ds.held_out(n, 0.05, 7), ds.held_out(n, 0.2, 7)
    assert np.all(big[small])                 # nested in the fraction
    assert not np.array_equal(ds.held_out(1000, 0.5, 1), ds.held_out(1000, 0.5, 2))


def test_normalize_bounds_and_invariance():
    rng = np.random.default_rng(1)
    v = (rng.standard_normal(1000) * 3 + 5).astype(np.float32)
    out, (lo, hi) = ds.normalize(v)
    assert out.min() == 0.0 and out.max() == 1.0
    assert lo == float(v.min()) and hi == float(v.max())
    out2, _ = ds.normalize((v.astype(np.float64) * 4 + 9).astype(np.float32))
    np.testing.assert_allclose(out2, out, atol=1e-6)
    const, _ = ds.normalize(np.full(5, 2.5, np.float32))
    assert np.all(const == 0.0)


def test_kmeans_by_hand():
    X = np.array([[0.0], [1.0], [10.0], [11.0]])
    C, a, inertia, changed, _ = ds.kmeans(X, np.array([[0.0], [10.0]]), 3)
    np.testing.assert_array_equal(C, [[0.5], [10.5]])
    np.testing.assert_array_equal(a, [0, 0, 1, 1])
    assert inertia == 4 * 0.25 and changed == 0


def test_kmeans_blobs_reach_their_means_and_inertia_falls():
    rng = np.random.default_rng(2)
    centers = np.array([[0, 0, 0], [10, 0, 0], [0, 10, 0], [0, 0, 10]], float)
    X = np.concatenate([c + rng.standard_normal((200, 3)) * 0.3 for c in centers])
    C0 = X[[5, 205, 405, 605]] + 0.5
    C, a, _, _, hist = ds.kmeans(X, C0, 10)
    for k in range(4):
        np.testing.assert_allclose(C[k], X[200 * k:200 * (k + 1)].mean(axis=0), rtol=1e-12)
        assert np.all(a[200 * k:200 * (k + 1)] == k)
    assert all(b <= a_ + 1e-12 for a_, b in zip(hist, hist[1:]))


def test_kmeans_ties_and_empty_clusters():
    X = np.array([[1.0, 0.0], [1.0, 0.0]])
    C, a, _, _, _ = ds.kmeans(X, np.array([[0.0, 0.0], [2.0, 0.0], [50.0, 50.0]]), 1)
    assert np.all(a == 0)                     # equal distances: lowest index
    np.testing.assert_array_equal(C[2], [50.0, 50.0])   # no rows: stays


def _kmeans_ties_high(X, C0, iters):
    X = np.asarray(X, float)
    C = np.array(C0, float)
    for t in range(iters + 1):
        d = ((X[:, None, :] - C[None]) ** 2).sum(2)
        a = len(C) - 1 - np.argmin(d[:, ::-1], axis=1)
        if t == iters:
            return C, a
        for k in range(len(C)):
            if (a == k).any():
                C[k] = X[a == k].mean(0)


def _normalize_by_max(val):
    v = np.asarray(val, np.float64)
    return (v / v.max()).astype(np.float32)


def test_planted_mistakes_fail_the_pins():
    X = np.array([[1.0, 0.0], [1.0, 0.0]])
    _, a = _kmeans_ties_high(X, np.array([[0.0, 0.0], [2.0, 0.0]]), 1)
    assert not np.all(a == 0)                 # the tie pin catches it
    # an off-by-one counter (output e instead of e + 1) breaks the published outputs
    assert [int(x) for x in ds.splitmix64(0, [0, 1, 2])] != SEED0
    # scaling by the maximum alone misses the lower bound
    rng = np.random.default_rng(1)
    v = (rng.standard_normal(1000) * 3 + 5).astype(np.float32)
    assert _normalize_by_max(v).min() != 0.0
