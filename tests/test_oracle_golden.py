"""The oracle reproduces its committed trajectory on the 100^3 workload."""
import json
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c1_trajectory_matches_golden():
    with open(os.path.join(HERE, "golden", "c1_oracle_trajectory.json")) as f:
        gold = json.load(f)
    p = synth.make_c1()
    G = p.core.astype(np.float64)
    A0 = [a.astype(np.float64) for a in p.factors]
    val = p.val.astype(np.float64)
    assert oracle.sse(G, A0, p.idx, val) == pytest.approx(gold["sse_init"], rel=1e-12)
    A, L, S = oracle.fit(G, A0, p.idx, val, p.lam, p.iters)
    np.testing.assert_allclose(S, gold["sse_per_iter"], rtol=1e-10)
    np.testing.assert_allclose(L, gold["loss_after_mode"], rtol=1e-10)
    np.testing.assert_allclose(A[0][:5], gold["rows_mode0_first5"], rtol=1e-8, atol=1e-12)
    np.testing.assert_allclose(A[2][-5:], gold["rows_mode2_last5"], rtol=1e-8, atol=1e-12)
    # Theorem 2 on this workload as well
    seq = np.asarray(L).ravel()
    assert np.all(seq[1:] <= seq[:-1] * (1 + 1e-12))
