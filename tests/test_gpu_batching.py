"""GPU tests of the batching form: graph replay and the autotuner.

* A captured iteration graph, replayed several times per call and over
  several calls (with the program's own synchronisations and a change of
  lambda that forces a re-capture in between), gives bitwise the same errors
  and factors as launching the kernels one by one.
* After the autotuner has picked work-range sizes, a mode update still
  matches the FP64 oracle per row (1e-5), and a second tuning run with the
  same cache file reuses the stored sizes.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import context, f64, log, row_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    assert torch.cuda.is_available()


@pytest.mark.parametrize("prec", [0, 2])
def test_graph_replay_bitwise_equal_to_eager(prec):
    import torch
    p = synth.make_small((60, 50, 40), (8, 8, 8), 6000, seed=21, skew=1.1)
    cg, _, _, _, fg = context(p, precision=prec)
    ce, _, _, _, fe = context(p, precision=prec)
    cg.set_options(precision=prec, use_graph=1)
    ce.set_options(precision=prec, use_graph=0)
    for call, lam in enumerate([0.01, 0.01, 0.05, 0.01]):
        sg, lg = cg.iterate(3, lam, strict=False)
        torch.cuda.synchronize()
        se, le = ce.iterate(3, lam, strict=False)
        torch.cuda.synchronize()
        assert np.array_equal(sg, se), (call, sg, se)
        assert np.array_equal(lg, le)
        for a, b in zip(fg, fe):
            assert torch.equal(a, b), call
    cg.close()
    ce.close()


def test_graph_replay_after_rebinding_model():
    import torch
    p = synth.make_small((40, 30, 20), (5, 5, 5), 3000, seed=22)
    c, idx, val, core, fac = context(p)
    c.iterate(2, p.lam)
    # bind a fresh copy: the captured graph must not keep the old pointers
    fac2 = [f.clone() for f in fac]
    core2 = core.clone()
    c.bind_model(core2, fac2)
    before = [f.clone() for f in fac]
    s2, _ = c.iterate(2, p.lam)
    for a, b in zip(fac, before):
        assert torch.equal(a, b)           # old buffers untouched
    assert not all(torch.equal(a, b) for a, b in zip(fac2, before))
    c.close()


@pytest.mark.parametrize("prec,dims,ranks", [
    (0, (80, 70, 60), (5, 5, 5)),
    (0, (20, 18, 16, 14, 12), (3, 3, 3, 3, 3)),
    (0, (30, 28, 26, 24), (10, 10, 10, 10)),         # tile shape searched too
    (0, (14, 13, 12, 11, 10), (8, 8, 8, 8, 8)),      # tile shape searched too
    (2, (80, 70, 60), (16, 16, 16)),
])
def test_autotune_then_update_matches_oracle(prec, dims, ranks, tmp_path):
    """The tuner picks the work-range size of every mode and, where both are
    compiled (FP64 at (4, 10) and (5, 8)), one or two entries per lane; the
    choice is cached ("key work [two]") and applied again from the cache."""
    p = synth.make_small(dims, ranks, 8000, seed=23, skew=1.2)
    if prec == 2:
        # integer data: the BF16 path is exact there
        rng = np.random.default_rng(5)
        p.core = rng.integers(-1, 2, size=ranks).astype(np.float32)
        p.factors = [rng.integers(-1, 2, size=(d, r)).astype(np.float32)
                     for d, r in zip(dims, ranks)]
        p.val = rng.integers(-3, 4, size=p.nnz).astype(np.float32)
    cache = str(tmp_path / "tune.txt")
    c, idx, val, core, fac = context(p, precision=prec)
    work = c.autotune(cache)
    log("autotuned work per mode", work)
    assert all(w > 0 for w in work)
    assert os.path.getsize(cache) > 0
    fields = [len(line.split()) for line in open(cache)]
    both = prec == 0 and (len(dims), ranks[0]) in ((4, 10), (5, 8))
    assert fields == [3 if both else 2] * len(dims)
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    v = p.val.astype(np.float64)
    for n in range(len(dims)):
        before = [f.clone() for f in fac]
        c.update_mode(n, p.lam)
        want = oracle.update_rows(G, A, p.idx, v, n, p.lam)
        got = f64(fac[n])
        nz = np.bincount(p.idx[n], minlength=dims[n]) > 0
        assert row_rel_err(got[nz], want[nz]).max() <= 1e-5
        for f, b in zip(fac, before):
            f.copy_(b)
    c2, *_ = context(p, precision=prec)
    assert c2.autotune(cache) == work
    c.close()
    c2.close()


@pytest.mark.parametrize("graph", [1, 0])
def test_iterate_early_stop_by_tolerance(graph):
    """options.tol stops ptk_iterate after the first iteration t >= 2 whose
    error sqrt(SSE) moved by at most tol times the previous one; the
    iterations it ran equal those of a run without it, bitwise, and the
    entries past them are NaN."""
    import paper_1710_02261_amd as ptk
    p = synth.make_small((40, 35, 30), (5, 5, 5), 6000, seed=71)
    ref, _, _, _, _ = context(p)
    ref.set_options(use_graph=graph)
    want, want_loss = ref.iterate(12, p.lam, strict=False)
    e = np.sqrt(want)
    for tol in (1.0, 1e-3, 1e-6):
        ctx, _, _, _, _ = context(p)
        ctx.set_options(use_graph=graph, tol=tol)
        got, loss = ctx.iterate(12, p.lam, strict=False)
        done = ctx.iterations_done()
        stop = next((t + 1 for t in range(1, 12) if abs(e[t] - e[t - 1]) <= tol * e[t - 1]), 12)
        assert done == stop, (tol, done, stop)
        assert np.array_equal(got[:done], want[:done])
        assert np.array_equal(loss[:done], want_loss[:done])
        assert np.all(np.isnan(got[done:])) and np.all(np.isnan(loss[done:]))
        ctx.close()
    ref.close()
    c = ptk.Context(p.dims, p.ranks)
    with pytest.raises(ptk.PtkError, match="tol"):
        c.set_options(tol=-1.0)
    c.close()
