"""ptk_fold_in_noalloc (the fold-in on the library's fixed device scratch)
against ptk_fold_in, through the C ABI: two calls in a row, the second with
fewer entries, both to the fold-in bar (per-row relative 1e-5; the two share
their kernels and, at these sizes, their work split, so they agree bitwise),
and both against the FP64 oracle. Also the size limit and the state after
calls of the allocating entry point."""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import log

pytestmark = pytest.mark.gpu


def _model():
    import torch
    import paper_1710_02261_amd as ptk
    rng = np.random.default_rng(91)
    dims, ranks = (300, 200, 100), (6, 5, 4)
    G, A = synth.planted_model(rng, dims, ranks)
    dev = torch.device("cuda:0")
    core = torch.from_numpy(np.ascontiguousarray(G, dtype=np.float32)).to(dev)
    fac = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev) for a in A]
    ctx = ptk.Context(dims, ranks)
    ctx.bind_model(core, fac)
    return ctx, G.astype(np.float64), [a.astype(np.float64) for a in A], dims, rng


def _request(rng, dims, n, k):
    idx = np.zeros((len(dims), k), dtype=np.int32)
    for m in range(len(dims)):
        if m != n:
            idx[m] = rng.integers(0, dims[m], k)
    val = rng.standard_normal(k).astype(np.float32)
    return idx, val


def test_noalloc_fold_in_matches_fold_in_twice():
    import torch
    ctx, G, A, dims, rng = _model()
    lam = 0.05
    n = 1
    prev = None
    for k in (4000, 700):                      # the second call is smaller
        idx, val = _request(rng, dims, n, k)
        ti = torch.from_numpy(idx).cuda()
        tv = torch.from_numpy(val).cuda()
        want = ctx.fold_in(n, ti, tv, lam).cpu().numpy().astype(np.float64)
        out = torch.full((A[n].shape[1],), float("nan"), dtype=torch.float32, device="cuda")
        got = ctx.fold_in_noalloc(n, ti, tv, lam, out).cpu().numpy().astype(np.float64)
        ora = oracle.fold_in(G, A, n, idx, val.astype(np.float64), lam)
        rel = np.linalg.norm(got - want) / np.linalg.norm(want)
        rel_o = np.linalg.norm(got - ora) / np.linalg.norm(ora)
        log("k=%d: noalloc vs fold_in rel %.3g (bitwise %s), vs oracle %.3g"
            % (k, rel, bool(np.array_equal(got, want)), rel_o))
        assert rel <= 1e-5 and rel_o <= 1e-5
        if prev is not None:
            assert not np.array_equal(got, prev)
        prev = got
    ctx.close()


def test_noalloc_fold_in_limit_and_empty_row():
    import torch
    import paper_1710_02261_amd as ptk
    ctx, G, A, dims, rng = _model()
    out = torch.zeros(A[0].shape[1], dtype=torch.float32, device="cuda")
    e = torch.zeros((3, 0), dtype=torch.int32, device="cuda")
    v = torch.zeros(0, dtype=torch.float32, device="cuda")
    ctx.fold_in_noalloc(0, e, v, 0.1, out)          # no entry: the row is 0
    assert torch.count_nonzero(out).item() == 0
    big = torch.zeros((3, (1 << 24) + 1), dtype=torch.int32, device="cuda")
    bv = torch.zeros((1 << 24) + 1, dtype=torch.float32, device="cuda")
    with pytest.raises(ptk.PtkError, match="limit"):
        ctx.fold_in_noalloc(0, big, bv, 0.1, out)
    ctx.close()
