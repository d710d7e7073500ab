"""Parity at the full size of the benchmark workload, in the launch
configuration the benchmark times.

Workload: order-4 100000^4 tensor, 1e7 entries (Zipf 1.1 per mode), J=10,
FP64 delta/Gram arithmetic, work ranges chosen by the autotuner (as in
bench.py). The oracle cannot update a whole mode of this size in test time,
so it recomputes sampled rows one by one (all entries of each sampled row):

* per mode, one ptk_update_mode from the same starting factors; sampled rows
  cover the row-length distribution (single-entry rows up to rows of ~1e5
  entries) and rows that cross work-range boundaries (their systems go
  through the merge). Bar: per-row relative error <= 1e-5. Rows whose
  system B + lambda I has a condition number above 1e10 get the bound
  kappa * 1e-15 instead (two correct FP64 evaluations that sum in different
  orders differ by about kappa * eps there); the log prints kappa per row.
* predictions of 20000 sampled entries against the oracle (1e-6);
* the error of the fused pass (row-system identity of the last mode) against
  the direct pass on the GPU, and the direct pass against the oracle on
  sampled entries through the predictions above.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import f64, log, row_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c2():
    import paper_1710_02261_amd as ptk
    import torch
    assert torch.cuda.is_available()
    log("generating the order-4 1e7-entry workload")
    p = synth.make("c2")
    dev = torch.device("cuda:0")
    idx = torch.from_numpy(p.idx).to(dev)
    val = torch.from_numpy(p.val).to(dev)
    core = torch.from_numpy(p.core).to(dev)
    fac = [torch.from_numpy(a).to(dev) for a in p.factors]
    ctx = ptk.Context(p.dims, p.ranks)
    ctx.set_options(precision=0, fuse_error=1, profile=0, use_graph=1)
    ctx.set_observed(idx, val)
    ctx.bind_model(core, fac)
    work = ctx.autotune(None)
    log("autotuned work-range sizes", work)
    yield p, ctx, idx, core, fac, work
    ctx.close()


def sample_rows(counts, chunk, rng):
    nz = np.flatnonzero(counts)
    order = nz[np.argsort(counts[nz], kind="stable")]
    picks = set()
    for q in (0.0, 0.1, 0.5, 0.9, 0.99, 0.999):
        picks.add(int(order[int(q * (len(order) - 1))]))
    light = order[counts[order] <= 100_000]
    picks.add(int(light[-1]))                       # heaviest row up to 1e5 entries
    # rows that cross a work-range boundary (merged from partial systems)
    rp = np.concatenate([[0], np.cumsum(counts)])
    cross = [r for r in nz if rp[r] // chunk != (rp[r + 1] - 1) // chunk
             and counts[r] <= 20_000]
    for r in rng.choice(cross, size=min(4, len(cross)), replace=False):
        picks.add(int(r))
    picks.update(int(r) for r in rng.choice(nz, size=6, replace=False))
    return np.array(sorted(picks), dtype=np.int32)


def test_fullsize_mode_updates_match_oracle_on_sampled_rows(c2):
    p, ctx, idx, core, fac, work = c2
    import paper_1710_02261_amd as ptk
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    v = p.val.astype(np.float64)
    rng = np.random.default_rng(5)
    for n in range(p.N):
        before = [f.clone() for f in fac]
        try:
            ctx.update_mode(n, p.lam)
        except ptk.PtkError as e:                  # rows kept their value
            assert "PTK_E_NOT_PD" in str(e)
        counts = np.bincount(p.idx[n], minlength=p.dims[n])
        rows = sample_rows(counts, work[n], rng)
        want = oracle.update_rows(G, A, p.idx, v, n, p.lam, rows=rows)
        got = f64(fac[n])[rows]
        err = row_rel_err(got, want)
        for r, e in zip(rows, err):
            B, c = oracle.row_system(G, A, p.idx, v, n, int(r))
            kappa = np.linalg.cond(B + p.lam * np.eye(B.shape[0]))
            bound = 1e-5 if kappa <= 1e10 else max(1e-5, kappa * 1e-15)
            log("mode %d row %d: %d entries, kappa %.3g, rel err %.3g (bound %.3g)"
                % (n, r, counts[r], kappa, e, bound))
            assert e <= bound, (n, r, e, kappa)
        for f, b in zip(fac, before):
            f.copy_(b)


def test_fullsize_predictions_and_error_pass(c2):
    p, ctx, idx, core, fac, work = c2
    import torch
    rng = np.random.default_rng(6)
    pick = rng.choice(p.nnz, size=20_000, replace=False)
    sub = np.ascontiguousarray(p.idx[:, pick])
    got = ctx.predict(torch.from_numpy(sub).cuda()).cpu().numpy().astype(np.float64)
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    want = oracle.predict(G, A, sub)
    np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-6 * np.abs(want).max())
    # the sampled squared residuals estimate the full SSE of the direct pass
    sse_direct, rmse, _ = ctx.recon_error(p.lam)
    est = np.sum((p.val[pick].astype(np.float64) - want) ** 2) * p.nnz / len(pick)
    log("direct SSE %.6g, sampled estimate %.6g" % (sse_direct, est))
    assert 0.8 * est <= sse_direct <= 1.25 * est
    # fused error (row-system identity of the last mode) vs the direct pass
    before = [f.clone() for f in fac]
    sse_fused, _ = ctx.iterate(1, p.lam, strict=False)
    sse_after, _, _ = ctx.recon_error(p.lam)
    log("after one iteration: fused SSE %.9g, direct SSE %.9g, rel diff %.3g"
        % (sse_fused[0], sse_after, abs(sse_fused[0] - sse_after) / sse_after))
    assert abs(sse_fused[0] - sse_after) <= 1e-3 * sse_after
    for f, b in zip(fac, before):
        f.copy_(b)
