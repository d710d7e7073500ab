"""GPU parity of the sparse-core row systems of the Approx variant (Alg. 4,
Sec. 3.3): once the removals have left few non-zero cells in G, delta
(eq. "delta") is summed over the listed non-zero cells only.

* Iterations of Alg. 2 with the removal, on cores with most cells already
  zero, each from the same state as the oracle (which sums delta over every
  cell, zeros included): factors per row 1e-5, error 1e-5, the removed cells
  as in the dense Approx test. Every Approx shape; at (4, 10) and (5, 8) the
  sparse kernel also keeps the deltas the residuals are formed from.
* The switch is taken on the device inside the captured iteration: a run
  whose core crosses the limit between iterations matches the dense path
  (sparse_limit < 0) to the same bound, and ptk_approx_stats reports the
  non-zero cells and the modes on the sparse kernel.
* An all-zero core: delta = 0, so every observed row solves to 0.
* Option refusals.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import context, f64, log, row_rel_err
from tests.test_gpu_approx import check_removal

pytestmark = pytest.mark.gpu

SHAPES = [((30, 25, 20), 3), ((30, 25, 20), 4), ((30, 25, 20), 5), ((40, 30, 20), 8),
          ((30, 25, 20), 10), ((30, 25, 20), 16), ((12, 11, 10, 9), 3),
          ((12, 11, 10, 9), 5), ((12, 11, 10, 9), 8), ((12, 11, 10, 9), 10),
          ((8, 7, 6, 5, 4), 3), ((8, 7, 6, 5, 4), 5), ((8, 7, 6, 5, 4), 8)]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    assert torch.cuda.is_available()


def sparse_problem(dims, J, seed, keep, nnz=4000):
    """Synthetic Zipf-skewed problem whose core keeps a `keep` fraction of
    its cells (the others set to zero, chosen at random)."""
    p = synth.make_small(dims, (J,) * len(dims), nnz, seed=seed, skew=1.1)
    rng = np.random.default_rng(seed + 1)
    cells = p.core.size
    drop = rng.choice(cells, size=cells - max(1, int(keep * cells)), replace=False)
    core = p.core.copy().reshape(-1)
    core[drop] = 0.0
    p.core = core.reshape(p.core.shape)
    return p


def replay(ctx, core, fac, p, rate, iters):
    """Run `iters` single iterations; each against the oracle from the same
    state, then both continue from the oracle's state."""
    import torch
    v = p.val.astype(np.float64)
    N = len(p.dims)
    start_nz = -1
    for t in range(iters):
        G = core.cpu().numpy().astype(np.float64)
        start_nz = int(np.count_nonzero(G))
        A = [f64(f) for f in fac]
        sse, _ = ctx.iterate(1, p.lam, strict=False)
        for n in range(N):
            A = oracle.update_mode(G, A, p.idx, v, n, p.lam)
            A[n] = A[n].astype(np.float32).astype(np.float64)
        want_sse = oracle.sse(G, A, p.idx, v)
        R = oracle.partial_error(G, A, p.idx, v)
        worst = 0.0
        for n in range(N):
            nz = np.bincount(p.idx[n], minlength=p.dims[n]) > 0
            e = row_rel_err(f64(fac[n])[nz], A[n][nz]).max()
            worst = max(worst, e)
            assert e <= 1e-5, (t, n, e)
        assert abs(sse[0] - want_sse) <= 1e-5 * want_sse
        G_gpu = core.cpu().numpy().astype(np.float64)
        check_removal(G, G_gpu, R, want_sse, rate)
        log("iteration", t, "non-zero cells", np.count_nonzero(G), "row err", worst)
        Go, _ = oracle.truncate(G, R, rate)
        core.copy_(torch.from_numpy(Go.astype(np.float32)))
        for f, a in zip(fac, A):
            f.copy_(torch.from_numpy(a.astype(np.float32)))
    return start_nz


@pytest.mark.parametrize("dims,J", SHAPES, ids=["%dd-J%d" % (len(d), j) for d, j in SHAPES])
def test_sparse_core_iterations_match_oracle(dims, J):
    p = sparse_problem(dims, J, seed=61, keep=0.12)
    ctx, idx, val, core, fac = context(p, profile=1)
    ctx.set_options(fuse_error=0, approx_rate=0.2, profile=1, use_graph=1, sparse_limit=1.0)
    last_nz = replay(ctx, core, fac, p, 0.2, 3)
    kt = ctx.kernel_times()
    assert "gram_sparse" in kt and "sparse_lists" in kt
    assert ctx.approx_stats() == (last_nz, (1 << len(dims)) - 1)
    kept = "approx_resid_kept" in kt
    assert kept == ((len(dims), J) in ((4, 10), (5, 8)))
    ctx.close()


@pytest.mark.parametrize("dims,J", [((40, 30, 20), 8), ((12, 11, 10, 9), 10),
                                    ((8, 7, 6, 5, 4), 8)])
def test_switch_inside_graph_matches_dense_path(dims, J):
    """Rate 0.5 from a core with 60% of its cells: 0.6, 0.3, 0.15 of the cells
    in the three iterations, so with a limit of 0.35 the first one runs the
    dense kernels and the next two the sparse one, in one captured graph."""
    import torch
    p = sparse_problem(dims, J, seed=62, keep=0.6)
    cs, _, _, core_s, fs = context(p)
    cd, _, _, core_d, fd = context(p)
    cs.set_options(fuse_error=1, approx_rate=0.5, use_graph=1, sparse_limit=0.35)
    cd.set_options(fuse_error=1, approx_rate=0.5, use_graph=1, sparse_limit=-1.0)
    ss, _ = cs.iterate(3, p.lam, strict=False)
    sd, _ = cd.iterate(3, p.lam, strict=False)
    torch.cuda.synchronize()
    np.testing.assert_allclose(ss, sd, rtol=1e-5)
    for n in range(len(dims)):
        a, b = f64(fs[n]), f64(fd[n])
        nz = np.bincount(p.idx[n], minlength=dims[n]) > 0
        assert row_rel_err(a[nz], b[nz]).max() <= 1e-5
    # the last iteration started from 0.15 of the cells, on the sparse kernel
    cells = J ** len(dims)
    left = int(0.6 * cells)
    left -= left // 2
    left -= left // 2
    assert cs.approx_stats() == (left, (1 << len(dims)) - 1)
    assert cd.approx_stats() == (-1, 0)
    # the same cells were removed (no near-ties at these sizes)
    assert torch.equal(core_s != 0, core_d != 0)
    cs.close()
    cd.close()


def test_all_zero_core_solves_rows_to_zero():
    import torch
    p = synth.make_small((20, 18, 16, 14), (5,) * 4, 3000, seed=63, skew=1.1)
    p.core = np.zeros_like(p.core)
    ctx, idx, val, core, fac = context(p)
    ctx.set_options(approx_rate=0.2, use_graph=1, sparse_limit=1.0)
    sse, _ = ctx.iterate(1, p.lam, strict=False)
    torch.cuda.synchronize()
    for f in fac:
        assert torch.count_nonzero(f).item() == 0
    want = float(np.sum(p.val.astype(np.float64) ** 2))
    assert abs(sse[0] - want) <= 1e-9 * want
    ctx.close()


def test_sparse_limit_refusals():
    import paper_1710_02261_amd as ptk
    p = synth.make_small((10, 9, 8), (3, 3, 3), 200, seed=64)
    ctx, *_ = context(p)
    for bad in (1.5, float("inf"), float("nan")):
        with pytest.raises(ptk.PtkError):
            ctx.set_options(approx_rate=0.2, sparse_limit=bad)
    ctx.set_options(approx_rate=0.2, sparse_limit=-3.0)     # never
    ctx.set_options(approx_rate=0.2, sparse_limit=1.0)      # always
    ctx.close()
