"""GPU parity on the shapes of the paper's synthetic scalability sweeps
(Sec. 4.2) that run on the generic row-system kernel: orders 6 to 10 with
J = 3, and ranks 7, 9 and 11 at order 3. Random tensors as in the paper
(values U[0,1) at uniform cells, U[0,1) initial model), small enough for
the oracle. Bar: one mode update per mode, per-row relative error <= 1e-5.

Each case runs with the delta sum sliced over the core cells as chosen
automatically (these observed sets are small, so it slices), unsliced
(delta_slices = 1: the one-wavefront-per-64-entries kernel) and with an odd
forced slice count; plus unequal ranks, rows crossing work ranges, a slice
count capped at one cell per slice, and the option's refusals.
"""
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


CASES = [((10,) * 6, 3, 800), ((8,) * 7, 3, 600), ((6,) * 8, 3, 500),
         ((5,) * 9, 3, 300), ((4,) * 10, 3, 300),
         ((60, 50, 40), 7, 3000), ((60, 50, 40), 9, 3000), ((60, 50, 40), 11, 3000)]


def check_updates(p, ctx, fac, tol=1e-5):
    dims = p.dims
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    v = p.val.astype(np.float64)
    worst = []
    for n in range(len(dims)):
        before = [f.clone() for f in fac]
        ctx.update_mode(n, p.lam)
        want = oracle.update_rows(G, A, p.idx, v, n, p.lam)
        nz = np.bincount(p.idx[n], minlength=dims[n]) > 0
        err = row_rel_err(f64(fac[n])[nz], want[nz])
        worst.append(float(err.max()))
        assert err.max() <= tol, (n, err.max())
        for f, b in zip(fac, before):
            f.copy_(b)
    return worst


@pytest.mark.parametrize("slices", [0, 1, 7], ids=["auto", "unsliced", "s7"])
@pytest.mark.parametrize("dims,J,nnz", CASES,
                         ids=["N%d-J%d" % (len(d), j) for d, j, _ in CASES])
def test_sweep_shape_updates_match_oracle(dims, J, nnz, slices):
    p = synth.make_random(dims, J, nnz, seed=12)
    ctx, idx, val, core, fac = context(p, delta_slices=slices)
    worst = check_updates(p, ctx, fac)
    log("sweep shape", dims, J, "slices", slices, "worst per-row error per mode", worst)
    ctx.close()


@pytest.mark.parametrize("slices", [0, 65535], ids=["auto", "capped"])
@pytest.mark.parametrize("dims,ranks", [((12, 10, 9, 8, 7, 6), (2, 3, 4, 3, 2, 5)),
                                        ((40, 30, 20, 10), (3, 4, 6, 20))],
                         ids=["N6-mixed", "N4-mixed"])
def test_sliced_unequal_ranks(dims, ranks, slices):
    p = synth.make_small(dims, ranks, 3000, seed=13, skew=1.1)
    ctx, idx, val, core, fac = context(p, delta_slices=slices)
    check_updates(p, ctx, fac)
    ctx.close()


def test_sliced_rows_across_work_ranges_and_sweep():
    # 64-entry ranges: long rows cross ranges and go through the merge; then
    # a whole ptk_iterate sweep (graph replay) against the oracle's sweep
    p = synth.make_small((30, 6, 5, 40, 5, 4), (3,) * 6, 8000, seed=14, skew=1.3)
    ctx, idx, val, core, fac = context(p, chunk_nnz=64, fuse_error=0)
    check_updates(p, ctx, fac)
    sse, _ = ctx.iterate(1, p.lam, strict=False)
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    v = p.val.astype(np.float64)
    for n in range(p.N):
        A = oracle.update_mode(G, A, p.idx, v, n, p.lam)
        A[n] = A[n].astype(np.float32).astype(np.float64)
    for n in range(p.N):
        nz = np.bincount(p.idx[n], minlength=p.dims[n]) > 0
        assert row_rel_err(f64(fac[n])[nz], A[n][nz]).max() <= 1e-5, n
    want = float(oracle.sse(G, A, p.idx, v))
    assert abs(sse[0] - want) <= 1e-5 * want
    ctx.close()


def test_delta_slices_option_refusals():
    import paper_1710_02261_amd as ptk
    p = synth.make_random((8,) * 6, 3, 300, seed=15)
    ctx = ptk.Context(p.dims, p.ranks)
    for bad in (-1, 65536):
        with pytest.raises(ptk.PtkError, match="PTK_E_INVALID"):
            ctx.set_options(delta_slices=bad)
    ctx.close()
    ctx, *_ = context(p)
    with pytest.raises(ptk.PtkError, match="PTK_E_STATE"):
        ctx.set_options(delta_slices=3)                    # after set_observed
    ctx.close()
