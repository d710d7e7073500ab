"""GPU parity of the steps either side of the fit (through the C ABI):

* min-max normalisation: bitwise equal to the oracle's FP64 scaling rounded to
  FP32, min and max exact; constant values; empty list;
* train/test split: the held-out set and both sides' order exactly as the
  oracle's SplitMix64 rule gives them, for several fractions and seeds,
  ragged tile tails, fractions 0 and 1, and the count mismatch refusal;
* error over an entry list (test RMSE) against the oracle's SSE, 1e-9;
* k-means over a factor's rows against the oracle's Lloyd iterations:
  centroids 1e-9 relative, inertia 1e-9, assignments equal wherever the two
  nearest centroids are not within 1e-9 of a tie; an empty cluster; K = 1;
  iters = 0; the size refusal;
* the whole chain on a small planted tensor: COO file -> read -> split ->
  normalise -> fit on the training side -> test RMSE, against the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import data_steps as ds
from tests.gpu_util import context, f64, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx3():
    import paper_1710_02261_amd as ptk
    import torch
    assert torch.cuda.is_available()
    c = ptk.Context((10, 10, 10), (3, 3, 3))
    yield c
    c.close()


@pytest.mark.parametrize("n", [1, 63, 1000, 300_001])
def test_normalize_matches_oracle(ctx3, n):
    import torch
    rng = np.random.default_rng(n)
    v = (rng.standard_normal(n) * 7 - 3).astype(np.float32)
    t = torch.from_numpy(v).cuda()
    lo, hi = ctx3.normalize_values(t)
    want, (wlo, whi) = ds.normalize(v)
    assert (lo, hi) == (wlo, whi)
    assert np.array_equal(t.cpu().numpy(), want)


def test_normalize_constant_and_empty(ctx3):
    import torch
    t = torch.full((100,), 4.5, dtype=torch.float32, device="cuda")
    assert ctx3.normalize_values(t) == (4.5, 4.5)
    assert torch.all(t == 0)
    assert ctx3.normalize_values(torch.empty(0, dtype=torch.float32, device="cuda")) == (0.0, 0.0)


@pytest.mark.parametrize("nnz,frac,seed", [(1, 0.5, 3), (1023, 0.1, 0), (1025, 0.1, 1),
                                           (200_000, 0.1, 12345), (50_000, 0.37, 2 ** 63 + 5),
                                           (5000, 0.0, 9), (5000, 1.0, 9)])
def test_split_matches_oracle(ctx3, nnz, frac, seed):
    import torch
    rng = np.random.default_rng(nnz)
    N = 3
    idx = rng.integers(0, 10, size=(N, nnz)).astype(np.int32)
    val = rng.standard_normal(nnz).astype(np.float32)
    it, vt, ie, ve = ctx3.split(torch.from_numpy(idx).cuda(), torch.from_numpy(val).cuda(),
                                frac, seed)
    m = ds.held_out(nnz, frac, seed)
    assert np.array_equal(ie.cpu().numpy(), idx[:, m])
    assert np.array_equal(ve.cpu().numpy(), val[m])
    assert np.array_equal(it.cpu().numpy(), idx[:, ~m])
    assert np.array_equal(vt.cpu().numpy(), val[~m])


def test_split_refuses_wrong_count(ctx3):
    import torch
    import ctypes as C
    import paper_1710_02261_amd as ptk
    idx = torch.zeros((3, 100), dtype=torch.int32, device="cuda")
    val = torch.zeros(100, dtype=torch.float32, device="cuda")
    out_i = torch.empty((3, 100), dtype=torch.int32, device="cuda")
    out_v = torch.empty(100, dtype=torch.float32, device="cuda")
    st = ctx3._lib.ptk_split_entries(ctx3._h, 3, 100, C.c_void_p(idx.data_ptr()),
                                     C.c_void_p(val.data_ptr()), 0.5, C.c_uint64(1), 7,
                                     C.c_void_p(out_i.data_ptr()), C.c_void_p(out_v.data_ptr()),
                                     C.c_void_p(out_i.data_ptr()), C.c_void_p(out_v.data_ptr()))
    assert st != 0
    assert "ntest" in ctx3._lib.ptk_last_error(ctx3._h).decode()
    with pytest.raises(ptk.PtkError, match="test_fraction"):
        ctx3.split(idx, val, 1.5, 0)


def test_entry_error_matches_oracle():
    import torch
    p = synth.make_small((40, 35, 30), (5, 5, 5), 6000, seed=61)
    ctx, idx, val, core, fac = context(p)
    rng = np.random.default_rng(61)
    m = 3001
    q = np.stack([rng.integers(0, d, m) for d in p.dims]).astype(np.int32)
    x = rng.standard_normal(m).astype(np.float32)
    sse, rmse = ctx.entry_error(torch.from_numpy(q).cuda(), torch.from_numpy(x).cuda())
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    want = float(oracle.sse(G, A, q, x.astype(np.float64)))
    assert abs(sse - want) <= 1e-9 * want
    assert abs(rmse - np.sqrt(want / m)) <= 1e-9 * rmse
    assert ctx.entry_error(torch.zeros((3, 0), dtype=torch.int32, device="cuda"),
                           torch.zeros(0, dtype=torch.float32, device="cuda")) == (0.0, 0.0)
    ctx.close()


def _kmeans_case(dims, ranks, n, K, iters, seed, planted=True):
    import torch
    p = synth.make_small(dims, ranks, 2000, seed=seed)
    rng = np.random.default_rng(seed)
    A = p.factors[n]
    if planted:                                   # rows around K planted centres
        cent = rng.standard_normal((K, ranks[n])) * 3
        lab = rng.integers(0, K, len(A))
        A[:] = (cent[lab] + rng.standard_normal(A.shape) * 0.5).astype(np.float32)
    ctx, idx, val, core, fac = context(p)
    C0 = A[rng.choice(len(A), K, replace=False)].astype(np.float64)
    Cg = torch.from_numpy(C0.copy()).cuda()
    assign, inertia, changed = ctx.kmeans(n, Cg, iters)
    Cw, aw, iw, chw, _ = ds.kmeans(A.astype(np.float64), C0, iters)
    np.testing.assert_allclose(Cg.cpu().numpy(), Cw, rtol=1e-9, atol=1e-12)
    assert abs(inertia - iw) <= 1e-9 * max(iw, 1e-30)
    got = assign.cpu().numpy()
    _, _, d = ds.assign_rows(A.astype(np.float64), Cw)
    s = np.sort(d, axis=1)
    tie = (s[:, 1] - s[:, 0]) <= 1e-9 * np.maximum(s[:, 1], 1e-30) if K > 1 else np.zeros(len(A), bool)
    assert np.array_equal(got[~tie], aw[~tie])
    log("kmeans", dims, "mode", n, "K", K, "iters", iters, "inertia", inertia, "changed",
        changed, "oracle", chw, "ties", int(tie.sum()))
    ctx.close()
    return changed, chw


@pytest.mark.parametrize("dims,ranks,n,K,iters", [
    ((3000, 40, 30), (8, 8, 8), 0, 6, 8),
    ((100000, 40, 30), (10, 10, 10), 0, 20, 5),
    ((500, 300, 20), (5, 16, 4), 1, 12, 10),
    ((500, 300, 20), (5, 16, 4), 2, 1, 3),
    ((700, 50, 20), (3, 3, 3), 0, 9, 0),
])
def test_kmeans_matches_oracle(dims, ranks, n, K, iters):
    _kmeans_case(dims, ranks, n, K, iters, seed=62 + K)


def test_kmeans_empty_cluster_and_refusal():
    import torch
    import paper_1710_02261_amd as ptk
    p = synth.make_small((300, 20, 20), (4, 4, 4), 1000, seed=63)
    ctx, idx, val, core, fac = context(p)
    A = p.factors[0].astype(np.float64)
    C0 = np.concatenate([A[:3], np.full((1, 4), 1e6)])   # the far centroid gets no rows
    Cg = torch.from_numpy(C0.copy()).cuda()
    assign, inertia, _ = ctx.kmeans(0, Cg, 4)
    Cw, aw, iw, _, _ = ds.kmeans(A, C0, 4)
    assert np.all(Cg.cpu().numpy()[3] == 1e6) and np.all(Cw[3] == 1e6)
    np.testing.assert_allclose(Cg.cpu().numpy(), Cw, rtol=1e-9)
    with pytest.raises(ptk.PtkError, match="K must be"):
        ctx.kmeans(0, torch.zeros((2000, 4), dtype=torch.float64, device="cuda"), 1)
    ctx.close()


def test_chain_file_split_normalize_fit_test_rmse(tmp_path):
    import torch
    import paper_1710_02261_amd as ptk
    p = synth.make_small((60, 50, 40), (4, 4, 4), 20000, seed=64)
    path = tmp_path / "x.tns"
    with open(path, "w") as f:
        for e in range(p.nnz):
            f.write("%d %d %d %r\n" % (p.idx[0, e] + 1, p.idx[1, e] + 1, p.idx[2, e] + 1,
                                       float(p.val[e])))
    nnz, dims = ptk.coo_scan(str(path), 3)
    idx_h, val_h = ptk.coo_read(str(path), 3, nnz)
    assert np.array_equal(idx_h, p.idx) and np.array_equal(val_h, p.val)
    ctx = ptk.Context(p.dims, p.ranks)
    idx, val = torch.from_numpy(idx_h).cuda(), torch.from_numpy(val_h).cuda()
    lo, hi = ctx.normalize_values(val)
    vn, _ = ds.normalize(val_h)
    assert np.array_equal(val.cpu().numpy(), vn)
    it, vt, ie, ve = ctx.split(idx, val, 0.1, 2024)
    m = ds.held_out(nnz, 0.1, 2024)
    ctx.set_options(fuse_error=0)
    ctx.set_observed(it, vt)
    core = torch.from_numpy(p.core).cuda()
    fac = [torch.from_numpy(a).cuda() for a in p.factors]
    ctx.bind_model(core, fac)
    ctx.iterate(3, p.lam, strict=False)
    sse, rmse = ctx.entry_error(ie, ve)
    # the oracle's sweeps, its factors rounded to FP32 after each mode as the
    # library stores them
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    tr_idx, tr_val = np.ascontiguousarray(p.idx[:, ~m]), vn[~m].astype(np.float64)
    for _ in range(3):
        for n in range(3):
            A = oracle.update_mode(G, A, tr_idx, tr_val, n, p.lam)
            A[n] = A[n].astype(np.float32).astype(np.float64)
    want = float(oracle.sse(G, A, np.ascontiguousarray(p.idx[:, m]), vn[m].astype(np.float64)))
    log("chain: test RMSE", rmse, "oracle", np.sqrt(want / m.sum()))
    assert abs(sse - want) <= 1e-5 * want
    ctx.close()
