"""GPU parity of the shared-index units (ptk_options.shared_units): the row
systems (eqs. "rowB", "rowC") formed from units of consecutive entries of a
row that share their index in the last other mode, the core contracted with
that mode's row once per unit (eq. "delta" summed in another order).

* Unit lists: per mode, the numbers of units of 1, 2, 4 and 8 entries, of
  long runs (64 entries or more, whose entries read a table of the core
  contracted with the shared row) and of their tasks equal those of the runs
  of equal (i_n, i_s) counted here from the COO input (exact), for the
  default cap and the caps 2, 4 and 8.
* Row systems to 1e-10 and one mode update to 1e-5 per row against the
  oracle, every unit shape, with work ranges that cut rows; the units and the
  fused kernels give the same row systems to 1e-12.
* Iterations in a captured graph with every row in the least-squares form
  (cond_limit = 1), whose kept deltas then come from the stored ones: every
  row of every iteration to 1e-5 against the oracle from the same state.
* Index tables (G contracted with a row of A^(s), one per value of i_s with
  64 entries or more, single-entry units for the rest):
  groups and tasks counted exactly, row systems, updates and graph
  iterations to the same bars; a mode with no value wide enough for a
  table.
* Auto: the work model keeps the fused kernels when nothing repeats and
  takes the index tables when the values of i_s repeat across rows; an
  empty observed set; option refusals.
"""
import numpy as np
import pytest

import oracle
import synth
from tests.gpu_util import context, f64, log, row_rel_err

pytestmark = pytest.mark.gpu

# (dims, J, nnz): small dims so that (row, i_s) pairs repeat, Zipf skew so
# that run lengths spread from 1 to hundreds
SHAPES = [((40, 30, 20), 16, 6001), ((30, 25, 20, 15), 10, 7003),
          ((12, 11, 10, 9, 8), 8, 5005)]
SIDS = ["%dd-J%d" % (len(d), j) for d, j, _ in SHAPES]


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    assert torch.cuda.is_available()


def problem(dims, J, nnz, seed):
    return synth.make_small(dims, (J,) * len(dims), nnz, seed=seed, skew=1.1)


LONG_RUN, LONG_TASK = 64, 128


def expected_units(p, n, emax):
    """Counters from the runs of equal (i_n, i_s), s the last mode other than
    n: a run of r >= 64 entries is long (one run, ceil(r / 128) tasks); any
    other gives floor(r / emax) units of emax, then the bits of r % emax."""
    N = len(p.dims)
    s = N - 1 if n != N - 1 else N - 2
    key = p.idx[n].astype(np.int64) * p.dims[s] + p.idx[s].astype(np.int64)
    _, runs = np.unique(key, return_counts=True)
    lng = runs >= LONG_RUN
    out = [0] * 6
    out[4] = int(lng.sum())
    out[5] = int(((runs[lng] + LONG_TASK - 1) // LONG_TASK).sum())
    short = runs[~lng]
    cmax = emax.bit_length() - 1
    out[cmax] = int((short // emax).sum())
    rest = short % emax
    for c in range(cmax):
        out[c] = int(((rest >> c) & 1).sum())
    return out


@pytest.mark.parametrize("dims,J,nnz", SHAPES, ids=SIDS)
@pytest.mark.parametrize("cap", [1, 2, 4, 8])
def test_unit_lists_count_runs(dims, J, nnz, cap):
    p = problem(dims, J, nnz, seed=71)
    ctx, *_ = context(p, shared_units=cap)
    emax = 8 if (J <= 10 and len(dims) <= 4) else 4
    emax = min(emax, cap) if cap > 1 else 2
    for n in range(len(dims)):
        counts, on = ctx.unit_stats(n)
        want = expected_units(p, n, emax)
        assert counts[:6] == want and counts[6:] == [0, 0, 0], (n, counts, want)
        assert on == 1
        N = len(dims)
        s = N - 1 if n != N - 1 else N - 2
        key = p.idx[n].astype(np.int64) * dims[s] + p.idx[s]
        _, runs = np.unique(key, return_counts=True)
        in_long = int(runs[runs >= LONG_RUN].sum())
        assert sum((1 << c) * counts[c] for c in range(4)) + in_long == nnz
    ctx.close()


@pytest.mark.parametrize("dims,J,nnz", SHAPES, ids=SIDS)
@pytest.mark.parametrize("form", [1, 16], ids=["units", "index"])
def test_row_systems_with_units_match_oracle(dims, J, nnz, form):
    p = problem(dims, J, nnz, seed=72)
    ctx, *_ = context(p, chunk_nnz=128, shared_units=form)
    ref, *_ = context(p, chunk_nnz=128, shared_units=-1)
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    val = p.val.astype(np.float64)
    for n in range(len(dims)):
        assert ctx.unit_stats(n)[1] == (2 if form == 16 else 1)
        assert ref.unit_stats(n)[1] == 0
        B, c = ctx.row_systems(n)
        B, c = f64(B), f64(c)
        Br, cr = ref.row_systems(n)
        Br, cr = f64(Br), f64(cr)
        scale = np.abs(Br).max()
        assert np.abs(B - Br).max() <= 1e-12 * scale
        assert np.abs(c - cr).max() <= 1e-12 * np.abs(cr).max()
        counts = np.bincount(p.idx[n], minlength=dims[n])
        rows = list(np.argsort(-counts)[:3]) + list(range(0, dims[n], max(1, dims[n] // 7)))
        for i in rows:
            Bo, co = oracle.row_system(G, A, p.idx, val, n, int(i))
            assert np.abs(B[i] - Bo).max() <= 1e-10 * max(np.abs(Bo).max(), 1e-300), (n, i)
            assert np.abs(c[i] - co).max() <= 1e-10 * max(np.abs(co).max(), 1e-300)
    ctx.close()
    ref.close()


@pytest.mark.parametrize("dims,J,nnz", SHAPES, ids=SIDS)
@pytest.mark.parametrize("cap,chunk", [(1, 0), (2, 64), (4, 192), (8, 64), (16, 0), (16, 64)])
def test_update_with_units_matches_oracle(dims, J, nnz, cap, chunk):
    p = problem(dims, J, nnz, seed=73)
    ctx, idx, val, core, fac = context(p, chunk_nnz=chunk, shared_units=cap)
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    v = p.val.astype(np.float64)
    worst = 0.0
    for n in range(p.N):
        before = [f.clone() for f in fac]
        ctx.update_mode(n, p.lam)
        got = f64(fac[n])
        want = oracle.update_rows(G, A, p.idx, v, n, p.lam)
        empty = np.bincount(p.idx[n], minlength=p.dims[n]) == 0
        assert np.all(got[empty] == 0.0)
        err = row_rel_err(got[~empty], want[~empty])
        worst = max(worst, float(err.max()))
        assert err.max() <= 1e-5, (n, err.max())
        for f, b in zip(fac, before):
            f.copy_(b)
    log("units", dims, J, "cap", cap, "chunk", chunk, "worst", worst)
    ctx.close()


@pytest.mark.parametrize("dims,J,nnz", SHAPES, ids=SIDS)
@pytest.mark.parametrize("form", [1, 16], ids=["units", "index"])
def test_graph_iterations_least_squares_from_stored_deltas(dims, J, nnz, form):
    """cond_limit = 1 sends every row to the least-squares form; from the
    second iteration on its deltas are the ones the stored-delta sweep kept."""
    p = problem(dims, J, nnz, seed=74)
    ctx, idx, val, core, fac = context(p, shared_units=form)
    ctx.set_options(cond_limit=1.0, use_graph=1, shared_units=form)
    G = p.core.astype(np.float64)
    v = p.val.astype(np.float64)
    for t in range(3):
        A = [f64(f) for f in fac]
        s1, _ = ctx.iterate(1, p.lam, strict=False)
        for n in range(p.N):
            A = oracle.update_mode(G, A, p.idx, v, n, p.lam)
            A[n] = A[n].astype(np.float32).astype(np.float64)
        worst = 0.0
        for n in range(p.N):
            nz = np.bincount(p.idx[n], minlength=p.dims[n]) > 0
            worst = max(worst, float(row_rel_err(f64(fac[n])[nz], A[n][nz]).max()))
        want = oracle.sse(G, A, p.idx, v)
        rows, _ = ctx.solve_stats()
        log("units least squares", dims, J, "iteration", t, "worst", worst, "ls rows", rows)
        assert rows > 0
        assert worst <= 1e-5
        assert abs(s1[0] - want) <= 1e-6 * want
    ctx.close()


def expected_index(p, n):
    """Index groups: a value of i_s with 64 entries or more has a table and
    ceil(count / 128) tasks, a smaller one a single-entry unit per entry."""
    N = len(p.dims)
    s = N - 1 if n != N - 1 else N - 2
    _, cnt = np.unique(p.idx[s], return_counts=True)
    wide = cnt >= 64
    return [int(wide.sum()), int(((cnt[wide] + 127) // 128).sum()), int(cnt[~wide].sum())]


@pytest.mark.parametrize("dims,J,nnz", SHAPES, ids=SIDS)
def test_index_groups_count_values(dims, J, nnz):
    p = problem(dims, J, nnz, seed=71)
    ctx, *_ = context(p, shared_units=16)
    for n in range(len(dims)):
        counts, on = ctx.unit_stats(n)
        assert on == 2
        assert counts[6:] == expected_index(p, n), (n, counts)
    ctx.close()


def test_index_form_without_tables():
    """Every value of i_s has fewer than 64 entries: no table at all, every
    entry a single-entry unit; row systems as the fused kernels' and one
    update against the oracle."""
    p = problem((30, 25, 20, 15), 10, 120, seed=77)
    ctx, idx, val, core, fac = context(p, shared_units=16)
    ref, *_ = context(p, shared_units=-1)
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    v = p.val.astype(np.float64)
    for n in range(p.N):
        counts, on = ctx.unit_stats(n)
        assert on == 2 and counts[6:] == [0, 0, p.nnz], (n, counts)
        B, c = ctx.row_systems(n)
        Br, cr = ref.row_systems(n)
        B, c, Br, cr = f64(B), f64(c), f64(Br), f64(cr)
        assert np.abs(B - Br).max() <= 1e-12 * np.abs(Br).max()
        assert np.abs(c - cr).max() <= 1e-12 * np.abs(cr).max()
    ctx.update_mode(0, p.lam)
    got = f64(fac[0])
    want = oracle.update_rows(G, A, p.idx, v, 0, p.lam)
    nz = np.bincount(p.idx[0], minlength=p.dims[0]) > 0
    assert row_rel_err(got[nz], want[nz]).max() <= 1e-5
    ctx.close()
    ref.close()


def test_auto_picks_by_the_work_model():
    # 4e4 entries over 10^6 values per mode: nothing repeats enough
    p = synth.make_small((1_000_000,) * 4, (10,) * 4, 40000, seed=75)
    ctx, *_ = context(p)
    for n in range(4):
        counts, on = ctx.unit_stats(n)
        assert on == 0 and counts[0] > 0.9 * p.nnz
    ctx.close()
    # few repeated (row, i_s) pairs, but each i_s value serves 133 entries on
    # average: the index tables win
    p = synth.make_small((300, 300, 300, 300), (10,) * 4, 40000, seed=75)
    ctx, *_ = context(p)
    assert all(ctx.unit_stats(n)[1] == 2 for n in range(4))
    ctx.close()


def test_empty_observed_set_and_refusals():
    import torch
    import paper_1710_02261_amd as ptk
    p = problem((30, 25, 20, 15), 10, 100, seed=76)
    ctx = ptk.Context(p.dims, p.ranks)
    for bad in (3, 5, -2, 32):
        with pytest.raises(ptk.PtkError):
            ctx.set_options(shared_units=bad)
    ctx.set_options(shared_units=1)
    idx = torch.zeros((4, 0), dtype=torch.int32, device="cuda")
    val = torch.zeros((0,), dtype=torch.float32, device="cuda")
    ctx.set_observed(idx, val)
    assert ctx.unit_stats(0) == ([0] * 9, 0)
    with pytest.raises(ptk.PtkError):
        ctx.set_options(shared_units=-1)            # after set_observed
    ctx.close()
