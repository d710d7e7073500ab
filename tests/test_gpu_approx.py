"""GPU parity of the Approx variant (Alg. 4, Sec. 3.3).

* R(beta) (eq. "recon_partial") for every core cell against the oracle,
  which evaluates the definition (the difference of the two squared
  residuals, entry by entry). That form loses about eps * SSE to
  cancellation, so the bound is |R_gpu - R_oracle| <= 1e-9 (SSE + |R|).
* The removal: the same number of cells (floor(p * nz)), and the same cells
  except where R lies within that bound of the cut (the ranking is a
  floating-point decision; such cells may go either way, and the test checks
  that what each side removed is valid for its own values).
* Iterations of Alg. 2 with the removal inside the captured graph: each
  iteration from the same state as the oracle (the oracle replays it with
  its factors rounded to float32 after each mode, as the library stores
  them), factors per row 1e-5, error 1e-5, removed cells as above; the
  states are then synchronised for the next iteration.
* Graph replay equals launching kernels one by one; a rate that removes
  nothing leaves the plain path; refusals.
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


SHAPES = [((30, 25, 20), 3), ((30, 25, 20), 5), ((40, 30, 20), 8), ((30, 25, 20), 10),
          ((30, 25, 20), 16), ((12, 11, 10, 9), 3), ((12, 11, 10, 9), 5),
          ((12, 11, 10, 9), 8), ((12, 11, 10, 9), 10), ((8, 7, 6, 5, 4), 3),
          ((8, 7, 6, 5, 4), 5), ((8, 7, 6, 5, 4), 8)]


def ids():
    return ["%dd-J%d" % (len(d), j) for d, j in SHAPES]


def problem(dims, J, seed, nnz=2500):
    return synth.make_small(dims, (J,) * len(dims), nnz, seed=seed, skew=1.1)


def model64(p):
    return p.core.astype(np.float64), [a.astype(np.float64) for a in p.factors]


def check_removal(G_before, G_gpu, R, sse, p):
    """Same count; same cells up to near-ties at the cut."""
    nz = G_before != 0.0
    k = int(np.floor(p * np.count_nonzero(nz)))
    rem_gpu = nz & (G_gpu == 0.0)
    assert np.count_nonzero(rem_gpu) == k
    kept = ~rem_gpu
    np.testing.assert_array_equal(G_gpu[kept], G_before[kept])
    if k == 0:
        return
    tol = 1e-9 * (sse + np.abs(R).max())
    flat = R[nz]
    cut = np.sort(flat)[::-1][k - 1]
    clear_in = nz & (R > cut + tol)
    clear_out = nz & (R < cut - tol)
    assert np.all(rem_gpu[clear_in]) and not np.any(rem_gpu[clear_out])


FORMS = [(d, j, 0) for d, j in SHAPES] + [(d, j, 1) for d, j in SHAPES if len(d) >= 4]


@pytest.mark.parametrize("dims,J,form", FORMS,
                         ids=["%dd-J%d-form%d" % (len(d), j, f) for d, j, f in FORMS])
def test_partial_error_matches_oracle(dims, J, form):
    """form 0 (auto) takes the row sums at orders 4 and 5, form 1 the
    per-cell groups."""
    p = problem(dims, J, seed=51)
    ctx, idx, val, core, fac = context(p)
    ctx.set_options(approx_form=form)
    R = ctx.partial_error().cpu().numpy()
    G, A = model64(p)
    v = p.val.astype(np.float64)
    want = oracle.partial_error(G, A, p.idx, v)
    sse = oracle.sse(G, A, p.idx, v)
    err = np.abs(R - want).max()
    log("partial error", dims, J, "max abs diff %.3g, SSE %.3g, max|R| %.3g"
        % (err, sse, np.abs(want).max()))
    assert err <= 1e-9 * (sse + np.abs(want).max())
    ctx.close()


@pytest.mark.parametrize("dims,J", SHAPES[::2], ids=ids()[::2])
@pytest.mark.parametrize("rate", [0.2, 0.55])
def test_truncate_matches_oracle_ranking(dims, J, rate):
    p = problem(dims, J, seed=52)
    ctx, idx, val, core, fac = context(p)
    G, A = model64(p)
    v = p.val.astype(np.float64)
    R = oracle.partial_error(G, A, p.idx, v)
    k = ctx.truncate(rate)
    G_gpu = core.cpu().numpy().astype(np.float64)
    assert k == int(np.floor(rate * np.count_nonzero(G)))
    check_removal(G, G_gpu, R, oracle.sse(G, A, p.idx, v), rate)
    # a second removal counts only the cells left
    k2 = ctx.truncate(rate)
    assert k2 == int(np.floor(rate * np.count_nonzero(G_gpu)))
    ctx.close()


@pytest.mark.parametrize("dims,J", [((30, 25, 20), 5), ((12, 11, 10, 9), 8),
                                    ((8, 7, 6, 5, 4), 3), ((12, 11, 10, 9), 10),
                                    ((8, 7, 6, 5, 4), 8)])
def test_approx_iterations_match_oracle(dims, J):
    """At (4, 10) and (5, 8) the last mode has the fewest rows and its
    two-entry row-system kernel keeps the deltas the residuals are formed
    from; the other shapes recompute them."""
    import torch
    p = problem(dims, J, seed=53, nnz=4000)
    ctx, idx, val, core, fac = context(p, profile=1)
    ctx.set_options(fuse_error=0, approx_rate=0.2, profile=1, use_graph=0)
    v = p.val.astype(np.float64)
    n_left = core.numel()
    for t in range(3):
        G = core.cpu().numpy().astype(np.float64)
        A = [f64(f) for f in fac]
        sse, _ = ctx.iterate(1, p.lam, strict=False)
        # the oracle replays the iteration from the same state
        for n in range(len(dims)):
            A = oracle.update_mode(G, A, p.idx, v, n, p.lam)
            A[n] = A[n].astype(np.float32).astype(np.float64)
        want_sse = oracle.sse(G, A, p.idx, v)
        R = oracle.partial_error(G, A, p.idx, v)
        for n in range(len(dims)):
            nz = np.bincount(p.idx[n], minlength=dims[n]) > 0
            assert row_rel_err(f64(fac[n])[nz], A[n][nz]).max() <= 1e-5
        assert abs(sse[0] - want_sse) <= 1e-5 * want_sse
        G_gpu = core.cpu().numpy().astype(np.float64)
        check_removal(G, G_gpu, R, want_sse, 0.2)
        n_left -= int(np.floor(0.2 * n_left))
        assert np.count_nonzero(G_gpu) == n_left
        log("approx iteration", t, "sse", sse[0], "core cells left", n_left)
        kept = "approx_resid_kept" in ctx.kernel_times()
        assert kept == ((len(dims), J) in ((4, 10), (5, 8)))
        # continue both from the oracle's state
        Go, _ = oracle.truncate(G, R, 0.2)
        core.copy_(torch.from_numpy(Go.astype(np.float32)))
        for f, a in zip(fac, A):
            f.copy_(torch.from_numpy(a.astype(np.float32)))
    ctx.close()


def test_approx_graph_replay_bitwise():
    import torch
    p = problem((30, 25, 20, 15), 5, seed=54, nnz=5000)
    cg, _, _, core_g, fg = context(p)
    ce, _, _, core_e, fe = context(p)
    cg.set_options(use_graph=1, approx_rate=0.2)
    ce.set_options(use_graph=0, approx_rate=0.2)
    for call in range(3):
        sg, lg = cg.iterate(2, p.lam, strict=False)
        torch.cuda.synchronize()
        se, le = ce.iterate(2, p.lam, strict=False)
        torch.cuda.synchronize()
        assert np.array_equal(sg, se) and np.array_equal(lg, le), call
        assert torch.equal(core_g, core_e), call
        for a, b in zip(fg, fe):
            assert torch.equal(a, b), call
    cg.close()
    ce.close()


def test_rate_removing_nothing_is_plain_path():
    import torch
    p = problem((30, 25, 20), 8, seed=55)
    ca, _, _, core_a, fa = context(p)
    cp, _, _, core_p, fp = context(p)
    ca.set_options(approx_rate=1e-4)       # floor(1e-4 * 512) = 0
    sa, _ = ca.iterate(3, p.lam, strict=False)
    sp, _ = cp.iterate(3, p.lam, strict=False)
    assert np.array_equal(sa, sp)
    assert torch.equal(core_a, core_p)
    for a, b in zip(fa, fp):
        assert torch.equal(a, b)
    ca.close()
    cp.close()


@pytest.mark.parametrize("dims,J", [((40, 30, 20, 6), 5), ((9, 8, 7, 7, 6), 3),
                                    ((60, 50, 40, 8), 10), ((10, 9, 8, 7, 5), 8)])
def test_row_sum_form_equals_cell_groups(dims, J):
    """The two forms of S1, S2 give R equal up to rounding order, on entries
    whose grouping mode (the last, fewest rows) has empty rows and one row
    holding most entries, so that row pieces cross many slices."""
    rng = np.random.default_rng(57)
    p = problem(dims, J, seed=57, nnz=6000)
    last = len(dims) - 1
    used = np.array([0, 2, dims[last] - 1])
    p.idx[last] = used[np.minimum(rng.geometric(0.25, p.idx.shape[1]) - 1, 2)]
    G, A = model64(p)
    v = p.val.astype(np.float64)
    Rs = []
    for form in (2, 1):
        ctx, idx, val, core, fac = context(p)
        ctx.set_options(approx_form=form)
        Rs.append(ctx.partial_error().cpu().numpy())
        ctx.close()
    want = oracle.partial_error(G, A, p.idx, v)
    sse = oracle.sse(G, A, p.idx, v)
    scale = sse + np.abs(want).max()
    log("row sums vs cell groups", dims, J, "diff %.3g, vs oracle %.3g, scale %.3g"
        % (np.abs(Rs[0] - Rs[1]).max(), np.abs(Rs[0] - want).max(), scale))
    assert np.abs(Rs[0] - Rs[1]).max() <= 1e-12 * scale
    assert np.abs(Rs[0] - want).max() <= 1e-9 * scale


def test_approx_refusals():
    import paper_1710_02261_amd as ptk
    p = problem((20, 20, 20), 4, seed=56, nnz=500)
    ctx, *_ = context(p)
    for bad in (1.0, -0.1, float("nan")):
        with pytest.raises(ptk.PtkError, match="PTK_E_INVALID"):
            ctx.set_options(approx_rate=bad)
    with pytest.raises(ptk.PtkError, match="PTK_E_INVALID"):
        ctx.truncate(1.5)
    with pytest.raises(ptk.PtkError, match="PTK_E_INVALID"):
        ctx.set_options(approx_form=3)
    ctx.set_options(approx_form=2)          # order 3: no row-sum form
    with pytest.raises(ptk.PtkError, match="PTK_E_UNSUPPORTED"):
        ctx.partial_error()
    ctx.close()
    ctx = ptk.Context((20, 20, 20), (3, 2, 4))
    with pytest.raises(ptk.PtkError, match="PTK_E_UNSUPPORTED"):
        ctx.set_options(approx_rate=0.2)
    ctx.close()
    ctx = ptk.Context((6,) * 6, (3,) * 6)
    with pytest.raises(ptk.PtkError, match="PTK_E_UNSUPPORTED"):
        ctx.set_options(approx_rate=0.2)
    ctx.close()
