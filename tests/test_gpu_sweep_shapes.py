"""GPU parity on the shapes of the paper's synthetic scalability sweeps
(Sec. 4.2) that run on the generic row-system kernel: orders 6 to 10 with
J = 3, and ranks 7, 9 and 11 at order 3. Random tensors as in the paper
(values U[0,1) at uniform cells, U[0,1) initial model), small enough for
the oracle. Bar: one mode update per mode, per-row relative error <= 1e-5.
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


@pytest.mark.parametrize("dims,J,nnz", CASES,
                         ids=["N%d-J%d" % (len(d), j) for d, j, _ in CASES])
def test_sweep_shape_updates_match_oracle(dims, J, nnz):
    p = synth.make_random(dims, J, nnz, seed=12)
    ctx, idx, val, core, fac = context(p)
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
        assert err.max() <= 1e-5, (n, err.max())
        for f, b in zip(fac, before):
            f.copy_(b)
    log("sweep shape", dims, J, "worst per-row error per mode", worst)
    ctx.close()
