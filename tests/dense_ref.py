"""Dense numpy formulations used to pin the oracle (tests only).

These are written from the definitions of Sec. 2 (Frobenius norm,
matricization, n-mode product, Tucker reconstruction) with numpy's einsum over
whole dense tensors. They share nothing with the oracle's loops and are only
usable on tiny tensors.
"""
import itertools
import string

import numpy as np


def full_tensor(G, A):
    """G x_1 A^(1) ... x_N A^(N) as a dense array (eq. "recon2" for all cells)."""
    N = G.ndim
    core = string.ascii_lowercase[:N]
    outs = string.ascii_uppercase[:N]
    spec = core + "," + ",".join(outs[n] + core[n] for n in range(N)) + "->" + outs
    return np.einsum(spec, G, *A, optimize=True)


def partial_tensor(G, A, n):
    """G x_k A^(k) for all k != n: shape (I_1..J_n..I_N)."""
    N = G.ndim
    core = string.ascii_lowercase[:N]
    outs = list(string.ascii_uppercase[:N])
    outs[n] = core[n]
    ops, specs = [G], [core]
    for k in range(N):
        if k != n:
            ops.append(A[k])
            specs.append(outs[k] + core[k])
    spec = ",".join(specs) + "->" + "".join(outs)
    return np.einsum(spec, *ops, optimize=True)


def deltas(G, A, idx, n):
    """delta^(n)_alpha for every observed alpha, from the dense partial tensor."""
    T = partial_tensor(G, A, n)          # axis n has length J_n
    T = np.moveaxis(T, n, -1)
    others = tuple(idx[k] for k in range(G.ndim) if k != n)
    return T[others]                     # (nnz, J_n)


def unfold(T, n):
    """Mode-n matricization with the column map of Sec. 2.1 (first mode fastest).

    Column of cell (i_1..i_N) = sum_{k != n} i_k * prod_{m < k, m != n} I_m
    (0-based form of the paper's 1-based formula).
    """
    dims = T.shape
    ncols = int(np.prod([d for k, d in enumerate(dims) if k != n]))
    M = np.zeros((dims[n], ncols), dtype=T.dtype)
    for cell in itertools.product(*[range(d) for d in dims]):
        col, stride = 0, 1
        for k in range(len(dims)):
            if k == n:
                continue
            col += cell[k] * stride
            stride *= dims[k]
        M[cell[n], col] = T[cell]
    return M


def loss(G, A, idx, val, lam):
    X = full_tensor(G, A)
    r = val - X[tuple(idx)]
    return float(r @ r + lam * sum(float(np.sum(a * a)) for a in A))
