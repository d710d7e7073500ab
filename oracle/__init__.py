"""FP64 CPU oracle for P-Tucker's row-wise ALS (ctypes front end).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product. It wraps the plain C file
``ptk_oracle.c`` (double precision, loops written from the paper's
definitions) and shares no code with the GPU library. Inputs are numpy arrays;
float32 inputs are widened to float64 exactly.

Functions and the passages they follow:

* ``delta``          -- eq. "delta" (Sec. 3.2), plain core-cell loop.
* ``predict``        -- eq. "recon2" (Sec. 2.2).
* ``sse`` / ``loss`` -- eq. "reconfull" squared / eq. "TF_PARTIAL".
* ``row_system``     -- eqs. "rowB", "rowC" for one row.
* ``solve``          -- eq. "rowupdate" as a Cholesky solve of a formed system.
* ``ls_solve``       -- eq. "rowupdate" as the regularised least-squares
  problem it is the normal equations of (Givens QR of the stacked matrix).
* ``update_rows`` / ``update_mode`` -- Alg. 3 for one mode, each row by the
  least-squares form (defined for every row and lambda > 0).
* ``fit``            -- Alg. 2 iterations (factor sweeps + error).
* ``partial_error`` / ``truncate`` / ``fit_approx`` -- the Approx variant
  (Alg. 4, eq. "recon_partial"): per-cell partial reconstruction error,
  removal of the top floor(p |G|) cells, Alg. 2 with the removal.
* ``fit_cached``     -- the same with the Cache variant of Alg. 3 (Sec. 3.3):
  table Pres, delta by division, rescale after each mode, plain products
  where a factor element is zero.
* ``qr`` / ``core_update`` / ``orthogonalize`` -- Alg. 2's final QR and core
  update (Sec. 3.1, n-mode product of Sec. 2.1).
* ``fold_in``        -- the row update for a new row with the model fixed.
* ``data_steps``     -- (numpy) the steps either side of the fit: SplitMix64
  train/test split, min-max normalisation, k-means over factor rows.

The C file is built with ``-O3`` for the host it runs on (``-march=native``)
and OpenMP: the rows of a mode are dealt to threads dynamically (Sec. 3.4),
each row computed by one thread in a fixed order, so results do not depend
on the thread count (``set_threads``). The library file name carries a tag of
the host CPU, so a copy built on another machine is never loaded.
"""
from __future__ import annotations

import ctypes as C
import hashlib
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ptk_oracle.c")
_FLAGS = ["-O3", "-march=native", "-fopenmp", "-std=c99", "-shared", "-fPIC"]
_lib = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)
_dpp = C.POINTER(_dp)


def host_cpu():
    """Model name and logical CPU count of this host (from /proc/cpuinfo)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count() or 1


def _lib_path():
    h = hashlib.sha1()
    with open(_SRC, "rb") as f:
        h.update(f.read())
    h.update(" ".join(_FLAGS).encode())
    h.update(host_cpu()[0].encode())
    try:     # the instruction-set flags, so -march=native matches this host
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("flags"):
                    h.update(line.encode())
                    break
    except OSError:
        pass
    return os.path.join(_HERE, "libptk_oracle_%s.so" % h.hexdigest()[:12])


def build(force: bool = False) -> str:
    """Compile the oracle with the host C compiler for this host's CPU."""
    lib = _lib_path()
    if force or not os.path.exists(lib):
        tmp = lib + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", *_FLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, lib)
    return lib


def _load(path=None):
    global _lib
    if _lib is not None and path is None:
        return _lib
    if path is None:
        path = os.environ.get("PTK_ORACLE_LIB")   # mutation tests only
    if path is None:
        path = build()
    lib = C.CDLL(path)
    sig = {
        "ora_delta": (None, [C.c_int, _ip, _dp, _dpp, C.c_int, _dp]),
        "ora_predict_one": (C.c_double, [C.c_int, _ip, _dp, _dpp]),
        "ora_predict": (None, [C.c_int, _ip, _dp, _dpp, C.c_int64, _ip, _dp]),
        "ora_sse": (C.c_double, [C.c_int, _ip, _dp, _dpp, C.c_int64, _ip, _dp]),
        "ora_loss": (C.c_double, [C.c_int, _lp, _ip, _dp, _dpp, C.c_int64, _ip,
                                  _dp, C.c_double]),
        "ora_solve": (C.c_int, [C.c_int, _dp, _dp, C.c_double, _dp]),
        "ora_ls_solve": (C.c_int, [C.c_int, C.c_int64, _dp, _dp, C.c_double, _dp]),
        "ora_set_threads": (C.c_int, [C.c_int]),
        "ora_row_system": (C.c_int, [C.c_int, _ip, _dp, _dpp, C.c_int64, _ip,
                                     _dp, C.c_int, C.c_int32, _dp, _dp]),
        "ora_update_rows": (C.c_int64, [C.c_int, _lp, _ip, _dp, _dpp, C.c_int64,
                                        _ip, _dp, C.c_int, C.c_double, C.c_int64,
                                        _ip, _dp]),
        "ora_update_mode": (C.c_int64, [C.c_int, _lp, _ip, _dp, _dpp, C.c_int64,
                                        _ip, _dp, C.c_int, C.c_double]),
        "ora_fit": (C.c_int64, [C.c_int, _lp, _ip, _dp, _dpp, C.c_int64, _ip,
                                _dp, C.c_double, C.c_int, _dp, _dp]),
        "ora_fit_cached": (C.c_int64, [C.c_int, _lp, _ip, _dp, _dpp, C.c_int64,
                                       _ip, _dp, C.c_double, C.c_int, _dp]),
        "ora_partial_error": (C.c_int, [C.c_int, _ip, _dp, _dpp, C.c_int64, _ip,
                                        _dp, _dp]),
        "ora_truncate": (C.c_int64, [C.c_int, _ip, _dp, _dp, C.c_double]),
        "ora_fit_approx": (C.c_int64, [C.c_int, _lp, _ip, _dp, _dpp, C.c_int64,
                                       _ip, _dp, C.c_double, C.c_int, C.c_double,
                                       _dp, _lp]),
        "ora_qr": (C.c_int, [C.c_int64, C.c_int, _dp, _dp]),
        "ora_core_update": (C.c_int, [C.c_int, _ip, _dp, C.c_int, _dp]),
        "ora_orthogonalize": (C.c_int, [C.c_int, _lp, _ip, _dp, _dpp, _dp]),
        "ora_fold_in": (C.c_int, [C.c_int, _ip, _dp, _dpp, C.c_int, C.c_int64,
                                  _ip, _dp, C.c_double, _dp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def use_library(path):
    """Point this module at another build of the oracle (mutation tests only).

    Returns the previously loaded library handle so the caller can restore it
    with ``restore_library``.
    """
    global _lib
    prev = _lib
    _lib = None
    _load(path)
    return prev


def restore_library(prev):
    global _lib
    _lib = prev


# ----------------------------------------------------------------------------
# marshalling
# ----------------------------------------------------------------------------
def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


def _i(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(_ip)


def _l(a):
    a = np.ascontiguousarray(a, dtype=np.int64)
    return a, a.ctypes.data_as(_lp)


def _ptrs(mats):
    keep = [np.ascontiguousarray(m, dtype=np.float64) for m in mats]
    arr = (_dp * len(keep))(*[k.ctypes.data_as(_dp) for k in keep])
    return keep, arr


def _shape(G, A):
    J = np.array(G.shape, dtype=np.int32)
    I = np.array([a.shape[0] for a in A], dtype=np.int64)
    for a, j in zip(A, J):
        if a.shape[1] != j:
            raise ValueError("factor width does not match the core")
    return I, J


# ----------------------------------------------------------------------------
# public functions
# ----------------------------------------------------------------------------
def delta(G, rows, n):
    """delta^(n) for one entry; rows[k] is the factor row a^(k)_{i_k}."""
    lib = _load()
    G, Gp = _d(G)
    J, Jp = _i(np.array(G.shape))
    rows = [np.asarray(r, dtype=np.float64) if k != n else np.zeros(J[k])
            for k, r in enumerate(rows)]
    keep, rp = _ptrs(rows)
    out = np.zeros(J[n])
    lib.ora_delta(len(J), Jp, Gp, rp, int(n), out.ctypes.data_as(_dp))
    return out


def predict(G, A, idx):
    lib = _load()
    G, Gp = _d(G)
    I, J = _shape(G, A)
    J, Jp = _i(J)
    keep, Ap = _ptrs(A)
    idx, ip = _i(idx)
    out = np.zeros(idx.shape[1])
    lib.ora_predict(len(J), Jp, Gp, Ap, idx.shape[1], ip, out.ctypes.data_as(_dp))
    return out


def sse(G, A, idx, val):
    lib = _load()
    G, Gp = _d(G)
    I, J = _shape(G, A)
    J, Jp = _i(J)
    keep, Ap = _ptrs(A)
    idx, ip = _i(idx)
    val, vp = _d(val)
    return lib.ora_sse(len(J), Jp, Gp, Ap, idx.shape[1], ip, vp)


def loss(G, A, idx, val, lam):
    lib = _load()
    G, Gp = _d(G)
    I, J = _shape(G, A)
    I, Ip = _l(I)
    J, Jp = _i(J)
    keep, Ap = _ptrs(A)
    idx, ip = _i(idx)
    val, vp = _d(val)
    return lib.ora_loss(len(J), Ip, Jp, Gp, Ap, idx.shape[1], ip, vp, float(lam))


def row_system(G, A, idx, val, n, row):
    """(B, c) of eqs. rowB/rowC for row ``row`` of mode ``n``."""
    lib = _load()
    G, Gp = _d(G)
    I, J = _shape(G, A)
    J, Jp = _i(J)
    keep, Ap = _ptrs(A)
    idx, ip = _i(idx)
    val, vp = _d(val)
    B = np.zeros((J[n], J[n]))
    c = np.zeros(J[n])
    rc = lib.ora_row_system(len(J), Jp, Gp, Ap, idx.shape[1], ip, vp, int(n),
                            int(row), B.ctypes.data_as(_dp), c.ctypes.data_as(_dp))
    if rc:
        raise RuntimeError("ora_row_system failed: %d" % rc)
    return B, c


def solve(B, c, lam):
    lib = _load()
    B, Bp = _d(B)
    c, cp = _d(c)
    a = np.zeros(c.shape[0])
    rc = lib.ora_solve(c.shape[0], Bp, cp, float(lam), a.ctypes.data_as(_dp))
    if rc:
        raise np.linalg.LinAlgError("B + lambda I is not positive definite")
    return a


def ls_solve(Delta, x, lam):
    """Solution of min ||x - Delta a||^2 + lam ||a||^2, i.e. of
    (Delta^T Delta + lam I) a = Delta^T x (eq. "rowupdate" with the entries'
    deltas as the rows of Delta), by the oracle's Givens QR."""
    lib = _load()
    Delta, Dp = _d(np.atleast_2d(Delta))
    x, xp = _d(x)
    a = np.zeros(Delta.shape[1])
    rc = lib.ora_ls_solve(Delta.shape[1], Delta.shape[0], Dp, xp, float(lam),
                          a.ctypes.data_as(_dp))
    if rc:
        raise RuntimeError("ora_ls_solve failed: %d" % rc)
    return a


def set_threads(t=0):
    """Threads of the row updates and residuals (0: leave as is). Returns the
    count in effect (1 when the oracle was built without OpenMP)."""
    return int(_load().ora_set_threads(int(t)))


def update_rows(G, A, idx, val, n, lam, rows=None, return_bad=False):
    """New values of the requested rows of A^(n) (all rows when None).

    Every row is solved by the least-squares form of eq. "rowupdate"; with
    return_bad=True the number of rows whose result is not finite (zero for
    finite inputs and lam > 0) is returned too."""
    lib = _load()
    G, Gp = _d(G)
    I, J = _shape(G, A)
    I, Ip = _l(I)
    J, Jp = _i(J)
    keep, Ap = _ptrs(A)
    idx, ip = _i(idx)
    val, vp = _d(val)
    if rows is None:
        out = np.zeros((I[n], J[n]))
        rp, nreq = None, 0
    else:
        rows, rp = _i(rows)
        nreq = rows.shape[0]
        out = np.zeros((nreq, J[n]))
    bad = lib.ora_update_rows(len(J), Ip, Jp, Gp, Ap, idx.shape[1], ip, vp,
                              int(n), float(lam), nreq, rp,
                              out.ctypes.data_as(_dp))
    if bad < 0:
        raise RuntimeError("ora_update_rows failed: %d" % bad)
    return (out, int(bad)) if return_bad else out


def update_mode(G, A, idx, val, n, lam):
    """Alg. 3 for mode n; returns a new list of factors."""
    A = [np.array(a, dtype=np.float64) for a in A]
    A[n] = update_rows(G, A, idx, val, n, lam)
    return A


def fit(G, A, idx, val, lam, iters):
    """Alg. 2 iterations. Returns (factors, loss after each mode, SSE per iter)."""
    lib = _load()
    G, Gp = _d(G)
    I, J = _shape(G, A)
    I, Ip = _l(I)
    J, Jp = _i(J)
    A = [np.array(a, dtype=np.float64) for a in A]
    arr = (_dp * len(A))(*[a.ctypes.data_as(_dp) for a in A])
    idx, ip = _i(idx)
    val, vp = _d(val)
    N = len(J)
    L = np.zeros(iters * N)
    S = np.zeros(iters)
    bad = lib.ora_fit(N, Ip, Jp, Gp, arr, idx.shape[1], ip, vp, float(lam),
                      int(iters), L.ctypes.data_as(_dp), S.ctypes.data_as(_dp))
    if bad < 0:
        raise RuntimeError("ora_fit failed: %d" % bad)
    return A, L.reshape(iters, N), S


def fit_cached(G, A, idx, val, lam, iters):
    """Alg. 2 iterations with the Cache variant. Returns (factors, SSE per iter)."""
    lib = _load()
    G, Gp = _d(G)
    I, J = _shape(G, A)
    I, Ip = _l(I)
    J, Jp = _i(J)
    A = [np.array(a, dtype=np.float64) for a in A]
    arr = (_dp * len(A))(*[a.ctypes.data_as(_dp) for a in A])
    idx, ip = _i(idx)
    val, vp = _d(val)
    S = np.zeros(iters)
    bad = lib.ora_fit_cached(len(J), Ip, Jp, Gp, arr, idx.shape[1], ip, vp, float(lam),
                             int(iters), S.ctypes.data_as(_dp))
    if bad < 0:
        raise RuntimeError("ora_fit_cached failed: %d" % bad)
    return A, S


def partial_error(G, A, idx, val):
    """R(beta) of eq. "recon_partial" for every core cell (shape of G)."""
    lib = _load()
    G, Gp = _d(G)
    I, J = _shape(G, A)
    J, Jp = _i(J)
    A = [np.ascontiguousarray(a, dtype=np.float64) for a in A]
    arr = (_dp * len(A))(*[a.ctypes.data_as(_dp) for a in A])
    idx, ip = _i(idx)
    val, vp = _d(val)
    R = np.zeros(G.shape)
    rc = lib.ora_partial_error(len(J), Jp, Gp, arr, idx.shape[1], ip, vp,
                               R.ctypes.data_as(_dp))
    if rc:
        raise RuntimeError("ora_partial_error failed: %d" % rc)
    return R


def truncate(G, R, p):
    """Alg. 4's removal on a copy of G. Returns (G', number removed)."""
    lib = _load()
    G = np.array(G, dtype=np.float64)
    J, Jp = _i(np.array(G.shape))
    R, Rp = _d(R)
    k = lib.ora_truncate(len(J), Jp, G.ctypes.data_as(_dp), Rp, float(p))
    if k < 0:
        raise RuntimeError("ora_truncate failed: %d" % k)
    return G, int(k)


def fit_approx(G, A, idx, val, lam, iters, p):
    """Alg. 2 with Alg. 4 each iteration. Returns (G, factors, SSE per iter
    (before the removal), non-zero core cells left after each iteration)."""
    lib = _load()
    G = np.array(G, dtype=np.float64)
    I, J = _shape(G, A)
    I, Ip = _l(I)
    J, Jp = _i(J)
    A = [np.array(a, dtype=np.float64) for a in A]
    arr = (_dp * len(A))(*[a.ctypes.data_as(_dp) for a in A])
    idx, ip = _i(idx)
    val, vp = _d(val)
    S = np.zeros(iters)
    C_ = np.zeros(iters, dtype=np.int64)
    bad = lib.ora_fit_approx(len(J), Ip, Jp, G.ctypes.data_as(_dp), arr, idx.shape[1],
                             ip, vp, float(lam), int(iters), float(p),
                             S.ctypes.data_as(_dp), C_.ctypes.data_as(_lp))
    if bad < 0:
        raise RuntimeError("ora_fit_approx failed: %d" % bad)
    return G, A, S, C_


def qr(A):
    """Thin Householder QR with diag(R) >= 0. Returns (Q, R)."""
    lib = _load()
    Q = np.array(A, dtype=np.float64)
    R = np.zeros((Q.shape[1], Q.shape[1]))
    rc = lib.ora_qr(Q.shape[0], Q.shape[1], Q.ctypes.data_as(_dp),
                    R.ctypes.data_as(_dp))
    if rc:
        raise ValueError("ora_qr failed: %d" % rc)
    return Q, R


def core_update(G, n, U):
    """G x_n U with the n-mode product of Sec. 2.1."""
    lib = _load()
    G = np.array(G, dtype=np.float64)
    J, Jp = _i(np.array(G.shape))
    U, Up = _d(U)
    rc = lib.ora_core_update(len(J), Jp, G.ctypes.data_as(_dp), int(n), Up)
    if rc:
        raise RuntimeError("ora_core_update failed: %d" % rc)
    return G


def orthogonalize(G, A):
    """Alg. 2's final step. Returns (G', A', [R^(n)])."""
    lib = _load()
    G = np.array(G, dtype=np.float64)
    I, J = _shape(G, A)
    I, Ip = _l(I)
    J, Jp = _i(J)
    A = [np.array(a, dtype=np.float64) for a in A]
    arr = (_dp * len(A))(*[a.ctypes.data_as(_dp) for a in A])
    R = np.zeros(int(np.sum(J.astype(np.int64) ** 2)))
    rc = lib.ora_orthogonalize(len(J), Ip, Jp, G.ctypes.data_as(_dp), arr,
                               R.ctypes.data_as(_dp))
    if rc:
        raise ValueError("ora_orthogonalize failed: %d" % rc)
    Rs, off = [], 0
    for j in J:
        Rs.append(R[off:off + j * j].reshape(j, j))
        off += j * j
    return G, A, Rs


def fold_in(G, A, n, idx, val, lam):
    """Row of mode n fitted to k new entries (idx [N][k]; row n ignored)."""
    lib = _load()
    G, Gp = _d(G)
    I, J = _shape(G, A)
    J, Jp = _i(J)
    keep, Ap = _ptrs(A)
    idx, ip = _i(idx)
    val, vp = _d(val)
    out = np.zeros(J[n])
    rc = lib.ora_fold_in(len(J), Jp, Gp, Ap, int(n), idx.shape[1], ip, vp,
                         float(lam), out.ctypes.data_as(_dp))
    if rc:
        raise RuntimeError("ora_fold_in failed: %d" % rc)
    return out
