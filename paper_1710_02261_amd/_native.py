"""ctypes binding of include/ptucker.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libptucker.so")
_lib = None

PTK_OK = 0
PREC_FP64_ACC = 0
PREC_FP32 = 1
PREC_BF16 = 2
PREC_BF16X3 = 3
_STATUS = {0: "PTK_OK", 1: "PTK_E_INVALID", 2: "PTK_E_NOMEM",
           3: "PTK_E_UNSUPPORTED", 4: "PTK_E_NOT_PD", 5: "PTK_E_HIP",
           6: "PTK_E_STATE", 7: "PTK_E_BUSY", 8: "PTK_E_DIVERGED"}

_vp = C.c_void_p
_i32 = C.c_int32
_i64 = C.c_int64
_dbl = C.c_double


class _Options(C.Structure):
    _fields_ = [("precision", _i32), ("chunk_nnz", _i32), ("fuse_error", _i32),
                ("profile", _i32), ("use_graph", _i32), ("pair_cache", _i32),
                ("approx_rate", _dbl), ("delta_slices", _i32), ("tol", _dbl),
                ("approx_form", _i32), ("cond_limit", _dbl), ("sparse_limit", _dbl),
                ("shared_units", _i32)]


class PtkError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        self.name = _STATUS.get(status, str(status))
        super().__init__("%s: %s" % (self.name, message))


def library_path() -> str:
    return _LIB_PATH


def load_library():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError("libptucker.so is not built; run "
                          "`python -m paper_1710_02261_amd.build` first")
    lib = C.CDLL(_LIB_PATH)
    sigs = {
        "ptk_create": [C.POINTER(_vp), _i32, C.POINTER(_i64), C.POINTER(_i32), _vp],
        "ptk_destroy": [_vp],
        "ptk_set_options": [_vp, C.POINTER(_Options)],
        "ptk_set_observed": [_vp, _i64, _vp, _vp],
        "ptk_bind_model": [_vp, _vp, C.POINTER(_vp)],
        "ptk_update_mode": [_vp, _i32, _dbl],
        "ptk_iterate": [_vp, _i32, _dbl, C.POINTER(_dbl), C.POINTER(_dbl)],
        "ptk_recon_error": [_vp, _dbl, C.POINTER(_dbl), C.POINTER(_dbl),
                            C.POINTER(_dbl)],
        "ptk_orthogonalize": [_vp],
        "ptk_predict": [_vp, _i64, _vp, _vp],
        "ptk_fold_in": [_vp, _i32, _i64, _vp, _vp, _dbl, _vp],
        "ptk_fold_in_noalloc": [_vp, _i32, _i64, _vp, _vp, _dbl, _vp],
        "ptk_delta": [_vp, _i32, _i64, _vp, _vp],
        "ptk_row_systems": [_vp, _i32, _vp, _vp],
        "ptk_kernel_times": [_vp, C.POINTER(_i32), C.POINTER(C.c_char_p),
                             C.POINTER(_i64), C.POINTER(_dbl)],
        "ptk_reset_timers": [_vp],
        "ptk_not_pd_count": [_vp, C.POINTER(_i64)],
        "ptk_solve_stats": [_vp, C.POINTER(_i64), C.POINTER(_i64)],
        "ptk_approx_stats": [_vp, C.POINTER(_i64), C.POINTER(_i32)],
        "ptk_unit_stats": [_vp, _i32, C.POINTER(_i64), C.POINTER(_i32)],
        "ptk_autotune": [_vp, C.c_char_p, C.POINTER(_i64)],
        "ptk_partial_error": [_vp, _vp],
        "ptk_truncate": [_vp, _dbl, C.POINTER(_i32)],
        "ptk_coo_scan": [C.c_char_p, _i32, C.POINTER(_i64), C.POINTER(_i64)],
        "ptk_coo_read": [C.c_char_p, _i32, _i64, _vp, _vp],
        "ptk_fp64_rates": [_i32, _vp],
        "ptk_normalize_values": [_vp, _i64, _vp, C.POINTER(_dbl)],
        "ptk_split_count": [_vp, _i64, _dbl, C.c_uint64, C.POINTER(_i64)],
        "ptk_split_entries": [_vp, _i32, _i64, _vp, _vp, _dbl, C.c_uint64, _i64, _vp, _vp,
                              _vp, _vp],
        "ptk_entry_error": [_vp, _i64, _vp, _vp, C.POINTER(_dbl), C.POINTER(_dbl)],
        "ptk_kmeans": [_vp, _i32, _i32, _i32, _vp, _vp, C.POINTER(_dbl)],
        "ptk_iterations_done": [_vp, C.POINTER(_i32)],
    }
    for name, args in sigs.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_int
    lib.ptk_last_error.argtypes = [_vp]
    lib.ptk_last_error.restype = C.c_char_p
    _lib = lib
    return lib


def _torch():
    import torch
    return torch


def _global_check(lib, st):
    if st != PTK_OK:
        msg = lib.ptk_last_error(None)
        raise PtkError(st, msg.decode() if msg else "")


def fp64_rates(iters=2000):
    """ptk_fp64_rates: sustained TFLOP/s of independent FP64 FMA chains, of
    the FP64 matrix cores, and of both at once, on the current device."""
    lib = load_library()
    out = (_dbl * 3)()
    _global_check(lib, lib.ptk_fp64_rates(int(iters), out))
    return {"fma_f64": out[0], "mfma_f64": out[1], "both": out[2]}


def coo_scan(path, N):
    """ptk_coo_scan: (entry count, dims) of a COO text file (1-based indices)."""
    lib = load_library()
    nnz = _i64(0)
    dims = (_i64 * int(N))()
    _global_check(lib, lib.ptk_coo_scan(os.fsencode(path), int(N), C.byref(nnz), dims))
    return int(nnz.value), tuple(int(d) for d in dims)


def coo_read(path, N, nnz=None):
    """ptk_coo_read: host arrays idx [N][nnz] int32 (0-based), val [nnz] float32."""
    lib = load_library()
    if nnz is None:
        nnz, _ = coo_scan(path, N)
    idx = np.empty((int(N), int(nnz)), dtype=np.int32)
    val = np.empty(int(nnz), dtype=np.float32)
    _global_check(lib, lib.ptk_coo_read(os.fsencode(path), int(N), int(nnz),
                                        idx.ctypes.data_as(_vp), val.ctypes.data_as(_vp)))
    return idx, val


def _dev_ptr(t, dtype, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a device tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return _vp(t.data_ptr())


class Context:
    """One ptk_ctx: an N-order tensor shape, core ranks and a HIP stream."""

    def __init__(self, dims, ranks, stream=None):
        torch = _torch()
        self._lib = load_library()
        self.dims = tuple(int(d) for d in dims)
        self.ranks = tuple(int(r) for r in ranks)
        self.N = len(self.dims)
        if len(self.ranks) != self.N:
            raise ValueError("dims and ranks differ in length")
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _vp()
        d = (_i64 * self.N)(*self.dims)
        r = (_i32 * self.N)(*self.ranks)
        st = self._lib.ptk_create(C.byref(h), self.N, d, r, _vp(stream.cuda_stream))
        if st != PTK_OK:
            raise PtkError(st, "ptk_create(%s, %s)" % (self.dims, self.ranks))
        self._h = h
        self._keep = []

    # -- plumbing ----------------------------------------------------------
    def _check(self, st):
        if st != PTK_OK:
            msg = self._lib.ptk_last_error(self._h)
            raise PtkError(st, msg.decode() if msg else "")

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ptk_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- C ABI calls ---------------------------------------------------------
    def set_options(self, precision=PREC_FP64_ACC, chunk_nnz=0, fuse_error=1,
                    profile=0, use_graph=1, pair_cache=0, approx_rate=0.0,
                    delta_slices=0, tol=0.0, approx_form=0, cond_limit=0.0,
                    sparse_limit=0.0, shared_units=0):
        o = _Options(precision, chunk_nnz, fuse_error, profile, use_graph, pair_cache,
                     float(approx_rate), delta_slices, float(tol), approx_form,
                     float(cond_limit), float(sparse_limit), shared_units)
        self._check(self._lib.ptk_set_options(self._h, C.byref(o)))

    def set_observed(self, idx, val):
        torch = _torch()
        if idx.dim() != 2 or idx.shape[0] != self.N:
            raise ValueError("idx must be [N, nnz]")
        nnz = int(idx.shape[1])
        if tuple(val.shape) != (nnz,):
            raise ValueError("val must be [nnz]")
        self._check(self._lib.ptk_set_observed(
            self._h, nnz, _dev_ptr(idx, torch.int32, "idx"),
            _dev_ptr(val, torch.float32, "val")))
        self.nnz = nnz

    def bind_model(self, core, factors):
        torch = _torch()
        if tuple(core.shape) != self.ranks:
            raise ValueError("core shape %s != ranks %s" % (tuple(core.shape), self.ranks))
        if len(factors) != self.N:
            raise ValueError("need one factor per mode")
        ptrs = (_vp * self.N)()
        for n, f in enumerate(factors):
            if tuple(f.shape) != (self.dims[n], self.ranks[n]):
                raise ValueError("factor %d has shape %s" % (n, tuple(f.shape)))
            ptrs[n] = _dev_ptr(f, torch.float32, "factor %d" % n)
        self._check(self._lib.ptk_bind_model(
            self._h, _dev_ptr(core, torch.float32, "core"), ptrs))
        self._keep = [core, *factors]

    def update_mode(self, n, lam):
        self._check(self._lib.ptk_update_mode(self._h, int(n), float(lam)))

    def iterate(self, iters, lam, strict=True):
        """Alg. 2 iterations; with strict=False the statuses PTK_E_NOT_PD (rows
        left unsolved) and PTK_E_DIVERGED (an error or loss not finite, or a
        rising loss) are not raised and the results are returned;
        ``last_status`` keeps the status either way."""
        sse = np.zeros(max(iters, 1))
        loss = np.zeros(max(iters, 1))
        st = self._lib.ptk_iterate(
            self._h, int(iters), float(lam),
            sse.ctypes.data_as(C.POINTER(_dbl)), loss.ctypes.data_as(C.POINTER(_dbl)))
        self.last_status = st
        if not (st in (4, 8) and not strict):
            self._check(st)
        return sse[:iters], loss[:iters]

    def autotune(self, cache_path=None):
        """Time work-range sizes per mode, keep the fastest; returns them."""
        out = (_i64 * self.N)()
        path = cache_path.encode() if cache_path else None
        self._check(self._lib.ptk_autotune(self._h, path, out))
        return [int(v) for v in out]

    def not_pd_count(self):
        n = _i64()
        self._check(self._lib.ptk_not_pd_count(self._h, C.byref(n)))
        return n.value

    def solve_stats(self):
        """(rows solved in least-squares form, most entries of such a row) of
        the last update_mode / iterate call."""
        a, b = _i64(), _i64()
        self._check(self._lib.ptk_solve_stats(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def approx_stats(self):
        """(non-zero core cells, bit mask of the modes on the sparse-core
        kernel) of the last iteration of the last iterate call; (-1, 0) when
        it listed no cells."""
        a, b = _i64(), _i32()
        self._check(self._lib.ptk_approx_stats(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def unit_stats(self, n):
        """([units of 1, 2, 4, 8 entries, long runs, their tasks, index
        values with a table, their tasks, single-entry units of the other
        values], path of
        mode n's row systems: 0 fused kernels, 1 units, 2 index tables) as
        built by set_observed."""
        cnt = (_i64 * 9)()
        on = _i32()
        self._check(self._lib.ptk_unit_stats(self._h, int(n), cnt, C.byref(on)))
        return [int(x) for x in cnt], int(on.value)

    def recon_error(self, lam=0.0):
        s, r, l = _dbl(), _dbl(), _dbl()
        self._check(self._lib.ptk_recon_error(self._h, float(lam), C.byref(s),
                                              C.byref(r), C.byref(l)))
        return s.value, r.value, l.value

    def orthogonalize(self):
        self._check(self._lib.ptk_orthogonalize(self._h))

    def predict(self, idx, out=None):
        torch = _torch()
        m = int(idx.shape[1])
        if out is None:
            out = torch.empty(m, dtype=torch.float32, device=idx.device)
        self._check(self._lib.ptk_predict(self._h, m, _dev_ptr(idx, torch.int32, "idx"),
                                          _dev_ptr(out, torch.float32, "out")))
        return out

    def fold_in(self, n, idx, val, lam, out=None):
        torch = _torch()
        k = int(idx.shape[1])
        if out is None:
            out = torch.empty(self.ranks[n], dtype=torch.float32, device=idx.device)
        iptr = _dev_ptr(idx, torch.int32, "idx") if k else _vp(0)
        vptr = _dev_ptr(val, torch.float32, "val") if k else _vp(0)
        self._check(self._lib.ptk_fold_in(self._h, int(n), k, iptr, vptr, float(lam),
                                          _dev_ptr(out, torch.float32, "out")))
        return out

    def fold_in_noalloc(self, n, idx, val, lam, out):
        """ptk_fold_in_noalloc: the fold-in on the library's fixed device
        scratch (no allocation); out is a caller-provided J_n float32 tensor."""
        torch = _torch()
        k = int(idx.shape[1])
        iptr = _dev_ptr(idx, torch.int32, "idx") if k else _vp(0)
        vptr = _dev_ptr(val, torch.float32, "val") if k else _vp(0)
        self._check(self._lib.ptk_fold_in_noalloc(self._h, int(n), k, iptr, vptr, float(lam),
                                                  _dev_ptr(out, torch.float32, "out")))
        return out

    def delta(self, n, idx):
        torch = _torch()
        m = int(idx.shape[1])
        out = torch.empty((m, self.ranks[n]), dtype=torch.float32, device=idx.device)
        self._check(self._lib.ptk_delta(self._h, int(n), m,
                                        _dev_ptr(idx, torch.int32, "idx"),
                                        _dev_ptr(out, torch.float32, "out")))
        return out

    def row_systems(self, n):
        torch = _torch()
        I, J = self.dims[n], self.ranks[n]
        dev = self._keep[0].device
        B = torch.empty((I, J, J), dtype=torch.float64, device=dev)
        c = torch.empty((I, J), dtype=torch.float64, device=dev)
        self._check(self._lib.ptk_row_systems(self._h, int(n),
                                              _dev_ptr(B, torch.float64, "B"),
                                              _dev_ptr(c, torch.float64, "c")))
        return B, c

    def partial_error(self):
        """R(beta) of eq. "recon_partial" for every core cell (float64, device)."""
        torch = _torch()
        dev = self._keep[0].device
        R = torch.empty(self.ranks, dtype=torch.float64, device=dev)
        self._check(self._lib.ptk_partial_error(self._h, _dev_ptr(R, torch.float64, "R")))
        return R

    def truncate(self, p):
        """One removal of Alg. 4 on the bound core; returns the cells removed."""
        k = _i32(0)
        self._check(self._lib.ptk_truncate(self._h, float(p), C.byref(k)))
        return int(k.value)

    def iterations_done(self):
        """Iterations the last iterate() ran (fewer when options.tol stopped it)."""
        n = _i32(0)
        self._check(self._lib.ptk_iterations_done(self._h, C.byref(n)))
        return int(n.value)

    # -- steps either side of the fit ----------------------------------------
    def normalize_values(self, val):
        """ptk_normalize_values in place; returns (min, max)."""
        torch = _torch()
        mm = (_dbl * 2)()
        n = int(val.numel())
        ptr = _dev_ptr(val, torch.float32, "val") if n else _vp(0)
        self._check(self._lib.ptk_normalize_values(self._h, n, ptr, mm))
        return float(mm[0]), float(mm[1])

    def split(self, idx, val, test_fraction=0.1, seed=0):
        """ptk_split_count + ptk_split_entries: (idx_train, val_train, idx_test,
        val_test) device tensors, each side in the original order."""
        torch = _torch()
        N, nnz = int(idx.shape[0]), int(idx.shape[1])
        nt = _i64(0)
        self._check(self._lib.ptk_split_count(self._h, nnz, float(test_fraction),
                                              C.c_uint64(int(seed)), C.byref(nt)))
        ntest = int(nt.value)
        dev = idx.device
        it = torch.empty((N, nnz - ntest), dtype=torch.int32, device=dev)
        vt = torch.empty(nnz - ntest, dtype=torch.float32, device=dev)
        ie = torch.empty((N, ntest), dtype=torch.int32, device=dev)
        ve = torch.empty(ntest, dtype=torch.float32, device=dev)

        def ptr(t, dt, name):
            return _dev_ptr(t, dt, name) if t.numel() else _vp(0)
        if nnz:
            self._check(self._lib.ptk_split_entries(
                self._h, N, nnz, ptr(idx, torch.int32, "idx"), ptr(val, torch.float32, "val"),
                float(test_fraction), C.c_uint64(int(seed)), ntest,
                ptr(it, torch.int32, "idx_train"), ptr(vt, torch.float32, "val_train"),
                ptr(ie, torch.int32, "idx_test"), ptr(ve, torch.float32, "val_test")))
        return it, vt, ie, ve

    def entry_error(self, idx, val):
        """ptk_entry_error: (sse, rmse) of the bound model over an entry list."""
        torch = _torch()
        m = int(idx.shape[1])
        sse, rmse = _dbl(0.0), _dbl(0.0)
        ip = _dev_ptr(idx, torch.int32, "idx") if m else _vp(0)
        vp = _dev_ptr(val, torch.float32, "val") if m else _vp(0)
        self._check(self._lib.ptk_entry_error(self._h, m, ip, vp, C.byref(sse), C.byref(rmse)))
        return float(sse.value), float(rmse.value)

    def kmeans(self, n, centroids, iters):
        """ptk_kmeans over the rows of the bound factor n from the given initial
        centroids (float64 [K][J_n] device, updated in place); returns
        (assignment int32 [I_n] device, inertia, rows changed in the last pass)."""
        torch = _torch()
        K = int(centroids.shape[0])
        if tuple(centroids.shape) != (K, self.ranks[n]):
            raise ValueError("centroids must be [K][J_n]")
        assign = torch.empty(self.dims[n], dtype=torch.int32, device=centroids.device)
        res = (_dbl * 2)()
        self._check(self._lib.ptk_kmeans(self._h, int(n), K, int(iters),
                                         _dev_ptr(centroids, torch.float64, "centroids"),
                                         _dev_ptr(assign, torch.int32, "assign"), res))
        return assign, float(res[0]), int(res[1])

    def kernel_times(self):
        cnt = _i32(64)
        names = (C.c_char_p * 64)()
        calls = (_i64 * 64)()
        ms = (_dbl * 64)()
        self._check(self._lib.ptk_kernel_times(self._h, C.byref(cnt), names, calls, ms))
        return {names[k].decode(): (int(calls[k]), float(ms[k]))
                for k in range(min(cnt.value, 64))}

    def reset_timers(self):
        self._check(self._lib.ptk_reset_timers(self._h))


class _ServerOpts(C.Structure):
    _fields_ = [("mem_budget_bytes", _i64), ("slots", _i32),
                ("max_batch_requests", _i32), ("queue_capacity", _i32),
                ("lambda_", _dbl)]


class _ServerStats(C.Structure):
    _fields_ = [("batches", _i64), ("requests", _i64), ("max_batch_requests", _i64),
                ("max_in_flight", _i64), ("queued", _i64)]


def _host_i32(a, rows):
    a = np.ascontiguousarray(a, dtype=np.int32)
    if a.ndim != 2 or a.shape[0] != rows:
        raise ValueError("idx must be [N, count]")
    return a


class Server:
    """ptk_server: continuous-batching fold-in / prediction loop on a context."""

    def __init__(self, ctx, lam, mem_budget_bytes=0, slots=0, max_batch_requests=0,
                 queue_capacity=0):
        lib = load_library()
        if not getattr(lib, "_server_sigs", False):
            u64p = C.POINTER(C.c_uint64)
            for name, args in {
                "ptk_server_create": [C.POINTER(_vp), _vp, C.POINTER(_ServerOpts)],
                "ptk_server_submit_foldin": [_vp, _i32, _i64, _vp, _vp, u64p],
                "ptk_server_submit_predict": [_vp, _i64, _vp, u64p],
                "ptk_server_poll": [_vp, C.c_uint64, _vp, _i64, C.POINTER(_i32),
                                    C.POINTER(C.c_int), C.POINTER(_dbl)],
                "ptk_server_wait": [_vp, C.c_uint64, _vp, _i64, _dbl, C.POINTER(C.c_int),
                                    C.POINTER(_dbl)],
                "ptk_server_get_stats": [_vp, C.POINTER(_ServerStats)],
                "ptk_server_destroy": [_vp],
            }.items():
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = C.c_int
            lib.ptk_server_last_error.argtypes = [_vp]
            lib.ptk_server_last_error.restype = C.c_char_p
            lib._server_sigs = True
        self._lib = lib
        self.ctx = ctx
        self.N = ctx.N
        o = _ServerOpts(int(mem_budget_bytes), int(slots), int(max_batch_requests),
                        int(queue_capacity), float(lam))
        h = _vp()
        st = lib.ptk_server_create(C.byref(h), ctx._h, C.byref(o))
        if st != PTK_OK:
            raise PtkError(st, "ptk_server_create")
        self._h = h

    def _check(self, st):
        if st != PTK_OK:
            msg = self._lib.ptk_server_last_error(self._h)
            raise PtkError(st, msg.decode() if msg else "")

    def submit_foldin(self, n, idx, val):
        idx = _host_i32(idx, self.N)
        val = np.ascontiguousarray(val, dtype=np.float32)
        t = C.c_uint64()
        self._check(self._lib.ptk_server_submit_foldin(
            self._h, int(n), int(idx.shape[1]), idx.ctypes.data_as(_vp),
            val.ctypes.data_as(_vp), C.byref(t)))
        return t.value

    def submit_predict(self, idx):
        idx = _host_i32(idx, self.N)
        t = C.c_uint64()
        self._check(self._lib.ptk_server_submit_predict(
            self._h, int(idx.shape[1]), idx.ctypes.data_as(_vp), C.byref(t)))
        return t.value

    def submit_foldin_ptr(self, n, k, idx_addr, val_addr):
        """submit_foldin from host addresses of contiguous int32 [N][k] indices
        and float32 [k] values (no conversion: for load generators)."""
        t = C.c_uint64()
        self._check(self._lib.ptk_server_submit_foldin(self._h, n, k, idx_addr, val_addr,
                                                       C.byref(t)))
        return t.value

    def submit_predict_ptr(self, m, idx_addr):
        """submit_predict from the host address of contiguous int32 [N][m]."""
        t = C.c_uint64()
        self._check(self._lib.ptk_server_submit_predict(self._h, m, idx_addr, C.byref(t)))
        return t.value

    def poll(self, ticket, size):
        out = np.zeros(max(int(size), 1), dtype=np.float32)
        done, st, lat = _i32(), C.c_int(), _dbl()
        self._check(self._lib.ptk_server_poll(self._h, ticket, out.ctypes.data_as(_vp),
                                              int(size), C.byref(done), C.byref(st),
                                              C.byref(lat)))
        if not done.value:
            return False, None, None, None
        return True, out[:size], st.value, lat.value

    def wait(self, ticket, size, timeout=60.0):
        """Blocks until the request finishes: (result, status, latency_ms)."""
        out = np.zeros(max(int(size), 1), dtype=np.float32)
        st, lat = C.c_int(), _dbl()
        self._check(self._lib.ptk_server_wait(self._h, ticket, out.ctypes.data_as(_vp),
                                              int(size), float(timeout), C.byref(st),
                                              C.byref(lat)))
        return out[:size], st.value, lat.value

    def stats(self):
        s = _ServerStats()
        self._check(self._lib.ptk_server_get_stats(self._h, C.byref(s)))
        return {k: getattr(s, k) for k, _ in _ServerStats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            self._lib.ptk_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
