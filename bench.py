"""Throughput of the row-wise sparse Tucker ALS on one MI355X.

Workload: order-4 tensor, 100,000 per mode, 10^7 distinct observed cells with
truncated Zipf(1.1) index skew per mode, ranks J=10, planted Tucker values
+ N(0, 0.1) noise, lambda = 0.01 (synthetic, seeded; ``synth.make_c2``).

One step = one iteration of Alg. 2: the four mode updates of
Alg. 3 and the reconstruction error, all on the GPU through the C ABI. The
metric is nnz x iterations / s over the timed steps, inputs resident in HBM.

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]

Prints one JSON line. Besides the throughput it reports the roofline of the
dominant kernel (delta + row-system kernel) from HIP-event durations taken
inside the library, and the FP64 oracle's throughput on a bounded sample of
the same workload on this host's CPU (``cpu_baseline``).
"""
from __future__ import annotations

import argparse
import gc
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "delta_index_c2_traffic.json")
KERNEL_SRC = [os.path.join(ROOT, "paper_1710_02261_amd", "csrc", f)
              for f in ("ptk_units.hip", "ptk_units.h", "ptk_device.h", "ptk_internal.h")]


def command_line():
    """The command that produced a record (kept with the record)."""
    return " ".join(["python", "bench.py"] + sys.argv[1:])


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fma_per_nnz_mode(N, J):
    """Algorithmic multiply-adds per (entry, mode): delta by the contraction
    chain J^N + J^(N-1) + ... + J^2, plus the packed Gram and rhs."""
    chain = sum(J ** k for k in range(2, N + 1))
    return chain + J * (J + 1) // 2 + J


def kernel_hash():
    """Hash of the sources that define the headline row-system kernel."""
    h = hashlib.sha256()
    for path in KERNEL_SRC:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_record(launch_nnz):
    """HBM bytes per launch of the dominant kernel from the committed PMC
    summary, or None when it is missing or the kernel source has changed."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


HEADLINE_KERNEL = "void ptk::k_delta_long<4, 10, 2>(ptk::LongArgs)"
# a precision form is reported with throughput when its RMSE after the run is
# at most this much above the FP64 path's (the comparison at equal RMSE)
USABLE_RMSE = 0.10
COPY_KERNEL_TAG = "MulFunctor<float>"


def traffic_summary(fetch_csv, write_csv, launches):
    """HBM traffic of the headline kernel from two rocprofv3 --pmc runs of
    `bench.py --no-cpu --no-variant --steps 2 --warmup 1 --copy-calibration`
    (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch): the last `launches`
    dispatches of the kernel, each counter scaled by what it reads for the
    copy kernel (256 MiB read and written). Writes TRAFFIC_FILE."""
    import csv

    def per_dispatch(path, counter):
        vals = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                key = int(r["Dispatch_Id"])
                name = r["Kernel_Name"]
                old = vals.get(key, (name, 0.0))
                vals[key] = (name, old[1] + float(r["Counter_Value"]))
        return [vals[k] for k in sorted(vals)]

    out = {"kernel": HEADLINE_KERNEL,
           "workload": "order-4 100000^4, 1e7 entries Zipf(1.1), J=10, FP64 arithmetic, "
                       "index tables, autotuned work ranges",
           "kernel_sha": kernel_hash()}
    cal = {"kernel": "torch.mul of 64 Mi float32 (reads and writes 256 MiB)"}
    for tag, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"),
                               ("write", write_csv, "WRITE_SIZE")):
        rows = per_dispatch(path, counter)
        copy = [v for n, v in rows if COPY_KERNEL_TAG in n]
        gram = [v for n, v in rows if n == HEADLINE_KERNEL][-launches:]
        if not copy or len(gram) < launches:
            raise SystemExit("traffic summary: missing copy or kernel dispatches in " + path)
        copy_kib = float(np.mean(copy))
        scale = 262144.0 / copy_kib
        raw = float(np.mean(gram))
        cal[tag + "_kib_read"] = copy_kib
        cal[tag + "_scale"] = scale
        out[tag + "_kib_raw_avg"] = raw
        out[tag + "_bytes_per_launch"] = raw * scale * 1024.0
    out["bytes_per_launch"] = out["fetch_bytes_per_launch"] + out["write_bytes_per_launch"]
    out["launches_averaged"] = launches
    out["calibration"] = cal
    out["commands"] = [
        "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 300 rocprofv3 --pmc FETCH_SIZE "
        "--kernel-trace -f csv -d $R/gpurun_out/pmc_fetch -o fetch -- python3 $R/bench.py "
        "--no-cpu --no-variant --steps 2 --warmup 1 --copy-calibration",
        "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 300 rocprofv3 --pmc WRITE_SIZE "
        "--kernel-trace -f csv -d $R/gpurun_out/pmc_write -o write -- python3 $R/bench.py "
        "--no-cpu --no-variant --steps 2 --warmup 1 --copy-calibration",
        "python bench.py --traffic-summary $R/gpurun_out/pmc_fetch/fetch_counter_collection.csv "
        "$R/gpurun_out/pmc_write/write_counter_collection.csv"]
    out["note"] = ("R = repository root; counters per dispatch in KiB; the averaged launches "
                   "are the last ones of the run (warm-up, timed and event-timed iterations, "
                   "after the autotuner). FETCH_SIZE counts L2 misses, served by HBM or the "
                   "Infinity Cache.")
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print(json.dumps(out))


def _oracle_rate(p, G, A, v, seconds, rng):
    """Seconds per entry-iteration of the oracle on a bounded sample of the
    workload: Alg. 3 row updates of random rows per mode (sized from a
    calibration on a few rows) and the error of random entries."""
    import oracle
    N = p.N
    per = seconds / (N + 1)
    t_per_nnz = []
    total_nnz, total_rows = 0, 0
    for n in range(N):
        cnt = np.bincount(p.idx[n], minlength=p.dims[n])
        nz = np.flatnonzero(cnt)
        order = rng.permutation(nz)
        csum = np.cumsum(cnt[order])
        k0 = int(np.searchsorted(csum, 2000)) + 1
        t0 = time.perf_counter()
        oracle.update_rows(G, A, p.idx, v, n, p.lam, rows=order[:k0])
        rate = max(time.perf_counter() - t0, 1e-3) / max(csum[k0 - 1], 1)
        target = max(2000, int(per / rate))
        k = int(np.searchsorted(csum, target)) + 1
        rows = order[k0:k0 + k]
        t0 = time.perf_counter()
        oracle.update_rows(G, A, p.idx, v, n, p.lam, rows=rows)
        dt = time.perf_counter() - t0
        nn = int(cnt[rows].sum())
        t_per_nnz.append(dt / nn)
        total_nnz += nn
        total_rows += len(rows)
    m = max(2000, int(per / max(t_per_nnz[0], 1e-9)))
    sel = rng.choice(p.nnz, size=min(m, p.nnz), replace=False)
    sub = np.ascontiguousarray(p.idx[:, sel])
    t0 = time.perf_counter()
    oracle.sse(G, A, sub, v[sel])
    t_err = (time.perf_counter() - t0) / len(sel)
    return sum(t_per_nnz) + t_err, total_rows, total_nnz, len(sel)


def host_cores():
    """(model, logical CPUs this process may use, physical cores of the host
    from lscpu or None)."""
    import oracle
    import subprocess
    model, _ = oracle.host_cpu()
    try:
        logical = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        logical = os.cpu_count() or 1
    physical = None
    try:
        out = subprocess.run(["lscpu", "-p=CORE,SOCKET"], capture_output=True, text=True,
                             timeout=10).stdout
        pairs = {tuple(l.split(",")) for l in out.splitlines() if l and not l.startswith("#")}
        physical = len(pairs) or None
    except (OSError, subprocess.SubprocessError):
        pass
    return model, logical, physical


def cpu_baseline(p, seconds=20.0):
    """FP64 oracle on a bounded sample of the workload: one thread, then all
    the threads this process may use (OpenMP, rows dealt dynamically as in
    the paper's Sec. 3.4). The value is the all-thread rate."""
    import oracle
    G = p.core.astype(np.float64)
    A = [a.astype(np.float64) for a in p.factors]
    v = p.val.astype(np.float64)
    model, logical, physical = host_cores()
    threads = min(logical, int(os.environ.get("OMP_NUM_THREADS", logical) or logical))
    prev = oracle.set_threads(0)
    try:
        oracle.set_threads(1)
        t1, rows1, nnz1, e1 = _oracle_rate(p, G, A, v, seconds / 2, np.random.default_rng(123))
        used = oracle.set_threads(threads)
        tm, rowsm, nnzm, em = _oracle_rate(p, G, A, v, seconds / 2, np.random.default_rng(124))
    finally:
        oracle.set_threads(prev)
    return {
        "value": 1.0 / tm,
        "unit": "nnz*iters/s",
        "cores": used,
        "kind": "oracle",
        "single_thread_value": 1.0 / t1,
        "cpu_model": model,
        "logical_cpus_available": logical,
        "physical_cores_host": physical,
        "build": "gcc -O3 -march=native -fopenmp",
        "sample": "FP64 oracle: Alg. 3 row updates of random rows of every mode "
                  "(%d rows, %d entries on %d threads; %d rows, %d entries on one "
                  "thread) and the error of random entries (%d / %d); seconds per "
                  "entry-iteration summed over the %d modes and the error pass"
                  % (rowsm, nnzm, used, rows1, nnz1, em, e1, p.N),
    }


WORKLOADS = {
    "c2": ("order-4 100000^4, 1e7 distinct cells, Zipf(1.1) per mode, J=10, "
           "planted Tucker + N(0,0.1), lambda=0.01, seed 1"),
    "c3": ("rating tensor 480000x18000x2000, 1e8 distinct cells, users Zipf(0.6), "
           "items Zipf(0.9), days uniform, ratings 1..5, J=16, lambda=0.01, seed 2"),
    "c4": ("order-5 10000^5, 5e7 distinct cells, lognormal(3,2) row weights per mode "
           "(1..1e5 per row), J=8, planted rank 4 + N(0,0.1), lambda=0.01, seed 3"),
}
PREC_NAMES = {"f64": 0, "f32": 1, "bf16": 2, "bf16x3": 3}
PREC_DTYPE = {"f64": "f64", "f32": "f32", "bf16": "bf16", "bf16x3": "bf16"}
PREC_PEAK = {"f64": 78.6e12, "f32": 157.3e12, "bf16": 2.5e15, "bf16x3": 2.5e15}


def serving(args):
    """Serving workload: continuous-batching server vs per-request calls."""
    import torch
    import synth
    import paper_1710_02261_amd as ptk

    t0 = time.perf_counter()
    G, A, reqs = synth.make_c5(n_foldin=args.requests)
    dims, J = (100_000, 50_000, 1_000), 16
    log("generated %d requests in %.1f s" % (len(reqs), time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    core = torch.from_numpy(G).to(dev)
    fac = [torch.from_numpy(a).to(dev) for a in A]
    ctx = ptk.Context(dims, (J, J, J))
    ctx.bind_model(core, fac)
    ctx.orthogonalize()                       # orthonormal factors, rotated core
    torch.cuda.synchronize()
    lam = 0.01
    sizes = [J if r[0] == "f" else r[2].shape[1] for r in reqs]
    kinds = np.array([r[0] == "f" for r in reqs])

    def submit(srv, r):
        return srv.submit_foldin(0, r[2], r[3]) if r[0] == "f" else srv.submit_predict(r[2])

    # contiguous host arrays and their addresses, prepared before any timing,
    # so that the generator does one call per request and nothing else
    prep = []
    for r in reqs:
        ix = np.ascontiguousarray(r[2], dtype=np.int32)
        if r[0] == "f":
            vv = np.ascontiguousarray(r[3], dtype=np.float32)
            prep.append((True, ix.shape[1], ix.ctypes.data, vv.ctypes.data, ix, vv))
        else:
            prep.append((False, ix.shape[1], ix.ctypes.data, 0, ix, None))

    def run_server(rate):
        """Submit the stream at its arrival times (Poisson at `rate` per
        second, or as fast as possible), from this thread only, then collect
        the results. The server's own thread runs the batches meanwhile. Each
        request's latency is measured by the library from its submit to its
        completion, so its completion time is at most the clock read right
        after its submit returned plus that latency; the served rate is the
        requests over the last completion, and collecting the results
        afterwards (client work) is not part of it. With no second Python
        thread and the cyclic garbage collector paused, the generator keeps to
        the schedule (its lag is reported)."""
        srv = ptk.Server(ctx, lam, slots=args.slots, max_batch_requests=args.max_batch)
        for r in reqs[:50]:                    # warm-up
            srv.wait(submit(srv, r), J if r[0] == "f" else r[2].shape[1])
        lag = np.zeros(len(reqs))
        after = np.zeros(len(reqs))
        tickets = [0] * len(reqs)
        rng = np.random.default_rng(7)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, len(reqs))) if rate else None
        sub_f, sub_p = srv.submit_foldin_ptr, srv.submit_predict_ptr
        clock = time.perf_counter
        gc.collect()
        gc.disable()
        try:
            start = clock()
            for i, (fold, m, ia, va, _, _) in enumerate(prep):
                if arrivals is not None:
                    due = arrivals[i]
                    while clock() - start < due:
                        pass
                    lag[i] = (clock() - start) - due
                tickets[i] = sub_f(0, m, ia, va) if fold else sub_p(m, ia)
                after[i] = clock() - start
        finally:
            gc.enable()
        lat = np.zeros(len(reqs))
        for i in range(len(reqs)):
            out, st, ms = srv.wait(tickets[i], sizes[i], timeout=600.0)
            if st != 0:
                raise RuntimeError("request %d failed with status %d" % (i, st))
            lat[i] = ms
        served = float(np.max(after + 1e-3 * lat))
        stats = srv.stats()
        srv.close()
        return served, lat, lag, stats

    def pct(x, q):
        return float(np.percentile(x, q)) if len(x) else None

    # saturation: the whole stream submitted as fast as possible
    served, lat, lag, st = run_server(None)
    sat = len(reqs) / served
    log("saturation: %.0f requests/s (%d batches, max %d in flight)" % (
        sat, st["batches"], st["max_in_flight"]))
    loads = {}
    for frac in args.loads:
        rate = frac * sat
        served2, lat2, lag2, st2 = run_server(rate)
        loads["%d%%" % round(100 * frac)] = {
            "offered_req_s": rate, "achieved_req_s": len(reqs) / served2,
            "foldin_p50_ms": pct(lat2[kinds], 50), "foldin_p99_ms": pct(lat2[kinds], 99),
            "predict_p50_ms": pct(lat2[~kinds], 50), "predict_p99_ms": pct(lat2[~kinds], 99),
            "generator_lag_p99_ms": 1e3 * pct(lag2, 99), "batches": st2["batches"],
            "max_in_flight": st2["max_in_flight"]}
        log("load %.0f%%: fold-in p50 %.3f ms p99 %.3f ms" % (
            100 * frac, loads["%d%%" % round(100 * frac)]["foldin_p50_ms"],
            loads["%d%%" % round(100 * frac)]["foldin_p99_ms"]))
    # per-request plain calls (synchronous, one at a time) on a prefix
    nplain = min(args.plain_requests, len(reqs))
    plat = np.zeros(nplain)
    tp = time.perf_counter()
    for i in range(nplain):
        r = reqs[i]
        t1 = time.perf_counter()
        idx = torch.from_numpy(r[2]).to(dev)
        if r[0] == "f":
            val = torch.from_numpy(r[3]).to(dev)
            ctx.fold_in(0, idx, val, lam).cpu()
        else:
            ctx.predict(idx).cpu()
        plat[i] = 1e3 * (time.perf_counter() - t1)
    plain_el = time.perf_counter() - tp
    pk = kinds[:nplain]
    out = {
        "metric": "serving: fold-in / prediction requests per second; p50/p99 ms",
        "value": sat, "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
        "data": "synthetic", "dtype": "f64",
        "config": {"workload": "order-3 model 100000x50000x1000, J=16, orthogonalised "
                               "planted N(0,1); %d fold-ins of mode 0 (k ~ lognormal(ln 50, "
                               "1.2) in [5, 5000]) and one prediction batch (1e3..1e5 "
                               "cells, log-uniform) per 20 fold-ins; Poisson arrivals"
                               % args.requests,
                   "requests": len(reqs), "foldins": int(kinds.sum()),
                   "slots": args.slots, "max_batch_requests": args.max_batch},
        "saturation": {"req_s": sat, "foldin_p50_ms": pct(lat[kinds], 50),
                       "foldin_p99_ms": pct(lat[kinds], 99), "batches": st["batches"],
                       "max_in_flight": st["max_in_flight"]},
        "poisson": loads,
        "plain_per_request": {"requests": nplain, "req_s": nplain / plain_el,
                              "foldin_p50_ms": pct(plat[pk], 50),
                              "foldin_p99_ms": pct(plat[pk], 99),
                              "predict_p50_ms": pct(plat[~pk], 50),
                              "predict_p99_ms": pct(plat[~pk], 99)},
    }
    ctx.close()
    out["command"] = command_line()
    print(json.dumps(out), flush=True)


# equal-rank shapes with an unrolled row-system kernel (the rest use the
# generic kernel)
FAST_SHAPES = {3: (3, 4, 5, 7, 8, 9, 10, 11, 16), 4: (3, 5, 8, 10), 5: (3, 5, 8)}


def sweeps(args):
    """The paper's four synthetic scalability sweeps (Sec. 4.2: order,
    dimensionality, observed entries, rank) and its Cache-variant comparison
    over orders 6-10 (Sec. 4.3, plain and pair cache) on one GPU: FP64
    arithmetic, graph replay, autotuned ranges; seconds per Alg. 2 iteration."""
    import paper_1710_02261_amd as ptk
    import synth
    import torch
    kinds = args.sweep or ["order", "dimensionality", "nnz", "rank", "cache"]
    table = []
    runs = [(kind, dims, J, nnz, cache) for kind in kinds
            for dims, J, nnz in synth.SWEEPS[kind]
            for cache in ((0, 1) if kind == "cache" else (0,))]
    for kind, dims, J, nnz, cache in runs:
        t0 = time.perf_counter()
        p = synth.make_random(dims, J, nnz, seed=11)
        gen = time.perf_counter() - t0
        dev = torch.device("cuda:0")
        idx = torch.from_numpy(p.idx).to(dev)
        val = torch.from_numpy(p.val).to(dev)
        core = torch.from_numpy(p.core).to(dev)
        fac = [torch.from_numpy(a).to(dev) for a in p.factors]
        ctx = ptk.Context(p.dims, p.ranks)
        ctx.set_options(precision=0, fuse_error=1, profile=0, use_graph=1,
                        pair_cache=cache)
        ctx.set_observed(idx, val)
        ctx.bind_model(core, fac)
        if nnz >= 100_000:
            ctx.autotune(None)
        steps = int(max(3, min(50, 2e8 // max(nnz, 1))))
        ctx.iterate(1, p.lam, strict=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.iterate(steps, p.lam, strict=False)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t1) / steps
        ctx.close()
        row = {"sweep": kind, "N": len(dims), "I": dims[0], "J": J, "nnz": nnz,
               "ms_per_iteration": 1e3 * sec, "nnz_iters_per_s": nnz / sec,
               "kernel": "fast" if J in FAST_SHAPES.get(len(dims), ()) else "generic",
               "pair_cache": cache}
        table.append(row)
        log("%-14s N=%2d I=%-9d J=%2d nnz=%-10d cache=%d %9.3f ms/iteration  "
            "%.3e nnz*iters/s  (generated in %.1f s)"
            % (kind, len(dims), dims[0], J, nnz, cache, 1e3 * sec, nnz / sec, gen))
        del idx, val, core, fac, p
    print(json.dumps({
        "metric": "seconds per Alg. 2 iteration on the synthetic scalability tensors",
        "value": None, "unit": "ms/iteration", "n_gpus": 1, "higher_is_better": False,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "random tensors of Sec. 4.2: values U[0,1) at uniform "
                               "distinct cells, equal ranks, U[0,1) initial model, seed 11",
                   "sweeps": kinds},
        "table": table, "command": command_line()}), flush=True)


def approx_trace(args, p, idx, val, core, fac0, use_graph):
    """Time K single iterations (each its own ptk_iterate call, bracketed by
    synchronisations) of three runs from the same start: no removal, the
    Approx variant with the dense row-system kernels (sparse_limit < 0), and
    the Approx variant with the sparse-core switch; record the non-zero core
    cells each iteration starts from. The first call of a run also captures
    its graph."""
    import torch
    import paper_1710_02261_amd as ptk
    rate = args.approx_rate if args.approx_rate > 0 else 0.2
    runs = [("plain", 0.0, -1.0), ("approx_dense", rate, -1.0),
            ("approx_sparse", rate, args.sparse_limit)]
    res = {}
    cells = int(core.numel())
    for name, r, lim in runs:
        fac = [f.clone() for f in fac0]
        core_run = core.clone()
        ctx = ptk.Context(p.dims, p.ranks)
        ctx.set_options(fuse_error=1, profile=0, use_graph=use_graph, approx_rate=r,
                        sparse_limit=lim)
        ctx.set_observed(idx, val)
        ctx.bind_model(core_run, fac)
        if not args.no_autotune:
            ctx.autotune(None)
        ms, nz, sse = [], [], []
        for t in range(args.approx_trace):
            nz.append(int(torch.count_nonzero(core_run)))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            s, _ = ctx.iterate(1, p.lam, strict=False)
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
            sse.append(float(s[0]))
            log("%s iteration %d: %.2f ms, non-zero cells %d (%.3f), rmse %.6g" % (
                name, t, ms[-1], nz[-1], nz[-1] / cells, np.sqrt(max(s[0], 0.0) / p.nnz)))
        ctx.close()
        res[name] = {"ms": ms, "nonzero_cells": nz,
                     "rmse": [float(np.sqrt(max(x, 0.0) / p.nnz)) for x in sse]}
    out = {"approx_trace": res, "approx_rate": rate, "core_cells": cells,
           "sparse_limit": args.sparse_limit,
           "config": {"workload": WORKLOADS[args.workload], "nnz": p.nnz,
                      "ranks": list(p.ranks), "dims": list(p.dims)},
           "note": "ms per iteration by host clock around one ptk_iterate call each "
                   "(graph replay); the first call of each run includes the capture",
           "command": command_line()}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", choices=sorted(WORKLOADS) + ["c5", "sweeps"],
                    default="c2")
    ap.add_argument("--sweep", nargs="*", choices=["order", "dimensionality", "nnz",
                                                   "rank", "cache"],
                    help="sweeps: which ones (default all five)")
    ap.add_argument("--requests", type=int, default=100_000, help="c5: fold-ins")
    ap.add_argument("--slots", type=int, default=2)
    ap.add_argument("--max-batch", type=int, default=1024)
    ap.add_argument("--loads", type=float, nargs="*", default=[0.25, 0.5, 0.75, 0.9])
    ap.add_argument("--plain-requests", type=int, default=10_000)
    ap.add_argument("--nnz", type=int, default=0, help="override the entry count")
    ap.add_argument("--precision", choices=sorted(PREC_NAMES), default="f64")
    ap.add_argument("--cpu-seconds", type=float, default=24.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-variant", action="store_true")
    ap.add_argument("--approx-rate", type=float, default=0.0,
                    help="Approx variant: core cells removed per iteration (0 = off)")
    ap.add_argument("--sparse-limit", type=float, default=0.0,
                    help="Approx variant: non-zero core fraction at or below which "
                         "delta is summed over the non-zero cells (0 = library "
                         "default, negative = never)")
    ap.add_argument("--approx-trace", type=int, default=0, metavar="K",
                    help="print ms and non-zero core cells of each of K single "
                         "iterations: no removal, Approx with the dense kernels, "
                         "Approx with the sparse-core switch; one JSON line, exit")
    ap.add_argument("--traffic-summary", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the headline kernel's HBM traffic record from two "
                         "rocprofv3 counter runs (see traffic_summary) and exit; no GPU")
    ap.add_argument("--fp64-ceiling", action="store_true",
                    help="print the sustained FP64 rates of the GPU (FMA loop, "
                         "matrix cores, both) as one JSON line and exit")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a 256 MiB copy kernel (HBM counter scale)")
    ap.add_argument("--pair-cache", action="store_true",
                    help="main run with the per-entry pair cache")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default work-range sizes")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch kernels one by one instead of replaying a graph")
    ap.add_argument("--shared-units", type=int, default=0, choices=[-1, 0, 1, 2, 4, 8],
                    help="ptk_options.shared_units (0 auto, -1 never, 1 always, "
                         "2/4/8 always with that cap)")
    args = ap.parse_args()

    if args.traffic_summary:
        # warm-up 1 + steps 2 + the event-timed pass, one launch per mode each
        traffic_summary(args.traffic_summary[0], args.traffic_summary[1], 5 * 4)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d requested)" % (args.gpus, world),
              file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_1710_02261_amd as ptk
    from paper_1710_02261_amd import _native
    if not os.path.exists(_native.library_path()):
        from paper_1710_02261_amd import build as hipbuild
        hipbuild.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.fp64_ceiling:
        rates = ptk.fp64_rates(2000)
        print(json.dumps({"fp64_rates_tflops": rates, "published_peak_tflops": 78.6,
                          "command": command_line()}), flush=True)
        return
    if args.workload == "sweeps":
        sweeps(args)
        return
    if args.workload == "c5":
        serving(args)
        return

    if args.copy_calibration:
        # a plain copy kernel of known size (reads and writes 256 MiB) that
        # calibrates the HBM byte counters of a profiled run
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
        log("copy calibration: 3 x (read 256 MiB, write 256 MiB)")

    t0 = time.perf_counter()
    kw = {"nnz": args.nnz} if args.nnz else {}
    p = synth.make(args.workload, **kw)
    log("generated %s (%d entries) in %.1f s" % (args.workload, p.nnz,
                                                time.perf_counter() - t0))
    dev = torch.device("cuda:0")
    idx = torch.from_numpy(p.idx).to(dev)
    val = torch.from_numpy(p.val).to(dev)
    core = torch.from_numpy(p.core).to(dev)
    fac0 = [torch.from_numpy(a).to(dev) for a in p.factors]
    N, J = p.N, p.ranks[0]

    use_graph = 0 if args.no_graph else 1
    if args.approx_trace:
        approx_trace(args, p, idx, val, core, fac0, use_graph)
        return

    def run(prec, cache=0, approx=0.0):
        fac = [f.clone() for f in fac0]
        core_run = core.clone()           # the Approx removal edits the core
        ctx = ptk.Context(p.dims, p.ranks)
        ctx.set_options(precision=PREC_NAMES[prec], fuse_error=1, profile=0,
                        use_graph=use_graph, pair_cache=cache, approx_rate=approx,
                        sparse_limit=args.sparse_limit, shared_units=args.shared_units)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        ctx.set_observed(idx, val)
        torch.cuda.synchronize()
        setup = time.perf_counter() - ts
        ctx.bind_model(core_run, fac)
        work, tune_s = None, 0.0
        if not args.no_autotune:
            ts = time.perf_counter()
            work = ctx.autotune(None)
            tune_s = time.perf_counter() - ts
        statuses = []
        if args.warmup:
            ctx.iterate(args.warmup, p.lam, strict=False)
            statuses.append(ctx.last_status)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sse, loss = ctx.iterate(args.steps, p.lam, strict=False)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t1
        statuses.append(ctx.last_status)
        not_pd = ctx.not_pd_count()
        ls_rows, ls_max = ctx.solve_stats()
        core_left = int(torch.count_nonzero(core_run))
        units = [ctx.unit_stats(n) for n in range(N)]
        # the model's error by a direct FP64 pass over all entries (untimed)
        _, rmse_direct, _ = ctx.recon_error(p.lam)
        # second pass with per-kernel HIP events on the library's stream
        ctx.set_options(precision=PREC_NAMES[prec], fuse_error=1, profile=1,
                        use_graph=use_graph, pair_cache=cache, approx_rate=approx,
                        sparse_limit=args.sparse_limit, shared_units=args.shared_units)
        ctx.reset_timers()
        ctx.iterate(args.steps, p.lam, strict=False)
        times = ctx.kernel_times()
        core_left_end = int(torch.count_nonzero(core_run))
        ctx.close()
        gname = ("gram_mfma" if prec.startswith("bf16")
                 else "gram_cache_write" if cache else "gram")
        calls, ms = times.get(gname, (0, 0.0))
        return {"elapsed": elapsed, "setup": setup, "sse": sse, "times": times,
                "not_pd": not_pd, "gram_ms": ms / max(calls, 1),
                "value": p.nnz * args.steps / elapsed,
                "rmse": float(rmse_direct), "work": work, "tune_s": tune_s,
                "core_left": core_left, "core_left_end": core_left_end,
                "ls_rows": ls_rows, "ls_max": ls_max,
                "units": units,
                "diverged": 8 in statuses,
                "status": max(statuses, key=lambda v: v != 0),
                "loss": [float(x) for x in loss],
                "rmse_fused": float(np.sqrt(max(sse[-1], 0.0) / p.nnz))}

    main_prec = args.precision
    cache_shapes = {3: (3, 4, 5, 8, 10, 16), 4: (3, 5, 8, 10), 5: (3, 5, 8)}
    cache_bytes = (p.nnz + 1) * ((J * J + 1) // 2 * 2) * 8
    cache_fits = cache_bytes <= 0.4 * torch.cuda.mem_get_info()[1]
    cache_ok = (len(set(p.ranks)) == 1 and not main_prec.startswith("bf16")
                and J in cache_shapes.get(N, ()) and cache_fits)
    if args.pair_cache and not cache_ok:
        raise SystemExit("bench.py: no pair-cache kernel for this workload and precision")
    r = run(main_prec, 1 if args.pair_cache else 0, args.approx_rate)
    log("%s: %.2f ms/step, %.3e nnz*iters/s" % (main_prec, 1e3 * r["elapsed"] / args.steps,
                                                  r["value"]))
    log("kernels: " + ", ".join("%s %.3f ms x%d" % (k, v[1] / max(v[0], 1), v[0])
                                for k, v in sorted(r["times"].items())))

    avg_s = r["gram_ms"] / 1e3
    unit_kernel = None
    if any(on for _, on in r["units"]) and not main_prec.startswith("bf16"):
        # shared-index units: the dominant kernel is the unit class with the
        # most time; its work is the multiply-adds the unit form executes
        # (J^(N-2) (J^2 + e (J + N - 3)) per unit of e entries)
        best = None
        on_modes = [u for u, on in r["units"] if on == 1]
        ix_modes = [n for n, (u, on) in enumerate(r["units"]) if on == 2]
        for c in range(6):
            name = ("delta_index" if c == 5 else "delta_long" if c == 4
                    else "delta_units%d" % (1 << c))
            calls, ms = r["times"].get(name, (0, 0.0))
            if calls and (best is None or ms > best[2]):
                best = (c, calls, ms)
        c, calls, ms = best
        if c == 5:
            # index tables (a kernel of their own, "index_tables"): the tasks
            # apply J^(N-1) + J^(N-2) multiply-adds per entry of the values
            # with 64 entries or more
            fl = 0.0
            for n in ix_modes:
                u = r["units"][n][0]
                fl += (p.nnz - u[8]) * (J ** (N - 1) + J ** (N - 2))
            unit_kernel = {"class": "index", "avg_ms": ms / calls,
                           "flops": 2.0 * fl / len(ix_modes)}
        elif c == 4:
            # long runs: a table of J^N multiply-adds per run, then
            # J^(N-1) + J^(N-2) per entry
            fl = 0.0
            for u in on_modes:
                entries = p.nnz - sum(u[k] << k for k in range(4))
                fl += u[4] * J ** N + entries * (J ** (N - 1) + J ** (N - 2))
            unit_kernel = {"class": "long", "avg_ms": ms / calls,
                           "flops": 2.0 * fl / len(on_modes)}
        else:
            e = 1 << c
            per_unit = J ** (N - 2) * (J * J + e * (J + N - 3))
            # single-entry units also serve the small values of index modes
            counted = [u[c] for u in on_modes] + ([r["units"][n][0][8] for n in ix_modes]
                                                 if c == 0 else [])
            unit_kernel = {"class": e, "avg_ms": ms / calls,
                           "flops": 2.0 * per_unit * sum(counted) / max(1, len(counted))}
        avg_s = unit_kernel["avg_ms"] / 1e3
    # Approx runs: each mode update launches the dense and the sparse-core
    # kernel, and the one not chosen (on the device, from the core's non-zero
    # cells) returns at once. Non-zero cells only fall during a run, so the
    # profiled pass used the sparse kernel throughout when the core was
    # within the limit at its start, and the dense one throughout when it was
    # still above it at its end; a pass that crossed has no roofline.
    sparse_kernel = None
    approx_mixed = False
    if args.approx_rate > 0 and r["times"].get("gram_sparse", (0, 0.0))[0] > 0:
        lim = 0.1 if args.sparse_limit == 0 else args.sparse_limit
        cells = J ** N
        nz0, nz1 = r["core_left"], r["core_left_end"]
        if lim >= 0 and nz0 <= lim * cells:
            calls, ms = r["times"]["gram_sparse"]
            # one multiply-add per non-zero cell (mean of the counts at the
            # start and end of the pass) plus the packed Gram and rhs
            sparse_kernel = {"avg_ms": ms / calls,
                             "flops": 2.0 * p.nnz * (0.5 * (nz0 + nz1) + J * (J + 1) // 2 + J)}
            avg_s = sparse_kernel["avg_ms"] / 1e3
        elif lim >= 0 and nz1 <= lim * cells:
            approx_mixed = True
    if main_prec.startswith("bf16"):
        # matrix-core work per entry and mode: stage 1 J^N (+2x for the split
        # products), Gram J^2 (+2x); the VALU part is not counted here
        mult = 3 if main_prec == "bf16x3" else 1
        flops = 2.0 * p.nnz * mult * (J ** N + J * J)
        bound, unit = "mfma", "TFLOP/s"
    elif unit_kernel:
        flops = unit_kernel["flops"]
        bound, unit = "alu", "TFLOP/s"
    elif sparse_kernel:
        flops = sparse_kernel["flops"]
        bound, unit = "alu", "TFLOP/s"
    else:
        flops = 2.0 * p.nnz * fma_per_nnz_mode(N, J)
        bound, unit = "alu", "TFLOP/s"
    achieved = flops / avg_s / 1e12
    peak = PREC_PEAK[main_prec] / 1e12
    traffic = traffic_record(p.nnz) if args.workload == "c2" and main_prec == "f64" else None
    # two entries per lane on the shapes where that wins (ptk_gram2.hip)
    dual = {(4, 10): 1, (5, 8): 2}
    kname = {"f64": ("k_gram_fast2<%d,%d,%d,double,false>" % (N, J, dual[(N, J)])
                     if (N, J) in dual else "k_gram_fast<%d,%d,U,double>" % (N, J)),
             "f32": "k_gram_fast<%d,%d,U,float>" % (N, J),
             "bf16": "k_gram_mfma<%d,%d,1>" % (N, J),
             "bf16x3": "k_gram_mfma<%d,%d,3>" % (N, J)}[main_prec]
    if args.pair_cache:
        kname = "k_gram_cache_write<%d,%d,%s>" % (N, J, "double" if main_prec == "f64"
                                                   else "float")
        traffic = None
    if unit_kernel:
        e = unit_kernel["class"]
        kname = ("k_delta_long<%d,%d,2> (index tables)" % (N, J)
                 if e == "index"
                 else "k_run_tables<%d,%d> + k_delta_long<%d,%d,2>" % (N, J, N, J) if e == "long"
                 else "k_delta_singles<%d,%d>" % (N, J) if e == 1
                 else "k_delta_units<%d,%d,%d,...>" % (N, J, e))
        if e != "index":           # the committed counters are of k_delta_long<4,10,2>
            traffic = None
    if sparse_kernel:
        kname = "k_gram_sparse<%d,%d,2>" % (N, J)
        traffic = None
    roofline = {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
                "frac": achieved / peak, "traffic": traffic, "kernel": kname,
                "avg_launch_ms": avg_s * 1e3, "flops_per_launch": flops}
    if approx_mixed:
        roofline = None
        log("roofline: none (the core crossed the sparse limit inside the profiled pass)")
    if roofline and main_prec == "f64":
        # context: what a plain loop of independent FP64 FMAs sustains here
        roofline["fma_loop_tflops"] = ptk.fp64_rates(2000)["fma_f64"]

    out = {
        "metric": "nnz*ALS-iters/s for row-wise factor update (1 GPU); fold-in p50/p99 ms",
        "value": r["value"],
        "unit": "nnz*iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * r["elapsed"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": PREC_DTYPE[main_prec],
        "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "nnz": p.nnz, "ranks": list(p.ranks), "dims": list(p.dims),
                   "step": "Alg. 2 iteration: %d mode updates + error" % N},
        "roofline": roofline,
        "setup_s": r["setup"],
        "autotune": {"work_per_mode": r["work"], "seconds": r["tune_s"]},
        "graph": bool(use_graph),
        "pair_cache": bool(args.pair_cache),
        "approx_rate": args.approx_rate,
        "core_cells_left": r["core_left"],
        "core_cells_left_profiled": r["core_left_end"],
        "rmse_after": r["rmse"],
        "rmse_after_fused": r["rmse_fused"],
        "not_pd_rows_timed": int(r["not_pd"]),
        "least_squares_rows_timed": int(r["ls_rows"]),
        "least_squares_max_entries": int(r["ls_max"]),
        "iterate_status": int(r["status"]),
        "loss_non_increasing": bool(all(b <= a * (1 + 1e-9)
                                        for a, b in zip(r["loss"], r["loss"][1:]))),
        "kernel_ms": {k: v[1] / max(v[0], 1) for k, v in r["times"].items()},
        "shared_units": {"option": args.shared_units,
                         "per_mode": [{"units_1_2_4_8_long_tasks_values_tasks_smallunits": u,
                                       "form": ["fused", "units", "index tables"][on]}
                                      for u, on in r["units"]]},
    }
    variants = {}
    if args.approx_rate > 0:
        # the same iterations without removal decide whether the Approx fit
        # is usable (also under --no-variant); an unusable one gets no
        # throughput
        v = run(main_prec, 1 if args.pair_cache else 0, 0.0)
        name = main_prec + " (no removal)"
        variants[name] = {"value": v["value"],
                          "ms_per_step": 1e3 * v["elapsed"] / args.steps,
                          "rmse_after": v["rmse"],
                          "rmse_rel_to_main": v["rmse"] / r["rmse"] - 1.0}
        log("%s: %.2f ms/step, rmse %.6g (main %.6g)" % (
            name, variants[name]["ms_per_step"], v["rmse"], r["rmse"]))
        out["rmse_rel_to_no_removal"] = r["rmse"] / v["rmse"] - 1.0
        out["usable"] = bool(out["rmse_rel_to_no_removal"] <= USABLE_RMSE and not r["diverged"])
        if not out["usable"]:
            out["value"] = None
            out["note"] = ("the Approx fit's RMSE is more than %d %% above that of the same "
                           "iterations without removal: not a usable fit on this workload, "
                           "no throughput reported (ms_per_step is the time of the failed "
                           "fit)" % round(100 * USABLE_RMSE))
            log("approx: unusable (rmse %.6g against %.6g without removal)" % (
                r["rmse"], v["rmse"]))
        out["variants"] = variants
    if not args.no_variant:
        if cache_ok:
            other = 0 if args.pair_cache else 1
            v = run(main_prec, other)
            name = main_prec + ("" if other == 0 else "+pair_cache")
            variants[name] = {"value": v["value"],
                              "ms_per_step": 1e3 * v["elapsed"] / args.steps,
                              "rmse_after": v["rmse"],
                              "rmse_rel_to_main": v["rmse"] / r["rmse"] - 1.0,
                              "kernel_ms": {k: t[1] / max(t[0], 1)
                                            for k, t in v["times"].items()}}
            log("%s: %.2f ms/step, rmse %.6g (main %.6g)" % (
                name, variants[name]["ms_per_step"], v["rmse"], r["rmse"]))
        runs = {}
        for prec in PREC_NAMES:
            if prec == main_prec:
                continue
            if prec.startswith("bf16") and not (N in (3, 4) and J in (8, 10, 16)
                                                and len(set(p.ranks)) == 1):
                continue
            runs[prec] = run(prec)
        # a form whose fit is not within USABLE_RMSE of the FP64 path's RMSE
        # after the same iterations (or that diverged) gets no throughput
        rmse64 = r["rmse"] if main_prec == "f64" else runs.get("f64", {}).get("rmse")
        for prec, v in runs.items():
            rel64 = v["rmse"] / rmse64 - 1.0 if rmse64 else None
            if v["diverged"] or (rel64 is not None and not (rel64 <= USABLE_RMSE)):
                why = ("error or loss not finite, or the loss rose" if v["diverged"] else
                       "RMSE more than %d %% above the FP64 path's" % round(100 * USABLE_RMSE))
                variants[prec] = {"unusable": True, "diverged": bool(v["diverged"]),
                                  "rmse_after": v["rmse"], "rmse_rel_to_f64": rel64,
                                  "note": why + ": not a usable form on this workload, "
                                          "no throughput reported"}
                log("%s: unusable (rmse %.6g, %s), no throughput reported" % (prec, v["rmse"], why))
                continue
            variants[prec] = {"value": v["value"], "ms_per_step": 1e3 * v["elapsed"] / args.steps,
                              "gram_ms": v["gram_ms"], "rmse_after": v["rmse"],
                              "rmse_rel_to_main": v["rmse"] / r["rmse"] - 1.0,
                              "rmse_rel_to_f64": rel64}
            log("%s: %.2f ms/step, rmse %.6g (main %.6g)" % (
                prec, variants[prec]["ms_per_step"], v["rmse"], r["rmse"]))
        if main_prec != "f64" and rmse64:
            out["rmse_rel_to_f64"] = r["rmse"] / rmse64 - 1.0
            out["usable"] = bool(out["rmse_rel_to_f64"] <= USABLE_RMSE and not r["diverged"])
        out["variants"] = variants
        out["variants_note"] = ("same workload, init and iteration count; rmse_after = "
                                "sqrt(SSE/nnz) by a direct FP64 pass after warmup+steps "
                                "iterations; a form whose RMSE is more than %d %% above the "
                                "FP64 path's is marked unusable and gets no throughput"
                                % round(100 * USABLE_RMSE))
    if not args.no_cpu and args.workload == "c2":
        t0 = time.perf_counter()
        out["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
        log("cpu baseline in %.1f s" % (time.perf_counter() - t0))
    out["command"] = command_line()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
