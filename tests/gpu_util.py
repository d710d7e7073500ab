"""Helpers of the GPU parity tests: move a synthetic workload to the device,
run the library through its binding, and compare with the FP64 oracle."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_device(p, device="cuda"):
    import torch
    idx = torch.from_numpy(np.ascontiguousarray(p.idx, dtype=np.int32)).to(device)
    val = torch.from_numpy(np.ascontiguousarray(p.val, dtype=np.float32)).to(device)
    core = torch.from_numpy(np.ascontiguousarray(p.core, dtype=np.float32)).to(device)
    fac = [torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(device)
           for a in p.factors]
    return idx, val, core, fac


def context(p, precision=0, chunk_nnz=0, fuse_error=1, profile=0, bind=True,
            pair_cache=0, delta_slices=0, shared_units=0):
    import paper_1710_02261_amd as ptk
    idx, val, core, fac = to_device(p)
    ctx = ptk.Context(p.dims, p.ranks)
    ctx.set_options(precision=precision, chunk_nnz=chunk_nnz, fuse_error=fuse_error,
                    profile=profile, pair_cache=pair_cache, delta_slices=delta_slices,
                    shared_units=shared_units)
    ctx.set_observed(idx, val)
    if bind:
        ctx.bind_model(core, fac)
    return ctx, idx, val, core, fac


def f64(t):
    return t.detach().cpu().numpy().astype(np.float64)


def row_rel_err(got, want):
    """Per-row relative error ||got - want|| / max(||want||, 1e-30)."""
    num = np.linalg.norm(got - want, axis=1)
    den = np.maximum(np.linalg.norm(want, axis=1), 1e-30)
    return num / den
