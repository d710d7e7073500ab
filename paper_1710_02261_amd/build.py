"""Build libptucker.so (gfx950) from the HIP sources in csrc/.

Every source is compiled with hipcc for gfx950 only, with packed FP32
instructions disabled, then linked into one shared library next to this file.

    python -m paper_1710_02261_amd.build
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libptucker.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["ptk_api.hip", "ptk_kernels.hip", "ptk_cache.hip", "ptk_approx.hip",
           "ptk_gram2.hip", "ptk_slice.hip", "ptk_solve.hip", "ptk_resolve.hip",
           "ptk_sparse.hip", "ptk_units.hip",
           "ptk_data.hip",
           "ptk_sort.hip", "ptk_finalize.hip", "ptk_mfma.hip", "ptk_server.hip",
           "ptk_ceiling.hip"]

CFLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-I", INCLUDE]
# Matrix-core results written to VGPRs (the VALU folds them right away; the
# accumulation-register form needs a move per result register).
MFMA_FLAGS = ["-mllvm", "-amdgpu-mfma-vgpr-form"]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
    extra = MFMA_FLAGS if src == "ptk_mfma.hip" else []
    cmd = [HIPCC, *CFLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-8000:]))
    return obj


def build(verbose: bool = False) -> str:
    """Compile and link; always rebuilds. Returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    workers = min(len(SOURCES), max(1, (os.cpu_count() or 4)))
    with cf.ThreadPoolExecutor(workers) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s" % r.stderr[-8000:])
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
