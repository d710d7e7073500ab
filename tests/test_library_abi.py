"""The C-ABI library loads and exports every call include/ptucker.h declares.

CPU only: loading the shared library needs the HIP runtime library, not a GPU;
no compute call is made.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ptucker.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ptk_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_1710_02261_amd import _native
    path = _native.library_path()
    if not os.path.exists(path):
        from paper_1710_02261_amd import build
        build.build()
    return ctypes.CDLL(path)


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for name in ["ptk_create", "ptk_destroy", "ptk_set_observed", "ptk_bind_model",
                 "ptk_update_mode", "ptk_iterate", "ptk_recon_error",
                 "ptk_orthogonalize", "ptk_predict", "ptk_fold_in", "ptk_last_error"]:
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_invalid_arguments_rejected_without_gpu(lib):
    """ptk_create rejects bad shapes before touching the device."""
    lib.ptk_create.restype = ctypes.c_int
    h = ctypes.c_void_p()
    dims = (ctypes.c_int64 * 3)(10, 10, 10)
    bad_ranks = (ctypes.c_int32 * 3)(5, 0, 5)
    assert lib.ptk_create(ctypes.byref(h), 3, dims, bad_ranks, None) == 1
    ranks = (ctypes.c_int32 * 3)(5, 5, 5)
    assert lib.ptk_create(ctypes.byref(h), 1, dims, ranks, None) == 1
    big = (ctypes.c_int32 * 3)(33, 5, 5)
    assert lib.ptk_create(ctypes.byref(h), 3, dims, big, None) == 1
    assert lib.ptk_destroy(None) == 0
