"""The COO text reader (ptk_coo_scan / ptk_coo_read): host code in the
library, run here without a GPU.

Checked against a plain Python reading of the same files: N 1-based indices
and a value per line, blanks or tabs between fields, CR LF line ends, blank
lines skipped, a '+' sign and exponents in values; files large enough to be
parsed by several threads; and the refusals (malformed lines with their
line number, index 0, a wrong field count, non-finite values, nnz that does
not match the file, a missing file).
"""
import os

import numpy as np
import pytest

from paper_1710_02261_amd import _native


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not os.path.exists(_native.library_path()):
        from paper_1710_02261_amd import build
        build.build()


def py_read(text, N):
    idx, val = [], []
    for line in text.splitlines():
        f = line.split()
        if not f:
            continue
        idx.append([int(x) - 1 for x in f[:N]])
        val.append(np.float32(float(f[N])))
    idx = np.array(idx, dtype=np.int32).T.reshape(N, -1)
    return np.ascontiguousarray(idx), np.array(val, dtype=np.float32)


def write(tmp_path, name, text):
    p = tmp_path / name
    p.write_bytes(text.encode())
    return str(p)


def test_small_file_with_mixed_layout(tmp_path):
    text = ("1 2 3 0.5\n"
            "\n"
            "4\t5\t6\t-1.25e-3\r\n"
            "   7 8 9   +3   \n"
            "10 1 1 1e2")                      # no final newline
    path = write(tmp_path, "a.tns", text)
    nnz, dims = _native.coo_scan(path, 3)
    assert nnz == 4 and dims == (10, 8, 9)
    idx, val = _native.coo_read(path, 3, nnz)
    want_idx, want_val = py_read(text, 3)
    np.testing.assert_array_equal(idx, want_idx)
    np.testing.assert_array_equal(val, want_val)


def test_large_file_parsed_in_pieces_matches(tmp_path):
    rng = np.random.default_rng(0)
    n, N = 150_000, 4
    ids = rng.integers(1, 100_000, size=(n, N))
    vals = rng.standard_normal(n).astype(np.float32)
    lines = [" ".join(map(str, ids[e])) + " " + repr(float(vals[e])) for e in range(n)]
    text = "\n".join(lines) + "\n"
    assert len(text) > 4 << 20                  # several reader threads
    path = write(tmp_path, "big.tns", text)
    nnz, dims = _native.coo_scan(path, N)
    assert nnz == n
    assert dims == tuple(int(d) for d in ids.max(axis=0))
    idx, val = _native.coo_read(path, N, nnz)
    np.testing.assert_array_equal(idx, (ids - 1).T.astype(np.int32))
    np.testing.assert_array_equal(val, vals)


def test_empty_file(tmp_path):
    path = write(tmp_path, "e.tns", "\n  \n")
    nnz, dims = _native.coo_scan(path, 3)
    assert nnz == 0 and dims == (0, 0, 0)
    idx, val = _native.coo_read(path, 3, 0)
    assert idx.shape == (3, 0) and val.shape == (0,)


@pytest.mark.parametrize("bad,line", [
    ("1 2 3 0.5\n0 2 3 1.0\n", 2),            # index 0 (indices start at 1)
    ("1 2 3 0.5\n\n1 2 1.0\n", 3),            # too few fields
    ("1 2 3 0.5 7\n", 1),                     # too many fields
    ("1 2 x 0.5\n", 1),                       # not an integer
    ("1 2 3 nan\n", 1),                       # not finite
    ("1 2 3 0.5\n1 2 3 1e99\n", 2),           # overflows float32
    ("1 2 3000000000 0.5\n", 1),              # index above 2^31 - 1
])
def test_malformed_lines_are_refused_with_their_number(tmp_path, bad, line):
    path = write(tmp_path, "bad.tns", bad)
    with pytest.raises(_native.PtkError, match="PTK_E_INVALID.*line %d" % line):
        _native.coo_scan(path, 3)


def test_read_refuses_wrong_count_and_missing_file(tmp_path):
    path = write(tmp_path, "c.tns", "1 1 1 1\n2 2 2 2\n")
    with pytest.raises(_native.PtkError, match="holds 2 entries"):
        _native.coo_read(path, 3, 3)
    with pytest.raises(_native.PtkError, match="cannot read"):
        _native.coo_scan(str(tmp_path / "missing.tns"), 3)
    with pytest.raises(_native.PtkError, match="N must be"):
        _native.coo_scan(path, 11)
