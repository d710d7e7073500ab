"""The oracle's pins catch plausible mistakes (mutation test, CPU only).

Each case plants one mistake in a private copy of the oracle's C source,
builds it, and runs the pin suite against it in a child process; the suite
must fail. The real oracle is never modified.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "ptk_oracle.c")

MUTANTS = {
    "drop_lambda": ("s = B[i * Jn + j] + (i == j ? lambda : 0.0);",
                    "s = B[i * Jn + j];"),
    "sign_of_rhs": ("c[p] += val[e] * delta[p];", "c[p] -= val[e] * delta[p];"),
    "gram_diagonal_only": ("B[p * Jn + q] += delta[p] * delta[q];",
                           "B[p * Jn + q] += delta[p] * delta[p];"),
    "delta_skips_last_cell": (
        "for (int j = 0; j < J[n]; ++j) out[j] = 0.0;\n    for (int64_t s = 0; s < S; ++s)",
        "for (int j = 0; j < J[n]; ++j) out[j] = 0.0;\n    for (int64_t s = 0; s < S - 1; ++s)"),
    "predict_drops_last_mode": ("for (int k = 0; k < N; ++k) p *= rows[k][beta[k]];",
                                "for (int k = 0; k < N - 1; ++k) p *= rows[k][beta[k]];"),
    "core_update_transposed": ("* U[j * J[n] + k];", "* U[k * J[n] + j];"),
    "qr_no_sign_fix": ("if (R[i * Jn + i] < 0.0) {", "if (R[i * Jn + i] < -1e300) {"),
    "back_substitution_index": ("s -= L[k * Jn + i] * a[k];", "s -= L[i * Jn + k] * a[k];"),
    "ls_half_regulariser": ("const double s = sqrt(lambda);",
                            "const double s = sqrt(0.5 * lambda);"),
    "ls_rotation_sign": ("d[q] = cs * d[q] - sn * t;", "d[q] = cs * d[q] + sn * t;"),
    "ls_rhs_not_rotated": ("z[j] = cs * t + sn * x;", "z[j] = t + sn * x;"),
    "ls_back_substitution_index": ("s -= R[j * Jn + q] * a[q];",
                                   "s -= R[q * Jn + j] * a[q];"),
    "ls_last_entry_dropped": ("for (int64_t t = 0; t < cnt; ++t) {\n        const int64_t e = ents[t];",
                              "for (int64_t t = 0; t + 1 < cnt; ++t) {\n        const int64_t e = ents[t];"),
    "heavy_row_skips_first_entry": (
        "for (int64_t t = 0; t < cnt; ++t)\n                ora_ls_add(Jn, R, z, dl + t * Jn, val[re[t]]);",
        "for (int64_t t = 1; t < cnt; ++t)\n                ora_ls_add(Jn, R, z, dl + t * Jn, val[re[t]]);"),
    "cache_no_zero_fallback": ("delta[beta[n]] += an != 0.0 ? Pres[e * S + s] / an",
                               "delta[beta[n]] += 1 ? Pres[e * S + s] / an"),
    "cache_no_rescale": ("Pres[e * S + s] / ao * rows[n][beta[n]]",
                         "Pres[e * S + s]"),
    "approx_error_sign": ("r += with * with - without * without;",
                          "r += without * without - with * with;"),
    "approx_count_ceil": ("(int64_t)floor(p * (double)nz)", "(int64_t)ceil(p * (double)nz)"),
    "approx_ties_reversed": ("return a < b ? -1 : (a > b ? 1 : 0);",
                             "return a > b ? -1 : (a < b ? 1 : 0);"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found exactly once"
    mutant = tmp_path / "mutant.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC",
                           str(mutant), "-o", str(lib), "-lm"])
    env = dict(os.environ, PTK_ORACLE_LIB=str(lib))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p",
                        "no:cacheprovider", os.path.join(ROOT, "tests",
                                                         "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, "pins did not catch mutant %s" % name
