"""The FP64 rate probe behind the roofline context (ptk_fp64_rates): the
three rates are finite, below the published FP64 peak of 78.6 TFLOP/s, and
above a floor that only a broken launch would miss; bad arguments are
refused."""
import math

import pytest

pytestmark = pytest.mark.gpu


def test_fp64_rates_are_plausible():
    import torch
    assert torch.cuda.is_available()
    import paper_1710_02261_amd as ptk
    r = ptk.fp64_rates(500)
    print(r, flush=True)
    for k in ("fma_f64", "mfma_f64", "both"):
        assert math.isfinite(r[k]) and 5.0 < r[k] < 160.0, (k, r[k])
    assert r["fma_f64"] < 78.6 * 1.05
    with pytest.raises(ptk.PtkError, match="PTK_E_INVALID"):
        ptk.fp64_rates(0)
