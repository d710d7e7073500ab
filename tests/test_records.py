"""The committed benchmark records (profiles/bench_*.json) are consistent
with themselves and with the counter summaries they cite (CPU only).

* Every record carries the fields of a bench line: metric, value, unit,
  one GPU, synthetic data, a named workload and the command that made it.
* Throughput records: value = entries / seconds per iteration, or no value
  for a fit marked unusable, with the reason.
* Rooflines: frac = achieved / peak with 0 < frac <= 1 against the
  published peak; achieved = flops per launch / average launch time.
* Index-table records: the flops per launch are the task kernel's
  J^(N-1) + J^(N-2) multiply-adds for every entry with a table, recounted
  from the unit statistics the record carries.
* The headline record's traffic is the bytes per launch of the committed
  counter summary, and its CPU baseline is the oracle's.
* Every profile the design notes and the README cite is committed.
"""
import glob
import json
import math
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PEAKS = {"TFLOP/s": (78.6, 157.3, 2500.0, 5000.0), "GB/s": (8000.0,)}


def load(path):
    text = open(path).read().strip()
    try:
        return json.loads(text)
    except json.JSONDecodeError:
        return json.loads(text.splitlines()[-1])


RECORDS = sorted(glob.glob(os.path.join(ROOT, "profiles", "bench_*.json")))


@pytest.mark.parametrize("path", RECORDS, ids=[os.path.basename(p) for p in RECORDS])
def test_record_fields(path):
    r = load(path)
    for key in ("metric", "value", "unit", "n_gpus", "higher_is_better", "dtype", "data",
                "config", "command"):
        assert key in r, key
    assert r["n_gpus"] == 1
    assert r["data"] == "synthetic"
    assert r["command"].startswith("python bench.py")
    if "ms_per_step" in r and r.get("unit") == "nnz*iters/s":
        if r["value"] is None:
            # a fit marked unusable reports no throughput, and says why
            assert r["usable"] is False and r["note"]
        else:
            nnz = r["config"]["nnz"]
            assert math.isclose(r["value"], nnz / (r["ms_per_step"] * 1e-3), rel_tol=1e-6)


@pytest.mark.parametrize("path", RECORDS, ids=[os.path.basename(p) for p in RECORDS])
def test_roofline_arithmetic(path):
    r = load(path)
    roof = r.get("roofline")
    if not roof:
        pytest.skip("no roofline in this record")
    assert roof["bound"] in ("hbm", "mfma", "alu")
    assert roof["peak"] in PEAKS[roof["unit"]]
    assert math.isclose(roof["frac"], roof["achieved"] / roof["peak"], rel_tol=1e-9)
    assert 0.0 < roof["frac"] <= 1.0, roof
    if "flops_per_launch" in roof:
        rate = roof["flops_per_launch"] / (roof["avg_launch_ms"] * 1e-3) / 1e12
        assert math.isclose(roof["achieved"], rate, rel_tol=1e-9)


@pytest.mark.parametrize("path", RECORDS, ids=[os.path.basename(p) for p in RECORDS])
def test_index_table_flops_recounted(path):
    r = load(path)
    roof = r.get("roofline") or {}
    if "(index tables)" not in roof.get("kernel", ""):
        pytest.skip("the dominant kernel is not the index-table task kernel")
    N = len(r["config"]["ranks"])
    J = r["config"]["ranks"][0]
    nnz = r["config"]["nnz"]
    modes = [m["units_1_2_4_8_long_tasks_values_tasks_smallunits"]
             for m in r["shared_units"]["per_mode"] if m["form"] == "index tables"]
    assert modes
    flops = sum(2.0 * (nnz - u[8]) * (J ** (N - 1) + J ** (N - 2)) for u in modes) / len(modes)
    assert math.isclose(roof["flops_per_launch"], flops, rel_tol=1e-9)


def test_headline_traffic_and_cpu_baseline():
    r = load(os.path.join(ROOT, "profiles", "bench_c2.json"))
    t = json.load(open(os.path.join(ROOT, "profiles", "delta_index_c2_traffic.json")))
    roof = r["roofline"]
    assert roof["kernel"].startswith("k_delta_long<4,10,2>")
    assert t["kernel"] == "void ptk::k_delta_long<4, 10, 2>(ptk::LongArgs)"
    assert math.isclose(roof["traffic"], t["bytes_per_launch"], rel_tol=1e-12)
    assert math.isclose(t["bytes_per_launch"],
                        t["fetch_bytes_per_launch"] + t["write_bytes_per_launch"], rel_tol=1e-12)
    cb = r["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] >= 1 and cb["value"] > 0 and cb["sample"]


def test_cited_profiles_exist():
    """Every file under profiles/ that the design notes or the README cite is
    committed (a path followed by * names a family of records)."""
    import re
    missing = []
    for doc in ("DESIGN.md", "README.md"):
        text = open(os.path.join(ROOT, doc)).read()
        for m in re.finditer(r"profiles/[A-Za-z0-9_.\-]+(\*?)", text):
            if m.group(1):
                continue
            path = m.group(0).rstrip(".,)")
            if not os.path.exists(os.path.join(ROOT, path)):
                missing.append((doc, path))
    assert not missing, missing
