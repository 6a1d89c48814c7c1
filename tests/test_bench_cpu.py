"""Host logic of bench.py: the HBM traffic summary built from rocprofv3 counter
files, and its lookup, which holds a figure only for the kernel source and the
tuned choice it was taken on."""
import csv
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def write_counters(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})


def test_traffic_summary_scales_and_keys_on_choice(tmp_path):
    b = load_bench()
    copy = "__amd_rocclr_copyBuffer(...)"
    c3 = "void hmm::" + b.TRAFFIC_KERNELS["c3_classify"][0] + "(hmm::DevPtrs, hmm::FwdLaunch)"
    # FETCH_SIZE counts half of a copy's read bytes (scale 2), WRITE_SIZE all of them
    write_counters(tmp_path / "f.csv", "FETCH_SIZE", [(copy, 262144.0)] * 4 + [(c3, 1000.0), (c3, 3000.0)])
    write_counters(tmp_path / "w.csv", "WRITE_SIZE", [(copy, 524288.0)] * 4 + [(c3, 10.0), (c3, 30.0)])
    choice = {"kernel": "tile32", "wg_per_cu": 4, "flags": 1}
    with open(tmp_path / "bench.json", "w") as fh:
        fh.write("[bench] log line\n")
        fh.write(json.dumps({"metric": "m", "tuning": {"c3_classify": {"choice": choice, "source": "cache"}}}) + "\n")
    out = str(tmp_path / "traffic.json")
    b.traffic_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "bench.json"), out=out)
    recs = json.load(open(out))["c3_classify"]
    assert len(recs) == 1
    rec = recs[0]
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["fetch_bytes_per_launch"] == pytest.approx(2000.0 * 1024 * 2.0)
    assert rec["write_bytes_per_launch"] == pytest.approx(20.0 * 1024)
    assert rec["launches"] == 2 and rec["choice"] == choice
    # kernels absent from the counters are not recorded
    assert set(json.load(open(out))) == {"c3_classify"}
    tuned = {"c3_classify": {"choice": choice}}
    got = b.measured_traffic("c3_classify", b.leg_choice(tuned, "c3_classify"), "tile32", path=out)
    assert got == pytest.approx(rec["bytes_per_launch"])
    # another cap or flag set, the heuristics' choice or another family: no figure
    for other in ({**choice, "flags": 0}, {**choice, "wg_per_cu": 2}, b.leg_choice({}, "c3_classify")):
        assert b.measured_traffic("c3_classify", other, "tile32", path=out) is None
    assert b.measured_traffic("c3_classify", choice, "tile16", path=out) is None

    # a run on another choice adds its record beside the first; a run on the same choice replaces it
    other = {**choice, "flags": 0}
    with open(tmp_path / "bench2.json", "w") as fh:
        fh.write(json.dumps({"tuning": {"c3_classify": {"choice": other}}}) + "\n")
    write_counters(tmp_path / "f2.csv", "FETCH_SIZE", [(copy, 262144.0)] * 4 + [(c3, 500.0)])
    write_counters(tmp_path / "w2.csv", "WRITE_SIZE", [(copy, 524288.0)] * 4 + [(c3, 5.0)])
    b.traffic_summary(str(tmp_path / "f2.csv"), str(tmp_path / "w2.csv"), str(tmp_path / "bench2.json"), out=out)
    assert b.measured_traffic("c3_classify", other, "tile32", path=out) == pytest.approx((1000.0 + 5.0) * 1024)
    assert b.measured_traffic("c3_classify", choice, "tile32", path=out) == pytest.approx(rec["bytes_per_launch"])
    b.traffic_summary(str(tmp_path / "f2.csv"), str(tmp_path / "w2.csv"), str(tmp_path / "bench2.json"), out=out)
    assert len(json.load(open(out))["c3_classify"]) == 2
    # records taken on other source are dropped at the next summary
    data = json.load(open(out))
    for r in data["c3_classify"]:
        r["kernel_source_hash"] = "0" * 16
    json.dump(data, open(out, "w"))
    b.traffic_summary(str(tmp_path / "f2.csv"), str(tmp_path / "w2.csv"), str(tmp_path / "bench2.json"), out=out)
    assert [r["choice"] for r in json.load(open(out))["c3_classify"]] == [other]


def test_leg_choice_defaults():
    b = load_bench()
    assert b.leg_choice({}, "c4_grad") == {"kernel": "auto", "wg_per_cu": 0, "flags": 0}
    assert b.leg_choice({"c4_grad": {"choice": {"kernel": "batched", "wg_per_cu": 1}}}, "c4_grad") == \
        {"kernel": "batched", "wg_per_cu": 1, "flags": 0}
    assert set(b.TRAFFIC_LEGS) == set(b.TRAFFIC_KERNELS)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
