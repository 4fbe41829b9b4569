"""Host logic of bench.py (no GPU): the single-GPU guard, the PMC summary's
calibration arithmetic and the rule that a traffic figure is reported only for
the kernel source it was measured on."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def _counters(d, rows):
    os.makedirs(d)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Value"])
        w.writeheader()
        for name, kib in rows:
            w.writerow({"Kernel_Name": name, "Counter_Value": kib})


def test_pmc_summary_scales_by_the_calibration_copy(tmp_path, capsys):
    half = bench.COPY_BYTES / 1024 / 2          # a counter that reads half the copied bytes
    _counters(tmp_path / "cf", [("__amd_rocclr_copyBuffer", half)])
    _counters(tmp_path / "cw", [("__amd_rocclr_copyBuffer", 2 * half)])
    # two launches of a backward sweep, one of the factorisation, one unclassified
    _counters(tmp_path / "f", [("void k_bwd_wave<float2, 16, 1>", 100.0),
                               ("void k_bwd_large<float2, 256, 32, 1>", 300.0),
                               ("void k_factor_large<float2, 16, 256>", 1000.0),
                               ("some_other_kernel", 5.0)])
    _counters(tmp_path / "w", [("void k_bwd_wave<float2, 16, 1>", 10.0),
                               ("void k_bwd_large<float2, 256, 32, 1>", 30.0),
                               ("void k_factor_large<float2, 16, 256>", 50.0),
                               ("some_other_kernel", 5.0)])
    bench.pmc_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"),
                      str(tmp_path / "cw"))
    out = capsys.readouterr().out
    line = next(ln for ln in out.splitlines() if ln.startswith("traffic_json: "))
    d = json.loads(line[len("traffic_json: "):])
    assert d["calibration"] == {"fetch": 2.0, "write": 1.0}
    sb = d["classes"]["sweep_bwd"]
    assert sb["launches"] == 2
    assert sb["fetch_per_launch"] == pytest.approx((100 + 300) * 1024 * 2.0 / 2)
    assert sb["write_per_launch"] == pytest.approx((10 + 30) * 1024 * 1.0 / 2)
    assert sb["bytes_per_launch"] == pytest.approx(sb["fetch_per_launch"] + sb["write_per_launch"])
    assert d["classes"]["front_lu"]["launches"] == 1
    assert set(d["classes"]) == {"sweep_bwd", "front_lu"}
    assert sb["source_sha"] == bench.source_sha("sweep_bwd")


def test_traffic_is_reported_only_for_the_measured_source(tmp_path, monkeypatch):
    summary = tmp_path / "pmc.md"
    good = {"launches": 3, "bytes_per_launch": 123.0, "source_sha": bench.source_sha("sweep_bwd")}
    stale = {"launches": 3, "bytes_per_launch": 456.0, "source_sha": "0000000000000000"}
    summary.write_text("# summary\n\ntraffic_json: " +
                       json.dumps({"classes": {"sweep_bwd": good, "sweep_fwd": stale}}) + "\n")
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(summary))
    assert bench.measured_traffic("sweep_bwd") == 123.0
    assert bench.measured_traffic("sweep_fwd") is None         # kernels changed since
    assert bench.measured_traffic("stencil") is None           # never measured
    monkeypatch.setattr(bench, "PMC_SUMMARY", str(tmp_path / "absent.md"))
    assert bench.measured_traffic("sweep_bwd") is None
