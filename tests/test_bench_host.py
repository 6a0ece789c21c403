"""Host checks of bench.py's reading of the committed counter runs (no GPU)."""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_counter_file_is_per_kernel_and_consistent():
    rec = json.load(open(os.path.join(ROOT, "profiles", "apply_c384_f64_pmc.json")))
    assert rec["kernels"], "no kernel in the counter file"
    for name, e in rec["kernels"].items():
        assert name.startswith("hbc::k_apply_win<double"), name
        hbm = (e["fetch_kib_per_dispatch_cold"] * rec["fetch_factor"]
               + e["write_kib_per_dispatch_cold"] * rec["write_factor"]) * 1024
        assert abs(hbm - e["hbm_bytes_per_launch"]) < 1e-6 * hbm
        assert abs(e["traffic_over_alg"] - hbm / rec["alg_bytes_per_launch"]) < 1e-9


def test_traffic_only_for_a_profiled_kernel_on_the_profiled_source(tmp_path, monkeypatch):
    h = bench.kernel_source_hash()
    rec = {"kernel_source_hash": h,
           "kernels": {"hbc::k_a<double>": {"hbm_bytes_per_launch": 123.0}}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "x.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.traffic_from_profile("x.json", "hbc::k_a<double>") == 123.0
    assert bench.traffic_from_profile("x.json", "hbc::k_b<double>") is None
    assert bench.traffic_from_profile("missing.json", "hbc::k_a<double>") is None
    rec["kernel_source_hash"] = "0" * 16
    (tmp_path / "profiles" / "x.json").write_text(json.dumps(rec))
    assert bench.traffic_from_profile("x.json", "hbc::k_a<double>") is None
