"""bench.py's counter post-processing (host logic, no GPU): the FETCH_SIZE /
WRITE_SIZE records of the assignment GEMMs (copy calibration, largest-grid
launches) and of the re-check on the reported path (dispatches split into
assignments at reset_small_kernel; the call is the assignment before the
first one holding a bound test and the run of those that do)."""
import csv
import hashlib
import json
import os
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))
import bench  # noqa: E402


def _write(dirpath, rows):
    os.makedirs(dirpath, exist_ok=True)
    with open(os.path.join(dirpath, "1_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Grid_Size",
                                          "Counter_Name", "Counter_Value"])
        w.writeheader()
        for i, (name, grid, val) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": grid,
                        "Counter_Name": "C", "Counter_Value": val})


def test_assign_traffic_calibration(tmp_path):
    gib = 1 << 20
    fetch = [("kmx::assign_kernel<2, 4, 4, 128, 8, 1, false, 4>(...)", 4000256, 1000.0),
             ("kmx::assign_kernel<2, 4, 4, 128, 8, 1, false, 4>(...)", 262144, 10.0),
             ("kmx::assign_kernel<2, 4, 4, 128, 8, 1, false, 4>(...)", 4000256, 1200.0)]
    fetch += [("__amd_rocclr_copyBuffer", 1 << 20, gib / 2.0)] * 3
    write = [(n, g, v / 10.0) for n, g, v in fetch[:3]] + [("__amd_rocclr_copyBuffer", 1 << 20,
                                                            float(gib))] * 3
    _write(str(tmp_path / "f"), fetch)
    _write(str(tmp_path / "w"), write)
    rec = bench.traffic_convert(str(tmp_path / "f"), str(tmp_path / "w"))
    assert rec["fetch_factor"] == pytest.approx(2.0) and rec["write_factor"] == pytest.approx(1.0)
    r = rec["assign_fp8"]
    # the largest-grid launches only: (1000 + 1200) / 2 KiB fetched, a tenth written
    assert r["fetch_kib"] == pytest.approx(1100.0) and r["write_kib"] == pytest.approx(110.0)
    assert r["hbm_bytes"] == pytest.approx((1100.0 * 2.0 + 110.0) * 1024.0)
    assert "assign_bf16" not in rec


def test_recheck_traffic_segments_the_bounded_call(tmp_path, monkeypatch):
    R, B, P, F = ("kmx::reset_small_kernel", "kmx::bounds_test_kernel",
                  "kmx::recheck_pair_kernel<32>", "kmx::recheck_full_kernel")
    rows = [(R, 64, 0.0), (P, 1, 500.0), (F, 1, 7.0)]          # an earlier path: not counted
    rows += [(R, 64, 0.0), (P, 1, 100.0), (F, 1, 1.0)]        # first assignment of the call
    rows += [(R, 64, 0.0), (B, 1, 3.0), (P, 1, 40.0), (F, 1, 2.0)] * 3
    rows += [(R, 64, 0.0), (P, 1, 900.0)]                      # a later path: not counted
    _write(str(tmp_path / "f"), rows)
    _write(str(tmp_path / "w"), [(n, g, v / 4.0) for n, g, v in rows])
    fk, nseg, nl = bench._recheck_bytes(str(tmp_path / "f"))
    assert (fk, nseg, nl) == (101.0 + 3 * 42.0, 4, 8)
    # the calibration comes from the assignment record in profiles/
    root = tmp_path / "root"
    (root / "profiles").mkdir(parents=True)
    src = root / "k.hip"
    src.write_text("kernel")
    (root / "profiles" / "assign_traffic_n4m_d512_k1000.json").write_text(
        json.dumps({"fetch_factor": 2.0, "write_factor": 1.0}))
    run = tmp_path / "run.log"
    run.write_text("[bench] ...\n" + json.dumps(
        {"config": {"d": 512}, "paths": {"bounded_routed_fp8": {"short_recheck_entries": 100}}})
        + "\n")
    monkeypatch.setattr(bench, "ROOT", str(root))
    monkeypatch.setattr(bench, "RECHECK_SOURCE", "k.hip")
    rec = bench.traffic_recheck_convert(str(tmp_path / "f"), str(tmp_path / "w"), str(run))
    hbm = ((101.0 + 126.0) * 2.0 + (101.0 + 126.0) / 4.0) * 1024.0
    assert rec["hbm_bytes"] == pytest.approx(hbm)
    assert rec["hbm_bytes_per_entry"] == pytest.approx(hbm / 100)
    assert rec["algorithmic_bytes_per_entry"] == 4.0 * 512 + 24
    assert rec["kernel_source_sha256"] == hashlib.sha256(b"kernel").hexdigest()
    # bench reports it per step while the source keeps that hash
    (root / "profiles" / "recheck_traffic_n4m_d512_k1000.json").write_text(json.dumps(rec))
    assert bench.measured_recheck_traffic(300, 3) == pytest.approx(hbm / 100 * 100)
    src.write_text("kernel, changed")
    assert bench.measured_recheck_traffic(300, 3) is None
