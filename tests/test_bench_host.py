"""Host-side part of bench.py that needs no GPU: the counter traffic record."""
import csv
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _write_counters(d, counter, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for disp, name, value in rows:
            w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_record_scales_by_the_copy_probe(tmp_path):
    """A kernel that reads 3 and writes 2 units while the copy probe reads and writes 1 unit each
    (the counters reporting half the copy's fetched bytes, as FETCH_SIZE does) moves 5 units;
    counters split over several rows of one dispatch are summed; the sources are hashed."""
    import bench

    mib = 4
    kib = mib * 1024
    k = "void vs::row_pass_kernel<float, float, 512, 1, false>(vs::PassArgs)"
    _write_counters(str(tmp_path / "f"), "FETCH_SIZE", [
        (1, "__amd_rocclr_copyBuffer", kib / 2), (2, k, 1.5 * kib / 2), (2, k, 1.5 * kib / 2),
        (3, k, 3 * kib / 2), (4, "other_kernel", 99.0)])
    _write_counters(str(tmp_path / "w"), "WRITE_SIZE", [
        (1, "__amd_rocclr_copyBuffer", kib), (2, k, 2 * kib), (3, k, 2 * kib)])
    rec = bench.traffic_record(str(tmp_path / "f"), str(tmp_path / "w"), "row_merged",
                               r"row_pass_kernel<float, float, 512, 1, false>", 2.0, mib, "fetch", "write", "test")
    assert rec["dispatches"] == 2
    assert rec["fetch_scale"] == pytest.approx(2.0) and rec["write_scale"] == pytest.approx(1.0)
    assert rec["traffic_bytes_per_dispatch"] == pytest.approx(5 * mib * 2 ** 20)
    assert rec["traffic_bytes_per_map_pass"] == pytest.approx(2.5 * mib * 2 ** 20)
    assert rec["source_files"] == bench.TRAFFIC_SOURCES["row_merged"] and len(rec["source_sha256"]) == 64

