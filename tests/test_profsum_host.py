"""rocprofv3 summary arithmetic (no GPU): the HBM counters of the iteration
and combine kernels are scaled by what the same counters read for the
calibration copy of known size; per-wave SQ figures divide by SQ_WAVES; the
last dispatch of a kernel is the one reported."""
import csv
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2308_01654_amd import profsum  # noqa: E402


def _write(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"], r)))


def test_traffic_scaled_by_the_calibration_copy(tmp_path):
    kib = profsum.COPY_BYTES / 1024.0
    # the fetch counter reads half the copy's bytes (scale 2), the write counter all of them
    # (scale 1); dimensions of one dispatch are summed; the last k_batch dispatch is used
    _write(tmp_path / "f", [
        (1, "mppi_impl::k_copy(...)", "FETCH_SIZE", kib / 4), (1, "mppi_impl::k_copy(...)", "FETCH_SIZE", kib / 4),
        (2, "void mppi_impl::k_batch<16, 3, false>(...)", "FETCH_SIZE", 999.0),
        (3, "void mppi_impl::k_combine<2>(...)", "FETCH_SIZE", 50.0),
        (4, "void mppi_impl::k_batch<16, 3, false>(...)", "FETCH_SIZE", 100.0)])
    _write(tmp_path / "w", [
        (1, "mppi_impl::k_copy(...)", "WRITE_SIZE", kib),
        (2, "void mppi_impl::k_batch<16, 3, false>(...)", "WRITE_SIZE", 1.0),
        (3, "void mppi_impl::k_combine<2>(...)", "WRITE_SIZE", 2.0),
        (4, "void mppi_impl::k_batch<16, 3, false>(...)", "WRITE_SIZE", 300.0)])
    out = tmp_path / "t.json"
    profsum.traffic(str(tmp_path / "f"), str(tmp_path / "w"), str(out))
    r = json.loads(out.read_text())
    assert abs(r["fetch_scale"] - 2.0) < 1e-12 and abs(r["write_scale"] - 1.0) < 1e-12
    assert r["fetch_bytes_per_launch"] == 100.0 * 1024 * 2
    assert r["write_bytes_per_launch"] == 300.0 * 1024
    assert r["hbm_bytes_per_launch"] == int(100.0 * 1024 * 2 + 300.0 * 1024)
    assert r["combine_fetch_bytes_per_launch"] == 50.0 * 1024 * 2
    assert r["kernel_source_sha256_16"] == profsum.kernel_source_hash()


def test_counters_per_wave_and_executed_flops(tmp_path):
    _write(tmp_path / "a", [
        (7, "void mppi_impl::k_batch<16, 3, false>(...)", "SQ_WAVES", 2048.0),
        (7, "void mppi_impl::k_batch<16, 3, false>(...)", "SQ_INSTS_VALU", 2048.0 * 10)])
    _write(tmp_path / "b", [
        (9, "void mppi_impl::k_batch<16, 3, false>(...)", "SQ_INSTS_VALU_FLOPS_FP32", 1000.0)])
    out = tmp_path / "c.json"
    profsum.counters([str(tmp_path / "a"), str(tmp_path / "b")], str(out))
    r = json.loads(out.read_text())
    assert r["per_wave"]["SQ_INSTS_VALU"] == 10.0
    # an FMA instruction counts 2 flops in the counter; every lane of the wave counts
    assert r["executed_fp32_flop_per_dispatch"] == 64.0 * 1000.0


def test_trace_record_of_the_most_frequent_launches(tmp_path):
    d = tmp_path / "t"
    d.mkdir()
    with open(d / "run_kernel_stats.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Name", "Calls", "TotalDurationNs", "AverageNs", "Percentage", "MinNs", "MaxNs", "StdDev"])
        w.writerow(["void mppi_impl::k_batch<16, 3, false>(...)", 200, 7000000, 35000.0, 80, 33000, 41000, 1])
        w.writerow(["void mppi_impl::k_batch<8, 3, false>(...)", 3, 300, 100.0, 1, 90, 110, 1])
        w.writerow(["void mppi_impl::k_combine<2>(...)", 200, 900000, 4500.0, 10, 4000, 5000, 1])
        w.writerow(["mppi_impl::k_copy(...)", 3, 300000, 100000.0, 9, 99000, 101000, 1])
    out = tmp_path / "trace.json"
    profsum.trace(str(d), str(out))
    r = json.loads(out.read_text())
    assert r["iteration"]["calls"] == 200 and r["iteration"]["average_ns"] == 35000.0
    assert "k_batch<16" in r["iteration"]["kernel"]
    assert r["combine"]["average_ns"] == 4500.0
    assert r["kernel_source_sha256_16"] == profsum.kernel_source_hash()
