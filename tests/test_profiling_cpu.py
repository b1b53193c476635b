"""CPU tests of the rocprofv3 summary helpers (paper_1811_01201_amd.profiling):
kernel names keep their template arguments, counters are averaged per
dispatch, and HBM traffic is scaled by the largest copy dispatch."""
import csv

import pytest

from paper_1811_01201_amd import profiling

HEAD = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HEAD)
        for disp, name, counter, value, t0, t1 in rows:
            w.writerow([disp, disp, 1, 1, 1, 1, 256, 7, name, 256, 0, 0, 8, 0, 16, counter, value, t0, t1])


def test_short_name_keeps_template_arguments():
    n = "void apsp::phase3_kernel<apsp::ArF32W, apsp::NoAlt, 256, 128, (apsp::P3Set)1, 8>(void*, long, int)"
    assert profiling.short_name(n) == "phase3_kernel<ArF32W, NoAlt, 256, 128, (P3Set)1, 8>"
    assert profiling.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_counters_average_per_dispatch(tmp_path):
    p = tmp_path / "c.csv"
    _write(p, [(1, "k<1>(int)", "X", 10, 0, 1000000), (2, "k<1>(int)", "X", 30, 0, 3000000),
               (3, "other(int)", "X", 5, 0, 500000)])
    c = profiling.counters([str(p)])
    assert c["k<1>"]["dispatches"] == 2 and c["k<1>"]["X"] == 20
    assert c["k<1>"]["avg_ms"] == pytest.approx(2.0)
    assert c["other"]["X"] == 5


def test_traffic_scales_by_the_largest_copy(tmp_path):
    f = tmp_path / "f.csv"
    w = tmp_path / "w.csv"
    # the restore copy of 4 KiB reads 2 KiB by the counter (scale 2) and writes 4 KiB (scale 1);
    # a 4-byte read-back copy must not enter the scale
    _write(f, [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 2.0, 0, 10), (2, "__amd_rocclr_copyBuffer",
               "FETCH_SIZE", 0.5, 0, 10), (3, "phase3_kernel<A>(x)", "FETCH_SIZE", 100.0, 0, 10)])
    _write(w, [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 4.0, 0, 10), (2, "__amd_rocclr_copyBuffer",
               "WRITE_SIZE", 0.25, 0, 10), (3, "phase3_kernel<A>(x)", "WRITE_SIZE", 50.0, 0, 10)])
    res = profiling.traffic(str(f), str(w), r"phase3_kernel", 4096)
    assert res["fetch_scale"] == pytest.approx(2.0) and res["write_scale"] == pytest.approx(1.0)
    k = res["kernels"]["phase3_kernel<A>"]
    assert k["fetch_bytes"] == pytest.approx(100 * 1024 * 2) and k["write_bytes"] == pytest.approx(50 * 1024)


def test_traffic_file_roundtrip_and_source_hash(tmp_path):
    p = tmp_path / "t.txt"
    p.write_text("# comment\nkernel=k<1>\ntraffic_bytes_per_launch=123\nsource_sha256=abc\n")
    d = profiling.read_traffic_file(str(p))
    assert d == {"kernel": "k<1>", "traffic_bytes_per_launch": "123", "source_sha256": "abc"}
    assert profiling.read_traffic_file(str(tmp_path / "missing.txt")) is None
    h = profiling.kernel_source_hash()
    assert len(h) == 64 and h == profiling.kernel_source_hash()
