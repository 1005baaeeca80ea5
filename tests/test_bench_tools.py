"""Host-side tools of bench.py (no GPU): the traffic summary that turns
rocprofv3 --pmc csv output into HBM bytes per launch, and the kernel-trace
summary.  Synthetic csv trees stand in for a profiler run."""
import csv
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

GEMM = "void bq::cgemm_f64<0, 64, 64, 16, 32, 32, 2, 0, 0, 1>(bq::GemmArgs)"
COMB = "void bq::combine_kernel<1>(bq::CombineArgs)"
COPY = "void at::native::elementwise_kernel<128, 4, direct_copy_kernel>(int)"


@pytest.fixture()
def bench(tmp_path, monkeypatch):
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    monkeypatch.setattr(mod, "TRAFFIC_FILE", str(tmp_path / "traffic.json"))
    return mod


def _pmc_tree(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, grid, value in rows:
            w.writerow({"Kernel_Name": name, "Grid_Size": grid, "Counter_Name": counter, "Counter_Value": value})


def test_traffic_takes_the_largest_launches_only(bench, tmp_path):
    """The benchmark run also launches the GEMM kernel at an eighth of the
    size (the slab leg): only the full-size launches count, and the copy
    calibration scales the counters (FETCH reads half the copied bytes)."""
    full_f, full_w, slab_f, slab_w = 1000.0, 300.0, 125.0, 40.0
    _pmc_tree(str(tmp_path / "f"), "FETCH_SIZE",
              [(GEMM, 16777216, full_f)] * 8 + [(GEMM, 2097152, slab_f)] * 32 + [(COMB, 134217728, 50.0)] * 6
              + [(COMB, 8192, 1.0)] * 3)
    _pmc_tree(str(tmp_path / "w"), "WRITE_SIZE",
              [(GEMM, 16777216, full_w)] * 8 + [(GEMM, 2097152, slab_w)] * 32 + [(COMB, 134217728, 70.0)] * 6
              + [(COMB, 8192, 2.0)] * 3)
    copy_bytes = 1 << 20
    _pmc_tree(str(tmp_path / "cf"), "FETCH_SIZE", [(COPY, 4096, copy_bytes / 1024 / 2)])
    _pmc_tree(str(tmp_path / "cw"), "WRITE_SIZE", [(COPY, 4096, copy_bytes / 1024)])
    bench.summarize_pmc(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "cf"), str(tmp_path / "cw"),
                        copy_bytes)
    out = json.load(open(bench.TRAFFIC_FILE))
    assert out["dispatches"] == [8, 8]
    assert out["fetch_scale"] == pytest.approx(2.0) and out["write_scale"] == pytest.approx(1.0)
    assert out["bytes_per_launch"] == pytest.approx((full_f * 2.0 + full_w) * 1024)
    assert out["combine_bytes_per_launch"] == pytest.approx((50.0 * 2.0 + 70.0) * 1024)
    # the bench line reports it only while the kernel source is unchanged
    assert bench.traffic_per_launch() == pytest.approx(out["bytes_per_launch"])
    out["kernel_source_sha256"] = "0" * 64
    json.dump(out, open(bench.TRAFFIC_FILE, "w"))
    assert bench.traffic_per_launch() is None


def test_trace_summary_groups_by_name_and_grid(bench, tmp_path):
    d = tmp_path / "trace"
    d.mkdir()
    with open(d / "run_kernel_trace.csv", "w", newline="") as f:
        fields = ["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Start_Timestamp", "End_Timestamp", "VGPR_Count",
                  "Accum_VGPR_Count", "Scratch_Size", "LDS_Block_Size"]
        w = csv.DictWriter(f, fieldnames=fields)
        w.writeheader()
        for i, (name, gx, dur) in enumerate([(GEMM, 16777216, 4e8), (GEMM, 16777216, 2e8), (GEMM, 2097152, 5e7),
                                            (COMB, 134217728, 7e6)]):
            w.writerow({"Kernel_Name": name, "Grid_Size_X": gx, "Grid_Size_Y": 1, "Start_Timestamp": 10 * i,
                        "End_Timestamp": 10 * i + int(dur), "VGPR_Count": 128, "Accum_VGPR_Count": 0,
                        "Scratch_Size": 0, "LDS_Block_Size": 69632})
    out = tmp_path / "sum.tsv"
    bench.summarize_trace(str(d), str(out))
    lines = out.read_text().splitlines()
    rows = [l.split("\t") for l in lines[1:]]
    assert rows[0][1] == "16777216" and rows[0][3] == "2" and float(rows[0][5]) == pytest.approx(300.0)
    assert {(r[1], r[3]) for r in rows} == {("16777216", "2"), ("2097152", "1"), ("134217728", "1")}
