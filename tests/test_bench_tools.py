"""Host-side checks of bench.py's profiler summarizers on small synthetic
rocprofv3-style CSV files (no GPU): the launch statistics behind the
committed kernel-trace summaries, the per-dispatch counter means behind the
traffic figures, and the clock each kernel family kept."""
import csv
import importlib.util
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


TRACE_HEADER = ["Kernel_Name", "Dispatch_Id", "Start_Timestamp", "End_Timestamp"]


def test_summarize_trace_orders_by_start_and_skips_warmup(tmp_path, capsys):
    bench = _bench()
    ring = "void stk::wave3d_ring_kernel<4>(stk::WaveLaunch)"
    other = "void stk::copy_kernel(float*)"
    # Dispatch ids deliberately out of time order; the other kernel must be
    # filtered out.  Durations (ns): 1000 (warm-up), 400, 500, 600.
    rows = [
        [ring, 7, 10_000, 10_400],
        [ring, 3, 1_000, 2_000],
        [other, 4, 3_000, 9_000],
        [ring, 9, 20_000, 20_500],
        [ring, 11, 30_000, 30_600],
    ]
    path = tmp_path / "k_kernel_trace.csv"
    _write(str(path), TRACE_HEADER, rows)
    out = bench.summarize_trace(str(path), "wave3d_ring_kernel", 1)
    assert out["launches_total"] == 4 and out["launches"] == 3 and out["skipped"] == 1
    assert out["kernels"] == [ring]
    assert out["mean_us"] == pytest.approx(0.5)
    assert out["median_us"] == pytest.approx(0.5)
    assert out["min_us"] == pytest.approx(0.4) and out["max_us"] == pytest.approx(0.6)
    assert out["sum_ms"] == pytest.approx(0.0015, abs=1e-3)
    assert "wave3d_ring_kernel" in capsys.readouterr().out


def test_summarize_trace_no_match_reports_zero_launches(tmp_path):
    bench = _bench()
    path = tmp_path / "k_kernel_trace.csv"
    _write(str(path), TRACE_HEADER, [["void a()", 1, 0, 10]])
    out = bench.summarize_trace(str(path), "absent_kernel", 0)
    assert out["launches"] == 0 and "mean_us" not in out


def test_summarize_counters_sums_instances_per_dispatch(tmp_path):
    bench = _bench()
    header = ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"]
    k = "void stk::zm3d_kernel<1>()"
    # FETCH_SIZE reported per dimension instance: two rows per dispatch that
    # must be summed before averaging over dispatches.
    rows = [
        [k, 1, "FETCH_SIZE", 100.0], [k, 1, "FETCH_SIZE", 50.0],
        [k, 2, "FETCH_SIZE", 200.0], [k, 2, "FETCH_SIZE", 10.0],
        [k, 1, "WRITE_SIZE", 30.0], [k, 2, "WRITE_SIZE", 50.0],
    ]
    a = tmp_path / "a_counter_collection.csv"
    _write(str(a), header, rows)
    out = bench.summarize_counters([str(a)])
    fetch = out[k]["FETCH_SIZE"]
    assert fetch["dispatches"] == 2
    assert fetch["mean"] == pytest.approx((150.0 + 210.0) / 2)
    assert sorted(fetch["values"]) == [150.0, 210.0]
    assert out[k]["WRITE_SIZE"]["mean"] == pytest.approx(40.0)


def test_summarize_clock_ghz_from_grbm_count(tmp_path):
    bench = _bench()
    d = tmp_path / "prof" / "host"
    ring = "void stk::wave3d_ring_kernel<4, 1>(stk::WaveLaunch, int)"
    copy = "void stk::copy_kernel(float*)"
    # 100 us at 2.1 GHz on 8 XCDs -> GRBM_COUNT = 8 * 2.1e9 * 1e-4 = 1.68e6,
    # reported as two instances; 200 us at 2.4 GHz for the copy kernel; a
    # 20 us dispatch is below the 50 us floor and must be dropped.
    _write(str(d / "run_kernel_trace.csv"), TRACE_HEADER, [
        [ring, 1, 0, 100_000],
        [copy, 2, 200_000, 400_000],
        [ring, 3, 500_000, 520_000],
    ])
    _write(str(d / "run_counter_collection.csv"),
           ["Kernel_Name", "Dispatch_Id", "Counter_Name", "Counter_Value"], [
               [ring, 1, "GRBM_COUNT", 1.0e6], [ring, 1, "GRBM_COUNT", 0.68e6],
               [copy, 2, "GRBM_COUNT", 8 * 2.4e9 * 2e-4],
               [ring, 3, "GRBM_COUNT", 8 * 2.4e9 * 2e-5],
           ])
    out = bench.summarize_clock(str(tmp_path / "prof"))
    ring_key = "stk::wave3d_ring_kernel<4, 1>"
    copy_key = "stk::copy_kernel"
    assert set(out) == {ring_key, copy_key}
    assert out[ring_key]["launches"] == 1
    assert out[ring_key]["ghz"][0] == pytest.approx(2.1, abs=1e-3)
    assert out[ring_key]["us"][0] == pytest.approx(100.0)
    assert out[copy_key]["ghz"][0] == pytest.approx(2.4, abs=1e-3)


def test_multi_gpu_request_exits_with_message(capsys, monkeypatch):
    bench = _bench()
    monkeypatch.setattr("sys.argv", ["bench.py", "--gpus", "2"])
    with pytest.raises(SystemExit) as e:
        bench.main()
    assert e.value.code == 2
    assert "one GPU" in capsys.readouterr().out
