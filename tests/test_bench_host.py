"""Host logic of bench.py (no GPU): kernel-name matching for the profiler's names, the
counter-derived traffic record (calibration scaling, the last `launches` dispatches, the
algorithmic bytes of a flop-bound class), the per-kernel counter totals, and the summary
of the GEMM tile autotuner's table."""
import csv
import json

import pytest

import bench


def _write_counters(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for d, k, c, v in rows:
            w.writerow(dict(Dispatch_Id=d, Kernel_Name=k, Counter_Name=c, Counter_Value=v))


def test_kernel_names_match_labels():
    m = bench._kernel_matches
    assert m("void pv::gemm_kernel<0, 64, 64>(pv::GemmDesc const*, int const*, int)", "gemm_kernel<0>+gemm_packed_kernel<0>")
    assert m("void pv::gemm_packed_kernel<0, 32, 32>(pv::GemmPack, int, int)", "gemm_kernel<0>+gemm_packed_kernel<0>")
    assert not m("void pv::gemm_kernel<1, 64, 64>(pv::GemmDesc const*, int const*, int)", "gemm_kernel<0>+gemm_packed_kernel<0>")
    assert not m("void pv::gemm_kernel<2, 64, 64>(x)", "gemm_kernel<0>")
    assert m("void pv::tridiag_step_kernel<8>(pv::EigDesc const*, int)", "tridiag_step_kernel")
    assert not m("pv::tridiag_step_kernelx(int)", "tridiag_step_kernel")


def test_traffic_record_scales_by_the_copy_and_takes_the_last_launches(tmp_path):
    K = "void pv::gemm_kernel<0, 64, 64>(a)"
    P = "void pv::gemm_packed_kernel<0, 32, 32>(b)"
    # warmup dispatches 1-2 (ignored), then the two launches of the last pass
    _write_counters(tmp_path / "f.csv", [(1, K, "FETCH_SIZE", 999.0), (2, P, "FETCH_SIZE", 999.0),
                                         (3, "pv::wstep_kernel(c)", "FETCH_SIZE", 5.0),
                                         (4, K, "FETCH_SIZE", 100.0), (5, P, "FETCH_SIZE", 300.0)])
    _write_counters(tmp_path / "w.csv", [(1, K, "WRITE_SIZE", 7.0), (2, P, "WRITE_SIZE", 7.0),
                                         (4, K, "WRITE_SIZE", 10.0), (5, P, "WRITE_SIZE", 30.0)])
    cal = 1 << 20  # 1 MiB copy: fetch reads half of it, write all of it
    _write_counters(tmp_path / "cf.csv", [(1, "copy", "FETCH_SIZE", cal / 1024 / 2)])
    _write_counters(tmp_path / "cw.csv", [(1, "copy", "WRITE_SIZE", cal / 1024)])
    line = {"config": {"workload": "w"},
            "roofline": {"kernel": "gemm_kernel<0>+gemm_packed_kernel<0>", "launches": 2, "unit": "TFLOP/s",
                         "achieved": 1.0, "avg_launch_ms": 0.01},
            "kernel_classes": {"gemm_f64_mfma": {"ms": 2.0, "calls": 4, "gbs": 50.0}}}
    (tmp_path / "b.json").write_text("# a log line\n" + json.dumps(line) + "\n")
    r = bench.pmc_traffic(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), str(tmp_path / "cf.csv"),
                          str(tmp_path / "cw.csv"), str(tmp_path / "b.json"), cal, "cmd")
    assert r["fetch_factor"] == pytest.approx(2.0) and r["write_factor"] == pytest.approx(1.0)
    assert r["read_bytes_per_launch"] == pytest.approx((100 + 300) * 1024 * 2.0 / 2)
    assert r["write_bytes_per_launch"] == pytest.approx((10 + 30) * 1024 / 2)
    assert r["traffic_bytes_per_launch"] == pytest.approx(r["read_bytes_per_launch"] + r["write_bytes_per_launch"])
    # 50 GB/s over 2 ms in 4 launches: 25 MB per launch
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(25e6)
    assert r["kernel_source_sha256"] == bench._kernel_hash()


def test_counter_totals_per_kernel(tmp_path):
    K = "void pv::gemm_kernel<0, 64, 64>(a)"
    _write_counters(tmp_path / "p.csv", [(1, K, "A", 1.0), (1, K, "B", 2.0), (2, K, "A", 3.0), (2, K, "B", 4.0),
                                         (3, "pv::wstep_kernel(c)", "A", 0.5)])
    lines = bench.pmc_summary(str(tmp_path / "p.csv")).splitlines()
    assert lines[0] == "| kernel | dispatches | A | B |"
    assert lines[2] == "| pv::gemm_kernel<0, 64, 64> | 2 | 4 | 6 |"
    assert lines[3] == "| pv::wstep_kernel | 1 | 0.5 | 0 |"


def test_tuner_summary_counts_decided_keys():
    rows = [dict(prec=0, tiles_log2=5, k_log2=6, choice=1, tflops64=1.0, tflops32=2.0),
            dict(prec=0, tiles_log2=10, k_log2=7, choice=1, tflops64=20.0, tflops32=22.0),
            dict(prec=0, tiles_log2=13, k_log2=7, choice=0, tflops64=31.0, tflops32=26.0),
            dict(prec=0, tiles_log2=3, k_log2=2, choice=-1, tflops64=0.0, tflops32=0.0)]
    s = bench.gemm_tiles_summary("tune", rows)
    assert (s["keys"], s["decided"], s["small_chosen"], s["rule_agrees"]) == (4, 3, 2, 2)
    assert s["table"][1] == [0, 10, 7, 1, 20.0, 22.0]
    assert bench.gemm_tiles_summary("rule", rows) == {"mode": "rule"}
