"""Host-side tools without a GPU: the rocprofv3 summary parsers, the benchmark's
refusal of several GPUs, and the CLI's argument handling."""
import csv
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write_counter_csv(path, rows):
    cols = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=cols)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(cols, r)))


def test_traffic_scales_counters_by_the_copy_calibration(tmp_path):
    from paper_1810_08142_amd import profiling
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    # a 1024 MiB copy reads 524288 KiB by FETCH_SIZE (factor 2) and writes 1048576 KiB
    _write_counter_csv(fetch, [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0, 0, 1),
                               (2, "ri::ppl::build_w_f64(double const*)", "FETCH_SIZE", 1000.0, 0, 1),
                               (3, "ri::ppl::build_w_f64(double const*)", "FETCH_SIZE", 3000.0, 0, 1)])
    _write_counter_csv(write, [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0, 0, 1),
                               (2, "ri::ppl::build_w_f64(double const*)", "WRITE_SIZE", 10.0, 0, 1),
                               (3, "ri::ppl::build_w_f64(double const*)", "WRITE_SIZE", 30.0, 0, 1)])
    d = profiling.traffic("build_w_f64", str(fetch), str(write), 1024, "h")
    assert d["launches"] == 2
    assert abs(d["copy_calibration"]["fetch_factor"] - 2.0) < 1e-12
    # per launch (2 * FETCH + 1 * WRITE) KiB, averaged
    assert abs(d["hbm_bytes_per_launch"] - ((2 * 1000 + 10) + (2 * 3000 + 30)) / 2 * 1024) < 1e-6


def test_mfma_summary(tmp_path):
    from paper_1810_08142_amd import profiling
    path = tmp_path / "m.csv"
    k = "ri::ppl::build_w_f64(double const*)"
    ns = 1_000_000  # 1 ms
    _write_counter_csv(path, [(5, k, "SQ_INSTS_VALU_MFMA_MOPS_F64", 1e8, 0, ns),
                              (5, k, "SQ_INSTS_VALU_MFMA_MOPS_BF16", 0.0, 0, ns),
                              (5, k, "SQ_VALU_MFMA_BUSY_CYCLES", 1024 * 1.2e6, 0, ns),
                              (5, k, "GRBM_GUI_ACTIVE", 8 * 2.4e6, 0, ns)])
    d = profiling.mfma("build_w_f64", str(path), 2.56e10, 78.6, "h")
    assert d["executed_mfma_flop_per_launch"] == 512 * 1e8
    assert abs(d["executed_tflops"] - 512e8 / 1e-3 / 1e12) < 1e-9
    assert abs(d["mfma_busy_frac"] - 0.5) < 1e-12
    assert abs(d["algorithmic_share"] - 2.56e10 / 5.12e10) < 1e-12


def test_profiler_names_match_one_kernel_exactly():
    from paper_1810_08142_amd.profiling import is_kernel
    assert is_kernel("ri::ppl::build_w_f64(double const*, int)", "build_w_f64")
    assert not is_kernel("ri::ppl::build_w_f64_diag(double const*, int)", "build_w_f64")
    assert is_kernel("ri::ppl::build_w_f64_diag(double const*, int)", "build_w_f64_diag")
    assert is_kernel("void ri::ppl::contract_f64<9>(double const*, long)", "contract_f64")
    assert not is_kernel("void ri::ppl::contract_f64<9>(double const*, long)", "contract_f")


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_bench_counter_summaries_are_keyed_to_the_sources():
    sys.path.insert(0, ROOT)
    import bench
    h = bench.source_hash()
    assert len(h) == 16
    for kernel in ("build_w_f64", "build_w_bf16x3"):
        p = os.path.join(ROOT, "profiles", f"{kernel}_c2_counters.json")
        if os.path.exists(p):
            d = json.load(open(p))
            assert d["kernel"] == kernel and "hbm_bytes_per_launch" in d


def test_cli_lists_its_commands():
    r = subprocess.run([sys.executable, "-m", "paper_1810_08142_amd.cli", "--help"], capture_output=True, text=True,
                       cwd=ROOT)
    assert r.returncode == 0
    for cmd in ("ccsd", "ttc", "shard"):
        assert cmd in r.stdout
