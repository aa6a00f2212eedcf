"""bench.py's profile summaries, on small synthetic rocprofv3 databases with known values:
HBM traffic from FETCH_SIZE and WRITE_SIZE scaled by the reference copy, kernel times in
microseconds as rocprofv3 stores them, and the VALU and clock figures."""
import json
import os
import sqlite3

import pytest

import bench

STEP = "void clbm::k_step2<float, false, 14, 512, unsigned int>(float const*, float*, clbm::LatticeConst, int, int, int)"
COPY = "clbm::k_stream_copy(HIP_vector_type<float, 4u>*, HIP_vector_type<float, 4u> const*, unsigned long)"


def _db(path, top=None, counters=None):
    con = sqlite3.connect(path)
    con.execute("create table top_kernels (name text, total_calls int, total_duration real, "
                "average real, percentage real)")
    con.execute("create table counters_collection (kernel_name text, grid_size int, value real, "
                "counter_name text)")
    for r in top or []:
        con.execute("insert into top_kernels values (?, ?, ?, ?, ?)", r)
    for r in counters or []:
        con.execute("insert into counters_collection values (?, ?, ?, ?)", r)
    con.commit()
    con.close()
    return str(path)


def test_traffic_summary(tmp_path):
    top = [(STEP, 210, 93368.2, 444.61, 90.0), (COPY, 12, 8394.1, 699.5, 8.1)]
    trace = _db(tmp_path / "t.db", top=top)
    fetch = _db(tmp_path / "f.db", counters=[(STEP, 1, 100.0, "FETCH_SIZE"), (STEP, 1, 100.0, "FETCH_SIZE"),
                                             (COPY, 1, 1048576.0, "FETCH_SIZE")])
    write = _db(tmp_path / "w.db", counters=[(STEP, 1, 300.0, "WRITE_SIZE"),
                                             (COPY, 1, 2097152.0, "WRITE_SIZE")])
    out = tmp_path / "out"
    bench.summarize_profiles(trace, fetch, write, "fp32", 64, ["cmd a", "cmd b", "cmd c"], out_dir=str(out))
    prof = json.load(open(out / "step_cavity64_fp32_hbm_traffic.json"))
    # the copy moves 2 GiB each way: FETCH_SIZE reads half of it (scale 2), WRITE_SIZE all
    assert prof["fetch_scale"] == pytest.approx(2.0) and prof["write_scale"] == pytest.approx(1.0)
    assert prof["traffic_bytes_per_launch"] == pytest.approx((100 * 2 + 300) * 1024)
    assert prof["algorithmic_bytes_per_launch"] == 112 * 64 * 64 * 2
    assert prof["steps_per_launch"] == 2 and prof["trace_avg_us"] == pytest.approx(444.61)
    md = open(out / "step_cavity64_fp32_rocprof.md").read()
    assert "| clbm::k_step2<float, false, 14, 512, unsigned int> | 210 | 93368.2 | 444.61 | 90.00 |" in md
    assert prof["source_digest"] in md


def test_valu_summary(tmp_path):
    db = _db(tmp_path / "v.db", top=[(STEP, 21, 10500.0, 500.0, 90.0)],
             counters=[(STEP, 1, 8e6, "GRBM_GUI_ACTIVE"), (STEP, 1, 2.048e8, "SQ_ACTIVE_INST_VALU"),
                       (STEP, 1, 1.5e8, "SQ_INSTS_VALU"), (STEP, 1, 1.0e8, "SQ_BUSY_CU_CYCLES")])
    bench.summarize_valu(db, "fp32", 64, "cmd", out_dir=str(tmp_path))
    prof = json.load(open(tmp_path / "step_cavity64_fp32_valu.json"))
    # 8e6 cycles over 8 XCDs in 500 us: 2.0 GHz; 2.048e8 x 4 / 1024 SIMDs / 1e6 cycles: 0.8 busy
    assert prof["clock_GHz"] == pytest.approx(2.0)
    assert prof["valu_busy"] == pytest.approx(0.8)
    # 1.5e8 wave-instructions in 500 us: 300 per ns against 256 x 2.4
    assert prof["valu_rate_G_per_s"] == pytest.approx(300.0)
    assert prof["valu_frac_of_peak"] == pytest.approx(300.0 / 614.4, abs=1e-4)
    assert prof["valu_instructions_per_node_launch"] == pytest.approx(1.5e8 * 64 / 4096)
    assert os.path.exists(tmp_path / "step_cavity64_fp32_valu.md")


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU: --gpus 2 exits with status 2 and says why, before any
    GPU work."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_launch_and_graph_counts():
    """Launches of a timed region and graph lengths: two-step launches end an odd count with
    one one-step launch; graphs hold an even number of steps between diagnostics."""
    assert bench.launches_of(2000, 2) == 1000 and bench.launches_of(21, 2) == 11
    assert bench.launches_of(21, 1) == 21
    assert bench.graph_steps(2000, 100) == 100 and bench.graph_steps(20, 100) == 20
    assert bench.graph_steps(15, 0) == 14 and bench.graph_steps(1, 100) == 0
    assert bench.arithmetic_dtype("fp16s") == "f32" and bench.arithmetic_dtype("fp32") == "f32"


def test_warmstart_summary_renders(tmp_path):
    """The warm-start summary writer on a small result of the shape the experiment returns."""
    inst = [{"Ra": 1e5, "Pr": 0.71, "Qstar": 1.0, "cold_steps": 1000, "warm_steps": 400,
             "cold_nu": 4.5, "warm_nu": 4.52, "cold_refined_nu": 4.51, "warm_refined_nu": 4.511,
             "cold_steps_to_nu": 2000, "warm_steps_to_nu": 500}]
    res = {"grid": 128, "train_states": 10, "train_requested": 10, "generate_seconds": 1.0,
           "generate_mlups": 100.0, "train_steps": 5, "train_batch": 2, "train_seconds": 0.5,
           "train_tflops": 1.0, "loss_first": 1.0, "loss_last": 0.1,
           "eval": {"cavities": 1, "side": 64, "both_converged": 1, "cold_steps_total": 1000,
                    "warm_steps_total": 400, "steps_ratio_warm_over_cold": 0.4, "median_ratio": 0.4,
                    "cold_seconds": 1.0, "warm_seconds": 0.5, "nu_rel_diff_max": 4e-3,
                    "nu_rel_diff_mean": 4e-3, "per_instance": inst,
                    "refine": {"tol": 1e-9, "nu_rel_diff_max": 2e-4, "nu_within_1e-3": 1,
                               "both_converged": 1, "warm_at_1e-7_vs_steady_max": 2e-3,
                               "cold_at_1e-7_vs_steady_max": 2e-3,
                               "warm_at_1e-7_within_1e-3_of_steady": 0,
                               "cold_at_1e-7_within_1e-3_of_steady": 0,
                               "cold_steps_to_tol_total": 3000, "warm_steps_to_tol_total": 1500,
                               "steps_ratio_to_tol": 0.5, "cold_steps_to_nu_1e-3_total": 2000,
                               "warm_steps_to_nu_1e-3_total": 500, "steps_ratio_to_nu_1e-3": 0.25,
                               "median_ratio_to_nu_1e-3": 0.25, "nu_settled_both": 1,
                               "nu_settle_chunk_steps": 100, "cold_seconds": 1.0, "warm_seconds": 0.5}}}
    out = tmp_path / "ws.md"
    bench.write_ws_summary(res, str(out), "python bench.py --warmstart")
    text = out.read_text()
    assert "0.25; 0.25" in text and "| 1.00e+05 | 0.71 | 1.00 | 1000 | 400 | 0.40 |" in text
    assert "cd /root/repo && python bench.py --warmstart" in text
