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
