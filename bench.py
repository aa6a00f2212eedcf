"""Benchmark of the fused thermal-CLBM step on one MI355X.

Workload: the 4096 x 4096 differentially heated cavity (Ra = 1e6, Pr = 0.71,
uniform heat source Q = 5e-6, Dirichlet side walls, adiabatic top and bottom,
U = 0.1), FP32 populations. This is the configuration whose working set
(1.88 GB of populations) exceeds the 256 MB Infinity Cache, so its HBM
roofline fraction is meaningful. One step = one launch of the fused
collide-and-stream kernel; the diagnostics reduction (residual, wall heat flux,
mass, NaN check) runs every --diag-every steps inside the timed region.

Prints one JSON line: MLUPS (million lattice-node updates per second, both
distributions), the roofline of the step kernel (algorithmic 112 B per node
update in FP32, 56 B in FP16 storage, over the kernel's average duration from
HIP events on the solver's stream) and the FP64 oracle's rate on the host cores.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled flow+thermal MLUPS & % HBM roofline; steps-to-steady warm vs cold"
HBM_PEAK_GBS = 8000.0
BYTES_PER_LUP = {"fp32": 112, "fp16s": 56}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def time_steps(torch, s, steps, diag_every):
    """Wall-clock time of `steps` steps (diagnostics every diag_every steps)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        n = min(diag_every, steps - done) if diag_every > 0 else steps - done
        s.step(n)
        done += n
        if diag_every > 0 and done % diag_every == 0:
            s.diagnostics()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def kernel_avg_ms(torch, s, launches):
    """Average duration of one fused-step launch: HIP events on the solver's stream
    around `launches` back-to-back launches."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.step(launches)
    e1.record(s.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / launches


def copy_ceiling(torch, clbm, nbytes=2 << 30, reps=10):
    """GB/s of the library's plain streaming copy (read + write) over nbytes buffers."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    src.fill_(1)
    for _ in range(2):
        clbm.clbm_stream_copy(dst, src)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        clbm.clbm_stream_copy(dst, src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2.0 * nbytes / (ms * 1e-3) / 1e9, ms


STEP_KERNEL_SOURCES = ("clbm_device.h", "clbm_kernels.h")


def source_digest():
    """Digest of the sources that define the fused step kernel, to tie a stored
    hardware-counter profile to the kernel it was taken from."""
    import hashlib
    h = hashlib.sha256()
    for f in STEP_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1801_04577_amd", "csrc", f), "rb") as fh:
            h.update(f.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(precision, n):
    """HBM bytes per step-kernel launch from the committed counter profile (FETCH_SIZE and
    WRITE_SIZE scaled by the same counters on the reference copy), or None when there is
    no profile for this kernel source and workload."""
    path = os.path.join(ROOT, "profiles", "step_cavity%d_%s_hbm_traffic.json" % (n, precision))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        prof = json.load(fh)
    if prof.get("source_digest") != source_digest():
        return None
    return prof.get("traffic_bytes_per_launch")


def cpu_baseline(prob, target_s=12.0):
    """The FP64 oracle on a 256-row strip of the same lattice and parameters, all host
    threads, steps chosen so the sample takes about target_s seconds."""
    import numpy as np
    import oracle
    strip = dict(prob, ny=256)
    nth = oracle.default_threads()
    o = oracle.Sim(strip, nthreads=nth)
    t0 = time.perf_counter()
    o.step(1)
    dt1 = time.perf_counter() - t0
    nsteps = max(1, int(target_s / max(dt1, 1e-3)))
    t0 = time.perf_counter()
    o.step(nsteps)
    dt = time.perf_counter() - t0
    lups = strip["nx"] * strip["ny"] * nsteps
    return {"value": round(lups / dt / 1e6, 3), "unit": "MLUPS", "cores": nth, "kind": "oracle",
            "sample": "FP64 oracle, %dx%d strip of the %dx%d cavity (same parameters), %d steps, %.1f s"
                      % (strip["nx"], strip["ny"], prob["nx"], prob["ny"], nsteps, dt)}


def summarize_profiles(trace_db, fetch_db, write_db, precision, n, command):
    """Write the kernel-time and HBM-traffic summaries under profiles/ from rocprofv3
    databases: one kernel-trace run and two counter runs (FETCH_SIZE, WRITE_SIZE). The
    counters are scaled by what they read for the reference copy (known bytes)."""
    import sqlite3
    import statistics

    def rows(db, sql, *a):
        con = sqlite3.connect(db)
        try:
            return list(con.execute(sql, a))
        finally:
            con.close()

    def short(name):
        return name.split("(")[0].replace("void ", "")

    top = rows(trace_db, "select name, total_calls, total_duration, average, percentage from top_kernels")
    counters = {}
    for db, cname in ((fetch_db, "FETCH_SIZE"), (write_db, "WRITE_SIZE")):
        per = {}
        for kname, grid, val in rows(db, "select kernel_name, grid_size, value from counters_collection "
                                     "where counter_name=?", cname):
            per.setdefault(short(kname), []).append((grid, val))
        counters[cname] = per
    copy_name = [k for k in counters["FETCH_SIZE"] if "k_stream_copy" in k][0]
    step_name = [k for k in counters["FETCH_SIZE"] if "k_step" in k][0]
    copy_bytes = 2 << 30  # bench.py's reference copy: 2 GiB read and 2 GiB written per launch
    f_copy = statistics.mean(v for _, v in counters["FETCH_SIZE"][copy_name])
    w_copy = statistics.mean(v for _, v in counters["WRITE_SIZE"][copy_name])
    f_step = statistics.mean(v for _, v in counters["FETCH_SIZE"][step_name])
    w_step = statistics.mean(v for _, v in counters["WRITE_SIZE"][step_name])
    sf, sw = copy_bytes / 1024 / f_copy, copy_bytes / 1024 / w_copy
    traffic = (f_step * sf + w_step * sw) * 1024
    alg = BYTES_PER_LUP[precision] * n * n
    tag = "step_cavity%d_%s" % (n, precision)
    step_row = [r for r in top if "k_step" in r[0]][0]
    prof = {
        "kernel": step_name, "workload": "cavity %dx%d Ra=1e6 Pr=0.71 Q=5e-6, %s" % (n, n, precision),
        "source_digest": source_digest(),
        "fetch_kib_per_dispatch": f_step, "write_kib_per_dispatch": w_step,
        "copy_fetch_kib_per_dispatch": f_copy, "copy_write_kib_per_dispatch": w_copy,
        "copy_bytes_read_and_written": copy_bytes,
        "fetch_scale": sf, "write_scale": sw,
        "traffic_bytes_per_launch": traffic, "algorithmic_bytes_per_launch": alg,
        "traffic_over_algorithmic": traffic / alg,
        "trace_avg_us": step_row[3], "trace_calls": step_row[1],
        "commands": command,
    }
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", tag + "_hbm_traffic.json"), "w") as fh:
        json.dump(prof, fh, indent=1)
    lines = ["# Kernel time and HBM traffic: %s" % prof["workload"], "",
             "Commands (run from the repository root on the GPU box):", ""]
    lines += ["    " + c for c in command]
    lines += ["", "## rocprofv3 --kernel-trace --stats (top kernels)", "",
              "| kernel | calls | total us | average us | % |", "|---|---|---|---|---|"]
    for name, calls, tot, avg, pct in top[:10]:
        lines.append("| %s | %d | %.1f | %.2f | %.2f |" % (short(name), calls, tot, avg, pct))
    lines += ["", "## HBM traffic per launch of the step kernel (rocprofv3 --pmc)", "",
              "| quantity | value |", "|---|---|",
              "| FETCH_SIZE, step kernel (KiB/dispatch) | %.1f |" % f_step,
              "| WRITE_SIZE, step kernel (KiB/dispatch) | %.1f |" % w_step,
              "| FETCH_SIZE, reference copy of 2 GiB (KiB/dispatch) | %.1f |" % f_copy,
              "| WRITE_SIZE, reference copy of 2 GiB (KiB/dispatch) | %.1f |" % w_copy,
              "| scale factors (known bytes / counter) | fetch %.4f, write %.4f |" % (sf, sw),
              "| traffic per launch (bytes) | %.4e |" % traffic,
              "| algorithmic bytes per launch (%d B x %d nodes) | %.4e |" % (BYTES_PER_LUP[precision], n * n, alg),
              "| traffic / algorithmic | %.4f |" % (traffic / alg),
              "", "Step-kernel source digest: %s" % prof["source_digest"]]
    with open(os.path.join(ROOT, "profiles", tag + "_rocprof.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({"written": tag, "traffic_over_algorithmic": traffic / alg}))


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-profiles":
        # --summarize-profiles TRACE_DB FETCH_DB WRITE_DB PRECISION N "cmd1" "cmd2" "cmd3"
        a = sys.argv[2:]
        summarize_profiles(a[0], a[1], a[2], a[3], int(a[4]), a[5:])
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--n", type=int, default=4096, help="cavity side")
    ap.add_argument("--precision", choices=["fp32", "fp16s"], default="fp32")
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch", default="", help="block_x,block_y,rows,remap")
    ap.add_argument("--kernel-launches", type=int, default=200)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import numpy as np
    import paper_1801_04577_amd as clbm
    import workloads as W

    clbm.ensure_built()
    torch.cuda.set_device(0)
    prob = W.cavity(args.n, Ra=1e6, Pr=0.71, Q=5e-6)
    prec = clbm.CLBM_FP16_SHIFTED if args.precision == "fp16s" else clbm.CLBM_FP32
    s = clbm.Solver(prob, prec)
    if args.launch:
        bx, by, rows, remap = [int(v) for v in args.launch.split(",")]
        s.set_launch(bx, by, rows, remap)
    T0 = torch.from_numpy(W.cavity_initial_T(prob, seed=12345).astype(np.float32))
    s.init(T=T0)
    log("bench: %dx%d %s, warmup %d" % (args.n, args.n, args.precision, args.warmup))
    time_steps(torch, s, args.warmup, args.diag_every)
    log("bench: timing %d steps" % args.steps)
    wall = time_steps(torch, s, args.steps, args.diag_every)
    nodes = args.n * args.n
    mlups = nodes * args.steps / wall / 1e6
    log("bench: %.3f ms/step, %.1f MLUPS" % (wall / args.steps * 1e3, mlups))
    kms = kernel_avg_ms(torch, s, args.kernel_launches)
    d = s.diagnostics()
    bpl = BYTES_PER_LUP[args.precision]
    achieved = bpl * nodes / (kms * 1e-3) / 1e9
    log("bench: step kernel %.4f ms avg, %.0f GB/s, nan %d" % (kms, achieved, d.nan_count))
    copy_gbs, copy_ms = copy_ceiling(torch, clbm)
    log("bench: reference copy %.0f GB/s" % copy_gbs)

    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "cavity %dx%d Ra=1e6 Pr=0.71 Q=5e-6 U=0.1, %s populations, "
                               "fused collide-and-stream, diagnostics every %d steps"
                               % (args.n, args.n, args.precision, args.diag_every),
                   "nx": args.n, "ny": args.n, "precision": args.precision,
                   "launch": s.get_launch()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(args.precision, args.n),
                     "algorithmic_bytes_per_launch": bpl * nodes,
                     "kernel": "k_step", "kernel_avg_ms": round(kms, 5), "bytes_per_lup": bpl,
                     "copy_ceiling_GBs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
    }
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
