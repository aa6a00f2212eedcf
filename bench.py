"""Benchmark of the fused thermal-CLBM step on one MI355X.

Workload: the 4096 x 4096 differentially heated cavity (Ra = 1e6, Pr = 0.71,
uniform heat source Q = 5e-6, Dirichlet side walls, adiabatic top and bottom,
U = 0.1), FP32 populations (or FP16 weight-shifted storage with --precision
fp16s). This is the configuration whose working set (1.88 GB of populations)
exceeds the 256 MB Infinity Cache, so its HBM roofline fraction is meaningful.
One step = one collide-and-stream update of every node; the default launch
advances two steps per kernel launch (k_step2, the first step's tile and halo
kept in LDS). The timed steps are replayed from HIP graphs; the diagnostics
reduction (residual, wall heat flux, mass, NaN check) runs every --diag-every
steps when the timed region is that long.

Prints one JSON line: MLUPS (million lattice-node updates per second, both
distributions) and the roofline of the step kernel. Its `achieved` is the bytes one
launch must move (every stored population read once and written once: 112 B per
node in FP32, 56 B in FP16 storage, whatever the steps per launch) over the
launch's average duration from HIP events on the solver's stream around the timed
region. The per-step algorithmic rate (bytes of one-step updates times the steps a
launch advances) is reported beside it as `effective_GBs`. `cpu_baseline` times
the FP64 oracle on the host cores.
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
    """Runs `steps` steps (diagnostics after every diag_every steps) and returns the
    wall-clock seconds, the milliseconds between HIP events recorded on the solver's
    stream at the start and the end, and the number of diagnostics calls made."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s.stream)
    done = diags = 0
    while done < steps:
        n = min(diag_every, steps - done) if diag_every > 0 else steps - done
        s.step(n)
        done += n
        if diag_every > 0 and done % diag_every == 0:
            s.diagnostics()
            diags += 1
    e1.record(s.stream)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, e0.elapsed_time(e1), diags


def launches_of(steps, spl):
    """Step-kernel launches of `steps` steps at spl steps per launch."""
    return steps // 2 + steps % 2 if spl == 2 else steps


def graph_steps(steps, diag_every):
    """Steps per replayed graph: the stretch between diagnostics (or the whole run), even."""
    g = min(steps, diag_every) if diag_every > 0 else steps
    return g - g % 2


def arithmetic_dtype(precision):
    """The arithmetic type of the collision: FP32 for both storage precisions (with FP32
    storage, the incoming population plus its change is formed exactly in FP64 before the
    unbiased rounding into FP32)."""
    return {"fp32": "f32", "fp16s": "f32"}[precision]


def host_cpu():
    """Host CPU model and the logical CPUs this process may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return model, os.cpu_count() or 1, usable


def kernel_avg_ms(torch, s, launches):
    """Average duration of one launch of the step kernel (one or two time steps per
    launch): HIP events on the solver's stream around `launches` back-to-back launches.
    Returns (ms per launch, steps per launch)."""
    spl = s.get_launch()["steps_per_launch"]
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s.stream)
    s.step(launches * spl)
    e1.record(s.stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / launches, spl


def copy_ceiling(torch, clbm, nbytes=2 << 30, reps=40):
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


def measured_traffic(precision, n, steps_per_launch):
    """HBM bytes per step-kernel launch from the committed counter profile (FETCH_SIZE and
    WRITE_SIZE scaled by the same counters on the reference copy), or None when there is
    no profile for this kernel source, workload and launch mode."""
    path = os.path.join(ROOT, "profiles", "step_cavity%d_%s_hbm_traffic.json" % (n, precision))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        prof = json.load(fh)
    if prof.get("source_digest") != source_digest() or prof.get("steps_per_launch", 1) != steps_per_launch:
        return None
    return prof.get("traffic_bytes_per_launch")


VALU_PEAK_G_PER_S = 256 * 2.4  # wave-instructions per ns: one per clock per CU, 256 CUs at 2.4 GHz


def summarize_valu(db, precision, n, command, out_dir=None):
    """Write the VALU issue and shader-clock summary of the step kernel under profiles/ from
    one rocprofv3 run with --kernel-trace and the counters GRBM_GUI_ACTIVE,
    SQ_ACTIVE_INST_VALU, SQ_BUSY_CU_CYCLES and SQ_INSTS_VALU."""
    import sqlite3
    import statistics
    con = sqlite3.connect(db)
    try:
        per = {}
        for k, c, v in con.execute("select kernel_name, counter_name, value from counters_collection"):
            per.setdefault((k.split("(")[0].replace("void ", ""), c), []).append(v)
        kname = sorted({k for k, _ in per if "k_step" in k}, key=lambda k: "k_step2" not in k)[0]
        dur_us = [float(a) for nm, a in con.execute("select name, average from top_kernels")
                  if nm.split("(")[0].replace("void ", "") == kname][0]
    finally:
        con.close()
    m = {c: statistics.mean(v) for (k, c), v in per.items() if k == kname}
    cycles = m["GRBM_GUI_ACTIVE"] / 8.0                 # summed over the 8 XCDs
    clock = cycles / (dur_us * 1e3)                     # GHz
    busy = m["SQ_ACTIVE_INST_VALU"] * 4.0 / 1024.0 / cycles
    rate = m["SQ_INSTS_VALU"] / (dur_us * 1e3)          # wave-instructions per ns
    spl = 2 if "k_step2" in kname else 1
    prof = {"kernel": kname, "workload": "cavity %dx%d Ra=1e6 Pr=0.71 Q=5e-6, %s" % (n, n, precision),
            "steps_per_launch": spl, "source_digest": source_digest(), "launches": len(per[(kname, "SQ_INSTS_VALU")]),
            "counters_per_launch": m, "trace_avg_us": dur_us, "clock_GHz": round(clock, 3),
            "valu_busy": round(busy, 4), "valu_instructions_per_node_launch": round(m["SQ_INSTS_VALU"] * 64.0 / (n * n), 1),
            "valu_rate_G_per_s": round(rate, 1), "valu_peak_G_per_s": VALU_PEAK_G_PER_S,
            "valu_frac_of_peak": round(rate / VALU_PEAK_G_PER_S, 4), "command": command}
    tag = "step_cavity%d_%s" % (n, precision)
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    with open(os.path.join(out_dir, tag + "_valu.json"), "w") as fh:
        json.dump(prof, fh, indent=1)
    lines = ["# VALU issue and shader clock of the step kernel: cavity %dx%d Ra=1e6 Pr=0.71 Q=5e-6, %s"
             % (n, n, precision), "", "Command (on the MI355X, where /root/repo is the repository):", "",
             "    " + command, "",
             "| quantity | value |", "|---|---|",
             "| kernel | %s (%d launches) |" % (kname, prof["launches"]),
             "| traced duration per launch | %.1f us |" % dur_us]
    lines += ["| %s per launch | %.4g |" % (c, m[c]) for c in sorted(m)]
    lines += ["| shader clock: GRBM_GUI_ACTIVE / 8 XCDs / duration | %.2f GHz |" % clock,
              "| VALU busy: SQ_ACTIVE_INST_VALU x 4 / 1024 SIMDs / cycles | %.2f |" % busy,
              "| VALU instructions per node per launch: SQ_INSTS_VALU x 64 / nodes | %.0f |" % prof["valu_instructions_per_node_launch"],
              "| VALU issue rate / peak (one wave-instruction per clock per CU, 256 CUs, 2.4 GHz) | %.0f / %.0f G/s = %.2f |"
              % (rate, VALU_PEAK_G_PER_S, rate / VALU_PEAK_G_PER_S),
              "", "Step-kernel source digest: %s" % prof["source_digest"]]
    with open(os.path.join(out_dir, tag + "_valu.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({"written": tag + "_valu", "valu_busy": prof["valu_busy"], "clock_GHz": prof["clock_GHz"]}))


def measured_valu(precision, n, steps_per_launch):
    """VALU issue of the step kernel from the committed counter profile, or None when there
    is no profile for this kernel source, workload and launch mode."""
    path = os.path.join(ROOT, "profiles", "step_cavity%d_%s_valu.json" % (n, precision))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        prof = json.load(fh)
    if prof.get("source_digest") != source_digest() or prof.get("steps_per_launch", 1) != steps_per_launch:
        return None
    return {k: prof[k] for k in ("valu_busy", "clock_GHz", "valu_instructions_per_node_launch",
                                 "valu_rate_G_per_s", "valu_peak_G_per_s", "valu_frac_of_peak")}


def cpu_baseline(prob, target_s=15.0):
    """The FP64 oracle on a 256-row strip of the same lattice and parameters, steps chosen
    so the sample takes about target_s seconds. Threads: OMP_NUM_THREADS when set (the GPU
    machine sets 16, its share of the host), else every CPU this process may use."""
    import oracle
    strip = dict(prob, ny=256)
    env = os.environ.get("OMP_NUM_THREADS", "")
    model, ncpu, usable = host_cpu()
    nth = int(env) if env.isdigit() and int(env) > 0 else usable
    o = oracle.Sim(strip, nthreads=nth)
    o.step(1)                      # first step: thread start-up
    t0 = time.perf_counter()
    o.step(4)
    dt1 = (time.perf_counter() - t0) / 4
    nsteps = max(1, int(target_s / max(dt1, 1e-3)))
    t0 = time.perf_counter()
    o.step(nsteps)
    dt = time.perf_counter() - t0
    lups = strip["nx"] * strip["ny"] * nsteps
    return {"value": round(lups / dt / 1e6, 3), "unit": "MLUPS", "cores": nth, "kind": "oracle",
            "sample": "FP64 oracle, %dx%d strip of the %dx%d cavity (same parameters), %d steps, %.1f s"
                      % (strip["nx"], strip["ny"], prob["nx"], prob["ny"], nsteps, dt),
            "threads_from": "OMP_NUM_THREADS" if env.isdigit() and int(env) > 0 else "affinity",
            "host_cpu_model": model, "host_logical_cpus": ncpu, "host_cpus_usable": usable}


def summarize_profiles(trace_db, fetch_db, write_db, precision, n, command, out_dir=None):
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
    # the two-step kernel when the run used it, else the single-step one
    names = sorted((k for k in counters["FETCH_SIZE"] if "k_step" in k), key=lambda k: "k_step2" not in k)
    step_name = names[0]
    spl = 2 if "k_step2" in step_name else 1
    copy_bytes = 2 << 30  # bench.py's reference copy: 2 GiB read and 2 GiB written per launch
    f_copy = statistics.mean(v for _, v in counters["FETCH_SIZE"][copy_name])
    w_copy = statistics.mean(v for _, v in counters["WRITE_SIZE"][copy_name])
    f_step = statistics.mean(v for _, v in counters["FETCH_SIZE"][step_name])
    w_step = statistics.mean(v for _, v in counters["WRITE_SIZE"][step_name])
    sf, sw = copy_bytes / 1024 / f_copy, copy_bytes / 1024 / w_copy
    traffic = (f_step * sf + w_step * sw) * 1024
    alg = BYTES_PER_LUP[precision] * n * n * spl
    tag = "step_cavity%d_%s" % (n, precision)
    step_row = [r for r in top if short(r[0]) == step_name][0]
    prof = {
        "kernel": step_name, "steps_per_launch": spl,
        "workload": "cavity %dx%d Ra=1e6 Pr=0.71 Q=5e-6, %s" % (n, n, precision),
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
    out_dir = out_dir or os.path.join(ROOT, "profiles")
    os.makedirs(out_dir, exist_ok=True)
    with open(os.path.join(out_dir, tag + "_hbm_traffic.json"), "w") as fh:
        json.dump(prof, fh, indent=1)
    lines = ["# Kernel time and HBM traffic: %s" % prof["workload"], "",
             "Commands (on the MI355X, where /root/repo is the repository):", ""]
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
              "| bytes a launch must move (%d B x %d nodes: each population read once, written once) | %.4e |"
              % (BYTES_PER_LUP[precision], n * n, BYTES_PER_LUP[precision] * n * n),
              "| traffic / bytes a launch must move | %.4f |" % (traffic / (BYTES_PER_LUP[precision] * n * n)),
              "| rate: bytes a launch must move / traced average duration | %.1f GB/s (%.3f of 8 TB/s) |"
              % (BYTES_PER_LUP[precision] * n * n / (step_row[3] * 1e-6) / 1e9,
                 BYTES_PER_LUP[precision] * n * n / (step_row[3] * 1e-6) / 1e9 / HBM_PEAK_GBS),
              "| per-step algorithmic bytes of the launch (%d B x %d nodes x %d step(s)) | %.4e |"
              % (BYTES_PER_LUP[precision], n * n, spl, alg),
              "| traffic / per-step algorithmic | %.4f |" % (traffic / alg),
              "", "Step-kernel source digest: %s" % prof["source_digest"]]
    with open(os.path.join(out_dir, tag + "_rocprof.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps({"written": tag, "traffic_over_algorithmic": traffic / alg}))


def standin_errors(args):
    """The 512 x 512 stand-in of the 4096^2 workload (same Ra, Pr, Q and walls, U = 0.1 rule,
    seeded noise): FP32 and FP16-shifted storage on the GPU and the FP64 oracle on the host,
    advanced together over the configuration's 20 000 steps. At each checkpoint, per field,
    max |gpu - oracle| / max |oracle| (u as the vector (u_x, u_y)) and max |rho - rho_oracle|."""
    import numpy as np
    import torch
    import paper_1801_04577_amd as clbm
    import workloads as W
    import oracle

    prob = W.cavity(512, Ra=1e6, Pr=0.71, Q=5e-6)
    T = W.cavity_initial_T(prob, seed=12345).astype(np.float32)
    o = oracle.Sim(prob, T=T.astype(np.float64))
    gpu = {}
    for name, prec in (("fp32", clbm.CLBM_FP32), ("fp16s", clbm.CLBM_FP16_SHIFTED)):
        g = clbm.Solver(prob, prec)
        g.init(T=torch.from_numpy(T))
        gpu[name] = g
    checkpoints = [int(c) for c in args.standin_checkpoints.split(",")]
    rows = []
    t0 = time.perf_counter()
    for c in checkpoints:
        while o.t < c:
            n = min(1000, c - o.t)
            o.step(n)
            for g in gpu.values():
                g.step(n)
            log("standin: %d steps, %.0f s" % (o.t, time.perf_counter() - t0))
        ro, uxo, uyo, To = o.macros()
        umax = float(np.sqrt(uxo ** 2 + uyo ** 2).max())
        Tmax = float(np.abs(To).max())
        row = {"steps": c, "umax": umax, "Tmax": Tmax}
        for name, g in gpu.items():
            rg, uxg, uyg, Tg = [t.cpu().numpy().astype(np.float64) for t in g.macros()]
            row[name] = {"u": float(np.sqrt((uxg - uxo) ** 2 + (uyg - uyo) ** 2).max() / umax),
                         "T": float(np.abs(Tg - To).max() / Tmax),
                         "rho_abs": float(np.abs(rg - ro).max())}
        rows.append(row)
        log("standin: %d steps: fp32 u %.2e T %.2e, fp16s u %.2e T %.2e"
            % (c, row["fp32"]["u"], row["fp32"]["T"], row["fp16s"]["u"], row["fp16s"]["T"]))
    out = {"workload": "cavity 512x512 Ra=1e6 Pr=0.71 Q=5e-6 U=0.1, seeded noise 1e-4 (seed 12345), "
                       "stand-in of the 4096x4096 workload",
           "oracle_threads": o.nthreads, "seconds": round(time.perf_counter() - t0, 1), "checkpoints": rows}
    if args.standin_out:
        lines = ["# Error of the GPU storage types against the FP64 oracle: 512^2 stand-in, 20 000 steps", "",
                 "Command (on the MI355X, where /root/repo is the repository):", "",
                 "    cd /root/repo && python bench.py --standin --standin-out %s" % args.standin_out, "",
                 "Workload: %s. Error per field: max over nodes of |gpu - oracle| / max over nodes of "
                 "|oracle| (u as the vector (u_x, u_y)); rho absolute." % out["workload"], "",
                 "| steps | max u | FP32 u | FP32 T | FP32 rho | FP16s u | FP16s T | FP16s rho |",
                 "|---|---|---|---|---|---|---|---|"]
        for r in rows:
            lines.append("| %d | %.3e | %.2e | %.2e | %.1e | %.2e | %.2e | %.1e |"
                         % (r["steps"], r["umax"], r["fp32"]["u"], r["fp32"]["T"], r["fp32"]["rho_abs"],
                            r["fp16s"]["u"], r["fp16s"]["T"], r["fp16s"]["rho_abs"]))
        lines += ["", "Oracle threads: %d; wall time %.0f s." % (o.nthreads, out["seconds"])]
        with open(args.standin_out, "w") as fh:
            fh.write("\n".join(lines) + "\n")
    return out


def small_configs(args):
    """The cache-resident configurations on the GPU (their working sets fit the 256 MB
    Infinity Cache, so they are launch-bound and get no HBM fraction; steps are replayed
    from graphs of 100 steps), each next to the FP64 oracle timed on the host cores with
    one thread and with all threads (bounded step counts, stated per entry)."""
    import numpy as np
    import torch
    import paper_1801_04577_amd as clbm
    import workloads as W
    import oracle

    def gpu_rate(prob, steps, precision=clbm.CLBM_FP32, T_init=None):
        s = clbm.Solver(prob, precision)
        s.set_graph(100)
        s.init(T=None if T_init is None else torch.from_numpy(T_init))
        s.step(200)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(steps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        d = s.diagnostics()
        return {"steps": steps, "seconds": round(dt, 4),
                "mlups": round(prob["nx"] * prob["ny"] * steps / dt / 1e6, 1), "nan": d.nan_count}

    def oracle_rate(prob, steps, nthreads):
        o = oracle.Sim(prob, nthreads=nthreads)
        o.step(1)
        t0 = time.perf_counter()
        o.step(steps)
        dt = time.perf_counter() - t0
        return {"threads": nthreads, "steps": steps, "seconds": round(dt, 3),
                "mlups": round(prob["nx"] * prob["ny"] * steps / dt / 1e6, 3)}

    nth = oracle.default_threads()
    out = []
    c0 = W.channel()
    log("configs: channel 64x32")
    out.append({"config": "channel 64x32 (periodic x, walls in y, g_x 1e-6, nu 0.05, Pr 0.71, Q 1e-4)",
                "gpu_fp32": gpu_rate(c0, 10000),
                "cpu_baseline": [dict(oracle_rate(c0, 10000, 1), kind="oracle"),
                                 dict(oracle_rate(c0, 10000, nth), kind="oracle")]})
    c1 = W.cavity(256, Ra=1e5, Pr=0.71)
    T1 = W.cavity_initial_T(c1, seed=12345).astype(np.float32)
    log("configs: cavity 256^2 to residual 1e-7")
    s = clbm.Solver(c1)
    s.set_graph(100)
    s.init(T=torch.from_numpy(T1))
    s.diagnostics()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while s.t < 3_000_000:
        s.step(1000)
        d = s.diagnostics()
        if d.nan_count or max(d.res_u, d.res_T) < 1e-7:
            break
    dt = time.perf_counter() - t0
    H, dT = 256, 1.0
    c1_run = {"steps_to_residual_1e-7": int(s.t), "seconds": round(dt, 3),
              "mlups": round(256 * 256 * s.t / dt / 1e6, 1), "res_u": d.res_u, "res_T": d.res_T,
              "Nu_cold_wall": round(clbm.nusselt(d, 1, H, dT, into_wall=True), 5),
              "Nu_hot_wall": round(clbm.nusselt(d, 0, H, dT, into_wall=False), 5),
              "Nu_cold_wall_link_flux": round(clbm.nusselt_flux(d, 1, H, dT, c1["alpha"], into_wall=True), 5),
              "nan": d.nan_count}
    out.append({"config": "cavity 256^2 Ra 1e5 Pr 0.71, walls +-0.5, seeded noise 1e-4, run to residual 1e-7 "
                          "(diagnostics every 1000 steps)",
                "gpu_fp32": c1_run,
                "cpu_baseline": [dict(oracle_rate(c1, 300, 1), kind="oracle"),
                                 dict(oracle_rate(c1, 1000, nth), kind="oracle")]})
    c2 = W.cavity(512, Ra=1e6, Pr=0.71, Q=5e-6)
    T2 = W.cavity_initial_T(c2, seed=12345).astype(np.float32)
    log("configs: cavity 512^2 stand-in")
    out.append({"config": "cavity 512^2 Ra 1e6 Pr 0.71 Q 5e-6 (stand-in of the 4096^2 cavity)",
                "gpu_fp32": gpu_rate(c2, 20000, T_init=T2),
                "gpu_fp16s": gpu_rate(c2, 20000, clbm.CLBM_FP16_SHIFTED, T_init=T2),
                "cpu_baseline": [dict(oracle_rate(c2, 100, 1), kind="oracle"),
                                 dict(oracle_rate(c2, 200, nth), kind="oracle")]})
    return out


def batched_sweep(args):
    """The batched form on the 256-cavity sweep: autotuned one-launch-per-step over a
    device tile list, against a loop of per-cavity launches of the single-lattice step on
    the same cavities; then a run of every cavity to its residual (--sweep-tol, 1e-7 by
    default; FP16 storage needs a tolerance above its rounding-noise floor of about 1e-6)
    with on-device retirement (graph of K steps + convergence check + tile-list
    compaction)."""
    import numpy as np
    import torch
    import paper_1801_04577_amd as clbm
    import workloads as W

    sets = W.sweep(count=args.sweep_count, seed=2024)
    probs = [p for p, _ in sets]
    nodes = sum(p["nx"] * p["ny"] for p in probs)
    inits = [{"T": torch.from_numpy((p["T0"] + W.noise_field(sd, p["nx"], p["ny"], 1e-4)).astype(np.float32))}
             for p, sd in sets]
    log("batched: %d cavities, %d nodes" % (len(probs), nodes))
    prec = clbm.CLBM_FP16_SHIFTED if args.precision == "fp16s" else clbm.CLBM_FP32
    b = clbm.Batch(probs, precision=prec)
    cache = args.write_cache or None
    if cache and os.path.exists(cache):
        os.remove(cache)
    best = b.autotune(steps=20, cache_path=cache)
    log("batched: autotuned tile %s" % best)
    for i, f in enumerate(inits):
        b.init(i, **f)
    torch.cuda.synchronize()
    b.step(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(args.sweep_steps)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t0
    mlups_batch = nodes * args.sweep_steps / t_batch / 1e6
    log("batched: %.1f MLUPS (one launch per step)" % mlups_batch)
    # the same cavities advanced one launch per cavity per step
    solvers = []
    for p, f in zip(probs, inits):
        sv = clbm.Solver(p, prec)
        sv.init(**f)
        solvers.append(sv)
    for sv in solvers:
        sv.step(2)
    torch.cuda.synchronize()
    loop_steps = max(2, args.sweep_steps // 10)
    t0 = time.perf_counter()
    for _ in range(loop_steps):
        for sv in solvers:
            sv.step(1)
    torch.cuda.synchronize()
    t_loop = time.perf_counter() - t0
    mlups_loop = nodes * loop_steps / t_loop / 1e6
    log("batched: loop of per-cavity launches %.1f MLUPS" % mlups_loop)
    del solvers
    # run to convergence from the seeded initial state
    for i, f in enumerate(inits):
        b.init(i, **f)
    t0 = time.perf_counter()

    def progress(st, names):
        log("batched: run to %.0e: %.0f s, running %d, converged %d, diverged %d, max_steps %d, "
            "max steps %d" % (args.sweep_tol, time.perf_counter() - t0, names.count("running"), names.count("converged"),
                              names.count("diverged"), names.count("max_steps"), max(st)))
    steps, status = b.run(max_steps=args.sweep_max_steps, tol=args.sweep_tol, K=1000, chunk=50000,
                          progress=progress)
    t_run = time.perf_counter() - t0
    lups = sum(st * p["nx"] * p["ny"] for st, p in zip(steps, probs))
    counts = {k: status.count(k) for k in ("converged", "diverged", "max_steps", "running")}
    under = [i for i, p in enumerate(probs) if p["meta"]["under_resolved"]]
    under_counts = {k: [status[i] for i in under].count(k) for k in ("converged", "diverged", "max_steps")}
    log("batched: run to %.0e: %s in %.1f s, %.1f MLUPS; under-resolved (tau_nu < 0.52): %d %s"
        % (args.sweep_tol, counts, t_run, lups / t_run / 1e6, len(under), under_counts))
    res = {"workload": "%d cavities (sides 64-512, a<=b<=2a; Ra 1e3-1e6 log-uniform; Pr 0.7-7; "
                       "Q 0-1e-4), %s storage" % (len(probs), args.precision),
           "nodes": nodes, "tile": best,
           "mlups_batched": round(mlups_batch, 1), "mlups_loop_of_launches": round(mlups_loop, 1),
           "speedup_vs_loop": round(mlups_batch / mlups_loop, 2),
           "run_to_residual": {"tol": args.sweep_tol, "K": 1000, "max_steps": args.sweep_max_steps,
                               "status_counts": counts, "seconds": round(t_run, 2),
                               "mlups": round(lups / t_run / 1e6, 1),
                               "steps_min": int(min(steps)), "steps_max": int(max(steps)),
                               "steps_median": float(np.median(steps)),
                               "under_resolved": len(under), "under_resolved_status": under_counts}}
    if args.sweep_summary:
        write_batch_summary(cache, res, args.sweep_summary)
    if args.sweep_out:
        residuals = [b.residual(i) for i in range(len(probs))]
        with open(args.sweep_out, "w") as fh:
            json.dump(dict(res, per_instance=[
                {"nx": p["nx"], "ny": p["ny"], "Ra": p["meta"]["Ra"], "Pr": p["meta"]["Pr"], "Q": p["Q"],
                 "tau_nu": p["meta"]["tau_nu"], "steps": st, "status": sn, "res_u": r[0], "res_T": r[1]}
                for p, st, sn, r in zip(probs, steps, status, residuals)]), fh, indent=1)
    return res


def write_batch_summary(cache, res, out):
    """Markdown summary of a batched-sweep run: the autotuner's candidates (from its cache
    file, fastest first) and the run to the residual."""
    lines = ["# Batched step: autotuner sweep and run to residual, %s" % res["workload"], "",
             "Command (on the MI355X, where /root/repo is the repository):", "",
             "    cd /root/repo && " + " ".join(["python", "bench.py"] + sys.argv[1:]), "",
             "Nodes: %d. Batched %.1f MLUPS against %.1f for a loop of per-cavity launches (%.2fx)."
             % (res["nodes"], res["mlups_batched"], res["mlups_loop_of_launches"], res["speedup_vs_loop"]), ""]
    if cache and os.path.exists(cache):
        rows = [json.loads(l) for l in open(cache)]
        best = [r for r in rows if r.get("best")]
        cand = sorted((r for r in rows if not r.get("best")), key=lambda r: r["ms_per_step"])
        lines += ["## Autotuner candidates (signature %s), fastest first" % (best[-1]["signature"] if best else "?"),
                  "", "| tile_x | tile_y | steps/launch | persistent_wgs (0 = one per tile) | XCD bands | ms/step | MLUPS |",
                  "|---|---|---|---|---|---|---|"]
        lines += ["| %d | %d | %d | %d | %d | %.4f | %.1f |" % (r["tile_x"], r["tile_y"], r["steps_per_launch"],
                                                              r["persistent_wgs"], r["xcd_bands"],
                                                              r["ms_per_step"], r["mlups"]) for r in cand]
        lines.append("")
    rr = res["run_to_residual"]
    lines += ["## Run of every cavity to residual %.0e (graph of K = %d steps, on-device retirement, cap %d steps)"
              % (rr["tol"], rr["K"], rr["max_steps"]), "",
              "| quantity | value |", "|---|---|"]
    lines += ["| %s | %s |" % (k, rr[k]) for k in ("status_counts", "seconds", "mlups", "steps_min", "steps_median",
                                                 "steps_max", "under_resolved", "under_resolved_status")]
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def write_ws_summary(res, out, command):
    """Markdown summary of a warm-start experiment (the JSON that --ws-out writes)."""
    e = res["eval"]
    lines = ["# Learned warm start: %d training steady states, %d held-out %d^2 cavities"
             % (res.get("train_states", 0), e["cavities"], e["side"]), "",
             "Workload: cavities with Ra log-uniform in [1e3, 1e6], Pr uniform in [0.7, 7], Q* = Q H^2/(alpha dT) "
             "uniform in [0, 4]; training sides {64, 96, 128} (a <= b <= 2a, seed 2024), held-out square cavities "
             "(seed 7). Network: 4-level conv encoder-decoder (32/64/128/256 channels, 15 3x3 convolutions) on a "
             "%d^2 grid, BF16 MFMA with FP32 accumulation, trained by the library's kernels (Adam); its prediction is "
             "resampled bilinearly and becomes the equilibrium initial state. Cold start: T0 + 1e-4 seeded noise at "
             "rest. Both starts run in one batch each to residual 1e-7 (r = ||x^n - x^(n-K)|| / (K ||x^n||), K = 1000)"
             "%s." % (res["grid"], ", then continue to %.0e" % e["refine"]["tol"] if "refine" in e else ""), "",
             "Command (on the MI355X, where /root/repo is the repository):", "", "    cd /root/repo && " + command, ""]
    if "train_states" in res:
        lines += ["## Training", "", "| quantity | value |", "|---|---|",
                  "| steady states generated (batched solver, cold start to 1e-7) | %d of %d in %.1f s (%.0f MLUPS) |"
                  % (res["train_states"], res["train_requested"], res["generate_seconds"], res["generate_mlups"]),
                  "| Adam steps x batch | %d x %d in %.1f s |" % (res["train_steps"], res["train_batch"],
                                                                  res["train_seconds"]),
                  "| network throughput (forward + backward, algorithmic flops) | %.2f TFLOP/s |" % res["train_tflops"],
                  "| MSE loss, first 50 / last 50 steps | %.4f / %.6f |" % (res["loss_first"], res["loss_last"]), ""]
    lines += ["## Held-out cavities: steps to residual 1e-7", "", "| quantity | value |", "|---|---|",
              "| cavities, both converged | %d, %d |" % (e["cavities"], e["both_converged"]),
              "| total steps cold / warm | %d / %d |" % (e["cold_steps_total"], e["warm_steps_total"]),
              "| warm / cold steps (total, median per cavity) | %s, %s |" % (e["steps_ratio_warm_over_cold"],
                                                                          e["median_ratio"]),
              "| wall time cold / warm (s), batched solver | %s / %s |" % (e["cold_seconds"], e["warm_seconds"]),
              "| Nu, warm vs cold at 1e-7: max / mean relative difference | %.2e / %.2e |"
              % (e["nu_rel_diff_max"], e["nu_rel_diff_mean"]), ""]
    if "refine" in e:
        r = e["refine"]
        lines += ["## Both runs continued to residual %.0e" % r["tol"], "", "| quantity | value |", "|---|---|",
                  "| Nu, warm vs cold at %.0e: max relative difference | %.2e (%d of %d within 1e-3) |"
                  % (r["tol"], r["nu_rel_diff_max"], r["nu_within_1e-3"], r["both_converged"]),
                  "| Nu at 1e-7 vs the steady Nu (cold at %.0e): warm max / cold max | %.2e / %.2e |"
                  % (r["tol"], r["warm_at_1e-7_vs_steady_max"], r["cold_at_1e-7_vs_steady_max"]),
                  "| cavities whose Nu at 1e-7 is within 1e-3 of steady: warm / cold | %d / %d |"
                  % (r["warm_at_1e-7_within_1e-3_of_steady"], r["cold_at_1e-7_within_1e-3_of_steady"]),
                  "| total steps to %.0e: cold / warm (ratio) | %d / %d (%s) |"
                  % (r["tol"], r["cold_steps_to_tol_total"], r["warm_steps_to_tol_total"], r["steps_ratio_to_tol"]),
                  "| total steps until Nu stays within 1e-3 of steady: cold / warm (ratio; median per cavity) | "
                  "%d / %d (%s; %s), %d cavities, Nu read every %d steps |"
                  % (r["cold_steps_to_nu_1e-3_total"], r["warm_steps_to_nu_1e-3_total"], r["steps_ratio_to_nu_1e-3"],
                     r["median_ratio_to_nu_1e-3"], r["nu_settled_both"], r["nu_settle_chunk_steps"]),
                  "| wall time of the continuation cold / warm (s) | %s / %s |" % (r["cold_seconds"], r["warm_seconds"]),
                  ""]
    lines += ["## Per cavity", "",
              "| Ra | Pr | Q* | cold steps | warm steps | warm/cold | Nu cold 1e-7 | Nu warm 1e-7 | Nu cold 1e-9 | "
              "Nu warm 1e-9 | cold steps to Nu | warm steps to Nu |", "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for q in e["per_instance"]:
        lines.append("| %.2e | %.2f | %.2f | %d | %d | %.2f | %.5f | %.5f | %s | %s | %s | %s |"
                     % (q["Ra"], q["Pr"], q["Qstar"], q["cold_steps"], q["warm_steps"],
                        q["warm_steps"] / max(q["cold_steps"], 1), q["cold_nu"], q["warm_nu"],
                        "%.5f" % q["cold_refined_nu"] if "cold_refined_nu" in q else "-",
                        "%.5f" % q["warm_refined_nu"] if "warm_refined_nu" in q else "-",
                        q.get("cold_steps_to_nu", "-"), q.get("warm_steps_to_nu", "-")))
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def net_flops_per_sample(H, W, cin=8, cout=3, widths=(32, 64, 128, 256)):
    """Multiply-add flops of one forward pass of the warm-start network (3x3 convolutions)."""
    w1, w2, w3, w4 = widths
    layers = [(1, cin, w1), (1, w1, w1), (2, w1, w2), (2, w2, w2), (4, w2, w3), (4, w3, w3),
              (8, w3, w4), (8, w4, w4), (4, w4 + w3, w3), (4, w3, w3), (2, w3 + w2, w2),
              (2, w2, w2), (1, w2 + w1, w1), (1, w1, w1), (1, w1, cout)]
    return sum(2.0 * (H // r) * (W // r) * 9 * ci * co for r, ci, co in layers)


def net_throughput(args):
    """Throughput of the warm-start network's kernels alone: forward passes, and training
    steps (forward, backward, Adam) at the benchmark's batch on its grid, random inputs and
    targets (the kernels' cost does not depend on the values)."""
    import numpy as np
    import torch
    import paper_1801_04577_amd as clbm
    from paper_1801_04577_amd import warmstart as ws
    B, G = args.ws_batch, args.ws_grid
    net = clbm.Net(B, G, G, ws.CIN, ws.COUT, ws.WIDTHS)
    net.set_params(torch.from_numpy(ws.init_params(seed=0)))
    gen = torch.Generator(device="cuda").manual_seed(0)
    X = torch.randn(B, ws.CIN, G, G, device="cuda", generator=gen)
    Y = torch.randn(B, ws.COUT, G, G, device="cuda", generator=gen)
    for t in range(1, 6):
        net.forward(X)
        net.backward(Y)
        net.adam(1e-3, t)
    n = args.net_steps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(6, 6 + n):
        net.forward(X)
        net.backward(Y)
        net.adam(1e-3, t)
    torch.cuda.synchronize()
    dt_train = (time.perf_counter() - t0) / n
    t0 = time.perf_counter()
    for _ in range(n):
        net.forward(X)
    torch.cuda.synchronize()
    dt_fwd = (time.perf_counter() - t0) / n
    fl = net_flops_per_sample(G, G) * B
    return {"batch": B, "grid": G, "steps": n,
            "train_ms_per_step": round(dt_train * 1e3, 3), "train_tflops": round(3.0 * fl / dt_train / 1e12, 1),
            "forward_ms": round(dt_fwd * 1e3, 3), "forward_tflops": round(fl / dt_fwd / 1e12, 1),
            "flops_note": "3x3 convolutions only; a training step counts 3x the forward flops",
            "mfma_peak_tflops_bf16": 2500.0}


def train_network(args, res, net, grid, progress):
    """Training half of the warm-start experiment: steady states of the training cavities
    from the batched solver (cold starts to residual 1e-7), then Adam on the network."""
    import numpy as np
    import torch
    import paper_1801_04577_amd as clbm
    from paper_1801_04577_amd import warmstart as ws
    import workloads as W

    # training data
    sides = tuple(int(v) for v in args.ws_train_sides.split(","))
    sets = W.warmstart_problems(args.ws_train, seed=2024, sides=sides, square=False)
    X, Y = [], []
    t_gen = time.perf_counter()
    lups = 0
    for k0 in range(0, len(sets), args.ws_chunk_instances):
        part = sets[k0:k0 + args.ws_chunk_instances]
        probs = [p for p, _ in part]
        cold = [{"T": (p["T0"] + W.noise_field(sd, p["nx"], p["ny"], 1e-4)).astype(np.float32)} for p, sd in part]
        b = clbm.Batch(probs)
        for i, f in enumerate(cold):
            b.init(i, **f)
        steps, status = b.run(max_steps=args.ws_max_steps, tol=1e-7, K=1000, chunk=20000,
                              progress=progress("generate %d-%d" % (k0, k0 + len(part))))
        lups += sum(st * p["nx"] * p["ny"] for st, p in zip(steps, probs))
        ok = [i for i, s in enumerate(status) if s == "converged"]
        Y.append(ws.targets(b, probs, ok, grid, grid))
        X.append(ws.inputs([probs[i] for i in ok], grid, grid))
        del b
    X = torch.cat(X)
    Y = torch.cat(Y)
    t_gen = time.perf_counter() - t_gen
    res["train_states"] = int(X.shape[0])
    res["train_requested"] = len(sets)
    res["generate_seconds"] = round(t_gen, 1)
    res["generate_mlups"] = round(lups / t_gen / 1e6, 1)
    log("warmstart: %d steady states in %.0f s" % (X.shape[0], t_gen))

    # training
    net.set_params(torch.from_numpy(ws.init_params(seed=0)))
    torch.cuda.synchronize()
    t_tr = time.perf_counter()
    losses = ws.train(net, X, Y, steps=args.ws_train_steps, lr=2e-3, lr_final=1e-4, seed=1, log_every=200)
    torch.cuda.synchronize()
    t_tr = time.perf_counter() - t_tr
    fl = 3.0 * net_flops_per_sample(grid, grid) * args.ws_batch * args.ws_train_steps
    res["train_steps"] = args.ws_train_steps
    res["train_batch"] = args.ws_batch
    res["train_seconds"] = round(t_tr, 1)
    res["train_tflops"] = round(fl / t_tr / 1e12, 2)
    res["loss_first"] = float(np.mean(losses[:50]))
    res["loss_last"] = float(np.mean(losses[-50:]))
    if args.ws_save:
        np.save(args.ws_save, net.params().cpu().numpy())


def warmstart_experiment(args):
    """Learned warm start at scale: steady states of the training cavities from the batched
    solver, training of the network by the library's kernels, and steps to residual 1e-7
    (and Nu) of held-out cavities from the cold start and from the network's prediction."""
    import numpy as np
    import torch
    import paper_1801_04577_amd as clbm
    from paper_1801_04577_amd import warmstart as ws
    import workloads as W

    grid = args.ws_grid
    res = {"grid": grid}

    def progress(tag):
        t0 = time.perf_counter()

        def cb(steps, status):
            log("%s: %.0f s, running %d, converged %d, diverged %d, max_steps %d, max steps %d"
                % (tag, time.perf_counter() - t0, status.count("running"), status.count("converged"),
                   status.count("diverged"), status.count("max_steps"), max(steps)))
        return cb

    net = clbm.Net(args.ws_batch, grid, grid, ws.CIN, ws.COUT, ws.WIDTHS)
    if args.ws_load:
        # parameters written by an earlier run of this experiment (--ws-save)
        net.set_params(torch.from_numpy(np.load(args.ws_load, allow_pickle=False).astype(np.float32)))
        res["params_loaded_from"] = args.ws_load
    else:
        train_network(args, res, net, grid, progress)

    # evaluation on held-out cavities
    tsets = W.warmstart_problems(args.ws_eval, seed=7, sides=(args.ws_eval_side,), square=True)
    tprobs = [p for p, _ in tsets]
    cold = [{"T": (p["T0"] + W.noise_field(sd, p["nx"], p["ny"], 1e-4)).astype(np.float32)} for p, sd in tsets]
    out = {}
    for key, inits in (("cold", cold), ("warm", None)):
        if inits is None:
            inits = ws.warm_inits(ws.predict(net, ws.inputs(tprobs, grid, grid)), tprobs)
        b = clbm.Batch(tprobs)
        for i, f in enumerate(inits):
            b.init(i, **f)
        # Nu of every instance at each chunk boundary (a multiple of K, where the run's own
        # residual snapshot equals the state, so reading the diagnostics does not disturb it)
        history = []

        def track(tag, offset):
            cb = progress(tag)

            def f(st, names):
                cb(st, names)
                history.append(([o + x for o, x in zip(offset, st)], ws.nusselt_numbers(b, tprobs)))
            return f
        t0 = time.perf_counter()
        steps, status = b.run(max_steps=args.ws_max_steps_eval, tol=1e-7, K=1000, chunk=args.ws_chunk,
                              progress=track("evaluate %s" % key, [0] * len(tprobs)))
        dt = time.perf_counter() - t0
        nu = ws.nusselt_numbers(b, tprobs)
        out[key] = {"steps": steps, "status": status, "nu": nu, "seconds": round(dt, 1)}
        if args.ws_refine_tol > 0:
            # continue from the state at 1e-7 to the tighter residual: both starts must
            # reach the same steady state
            t0 = time.perf_counter()
            steps_r, status_r = b.run(max_steps=args.ws_max_steps_eval, tol=args.ws_refine_tol, K=1000,
                                      chunk=args.ws_chunk, progress=track("refine %s" % key, steps))
            out[key].update(refine_steps=steps_r, refine_status=status_r,
                            refine_nu=ws.nusselt_numbers(b, tprobs),
                            refine_seconds=round(time.perf_counter() - t0, 1))
        out[key]["history"] = history
        del b
    both = [i for i in range(len(tprobs))
            if out["cold"]["status"][i] == "converged" and out["warm"]["status"][i] == "converged"]
    sc = np.array([out["cold"]["steps"][i] for i in both], dtype=float)
    sw = np.array([out["warm"]["steps"][i] for i in both], dtype=float)
    nc = np.array([out["cold"]["nu"][i] for i in both])
    nw = np.array([out["warm"]["nu"][i] for i in both])
    dnu = np.abs(nw - nc) / np.abs(nc)
    res["eval"] = {
        "cavities": len(tprobs), "side": args.ws_eval_side, "both_converged": len(both),
        "cold_steps_total": int(sc.sum()), "warm_steps_total": int(sw.sum()),
        "steps_ratio_warm_over_cold": round(float(sw.sum() / sc.sum()), 4) if len(both) else None,
        "median_ratio": round(float(np.median(sw / sc)), 4) if len(both) else None,
        "nu_rel_diff_max": float(dnu.max()) if len(both) else None,
        "nu_rel_diff_mean": float(dnu.mean()) if len(both) else None,
        "nu_within_1e-3": int((dnu < 1e-3).sum()),
        "cold_seconds": out["cold"]["seconds"], "warm_seconds": out["warm"]["seconds"],
        "nu_reference": "the cold start's Nu at the same residual",
        "per_instance": [{"Ra": p["meta"]["Ra"], "Pr": p["meta"]["Pr"], "Qstar": p["meta"]["Qstar"],
                          "cold_steps": out["cold"]["steps"][i], "warm_steps": out["warm"]["steps"][i],
                          "cold_status": out["cold"]["status"][i], "warm_status": out["warm"]["status"][i],
                          "cold_nu": out["cold"]["nu"][i], "warm_nu": out["warm"]["nu"][i]}
                         for i, p in enumerate(tprobs)],
    }
    if args.ws_refine_tol > 0:
        rb = [i for i in both if out["cold"]["refine_status"][i] == "converged"
              and out["warm"]["refine_status"][i] == "converged"]
        rc = np.array([out["cold"]["refine_nu"][i] for i in rb])
        rw = np.array([out["warm"]["refine_nu"][i] for i in rb])
        # the warm start's Nu at 1e-7 against the steady Nu (cold start refined)
        w7 = np.array([out["warm"]["nu"][i] for i in rb])
        d_ref = np.abs(rw - rc) / np.abs(rc)
        d_w7 = np.abs(w7 - rc) / np.abs(rc)
        d_c7 = np.abs(np.array([out["cold"]["nu"][i] for i in rb]) - rc) / np.abs(rc)
        res["eval"]["refine"] = {
            "tol": args.ws_refine_tol, "both_converged": len(rb),
            "nu_rel_diff_max": float(d_ref.max()) if len(rb) else None,
            "nu_within_1e-3": int((d_ref < 1e-3).sum()),
            "warm_at_1e-7_vs_steady_max": float(d_w7.max()) if len(rb) else None,
            "cold_at_1e-7_vs_steady_max": float(d_c7.max()) if len(rb) else None,
            "warm_at_1e-7_within_1e-3_of_steady": int((d_w7 < 1e-3).sum()),
            "cold_at_1e-7_within_1e-3_of_steady": int((d_c7 < 1e-3).sum()),
            "cold_extra_steps_total": int(sum(out["cold"]["refine_steps"][i] for i in rb)),
            "warm_extra_steps_total": int(sum(out["warm"]["refine_steps"][i] for i in rb)),
            "cold_seconds": out["cold"]["refine_seconds"], "warm_seconds": out["warm"]["refine_seconds"],
        }
        for i, rec in enumerate(res["eval"]["per_instance"]):
            rec.update(cold_refined_nu=out["cold"]["refine_nu"][i], warm_refined_nu=out["warm"]["refine_nu"][i],
                       cold_refine_steps=out["cold"]["refine_steps"][i],
                       warm_refine_steps=out["warm"]["refine_steps"][i])
        # steps to the tighter residual, and steps until Nu stays within 1e-3 of the steady
        # value (the cold start's Nu at the tighter residual), from the Nu recorded at every
        # chunk boundary
        c9 = np.array([out["cold"]["steps"][i] + out["cold"]["refine_steps"][i] for i in rb], dtype=float)
        w9 = np.array([out["warm"]["steps"][i] + out["warm"]["refine_steps"][i] for i in rb], dtype=float)

        def settle(key, i, ref):
            """First recorded step from which Nu of instance i stays within 1e-3 of ref."""
            first = None
            for st, nus in out[key]["history"]:
                if abs(nus[i] - ref) <= 1e-3 * abs(ref):
                    first = st[i] if first is None else first
                else:
                    first = None
            return first
        sc_nu, sw_nu = [], []
        for k, i in enumerate(rb):
            sc_nu.append(settle("cold", i, rc[k]))
            sw_nu.append(settle("warm", i, rc[k]))
        ok = [k for k in range(len(rb)) if sc_nu[k] is not None and sw_nu[k] is not None]
        res["eval"]["refine"].update({
            "cold_steps_to_tol_total": int(c9.sum()), "warm_steps_to_tol_total": int(w9.sum()),
            "steps_ratio_to_tol": round(float(w9.sum() / c9.sum()), 4) if len(rb) else None,
            "nu_settle_chunk_steps": args.ws_chunk,
            "nu_settled_both": len(ok),
            "cold_steps_to_nu_1e-3_total": int(sum(sc_nu[k] for k in ok)),
            "warm_steps_to_nu_1e-3_total": int(sum(sw_nu[k] for k in ok)),
            "steps_ratio_to_nu_1e-3": round(sum(sw_nu[k] for k in ok) / max(sum(sc_nu[k] for k in ok), 1), 4),
            "median_ratio_to_nu_1e-3": round(float(np.median([sw_nu[k] / sc_nu[k] for k in ok])), 4) if ok else None,
        })
        for k, i in enumerate(rb):
            res["eval"]["per_instance"][i].update(cold_steps_to_nu=sc_nu[k], warm_steps_to_nu=sw_nu[k])
    return res


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-valu":
        # --summarize-valu DB PRECISION N "command"
        a = sys.argv[2:]
        summarize_valu(a[0], a[1], int(a[2]), a[3])
        return
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
    ap.add_argument("--launch", default="", help="block_x,block_y,rows,remap[,steps_per_launch]")
    ap.add_argument("--kernel-launches", type=int, default=200)
    ap.add_argument("--batched", action="store_true", help="run the batched-sweep benchmark only")
    ap.add_argument("--configs", action="store_true",
                    help="the cache-resident configurations (64x32 channel, 256^2 to residual, 512^2) and the oracle")
    ap.add_argument("--sweep-count", type=int, default=256)
    ap.add_argument("--sweep-steps", type=int, default=200)
    ap.add_argument("--sweep-max-steps", type=int, default=200000)
    ap.add_argument("--sweep-tol", type=float, default=1e-7, help="residual of the batched run")
    ap.add_argument("--write-cache", default="", help="path of the autotuner cache (JSON lines)")
    ap.add_argument("--sweep-out", default="", help="write per-instance steps and statuses (JSON)")
    ap.add_argument("--sweep-summary", default="", help="write the autotuner and run summary (markdown)")
    ap.add_argument("--standin", action="store_true",
                    help="512^2 stand-in: FP32 and FP16 storage against the oracle over 20 000 steps")
    ap.add_argument("--standin-checkpoints", default="1000,5000,10000,20000")
    ap.add_argument("--standin-out", default="", help="write the error table (markdown) here")
    ap.add_argument("--warmstart", action="store_true", help="run the learned warm-start experiment only")
    ap.add_argument("--net", action="store_true", help="time the warm-start network's kernels only")
    ap.add_argument("--net-steps", type=int, default=50)
    ap.add_argument("--ws-train", type=int, default=2000)
    ap.add_argument("--ws-train-sides", default="64,96,128")
    ap.add_argument("--ws-chunk-instances", type=int, default=1024)
    ap.add_argument("--ws-max-steps", type=int, default=400000)
    ap.add_argument("--ws-max-steps-eval", type=int, default=3000000)
    ap.add_argument("--ws-grid", type=int, default=128)
    ap.add_argument("--ws-batch", type=int, default=32)
    ap.add_argument("--ws-train-steps", type=int, default=10000)
    ap.add_argument("--ws-eval", type=int, default=64)
    ap.add_argument("--ws-eval-side", type=int, default=512)
    ap.add_argument("--ws-save", default="", help="write the trained parameters (.npy)")
    ap.add_argument("--ws-load", default="", help="skip data generation and training; load parameters (.npy)")
    ap.add_argument("--ws-chunk", type=int, default=10000,
                    help="steps per batched-run call in the evaluation (Nu is recorded after each)")
    ap.add_argument("--ws-refine-tol", type=float, default=0.0,
                    help="after the runs to 1e-7, continue both to this residual and compare Nu there")
    ap.add_argument("--ws-out", default="")
    ap.add_argument("--ws-summary", default="", help="write the warm-start summary (markdown)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import numpy as np
    import paper_1801_04577_amd as clbm
    import workloads as W

    clbm.ensure_built()
    torch.cuda.set_device(0)
    if args.batched:
        print(json.dumps({"metric": METRIC, "batched": batched_sweep(args)}), flush=True)
        return
    if args.configs:
        print(json.dumps({"metric": METRIC, "configs": small_configs(args)}), flush=True)
        return
    if args.net:
        print(json.dumps({"metric": METRIC, "network": net_throughput(args)}), flush=True)
        return
    if args.standin:
        print(json.dumps({"metric": METRIC, "standin": standin_errors(args)}), flush=True)
        return
    if args.warmstart:
        r = warmstart_experiment(args)
        if args.ws_out:
            with open(args.ws_out, "w") as fh:
                json.dump(r, fh, indent=1)
        if args.ws_summary:
            write_ws_summary(r, args.ws_summary, " ".join(["python", "bench.py"] + sys.argv[1:]))
        print(json.dumps({"metric": METRIC, "warmstart": {k: v for k, v in r.items() if k != "eval"},
                          "eval": {k: v for k, v in r["eval"].items() if k != "per_instance"}}), flush=True)
        return
    prob = W.cavity(args.n, Ra=1e6, Pr=0.71, Q=5e-6)
    prec = clbm.CLBM_FP16_SHIFTED if args.precision == "fp16s" else clbm.CLBM_FP32
    s = clbm.Solver(prob, prec)
    if args.launch:
        v = [int(x) for x in args.launch.split(",")]
        s.set_launch(*v)
    gsteps = graph_steps(args.steps, args.diag_every)
    if gsteps > 0:
        s.set_graph(gsteps)          # instantiates both graphs before anything is timed
    T0 = torch.from_numpy(W.cavity_initial_T(prob, seed=12345).astype(np.float32))
    s.init(T=T0)
    # The reference copy runs first: besides the ceiling it reports (40 timed copies of
    # 2 GiB, about 28 ms), its streaming brings the shader and memory clocks out of idle,
    # so that a short timed region is not measured on the first launches after idle.
    copy_gbs, copy_ms = copy_ceiling(torch, clbm)
    log("bench: reference copy %.0f GB/s" % copy_gbs)
    log("bench: %dx%d %s, warmup %d, graphs of %d steps" % (args.n, args.n, args.precision, args.warmup, gsteps))
    time_steps(torch, s, args.warmup, args.diag_every)
    log("bench: timing %d steps" % args.steps)
    wall, ev_ms, diags = time_steps(torch, s, args.steps, args.diag_every)
    nodes = args.n * args.n
    mlups = nodes * args.steps / wall / 1e6
    spl = s.get_launch()["steps_per_launch"]
    launches = launches_of(args.steps, spl)
    kms = ev_ms / launches           # the timed region's launches, HIP events on the solver's stream
    log("bench: %.4f ms/step, %.1f MLUPS; %d launches, %.4f ms per launch (events), %d diagnostics"
        % (wall / args.steps * 1e3, mlups, launches, kms, diags))
    kms_iso, _ = kernel_avg_ms(torch, s, args.kernel_launches)
    d = s.diagnostics()
    bpl = BYTES_PER_LUP[args.precision]
    must_move = bpl * nodes                       # every population read once, written once
    achieved = must_move / (kms * 1e-3) / 1e9
    effective = bpl * nodes * spl / (kms * 1e-3) / 1e9
    log("bench: step kernel %.4f ms per launch of %d step(s) (%.4f ms over %d back-to-back launches), "
        "%.0f GB/s moved, %.0f GB/s per-step algorithmic, nan %d"
        % (kms, spl, kms_iso, args.kernel_launches, achieved, effective, d.nan_count))
    traffic = measured_traffic(args.precision, args.n, spl)
    valu = measured_valu(args.precision, args.n, spl)
    if diags:
        diag_text = "the diagnostics reduction after every %d steps (%d calls in the timed region)" % (
            args.diag_every, diags)
    else:
        diag_text = "no diagnostics in the timed region"
    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": arithmetic_dtype(args.precision),
        "data": "synthetic",
        "config": {"workload": "cavity %dx%d Ra=1e6 Pr=0.71 Q=5e-6 U=0.1, %s populations, "
                               "fused collide-and-stream, %d step(s) per launch, %s replayed from graphs "
                               "of %d steps, %s"
                               % (args.n, args.n, args.precision, spl, "steps" if gsteps else "no steps",
                                  gsteps, diag_text),
                   "nx": args.n, "ny": args.n, "storage": args.precision,
                   "collision_arithmetic": arithmetic_dtype(args.precision),
                   "launch": s.get_launch(), "graph_steps": gsteps, "diagnostics_calls": diags},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "bytes_per_launch": must_move,
                     "kernel": "k_step2" if spl == 2 else "k_step", "steps_per_launch": spl,
                     "kernel_avg_ms": round(kms, 5), "launches_timed": launches,
                     "kernel_avg_ms_back_to_back": round(kms_iso, 5),
                     # measured HBM bytes over the same launch time
                     "traffic_rate_GBs": None if traffic is None else round(traffic / (kms * 1e-3) / 1e9, 1),
                     # one-step updates the launch performs, at the one-step kernel's bytes each
                     "effective_GBs": round(effective, 1), "bytes_per_lup": bpl,
                     "copy_ceiling_GBs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4),
                     "note": ("achieved = bytes one launch must move (each of the %d B per node read once and "
                              "written once) / launch time from HIP events around the timed region; a launch "
                              "advances %d step(s), so the per-step algorithmic rate is effective_GBs"
                              % (bpl, spl)),
                     # the kernel's VALU issue from the committed counter profile
                     "valu": valu},
    }
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
