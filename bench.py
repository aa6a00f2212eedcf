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


def main():
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

    out = {
        "metric": METRIC, "value": round(mlups, 2), "unit": "MLUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall / args.steps * 1e3, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "cavity %dx%d Ra=1e6 Pr=0.71 Q=5e-6 U=0.1, %s populations, "
                               "fused collide-and-stream, diagnostics every %d steps"
                               % (args.n, args.n, args.precision, args.diag_every),
                   "nx": args.n, "ny": args.n, "precision": args.precision,
                   "launch": s.get_launch()},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel_avg_ms": round(kms, 5), "bytes_per_lup": bpl},
    }
    if not args.no_cpu_baseline:
        log("bench: timing the FP64 oracle on the host")
        out["cpu_baseline"] = cpu_baseline(prob)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
