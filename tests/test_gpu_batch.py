"""Batched form: many lattices of uneven size and parameters advanced by one kernel
launch per step over a device tile list, with on-device convergence checks and
retirement (C ABI clbm_batch_*). Each instance must evolve exactly as the same lattice
advanced alone (same per-node arithmetic), and the oracle bar applies to both."""
import json
import os

import numpy as np
import pytest

import workloads as W
from parity import f32, field_errors, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    import paper_1801_04577_amd as clbm
    assert torch.cuda.is_available()
    clbm.ensure_built()


def mixed_problems():
    probs = [W.cavity(64, 96, Ra=1e4, Pr=0.71),
             W.cavity(130, 67, Ra=1e5, Pr=2.0, Q=5e-5),
             W.channel(nx=70, ny=33),
             W.cavity(33, 33, Ra=3e3, Pr=6.0),
             W.couette(nx=65, ny=20, U=0.02, Q=1e-4),
             W.cavity(200, 120, Ra=1e6, Pr=0.7, Q=1e-5)]
    fields = []
    for k, p in enumerate(probs):
        fields.append({"T": f32(p["T0"] + W.noise_field(k + 1, p["nx"], p["ny"], 1e-4))})
    return probs, fields


def run_single(prob, fields, steps, precision=0):
    import torch
    import paper_1801_04577_amd as clbm
    s = clbm.Solver(prob, precision)
    s.init(**{k: torch.from_numpy(v) for k, v in fields.items()})
    s.step(steps)
    return s


@pytest.mark.parametrize("launch", [None, dict(tile_x=128, tile_y=2, persistent_wgs=0),
                                    dict(tile_x=64, tile_y=8, persistent_wgs=64),
                                    dict(tile_x=64, tile_y=14, persistent_wgs=0, steps_per_launch=2),
                                    dict(tile_x=64, tile_y=14, persistent_wgs=40, steps_per_launch=2),
                                    dict(tile_x=64, tile_y=14, persistent_wgs=40, steps_per_launch=2,
                                         xcd_bands=0),
                                    dict(tile_x=64, tile_y=6, persistent_wgs=0, steps_per_launch=2),
                                    dict(tile_x=64, tile_y=30, persistent_wgs=24, steps_per_launch=2),
                                    dict(tile_x=64, tile_y=22, persistent_wgs=0, steps_per_launch=2)])
@pytest.mark.parametrize("precision", [0, 1])
def test_batch_equals_single_lattices(launch, precision):
    """Every launch shape and both storage types: each instance bitwise equal to its
    lattice advanced alone (151 steps: two-step launches end with a one-step launch)."""
    import torch
    import paper_1801_04577_amd as clbm
    probs, fields = mixed_problems()
    b = clbm.Batch(probs, launch=launch, precision=precision)
    for i, f in enumerate(fields):
        b.init(i, **{k: torch.from_numpy(v) for k, v in f.items()})
    b.step(151)
    for i, (p, f) in enumerate(zip(probs, fields)):
        s = run_single(p, f, 151, precision)
        for x, y in zip(b.macros(i), s.macros()):
            assert torch.equal(x, y), (i, launch, precision)


@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-2)])
def test_batch_instance_matches_oracle(precision, tol):
    import torch
    import paper_1801_04577_amd as clbm
    probs, fields = mixed_problems()
    b = clbm.Batch(probs, precision=precision)
    for i, f in enumerate(fields):
        b.init(i, **{k: torch.from_numpy(v) for k, v in f.items()})
    b.step(300)
    for i in (1, 4, 5):
        o = run_oracle(probs[i], 300, fields[i])

        class View:  # field_errors reads .macros()
            def macros(self_inner):
                return b.macros(i)
        e = field_errors(o, View())
        print("batch instance %d, %s: u %.2e T %.2e" % (i, "fp32" if precision == 0 else "fp16s",
                                                       e["u"], e["T"]), flush=True)
        assert e["u"] <= tol and e["T"] <= tol, (i, e)


def test_batch_step_after_retirement():
    """clbm_batch_step advances every instance, the ones a run has retired included: after
    a run has retired the first cavity and not the second, two more steps leave each
    instance bitwise equal to its lattice advanced alone to its own step count plus two,
    and a resumed run still treats the first as retired."""
    import torch
    import paper_1801_04577_amd as clbm
    probs = [W.cavity(24, 24, Ra=1e3, Pr=0.71), W.cavity(48, 40, Ra=1e5, Pr=0.71)]
    fields = [{"T": f32(p["T0"] + W.noise_field(i, p["nx"], p["ny"], 1e-4))} for i, p in enumerate(probs)]
    b = clbm.Batch(probs)
    for i, f in enumerate(fields):
        b.init(i, **{k: torch.from_numpy(v) for k, v in f.items()})
    steps, status = b.run(max_steps=400000, tol=1e-6, K=200, chunk=1000, max_calls=1)
    while status[0] != "converged":
        steps, status = b.run(max_steps=400000, tol=1e-6, K=200, chunk=1000, max_calls=1, reset=False)
    assert status[1] == "running", (steps, status)
    b.step(2)
    for i, (p, f) in enumerate(zip(probs, fields)):
        s = run_single(p, f, steps[i] + 2)
        for x, y in zip(b.macros(i), s.macros()):
            assert torch.equal(x, y), (i, steps)
    s2, st2 = b.run(max_steps=400000, tol=1e-6, K=200, chunk=200, max_calls=1, reset=False)
    assert st2[0] == "converged" and s2[0] == steps[0]


def test_batch_run_converges_and_retires():
    """Small cavities converge at different times; each retired instance stays frozen
    while the others continue, and reports the step of its last window."""
    import torch
    import paper_1801_04577_amd as clbm
    probs = [W.cavity(24, 24, Ra=1e3, Pr=0.71), W.cavity(32, 24, Ra=1e4, Pr=0.71),
             W.cavity(40, 40, Ra=2e4, Pr=1.0)]
    b = clbm.Batch(probs)
    for i, p in enumerate(probs):
        b.init(i, T=torch.from_numpy(f32(p["T0"] + W.noise_field(i, p["nx"], p["ny"], 1e-4))))
    steps, status = b.run(max_steps=400000, tol=1e-6, K=200)
    assert status == ["converged"] * 3, (steps, status)
    assert all(s % 200 == 0 and s > 0 for s in steps)
    assert len(set(steps)) > 1
    for i in range(3):
        ru, rT = b.residual(i)
        assert max(ru, rT) < 1e-6
    # frozen after retirement: a second run with tol=inf retires everything after one window
    s2, st2 = b.run(max_steps=1000, tol=float("inf"), K=200)
    assert st2 == ["converged"] * 3 and s2 == [200] * 3


@pytest.mark.parametrize("K", [150, 200])
def test_batch_run_two_step_equals_one_step(K):
    """The replayed run graph with two-step launches (K/2 odd: two one-step launches
    keep the buffer parity) ends in the same states, step counts and statuses as the
    one-step graph."""
    import torch
    import paper_1801_04577_amd as clbm
    probs = [W.cavity(24, 24, Ra=1e3, Pr=0.71), W.cavity(70, 33, Ra=1e4, Pr=0.71, Q=1e-5),
             dict(W.viscous_channel(20, nx=66), Q=1e-6)]
    out = []
    for launch in (dict(tile_x=64, tile_y=4, steps_per_launch=1),
                   dict(tile_x=64, tile_y=14, steps_per_launch=2)):
        b = clbm.Batch(probs, launch=launch)
        for i, p in enumerate(probs):
            b.init(i, T=torch.from_numpy(f32(p["T0"] + W.noise_field(i, p["nx"], p["ny"], 1e-4))))
        steps, status = b.run(max_steps=3 * K, tol=1e-12, K=K)
        out.append((steps, status, [b.macros(i) for i in range(len(probs))]))
    assert out[0][0] == out[1][0] and out[0][1] == out[1][1]
    for ma, mb in zip(out[0][2], out[1][2]):
        for x, y in zip(ma, mb):
            assert torch.equal(x, y)


def test_batch_divergence_and_max_steps():
    import torch
    import paper_1801_04577_amd as clbm
    probs = [W.cavity(32, 32, Ra=1e4), W.cavity(48, 40, Ra=1e5)]
    b = clbm.Batch(probs)
    T = f32(np.zeros((32, 32)))
    T[5, 7] = np.nan
    b.init(0, T=torch.from_numpy(T))
    b.init(1)
    steps, status = b.run(max_steps=600, tol=0.0, K=200)
    assert status == ["diverged", "max_steps"], status
    assert steps == [200, 600]


def test_autotune_writes_cache_and_keeps_results(tmp_path):
    import torch
    import paper_1801_04577_amd as clbm
    probs, fields = mixed_problems()
    cache = str(tmp_path / "tune.jsonl")
    b = clbm.Batch(probs)
    assert b.cached_launch(cache) is None
    best = b.autotune(steps=4, cache_path=cache)
    lines = [json.loads(l) for l in open(cache)]
    # at least 12 one-step shapes and 4 two-step heights x 2 dealing orders, one workgroup
    # per tile (persistent counts at or above the tile count are skipped), and the best line
    assert len(lines) >= 12 + 8 + 1 and all(l["ms_per_step"] > 0 for l in lines)
    assert {l["tile_y"] for l in lines if l.get("steps_per_launch") == 2} == {6, 14, 22, 30}
    assert {l["xcd_bands"] for l in lines if l.get("steps_per_launch") == 2} == {0, 1}
    assert lines[-1]["best"] == 1 and len({l["signature"] for l in lines}) == 1
    assert best["tile_x"] % 64 == 0
    # read back: a batch of the same workload takes the cached launch, another one does not
    again = clbm.Batch(probs, tune_cache=cache)
    assert again.tuned_from_cache and again.cached_launch(cache) == best
    other = clbm.Batch(probs[:-1], tune_cache=cache)
    assert not other.tuned_from_cache
    for i, f in enumerate(fields):
        b.init(i, **{k: torch.from_numpy(v) for k, v in f.items()})
    b.step(40)
    ref = clbm.Batch(probs)
    for i, f in enumerate(fields):
        ref.init(i, **{k: torch.from_numpy(v) for k, v in f.items()})
    ref.step(40)
    for i in range(len(probs)):
        for x, y in zip(b.macros(i), ref.macros(i)):
            assert torch.equal(x, y)
