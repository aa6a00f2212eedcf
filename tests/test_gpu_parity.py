"""GPU (HIP, gfx950) fused step against the FP64 oracle, through the C ABI.

Bar (FP32 storage and arithmetic): after 1000 steps of the laminar workloads the
velocity and temperature agree with the oracle to a max relative error of 1e-5
(metric in tests/parity.py). Randomised small lattices (ragged sizes, every wall
type, moving walls, all source terms) are held to the same bar after 200 steps.
Post-collision populations are compared element by element.
"""
import math

import numpy as np
import pytest

import workloads as W
from parity import field_errors, f32, gpu_fields, population_errors, run_gpu, run_oracle

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    import paper_1801_04577_amd as clbm
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    clbm.ensure_built()


def report(name, e):
    print("%s: u %.3e  T %.3e  rho_abs %.3e  (umax %.3e Tmax %.3e)"
          % (name, e["u"], e["T"], e["rho_abs"], e["umax"], e["Tmax"]), flush=True)


def test_channel_64x32_1000_steps():
    prob = W.channel()
    o = run_oracle(prob, 1000)
    s = run_gpu(prob, 1000)
    e = field_errors(o, s)
    report("channel 64x32", e)
    assert e["u"] <= TOL and e["T"] <= TOL and e["rho_abs"] <= 1e-6
    p = population_errors(o, s, prob["T0"])
    print("populations", p)
    assert p["f"] <= TOL and p["g"] <= TOL


def test_cavity_256_1000_steps():
    prob = W.cavity(256, Ra=1e5, Pr=0.71)
    T = f32(W.cavity_initial_T(prob, seed=12345))
    o = run_oracle(prob, 1000, {"T": T})
    s = run_gpu(prob, 1000, {"T": T})
    e = field_errors(o, s)
    report("cavity 256 Ra=1e5", e)
    assert e["u"] <= TOL and e["T"] <= TOL and e["rho_abs"] <= 1e-6


def random_case(seed):
    rng = np.random.default_rng(seed)
    nx, ny = int(rng.integers(1, 140)), int(rng.integers(2, 90))
    px, py = rng.random() < 0.4, rng.random() < 0.3
    if not px and nx < 2:
        nx = 2

    def wall():
        kind = rng.integers(0, 3)
        u = float(rng.uniform(-0.05, 0.05)) if rng.random() < 0.4 else 0.0
        if kind == 0:
            return W.dirichlet(rng.uniform(-1, 1), u)
        if kind == 1:
            return W.adiabatic(u)
        return W.robin(rng.uniform(0.2, 2), rng.uniform(0.1, 2), rng.uniform(-1, 1), u)

    sides = [W.PERIODIC, W.PERIODIC] if px else [wall(), wall()]
    sides += [W.PERIODIC, W.PERIODIC] if py else [wall(), wall()]
    prob = W.problem(nx, ny, rng.uniform(0.01, 0.3), rng.uniform(0.01, 0.3), sides,
                     g_beta=rng.uniform(0, 1e-3), T0=rng.uniform(-0.3, 0.3),
                     Fx=rng.uniform(-1e-5, 1e-5), Fy=rng.uniform(-1e-5, 1e-5),
                     Q=rng.uniform(-1e-4, 1e-4))
    if rng.random() < 0.5:
        prob.update(s_b=rng.uniform(0.6, 1.6), s_4=rng.uniform(0.6, 1.6),
                    lambda_2=rng.uniform(0.5, 1.5))
    fields = {
        "rho": f32(1.0 + 1e-3 * rng.uniform(-1, 1, (ny, nx))),
        "ux": f32(0.02 * rng.uniform(-1, 1, (ny, nx))),
        "uy": f32(0.02 * rng.uniform(-1, 1, (ny, nx))),
        "T": f32(prob["T0"] + 0.5 * rng.uniform(-1, 1, (ny, nx))),
    }
    return prob, fields


@pytest.mark.parametrize("seed", range(12))
def test_random_lattices(seed):
    prob, fields = random_case(seed)
    o = run_oracle(prob, 200, fields)
    s = run_gpu(prob, 200, fields)
    e = field_errors(o, s)
    report("random %d (%dx%d)" % (seed, prob["nx"], prob["ny"]), e)
    assert e["u"] <= TOL and e["T"] <= TOL and e["rho_abs"] <= 1e-6
    p = population_errors(o, s, prob["T0"])
    assert p["f"] <= TOL and p["g"] <= TOL, p


@pytest.mark.parametrize("nx,ny,walls", [(1, 2, "y"), (2, 2, "xy"), (2, 1, "x"), (1, 1, "none"),
                                         (300, 2, "xy"), (2, 257, "xy")])
def test_degenerate_sizes(nx, ny, walls):
    sides = ([W.dirichlet(0.5), W.dirichlet(-0.5)] if "x" in walls else [W.PERIODIC] * 2) + \
            ([W.adiabatic(0.01), W.dirichlet(0.1)] if "y" in walls else [W.PERIODIC] * 2)
    prob = W.problem(nx, ny, 0.1, 0.08, sides, g_beta=1e-3, Fx=1e-5, Q=1e-4)
    rng = np.random.default_rng(nx * 1000 + ny)
    fields = {"T": f32(rng.uniform(-0.5, 0.5, (ny, nx))), "ux": f32(0.01 * rng.uniform(-1, 1, (ny, nx)))}
    o = run_oracle(prob, 100, fields)
    s = run_gpu(prob, 100, fields)
    e = field_errors(o, s)
    report("degenerate %dx%d" % (nx, ny), e)
    assert e["u"] <= TOL and e["T"] <= TOL


def test_init_state_matches_oracle():
    """t = 0: the GPU stores the collided equilibrium; its macros and post-collision
    populations equal the oracle's (Eq. 9, 19 and one collision)."""
    prob, fields = random_case(99)
    o = run_oracle(prob, 0, fields)
    s = run_gpu(prob, 0, fields)
    e = field_errors(o, s)
    assert e["u"] <= 1e-6 and e["T"] <= 1e-6
    p = population_errors(o, s, prob["T0"])
    assert p["f"] <= 1e-6 and p["g"] <= 1e-6, p


def test_diagnostics_match_oracle():
    import paper_1801_04577_amd as clbm
    prob = W.cavity(96, 80, Ra=1e5, Pr=0.71, Q=2e-5)
    T = f32(W.cavity_initial_T(prob, seed=5))
    o = run_oracle(prob, 400, {"T": T})
    s = run_gpu(prob, 400, {"T": T})
    d = s.diagnostics()
    ro = o.macros()[0]
    assert d.mass == pytest.approx(ro.sum(), rel=1e-7)
    assert d.nan_count == 0
    walls = [o.wall_values(side) for side in range(4)]
    # one gradient scale for all walls: adiabatic walls have dT/dn = 0 exactly
    scale = max(np.abs(dTdn).max() for _, dTdn in walls)
    for side, (Tw, dTdn) in enumerate(walls):
        assert abs(d.dTdn[side] - dTdn.mean()) <= 1e-4 * scale, side
        assert d.T_wall[side] == pytest.approx(Tw.mean(), abs=1e-5)
    # heat carried by the bounced links, 2 g*_out - c_T^2 T_w (Eq. 26), from the oracle's
    # post-collision populations at the wall nodes
    _, g = o.post_collision()
    g_out = [g[:, 0, 3], g[:, -1, 1], g[0, :, 4], g[-1, :, 2]]
    flux = [float(np.mean(2.0 * go - 0.4 * Tw)) for go, (Tw, _) in zip(g_out, walls)]
    fscale = max(abs(v) for v in flux)
    for side in range(4):
        assert abs(d.wall_flux[side] - flux[side]) <= 1e-4 * fscale, (side, d.wall_flux[side], flux[side])
    # residual: the snapshot is the state of the previous call
    s.step(100)
    d2 = s.diagnostics()
    assert d2.K == 100 and d2.res_u > 0 and d2.res_T > 0
    rg, uxg, uyg, Tg = gpu_fields(s)
    assert d2.sum_u2 == pytest.approx(float((uxg ** 2 + uyg ** 2).sum()), rel=1e-5)
    assert d2.sum_T2 == pytest.approx(float((Tg ** 2).sum()), rel=1e-5)


def test_graph_replay_is_bitwise_identical():
    import torch
    prob, fields = random_case(7)
    a = run_gpu(prob, 130, fields)
    b = run_gpu(prob, 130, fields, graph=16)
    for x, y in zip(a.populations(), b.populations()):
        assert torch.equal(x, y)


@pytest.mark.parametrize("launch", [dict(block_x=64, block_y=4), dict(block_x=128, block_y=2, rows_per_thread=2),
                                    dict(block_x=64, block_y=1, rows_per_thread=4, xcd_remap=1),
                                    dict(block_x=256, block_y=1, rows_per_thread=1, xcd_remap=1)])
def test_launch_shapes_are_bitwise_identical(launch):
    import torch
    prob, fields = random_case(3)
    a = run_gpu(prob, 60, fields)
    b = run_gpu(prob, 60, fields, launch=launch)
    for x, y in zip(a.populations(), b.populations()):
        assert torch.equal(x, y)


@pytest.mark.parametrize("seed", [0, 3, 5, 9, 11])
@pytest.mark.parametrize("steps", [1, 2, 37])
def test_two_step_launches_equal_single_steps(seed, steps):
    """Two time steps per launch (intermediate state in LDS) against one step per launch:
    bitwise identical states, also for an odd count (the last step runs alone) and through
    replayed graphs of 6 steps (three two-step launches)."""
    import torch
    prob, fields = random_case(seed)
    a = run_gpu(prob, steps, fields, launch=dict(block_x=256, steps_per_launch=1))
    b = run_gpu(prob, steps, fields, launch=dict(steps_per_launch=2))
    c = run_gpu(prob, steps + 12, fields, launch=dict(steps_per_launch=2), graph=6)
    d = run_gpu(prob, steps + 12, fields, launch=dict(block_x=256, steps_per_launch=1))
    for x, y in zip(a.populations(), b.populations()):
        assert torch.equal(x, y)
    for x, y in zip(c.populations(), d.populations()):
        assert torch.equal(x, y)


def test_two_step_launch_viscous_and_fp16_rules():
    import torch
    import paper_1801_04577_amd as clbm
    prob = dict(W.viscous_channel(32, nx=150), Q=1e-6)
    a = run_gpu(prob, 41, None, launch=dict(block_x=256, steps_per_launch=1))
    b = run_gpu(prob, 41, None, launch=dict(steps_per_launch=2))
    for x, y in zip(a.populations(), b.populations()):
        assert torch.equal(x, y)
    s = clbm.Solver(W.channel(), clbm.CLBM_FP16_SHIFTED)
    assert s.get_launch()["steps_per_launch"] == 2
    s.set_launch(steps_per_launch=1)
    assert s.get_launch()["steps_per_launch"] == 1
    with pytest.raises(clbm.ClbmError):
        s.set_launch(steps_per_launch=3)


@pytest.mark.parametrize("case", ["seed0", "seed5", "seed11", "walls", "periodic", "viscous", "wide"])
@pytest.mark.parametrize("steps", [2, 37])
def test_two_step_launches_equal_single_steps_fp16(case, steps):
    """FP16 storage, two steps per launch (64 x 14 tiles, the intermediate state rounded
    into binary16 in LDS) against one step per launch: bitwise identical states, also
    through replayed graphs of 6 steps."""
    import torch
    import paper_1801_04577_amd as clbm
    prob, fields = random_case(int(case[4:])) if case.startswith("seed") else _interior_case(case)
    h = clbm.CLBM_FP16_SHIFTED
    a = run_gpu(prob, steps, fields, precision=h, launch=dict(block_x=256, steps_per_launch=1))
    b = run_gpu(prob, steps, fields, precision=h, launch=dict(steps_per_launch=2))
    c = run_gpu(prob, steps + 12, fields, precision=h, launch=dict(steps_per_launch=2), graph=6)
    d = run_gpu(prob, steps + 12, fields, precision=h, launch=dict(block_x=256, steps_per_launch=1))
    for x, y in zip(a.populations(), b.populations()):
        assert torch.equal(x, y)
    for x, y in zip(c.populations(), d.populations()):
        assert torch.equal(x, y)


def test_checkpoint_resume_bitwise():
    import torch
    prob, fields = random_case(11)
    a = run_gpu(prob, 80, fields)
    s = run_gpu(prob, 30, fields)
    buf, t = s.save()
    s.step(10)                 # move on, then restore
    s.load(buf, t)
    s.step(50)
    assert s.t == 80
    for x, y in zip(a.populations(), s.populations()):
        assert torch.equal(x, y)


def test_determinism():
    import torch
    prob, fields = random_case(4)
    a = run_gpu(prob, 100, fields)
    b = run_gpu(prob, 100, fields)
    da, db = a.diagnostics(), b.diagnostics()
    assert da.mass == db.mass and da.sum_u2 == db.sum_u2 and list(da.dTdn) == list(db.dTdn)
    for x, y in zip(a.populations(), b.populations()):
        assert torch.equal(x, y)


def _interior_case(kind):
    """Lattices wide and tall enough that most two-step tiles (64 x 14 plus a ring) and
    most one-step blocks lie strictly inside: they take the interior gather."""
    nx, ny = (800, 40) if kind == "wide" else (300, 100)
    rng = np.random.default_rng({"walls": 1, "periodic": 2, "viscous": 3, "wide": 4}[kind])
    robin = [W.robin(1, 0.5, 0.05, 0.03), W.robin(0.5, 1, -0.05, -0.02), W.robin(1, 1, 0, 0.01),
             W.dirichlet(0.0, u_wall=-0.04)]
    if kind == "periodic":
        prob = W.problem(nx, ny, 0.05, 0.05, [W.PERIODIC] * 4, Fx=2e-6, Fy=1e-6, Q=1e-5)
    elif kind == "viscous":
        prob = W.problem(nx, ny, 0.07, 0.05, [W.PERIODIC, W.PERIODIC] + robin[2:], Fx=3e-6, Q=1e-5,
                         T0=0.05, viscous_heating=True)
    else:
        prob = W.problem(nx, ny, 0.07, 0.05, robin, g_beta=1e-4, Fx=3e-6, Q=1e-5, T0=0.05)
    fields = {"ux": f32(0.02 * rng.uniform(-1, 1, (ny, nx))), "uy": f32(0.02 * rng.uniform(-1, 1, (ny, nx))),
              "T": f32(prob["T0"] + 0.1 * rng.uniform(-1, 1, (ny, nx)))}
    return prob, fields


@pytest.mark.parametrize("kind", ["walls", "periodic", "viscous", "wide"])
def test_interior_tiles(kind):
    """Interior tiles and blocks skip the wall logic and address their sources through row
    pointers: two-step launches and one-step launches of several shapes give the same state
    bit for bit, and that state matches the oracle."""
    import torch
    prob, fields = _interior_case(kind)
    steps = 41
    runs = [run_gpu(prob, steps, fields, launch=dict(steps_per_launch=2))]
    for bx, by, rows, remap in [(256, 1, 1, 0), (64, 4, 1, 1), (128, 2, 2, 0), (32, 2, 1, 0)]:
        runs.append(run_gpu(prob, steps, fields, launch=dict(block_x=bx, block_y=by, rows_per_thread=rows,
                                                               xcd_remap=remap, steps_per_launch=1)))
    for r in runs[1:]:
        for x, y in zip(runs[0].populations(), r.populations()):
            assert torch.equal(x, y)
    o = run_oracle(prob, steps, fields)
    e = field_errors(o, runs[0])
    report("interior %s (%dx%d)" % (kind, prob["nx"], prob["ny"]), e)
    assert e["u"] <= TOL and e["T"] <= TOL and e["rho_abs"] <= 1e-6
    p = population_errors(o, runs[0], prob["T0"])
    assert p["f"] <= TOL and p["g"] <= TOL, p


@pytest.mark.parametrize("kind", ["walls", "wide"])
def test_interior_blocks_fp16(kind):
    """FP16 storage: one-step launches of several shapes (interior and generic blocks mixed
    differently) give the same state bit for bit."""
    import torch
    import paper_1801_04577_amd as clbm
    prob, fields = _interior_case(kind)
    runs = [run_gpu(prob, 23, fields, precision=clbm.CLBM_FP16_SHIFTED,
                    launch=dict(block_x=bx, block_y=by, rows_per_thread=rows, xcd_remap=remap))
            for bx, by, rows, remap in [(256, 1, 1, 0), (64, 4, 1, 1), (512, 1, 2, 0), (32, 2, 1, 0)]]
    for r in runs[1:]:
        for x, y in zip(runs[0].populations(), r.populations()):
            assert torch.equal(x, y)


@pytest.mark.parametrize("rows", [6, 14, 22, 30])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("case", ["seed3", "walls", "periodic", "viscous"])
def test_two_step_tile_heights(rows, precision, case):
    """Two-step tiles of 64 x 6, 14, 22 and 30 nodes (256, 512, 512 and 1024 threads; three
    rows per wave at 22) give the state of
    one-step launches bit for bit, for both storage types, at walls, in interior tiles, in
    a fully periodic lattice and with viscous heating; 37 steps end with a one-step launch."""
    import torch
    prob, fields = random_case(int(case[4:])) if case.startswith("seed") else _interior_case(case)
    a = run_gpu(prob, 37, fields, precision=precision, launch=dict(block_x=256, steps_per_launch=1))
    b = run_gpu(prob, 37, fields, precision=precision,
                launch=dict(steps_per_launch=2, xcd_remap=1, two_step_rows=rows))
    assert b.get_launch()["two_step_rows"] == rows
    for x, y in zip(a.populations(), b.populations()):
        assert torch.equal(x, y), (rows, precision, case)
