"""Viscous-dissipation heat source (Sec. 3.2) on the GPU against the FP64 oracle.

The source nu [(d_x u_y + d_y u_x)^2 + (d_x u_x - d_y u_y)^2] is evaluated inside the
fused step from the pre-collision central moments, and recovered from the stored
post-collision moments wherever a temperature is read back (wall extrapolation of
Eq. 28, macroscopic fields, diagnostics). Bar: the FP32 parity bar of the fused step,
max relative error 1e-5 on u and T (metric in tests/parity.py).
"""
import math

import numpy as np
import pytest

import workloads as W
from parity import f32, field_errors, population_errors, run_gpu, run_oracle

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


def lid_problem(nx=48, ny=40):
    """Moving lid over a closed box; every wall held at or relaxed towards T = 0, so all
    the heat in the box comes from viscous dissipation (shear and extension)."""
    sides = [W.dirichlet(0.0), W.robin(1.0, 0.5, 0.0), W.adiabatic(), W.dirichlet(0.0, u_wall=0.05)]
    return W.problem(nx, ny, 0.05, 0.04, sides, viscous_heating=True)


@pytest.mark.parametrize("transpose", [False, True])
def test_channel_1000_steps(transpose):
    prob = W.viscous_channel(32, nx=24, umax=0.02, transpose=transpose)
    o = run_oracle(prob, 1000)
    s = run_gpu(prob, 1000)
    e = field_errors(o, s)
    report("viscous channel%s" % (" (turned)" if transpose else ""), e)
    assert e["u"] <= TOL and e["T"] <= TOL and e["rho_abs"] <= 1e-6
    p = population_errors(o, s, prob["T0"])
    assert p["f"] <= TOL and p["g"] <= TOL


def test_lid_driven_box_1000_steps():
    prob = lid_problem()
    o = run_oracle(prob, 1000)
    s = run_gpu(prob, 1000)
    e = field_errors(o, s)
    report("viscous lid box 48x40", e)
    assert e["Tmax"] > 0
    assert e["u"] <= TOL and e["T"] <= TOL and e["rho_abs"] <= 1e-6


@pytest.mark.parametrize("seed", range(4))
def test_random_flows_200_steps(seed):
    """Ragged lattices, random walls (moving or not), random initial velocity so that
    both strain terms are large from the first step."""
    rng = np.random.default_rng(100 + seed)
    nx, ny = int(rng.integers(2, 120)), int(rng.integers(2, 80))
    px = rng.random() < 0.5

    def wall():
        u = float(rng.uniform(-0.05, 0.05))
        return W.robin(rng.uniform(0.2, 2), rng.uniform(0.1, 2), rng.uniform(-0.1, 0.1), u)

    sides = ([W.PERIODIC, W.PERIODIC] if px else [wall(), wall()]) + [wall(), wall()]
    prob = W.problem(nx, ny, rng.uniform(0.01, 0.3), rng.uniform(0.01, 0.3), sides,
                     Fx=rng.uniform(-1e-5, 1e-5), Fy=rng.uniform(-1e-5, 1e-5),
                     Q=rng.uniform(0, 1e-6), T0=rng.uniform(-0.1, 0.1), viscous_heating=True)
    fields = {"ux": f32(W.noise_field(seed * 3 + 1, nx, ny, 0.03)),
              "uy": f32(W.noise_field(seed * 3 + 2, nx, ny, 0.03)),
              "T": f32(prob["T0"] + W.noise_field(seed * 3 + 3, nx, ny, 1e-3))}
    o = run_oracle(prob, 200, fields)
    s = run_gpu(prob, 200, fields)
    e = field_errors(o, s)
    report("viscous random %d (%dx%d)" % (seed, nx, ny), e)
    assert e["u"] <= TOL and e["T"] <= TOL


def test_poiseuille_steady_closed_form():
    """Steady channel at h = 16: the GPU reproduces the oracle's steady profile and so
    the closed form of Sec. 3.2 to the oracle's own discretisation error."""
    ny = 32
    prob = W.viscous_channel(ny)
    steps = int(6 * ny * ny / prob["alpha"])
    o = run_oracle(prob, steps, nthreads=1)
    s = run_gpu(prob, steps, graph=500)
    Tg = s.macros()[3].cpu().numpy().astype(np.float64)[:, 0]
    To = o.macros()[3][:, 0]
    Ta = W.viscous_channel_exact(ny)
    e_or = math.sqrt(np.sum((To - Ta) ** 2) / np.sum(Ta ** 2))
    e_gpu = math.sqrt(np.sum((Tg - Ta) ** 2) / np.sum(Ta ** 2))
    rel = float(np.abs(Tg - To).max() / np.abs(To).max())
    print("steady viscous channel ny=32: E2 oracle %.4e gpu %.4e, max rel diff %.2e"
          % (e_or, e_gpu, rel), flush=True)
    assert rel <= TOL
    assert e_gpu < 2.5e-3


def test_diagnostics_wall_flux():
    """Wall values under viscous heating: the mean outward gradient at each channel wall
    balances half the dissipated heat (steady energy balance alpha dT/dn = -int Q dy / 2)."""
    import paper_1801_04577_amd as clbm
    ny = 32
    prob = W.viscous_channel(ny)
    s = run_gpu(prob, int(6 * ny * ny / prob["alpha"]), graph=500)
    d = s.diagnostics()
    h = ny / 2.0
    F = prob["Fx"]
    # int_{-h}^{h} nu (F y / nu)^2 dy = 2 F^2 h^3 / (3 nu)
    total = 2.0 * F * F * h ** 3 / (3.0 * prob["nu"])
    for side in (2, 3):
        flux = -prob["alpha"] * d.dTdn[side]
        print("side", side, "flux", flux, "expected", total / 2.0, flush=True)
        assert abs(flux - total / 2.0) < 0.02 * total / 2.0


def test_batch_with_viscous_instances():
    """Instances with and without viscous heating in one batch: each evolves bit for bit
    as the same lattice advanced alone."""
    import torch
    import paper_1801_04577_amd as clbm
    probs = [W.viscous_channel(32, nx=40), lid_problem(50, 37), W.cavity(48, 40, Ra=1e4),
             W.viscous_channel(20, nx=33, transpose=True)]
    b = clbm.Batch(probs)
    for i in range(len(probs)):
        b.init(i)
    b.step(300)
    for i, p in enumerate(probs):
        s = clbm.Solver(p)
        s.init()
        s.step(300)
        for x, y in zip(b.macros(i), s.macros()):
            assert torch.equal(x, y), i


def test_fp16_viscous_random():
    """FP16 storage with viscous heating: the shifted-storage bar (1e-2) on a flow whose
    dissipation is large from the first step."""
    import paper_1801_04577_amd as clbm
    nx, ny = 64, 48
    sides = [W.dirichlet(0.0), W.dirichlet(0.0), W.dirichlet(0.0), W.dirichlet(0.0, u_wall=0.08)]
    prob = W.problem(nx, ny, 0.02, 0.02, sides, viscous_heating=True)
    fields = {"ux": f32(W.noise_field(91, nx, ny, 0.05)), "uy": f32(W.noise_field(92, nx, ny, 0.05))}
    o = run_oracle(prob, 300, fields)
    s = run_gpu(prob, 300, fields, precision=clbm.CLBM_FP16_SHIFTED)
    e = field_errors(o, s)
    report("viscous fp16s 64x48", e)
    assert e["u"] <= 1e-2 and e["T"] <= 2e-2


def test_poiseuille_grid_convergence():
    """Sec. 3.2 grid study on the GPU: E2 against the closed form falls at second order
    (the paper fits a slope of 2.05)."""
    errs = []
    for ny in (8, 16, 32, 64):
        prob = W.viscous_channel(ny)
        s = run_gpu(prob, int(6 * ny * ny / prob["alpha"]), graph=500)
        T = s.macros()[3].cpu().numpy().astype(np.float64)[:, 0]
        Ta = W.viscous_channel_exact(ny)
        errs.append(math.sqrt(np.sum((T - Ta) ** 2) / np.sum(Ta ** 2)))
    slopes = [math.log2(errs[k] / errs[k + 1]) for k in range(len(errs) - 1)]
    print("viscous channel E2", ["%.3e" % e for e in errs], "slopes", ["%.3f" % v for v in slopes],
          flush=True)
    assert all(1.9 < v < 2.2 for v in slopes)


def test_couette_viscous_heating_steady():
    """Thermal Couette flow with viscous heating: steady GPU state against the oracle's
    (parity bar) and against the closed form (O(Ma^2) departure, as in the oracle)."""
    ny, U = 16, 0.01
    prob = W.couette(nx=8, ny=ny, nu=0.1, alpha=0.1, U=U, Tc=0.0, Th=0.0)
    prob["viscous_heating"] = True
    steps = int(8 * ny * ny / 0.1)
    o = run_oracle(prob, steps, nthreads=1)
    s = run_gpu(prob, steps, graph=512)
    e = field_errors(o, s)
    report("viscous Couette steady", e)
    assert e["u"] <= TOL and e["T"] <= TOL
    T = s.macros()[3].cpu().numpy().astype(np.float64)[:, 0]
    y = np.arange(ny) + 0.5
    heat = 0.1 * U * U / (2 * 0.1 * ny * ny) * y * (ny - y)
    assert np.abs(T - heat).max() / np.abs(heat).max() < 2e-6
