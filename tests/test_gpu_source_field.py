"""A heat source given per node (Q + Q_field, Sec. 3.2's spatially variable source in
Eq. 23-25) on the GPU, through the C ABI, against the oracle:
  * random two-dimensional fields in walled and periodic lattices, with buoyancy, Robin
    walls and viscous heating: FP32 within the 1e-5 bar after 300 steps, FP16 within 1e-2;
  * every launch shape (one-step blocks, two-step tiles of each height, the interior
    paths) gives the same state bit for bit;
  * steady diffusion with a source linear across the channel reaches the cubic closed
    form that the oracle reproduces to round-off;
  * batched instances with and without fields (and with viscous heating) evolve bit for
    bit as the same lattices advanced alone.
The fields are rounded to float32 first, so both sides use the same values."""
import math

import numpy as np
import pytest

import workloads as W
from parity import f32, field_errors, run_gpu, run_oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    import paper_1801_04577_amd as clbm
    assert torch.cuda.is_available()
    clbm.ensure_built()


def field_case(kind, seed=0):
    rng = np.random.default_rng(seed)
    if kind == "cavity":
        prob = W.cavity(150, 70, Ra=1e5, Pr=0.71, Q=1e-5)
    elif kind == "robin":
        prob = W.problem(130, 90, 0.07, 0.05, [W.robin(1, 0.5, 0.05, 0.03), W.robin(0.5, 1, -0.05, -0.02),
                                               W.robin(1, 1, 0, 0.01), W.dirichlet(0.0, u_wall=-0.04)],
                         g_beta=1e-4, Fx=3e-6, Q=1e-5, T0=0.05)
    elif kind == "periodic":
        prob = W.problem(200, 60, 0.05, 0.05, [W.PERIODIC] * 4, Fx=2e-6, Fy=1e-6, Q=0.0)
    else:  # viscous heating and a field together
        prob = W.problem(140, 48, 0.07, 0.05, [W.PERIODIC, W.PERIODIC, W.dirichlet(0.0), W.dirichlet(0.1)],
                         Fx=4e-6, Q=1e-6, viscous_heating=True)
    ny, nx = prob["ny"], prob["nx"]
    y, x = np.mgrid[0:ny, 0:nx]
    q = 5e-5 * (1 + np.sin(2 * math.pi * x / nx) * np.cos(math.pi * y / ny)) + rng.uniform(0, 2e-5, (ny, nx))
    prob["Q_field"] = f32(q).astype(np.float64)
    fields = {"T": f32(prob["T0"] + 0.05 * rng.uniform(-1, 1, (ny, nx))),
              "ux": f32(0.01 * rng.uniform(-1, 1, (ny, nx)))}
    return prob, fields


@pytest.mark.parametrize("kind", ["cavity", "robin", "periodic", "viscous"])
@pytest.mark.parametrize("precision,tol", [(0, 1e-5), (1, 1e-2)])
def test_field_matches_oracle(kind, precision, tol):
    prob, fields = field_case(kind)
    o = run_oracle(prob, 300, fields)
    s = run_gpu(prob, 300, fields, precision=precision)
    e = field_errors(o, s)
    print("source field %s, %s: u %.2e T %.2e" % (kind, "fp32" if precision == 0 else "fp16s", e["u"], e["T"]),
          flush=True)
    assert e["u"] <= tol and e["T"] <= tol


@pytest.mark.parametrize("kind", ["cavity", "robin", "periodic", "viscous"])
def test_field_launch_shapes_bitwise(kind):
    import torch
    prob, fields = field_case(kind, seed=1)
    runs = [run_gpu(prob, 37, fields, launch=dict(block_x=256, steps_per_launch=1))]
    runs.append(run_gpu(prob, 37, fields, launch=dict(block_x=64, block_y=4, rows_per_thread=2,
                                                      xcd_remap=1, steps_per_launch=1)))
    for rows in (6, 14, 22, 30):
        runs.append(run_gpu(prob, 37, fields, launch=dict(steps_per_launch=2, xcd_remap=1, two_step_rows=rows)))
    for r in runs[1:]:
        for x, y in zip(runs[0].populations(), r.populations()):
            assert torch.equal(x, y), kind


def test_linear_source_steady_closed_form():
    """alpha T'' + a + b y = 0 between walls at T = 0: the cubic closed form, within the
    FP32 storage's resolution of the steady state (the oracle meets it to round-off)."""
    import torch
    import paper_1801_04577_amd as clbm
    L, alpha, a, b = 12, 0.1, 2e-3, 1e-3
    y = np.arange(L) + 0.5
    prob = W.problem(64, L, 0.1, alpha, [W.PERIODIC, W.PERIODIC, W.dirichlet(0.0), W.dirichlet(0.0)])
    prob["Q_field"] = np.broadcast_to(f32(a + b * y)[:, None], (L, 64)).astype(np.float64)
    s = clbm.Solver(prob)
    s.set_graph(100)
    s.step(int(40 * L * L / alpha) + 2000)
    T = s.macros()[3].cpu().numpy().astype(np.float64)
    qy = f32(a + b * y).astype(np.float64)
    # closed form for the float32 source values (linear in y up to their rounding)
    exact = (-(a * y ** 2 / 2 + b * y ** 3 / 6) + (a * L / 2 + b * L ** 2 / 6) * y) / alpha
    err = math.sqrt(float(np.sum((T - exact[:, None]) ** 2) / (64 * np.sum(exact ** 2))))
    print("linear source, steady: E2 %.2e (source rounding %.1e)" % (err, np.abs(qy - (a + b * y)).max()),
          flush=True)
    assert err < 1e-5
    assert np.abs(T - T[:, :1]).max() < 1e-6 * np.abs(exact).max()


@pytest.mark.parametrize("precision", [0, 1])
def test_batch_with_fields_equals_single(precision):
    import torch
    import paper_1801_04577_amd as clbm
    cases = [field_case("cavity", 2), field_case("viscous", 3), (W.cavity(64, 80, Ra=1e4), {}),
             field_case("robin", 4)]
    probs = [p for p, _ in cases]
    b = clbm.Batch(probs, precision=precision)
    for i, (_, f) in enumerate(cases):
        b.init(i, **{k: torch.from_numpy(v) for k, v in f.items()})
    b.step(41)
    for i, (p, f) in enumerate(cases):
        s = run_gpu(p, 41, f, precision=precision)
        for x, y in zip(b.macros(i), s.macros()):
            assert torch.equal(x, y), (i, precision)
