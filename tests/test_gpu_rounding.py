"""Unbiased rounding into storage, seen through the conserved quantities.

A fully periodic lattice in a uniform state stays uniform. Each collision adds exactly F
to the momentum density (Eq. 7 changes the central moments k10, k01 by the force) and Q
to the sum of the temperature populations (Eq. 23 changes the thermal k00 by Q), and the
streaming conserves both sums. The stored post-collision state after n steps therefore
carries momentum rho0 u0 + (n + 1) F and sum g = T_init + (n + 1) Q exactly (the initial
collision adds the first F and Q), and its mass is unchanged. The test compares the
sums after n steps with the same sums right after initialisation (whose equilibrium,
evaluated in FP32 from float32 fields, carries its own few-ulp offset), so the gain
must be n F and n Q.

Here F and Q are about 40 times smaller than half a unit in the last place of the stored
populations: rounding to nearest would return every population unchanged and the sums
would not grow at all. The unbiased rounding must reproduce the growth on average over
the lattice. The sums are formed in FP64 on the host from the exported populations; the
noise of the lattice mean is about ulp * sqrt(k n / (4 N)) for k rounded populations per
node, N nodes and n steps, 0.2% of the signal in FP32 and about 1.5% in FP16.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

N_SIDE, STEPS, U0, T_INIT = 512, 4000, 0.05, 0.3


def _run(precision, F, Q):
    import torch
    import paper_1801_04577_amd as clbm
    prob = W.problem(N_SIDE, N_SIDE, 0.1, 0.1, [W.PERIODIC] * 4, Fx=F, Q=Q)
    s = clbm.Solver(prob, precision)
    ux = torch.full((N_SIDE, N_SIDE), U0, dtype=torch.float32)
    T = torch.full((N_SIDE, N_SIDE), T_INIT, dtype=torch.float32)
    s.init(ux=ux, T=T)
    before = _sums(s)
    s.step(STEPS)
    after = _sums(s)
    return [b - a for a, b in zip(before, after)]


def _sums(s):
    """Lattice means of rho - 1, j_x, j_y and sum g - T0 (T0 = 0), in FP64."""
    f, g = (t.cpu().numpy().astype(np.float64) for t in s.populations())
    nodes = N_SIDE * N_SIDE
    mass = f.sum() / nodes
    jx = (f[1] - f[3] + f[5] - f[6] - f[7] + f[8]).sum() / nodes
    jy = (f[2] - f[4] + f[5] + f[6] - f[7] - f[8]).sum() / nodes
    return mass, jx, jy, g.sum() / nodes


@pytest.mark.parametrize("precision,inc,rtol,mass_tol", [(0, 1e-10, 0.02, 1e-8), (1, 1e-7, 0.08, 3e-5)])
def test_sub_ulp_force_and_source_accumulate(precision, inc, rtol, mass_tol):
    dmass, djx, djy, dsg = _run(precision, inc, inc)
    want = STEPS * inc
    print("precision %d: momentum gain %.6e, heat gain %.6e (exact %.6e), mass change %.2e, j_y change %.2e"
          % (precision, djx, dsg, want, dmass, djy), flush=True)
    assert abs(djx / want - 1.0) < rtol
    assert abs(dsg / want - 1.0) < rtol
    assert abs(dmass) < mass_tol
    assert abs(djy) < rtol * want
