"""clbm_diagnostics_noalloc against clbm_diagnostics, through the C ABI.

The allocation-free variant runs the same reduction kernels with their partial and final
sums in the library's fixed device array instead of the handle's workspace. Two handles
advanced identically hold bitwise equal states (the stored rounding is a deterministic
function of the node and its results), so the two entry points must return identical
diagnostics: residuals against the previous snapshot, mass, wall gradients, wall
temperatures, wall heat fluxes and the NaN count. The first lattice needs the full
reduction grid (more nodes than 1024 workgroups of 256 cover in one pass); the second,
smaller one then reuses the array, whose partials beyond its own grid still hold the
first lattice's values.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

FIELDS = ("step", "K", "res_u", "res_T", "mass", "sum_u2", "sum_du2", "sum_T2", "sum_dT2",
          "nan_count")
SIDE_FIELDS = ("dTdn", "T_wall", "wall_flux")


def _same(da, db):
    for f in FIELDS:
        assert getattr(da, f) == getattr(db, f), f
    for f in SIDE_FIELDS:
        assert list(getattr(da, f)) == list(getattr(db, f)), f


def _pair(prob, precision, rounds):
    import torch
    import paper_1801_04577_amd as clbm
    T = torch.from_numpy(W.cavity_initial_T(prob, seed=5).astype(np.float32))
    a, b = clbm.Solver(prob, precision), clbm.Solver(prob, precision)
    a.init(T=T)
    b.init(T=T)
    out = []
    for n in rounds:
        a.step(n)
        b.step(n)
        da, db = a.diagnostics(), b.diagnostics(noalloc=True)
        _same(da, db)
        out.append(db)
    return out


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_matches_workspace_diagnostics(precision):
    big = W.cavity(600, 500, Ra=1e5, Pr=0.71, Q=1e-5)       # 300 000 nodes: capped grid
    small = W.cavity(70, 40, Ra=1e4, Pr=0.71)               # 11 workgroups
    print("no-alloc diagnostics, precision %d: 600x500 then 70x40" % precision, flush=True)
    d_big = _pair(big, precision, [20, 30])
    d_small = _pair(small, precision, [10, 25])
    for d, n in ((d_big[-1], 600 * 500), (d_small[-1], 70 * 40)):
        assert d.nan_count == 0
        assert d.K > 0 and d.res_u > 0.0 and d.res_T > 0.0
        assert abs(d.mass - n) < 1e-3 * n
