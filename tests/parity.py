"""Helpers for GPU-vs-oracle parity tests (imported by the test modules only).

Error metric per field: max over nodes of |gpu - oracle| divided by max over nodes
of |oracle| (a pointwise relative error is undefined where the reference is zero,
e.g. u_y in a channel or T at an isothermal wall). The velocity is judged as the
vector (u_x, u_y): max |u_gpu - u_oracle| / max |u_oracle|. Density is judged by
max |rho_gpu - rho_oracle| (absolute; rho = 1 + O(Ma^2)).
"""
import numpy as np

import oracle


def f32(a):
    """Round an input field to float32 so the oracle and the GPU start from the same
    values (the GPU takes float32 fields)."""
    return None if a is None else np.asarray(a, dtype=np.float32)


def run_oracle(prob, steps, fields=None, nthreads=None):
    fields = fields or {}
    kw = {k: (None if v is None else np.asarray(v, np.float64)) for k, v in fields.items()}
    o = oracle.Sim(prob, nthreads=nthreads, **kw)
    o.step(steps)
    return o


def run_gpu(prob, steps, fields=None, precision=0, launch=None, graph=0):
    import torch
    import paper_1801_04577_amd as clbm
    fields = fields or {}
    s = clbm.Solver(prob, precision)
    if launch:
        s.set_launch(**launch)
    if graph:
        s.set_graph(graph)
    s.init(**{k: (None if v is None else torch.from_numpy(np.ascontiguousarray(v)))
              for k, v in fields.items()})
    s.step(steps)
    torch.cuda.synchronize()
    return s


def gpu_fields(s):
    return [t.cpu().numpy().astype(np.float64) for t in s.macros()]


def field_errors(o, s):
    ro, uxo, uyo, To = o.macros()
    rg, uxg, uyg, Tg = gpu_fields(s)
    umax = float(np.sqrt(uxo ** 2 + uyo ** 2).max())
    du = float(np.sqrt((uxg - uxo) ** 2 + (uyg - uyo) ** 2).max())
    Tmax = float(np.abs(To).max())
    dT = float(np.abs(Tg - To).max())
    return {
        "u": du / umax if umax > 0 else du,
        "T": dT / Tmax if Tmax > 0 else dT,
        "rho_abs": float(np.abs(rg - ro).max()),
        "u_abs": du, "T_abs": dT, "umax": umax, "Tmax": Tmax,
    }


def population_errors(o, s, T0):
    """Post-collision populations as deviations: f* - w and g* - T0/5."""
    fo, go = o.post_collision()
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    fo = np.moveaxis(fo - w, -1, 0)
    go = np.moveaxis(go - T0 / 5.0, -1, 0)
    fg, gg = [t.cpu().numpy().astype(np.float64) for t in s.populations()]
    ef = float(np.abs(fg - fo).max() / max(np.abs(fo).max(), 1e-300))
    eg = float(np.abs(gg - go).max() / max(np.abs(go).max(), 1e-300))
    return {"f": ef, "g": eg}
