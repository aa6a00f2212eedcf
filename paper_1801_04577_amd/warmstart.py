"""Learned warm start for the thermal cascaded LBM.

A convolutional encoder-decoder (the library's clbm_net_* kernels, BF16 MFMA) maps the
dimensionless description of a cavity problem (Ra, Pr, Q*, wall data; clbm_problem_encode
and clbm_net_features) to its steady fields on a fixed grid, in the problem's own units:
u/U, v/U with U = sqrt(g beta dT H), and (T - T0)/dT. The prediction is resampled onto
the lattice (clbm_resample_bilinear) and becomes the initial state of the solver
(clbm_batch_init, equilibrium at the predicted u and T). The cold start, T = T0 plus a
seeded perturbation, is the fallback and the reference: both runs go to the same residual
and their Nusselt numbers are compared.

This module orchestrates library calls; every array operation of the method runs in
the library's kernels.
"""
import time

import numpy as np

from . import (Batch, Net, features, nusselt, problem_code, resample)

CIN, COUT = 8, 3
WIDTHS = (32, 64, 128, 256)
# outputs are trained as (OUT_SCALE * u/U, OUT_SCALE * v/U, (T - T0)/dT) so all three are O(1)
OUT_SCALE = 5.0


def layer_shapes(cin=CIN, cout=COUT, widths=WIDTHS):
    """(out, in) channels of the 15 convolutions in the canonical order of include/clbm.h."""
    w1, w2, w3, w4 = widths
    return [(w1, cin), (w1, w1), (w2, w1), (w2, w2), (w3, w2), (w3, w3), (w4, w3), (w4, w4),
            (w3, w4 + w3), (w3, w3), (w2, w3 + w2), (w2, w2), (w1, w2 + w1), (w1, w1), (cout, w1)]


def init_params(seed, cin=CIN, cout=COUT, widths=WIDTHS):
    """He-uniform weights and zero biases as one canonical float32 vector (seeded)."""
    rng = np.random.default_rng(seed)
    parts = []
    for co, ci in layer_shapes(cin, cout, widths):
        lim = np.sqrt(6.0 / (ci * 9))
        parts.append(rng.uniform(-lim, lim, co * ci * 9))
        parts.append(np.zeros(co))
    return np.concatenate(parts).astype(np.float32)


def solve(probs, inits, max_steps, tol, K, launch=None):
    """Advance every problem from its initial fields to the residual tol (batched form).
    inits[i] is a dict of fields (rho, ux, uy, T; host arrays or device tensors) or None
    for the rest state. Returns the Batch, steps, status."""
    b = Batch(probs, launch=launch)
    for i, f in enumerate(inits):
        b.init(i, **(f or {}))
    steps, status = b.run(max_steps=max_steps, tol=tol, K=K)
    return b, steps, status


def targets(batch, probs, idx, H, W):
    """Normalised steady fields of instances idx resampled onto the H x W network grid,
    [len(idx)][3][H][W] on the device."""
    import torch
    out = torch.empty(len(idx), COUT, H, W, dtype=torch.float32, device="cuda")
    for j, i in enumerate(idx):
        c = problem_code(probs[i])
        rho, ux, uy, T = batch.macros(i)
        src = torch.stack([ux, uy, T])
        p = probs[i]
        out[j] = resample(src, H, W, scale=[OUT_SCALE / c.u_scale, OUT_SCALE / c.u_scale, 1.0 / c.t_scale],
                          shift=[0.0, 0.0, -p["T0"] / c.t_scale])
    return out


def inputs(probs, H, W):
    return features([problem_code(p) for p in probs], H, W)


def train(net, X, Y, steps, lr=1e-3, seed=0, log_every=0, lr_final=None):
    """Adam on minibatches of net's batch size drawn from (X, Y) (device tensors)."""
    import torch
    B = net.shape_in[0]
    n = X.shape[0]
    rng = np.random.default_rng(seed)
    losses = []
    order = np.array([], dtype=np.int64)
    for t in range(1, steps + 1):
        if order.size < B:
            order = np.concatenate([order, rng.permutation(n)])
        pick = torch.as_tensor(order[:B], device=X.device)
        order = order[B:]
        net.forward(X.index_select(0, pick))
        losses.append(net.backward(Y.index_select(0, pick)))
        rate = lr if lr_final is None else lr * (lr_final / lr) ** ((t - 1) / max(steps - 1, 1))
        net.adam(rate, t)
        if log_every and t % log_every == 0:
            print("train step %d loss %.4e" % (t, float(np.mean(losses[-log_every:]))), flush=True)
    return losses


def predict(net, X):
    """Network outputs for all rows of X, in batches of net's batch size."""
    import torch
    B = net.shape_in[0]
    n = X.shape[0]
    outs = []
    for k in range(0, n, B):
        chunk = X[k:k + B]
        if chunk.shape[0] < B:
            pad = chunk[:1].expand(B - chunk.shape[0], *chunk.shape[1:])
            chunk = torch.cat([chunk, pad])
        outs.append(net.forward(chunk)[:min(B, n - k)].clone())
    return torch.cat(outs)


def warm_inits(pred, probs):
    """Predicted normalised fields -> lattice fields (u_x, u_y, T) of each problem."""
    out = []
    for j, p in enumerate(probs):
        c = problem_code(p)
        f = resample(pred[j], p["ny"], p["nx"], scale=[c.u_scale / OUT_SCALE, c.u_scale / OUT_SCALE, c.t_scale],
                     shift=[0.0, 0.0, p["T0"]])
        out.append({"ux": f[0], "uy": f[1], "T": f[2]})
    return out


def nusselt_numbers(batch, probs):
    """Mean heat flux into the cold wall (x+) in units of k dT/H for every instance."""
    out = []
    for i, p in enumerate(probs):
        d = batch.diagnostics(i)
        c = problem_code(p)
        out.append(nusselt(d, 1, p["ny"], c.t_scale, into_wall=True))
    return out


def compare(net, probs, cold, grid, max_steps, tol, K, refine_tol=None):
    """Cold start (initial fields `cold`, one dict per problem) and network warm start of
    the same problems to the same residual: per-instance steps, status and Nusselt
    numbers of both. With refine_tol both runs are then continued to that residual and
    their Nusselt numbers reported again (they must reach the same steady state), with
    the steps each continuation took."""
    t0 = time.perf_counter()
    bc, steps_c, st_c = solve(probs, cold, max_steps, tol, K)
    nu_c = nusselt_numbers(bc, probs)
    t1 = time.perf_counter()
    X = inputs(probs, grid, grid)
    pred = predict(net, X)
    bw, steps_w, st_w = solve(probs, warm_inits(pred, probs), max_steps, tol, K)
    nu_w = nusselt_numbers(bw, probs)
    t2 = time.perf_counter()
    out = {"cold_steps": steps_c, "cold_status": st_c, "cold_nu": nu_c,
           "warm_steps": steps_w, "warm_status": st_w, "warm_nu": nu_w,
           "cold_seconds": t1 - t0, "warm_seconds": t2 - t1}
    if refine_tol is not None:
        for key, b in (("cold", bc), ("warm", bw)):
            steps, status = b.run(max_steps=max_steps, tol=refine_tol, K=K)
            out[key + "_refined_nu"] = nusselt_numbers(b, probs)
            out[key + "_refined_status"] = status
            out[key + "_refined_steps"] = steps
    return out
