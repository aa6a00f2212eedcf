"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

This module holds problem descriptions and seeded random inputs only: no
lattice Boltzmann arithmetic. Both the FP64 oracle and the GPU library take
the same plain-dict problem and the same host arrays from here.

Problem dict keys: ``nx, ny, nu, alpha, g_beta, T0, Fx, Fy, Q``, ``viscous_heating``
(add the local viscous dissipation to Q, Sec. 3.2) and ``sides``
(four dicts, order x-, x+, y-, y+: ``kind`` "periodic"/"wall", ``u_wall``,
Robin data ``b1, b2, b3`` of ``b1 dT/dn + b2 T = b3`` with n the outward
normal). Optional rate overrides ``s_b, s_4, s_3, lambda_0, lambda_2``.

The natural-convection parameters follow the problem statement of Sec. 3.3 of
Fei & Luo (arXiv:1801.04577): Ra = g beta dT H^3/(nu alpha), Pr = nu/alpha and
a characteristic velocity U = sqrt(g beta dT H), so nu = U H sqrt(Pr/Ra),
alpha = nu/Pr and g beta = U^2/(H dT).
"""
import math

import numpy as np

PERIODIC = {"kind": "periodic"}


def dirichlet(T, u_wall=0.0):
    """Wall held at temperature T: b1 = 0, b2 = 1, b3 = T."""
    return {"kind": "wall", "b1": 0.0, "b2": 1.0, "b3": float(T), "u_wall": float(u_wall)}


def adiabatic(u_wall=0.0):
    """Insulated wall: b1 = 1, b2 = 0, b3 = 0."""
    return {"kind": "wall", "b1": 1.0, "b2": 0.0, "b3": 0.0, "u_wall": float(u_wall)}


def robin(b1, b2, b3, u_wall=0.0):
    return {"kind": "wall", "b1": float(b1), "b2": float(b2), "b3": float(b3),
            "u_wall": float(u_wall)}


def problem(nx, ny, nu, alpha, sides, g_beta=0.0, T0=0.0, Fx=0.0, Fy=0.0, Q=0.0,
            viscous_heating=False, **rates):
    p = {"nx": int(nx), "ny": int(ny), "nu": float(nu), "alpha": float(alpha),
         "g_beta": float(g_beta), "T0": float(T0), "Fx": float(Fx), "Fy": float(Fy),
         "Q": float(Q), "viscous_heating": bool(viscous_heating),
         "sides": [dict(s) for s in sides]}
    for k, v in rates.items():
        assert k in ("s_b", "s_4", "s_3", "lambda_0", "lambda_2"), k
        p[k] = v
    return p


# --------------------------------------------------------------------------
# Counter-based noise: splitmix64 of (seed, node index)
# --------------------------------------------------------------------------

_M64 = np.uint64(0xFFFFFFFFFFFFFFFF)


def splitmix64(x):
    """SplitMix64 output function (Steele, Lea, Flood 2014) on uint64 arrays."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed, n):
    """n uniforms in [0, 1) from splitmix64(seed * 2^32 + k), k = 0..n-1."""
    with np.errstate(over="ignore"):
        ctr = (np.uint64(seed) << np.uint64(32)) + np.arange(n, dtype=np.uint64)
    z = splitmix64(ctr)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def noise_field(seed, nx, ny, amplitude):
    """amplitude * U(-1, 1) per node, [ny][nx] row-major, node index y*nx + x."""
    return noise_rows(seed, nx, 0, ny, amplitude)


def noise_rows(seed, nx, y0, y1, amplitude):
    """Rows y0..y1-1 of noise_field(seed, nx, ny, amplitude) for any ny >= y1 (the
    counter of node (x, y) is y*nx + x, so a strip is generated on its own)."""
    with np.errstate(over="ignore"):
        ctr = ((np.uint64(seed) << np.uint64(32)) + np.uint64(y0 * nx)
               + np.arange((y1 - y0) * nx, dtype=np.uint64))
    z = splitmix64(ctr)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return amplitude * (2.0 * u.reshape(y1 - y0, nx) - 1.0)


# --------------------------------------------------------------------------
# Named problems
# --------------------------------------------------------------------------

def channel(nx=64, ny=32, nu=0.05, Pr=0.71, gx=1e-6, Q=1e-4, Tw=0.0):
    """Body-force channel: periodic in x, no-slip walls in y at temperature Tw,
    uniform heat source Q, no buoyancy. 64x32 at nu = 0.05, gx = 1e-6, Q = 1e-4 is the
    small FP32-vs-FP64 parity workload."""
    return problem(nx, ny, nu, nu / Pr, [PERIODIC, PERIODIC, dirichlet(Tw), dirichlet(Tw)],
                   Fx=gx, Q=Q)


def cavity_params(H, Ra, Pr, U=0.1, dT=1.0):
    nu = U * H * math.sqrt(Pr / Ra)
    return nu, nu / Pr, U * U / (H * dT)


def cavity(nx, ny=None, Ra=1e5, Pr=0.71, Q=0.0, Th=0.5, Tc=-0.5, U=0.1):
    """Differentially heated cavity (Sec. 3.3): hot wall at x-, cold wall at x+,
    adiabatic bottom and top, gravity along -y, H = ny."""
    ny = nx if ny is None else ny
    nu, alpha, gb = cavity_params(ny, Ra, Pr, U, Th - Tc)
    return problem(nx, ny, nu, alpha, [dirichlet(Th), dirichlet(Tc), adiabatic(), adiabatic()],
                   g_beta=gb, T0=0.5 * (Th + Tc), Q=Q)


def cavity_initial_T(prob, seed=12345, amplitude=1e-4):
    return prob["T0"] + noise_field(seed, prob["nx"], prob["ny"], amplitude)


def couette(nx=4, ny=16, nu=0.1, alpha=0.1, U=0.01, Tc=0.0, Th=1.0, Q=0.0):
    """Bottom wall at rest (Tc), top wall moving with U along x (Th); periodic in x."""
    return problem(nx, ny, nu, alpha, [PERIODIC, PERIODIC, dirichlet(Tc), dirichlet(Th, U)], Q=Q)


def diffusion_source(alpha, bottom, top, L=6, dT=1.0, **rates):
    """Steady diffusion with a uniform heat source between two walls (Sec. 3.1): one
    periodic column of L nodes, Q = 2 alpha dT / L^2, so that with T = 0 at the bottom
    and T = dT at the top the steady profile is T = dT (y/L)(2 - y/L)."""
    Q = 2.0 * alpha * dT / L ** 2
    return problem(1, L, 0.1, alpha, [PERIODIC, PERIODIC, bottom, top], Q=Q, **rates)


def diffusion_source_exact(L=6, T0=0.0, dT=1.0):
    y = np.arange(L) + 0.5
    return T0 + dT * (y / L) * (2.0 - y / L)


def viscous_channel(ny, nx=4, nu=0.1, alpha=0.1, umax=0.01, Tw=0.0, transpose=False):
    """Body-force Poiseuille flow with viscous heating (Sec. 3.2): walls at Tw, no
    buoyancy, half-width h = ny/2, force chosen so that the centre speed is umax.
    transpose=True turns the channel by 90 degrees (flow along y, walls at x = 0, nx)."""
    h = ny / 2.0
    F = 2.0 * nu * umax / (h * h)
    walls = [dirichlet(Tw), dirichlet(Tw)]
    if transpose:
        p = problem(ny, nx, nu, alpha, walls + [PERIODIC, PERIODIC], Fy=F)
    else:
        p = problem(nx, ny, nu, alpha, [PERIODIC, PERIODIC] + walls, Fx=F)
    p["viscous_heating"] = True
    return p


def viscous_channel_exact(ny, nu=0.1, alpha=0.1, umax=0.01, Tw=0.0):
    """Steady temperature of the viscous-heating channel at the node centres
    (Sec. 3.2): Tw + (h^2 F/2)^2 (1 - (y/h)^4)/(3 nu alpha), y from the centre line."""
    h = ny / 2.0
    F = 2.0 * nu * umax / (h * h)
    y = np.arange(ny) + 0.5 - h
    return Tw + (h * h * F / 2.0) ** 2 * (1.0 - (y / h) ** 4) / (3.0 * nu * alpha)


# Sizes of the workloads named in the benchmark and the tests.
CHANNEL_64x32 = dict(nx=64, ny=32)
CAVITY_256 = dict(n=256, Ra=1e5, Pr=0.71)
CAVITY_4096 = dict(n=4096, Ra=1e6, Pr=0.71, Q=5e-6)
CAVITY_512_STANDIN = dict(n=512, Ra=1e6, Pr=0.71, Q=5e-6)


def large_cavity(n=4096):
    return cavity(n, Ra=1e6, Pr=0.71, Q=5e-6)


# --------------------------------------------------------------------------
# Batched sweep: many cavities of uneven size and parameters
# --------------------------------------------------------------------------

SWEEP_SIDES = list(range(64, 513, 32))


def sweep(count=256, seed=2024, sides=SWEEP_SIDES, ra_range=(1e3, 1e6), pr_range=(0.7, 7.0),
          q_range=(0.0, 1e-4), U=0.1, tau_max=2.0):
    """Seeded list of (problem, seed) pairs. Sides a <= b <= 2a drawn from `sides`,
    orientation by coin flip; Ra log-uniform, Pr and Q uniform. Where the U = 0.1 rule
    would give a relaxation time above tau_max the characteristic velocity is lowered
    so that nu = (tau_max - 1/2)/3. meta["under_resolved"] marks the instances whose
    shear relaxation time tau_nu = 3 nu + 1/2 is below 0.52 (thin boundary layers at
    high Ra on small grids; flagged, not changed)."""
    u = uniform01(seed, count * 8).reshape(count, 8)
    pairs = [(a, b) for a in sides for b in sides if a <= b <= 2 * a]
    out = []
    for k in range(count):
        a, b = pairs[min(int(u[k, 0] * len(pairs)), len(pairs) - 1)]
        nx, ny = (a, b) if u[k, 1] < 0.5 else (b, a)
        Ra = 10.0 ** (math.log10(ra_range[0]) + u[k, 2] * (math.log10(ra_range[1]) - math.log10(ra_range[0])))
        Pr = pr_range[0] + u[k, 3] * (pr_range[1] - pr_range[0])
        Q = q_range[0] + u[k, 4] * (q_range[1] - q_range[0])
        Uk = U
        nu = Uk * ny * math.sqrt(Pr / Ra)
        nu_max = (tau_max - 0.5) / 3.0
        if nu > nu_max:
            Uk = U * nu_max / nu
        prob = cavity(nx, ny, Ra=Ra, Pr=Pr, Q=Q, U=Uk)
        tau_nu = 3.0 * prob["nu"] + 0.5
        prob["meta"] = {"Ra": Ra, "Pr": Pr, "U": Uk, "tau_nu": tau_nu, "under_resolved": tau_nu < 0.52}
        out.append((prob, int(seed * 1000 + k)))
    return out


# --------------------------------------------------------------------------
# Warm-start sets: cavities described by (Ra, Pr, Q*) with Q* = Q H^2/(alpha dT)
# --------------------------------------------------------------------------

def warmstart_problems(count, seed, sides=(64,), square=True, ra_range=(1e3, 1e6),
                       pr_range=(0.7, 7.0), qstar_range=(0.0, 4.0), U=0.1, tau_max=2.0):
    """Seeded cavities for the learned warm start: Ra log-uniform, Pr uniform, the
    source given through Q* uniform (so that the internal heating stays comparable to
    the wall-driven flow at every size), sides drawn from `sides` (square or a <= b <= 2a),
    the velocity scale lowered where U would give tau_nu > tau_max. Returns a list of
    (problem, noise_seed)."""
    u = uniform01(seed, count * 8).reshape(count, 8)
    out = []
    for k in range(count):
        if square:
            nx = ny = int(sides[min(int(u[k, 0] * len(sides)), len(sides) - 1)])
        else:
            pairs = [(a, b) for a in sides for b in sides if a <= b <= 2 * a]
            a, b = pairs[min(int(u[k, 0] * len(pairs)), len(pairs) - 1)]
            nx, ny = (a, b) if u[k, 1] < 0.5 else (b, a)
        Ra = 10.0 ** (math.log10(ra_range[0]) + u[k, 2] * (math.log10(ra_range[1]) - math.log10(ra_range[0])))
        Pr = pr_range[0] + u[k, 3] * (pr_range[1] - pr_range[0])
        qs = qstar_range[0] + u[k, 4] * (qstar_range[1] - qstar_range[0])
        Uk = U
        nu = Uk * ny * math.sqrt(Pr / Ra)
        nu_max = (tau_max - 0.5) / 3.0
        if nu > nu_max:
            Uk = U * nu_max / nu
        nu, alpha, _ = cavity_params(ny, Ra, Pr, Uk, 1.0)
        prob = cavity(nx, ny, Ra=Ra, Pr=Pr, Q=qs * alpha / (ny * ny), U=Uk)
        prob["meta"] = {"Ra": Ra, "Pr": Pr, "Qstar": qs, "U": Uk}
        out.append((prob, int(seed * 1000 + k)))
    return out
