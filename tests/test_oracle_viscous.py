"""Pins of the oracle's viscous-dissipation heat source (Sec. 3.2) on the CPU.

  * node level: populations built from the first-order Chapman-Enskog solution
    f = f_eq(rho, u) - (w_i rho / (c_s^2 s_nu)) (e_i e_i - c_s^2 I) : grad u carry a
    known velocity gradient; the source the oracle adds must be
    nu [(d_x u_y + d_y u_x)^2 + (d_x u_x - d_y u_y)^2] of that gradient;
  * Poiseuille channel: the steady temperature matches the closed form of Sec. 3.2
    and the global relative error falls at second order with the grid (the paper
    reports a fitted slope of 2.05);
  * the channel turned by 90 degrees gives the same profile (the d_x u_y term);
  * without flow the option changes nothing; with buoyancy it is refused.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W

CS2 = 1.0 / 3.0
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1])
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1])
WT = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)


def chapman_enskog_f(rho, ux, uy, G, s_nu):
    """f_eq of the oracle plus the first-order non-equilibrium part for the velocity
    gradient G[a][b] = d_a u_b (lattice units, dt = 1)."""
    f_eq, _ = oracle.equilibrium(rho, ux, uy, 0.0)
    e = np.stack([EX, EY], axis=1).astype(float)
    contr = np.einsum("ia,ib,ab->i", e, e, G) - CS2 * np.trace(G)
    return f_eq - WT * rho / (CS2 * s_nu) * contr


def dissipation_exact(nu, G):
    return nu * ((G[0, 1] + G[1, 0]) ** 2 + (G[0, 0] - G[1, 1]) ** 2)


@pytest.mark.parametrize("seed", range(6))
def test_source_from_chapman_enskog_populations(seed):
    rng = np.random.default_rng(seed)
    nu = [0.02, 0.05, 0.1, 0.3, 0.5, 0.01][seed]
    prob = W.problem(4, 4, nu, 0.1, [W.PERIODIC] * 4, viscous_heating=True)
    s_nu = oracle.rates(prob)[0]
    rho = 1.0 + 0.05 * rng.uniform(-1, 1)
    ux, uy = 0.05 * rng.uniform(-1, 1, 2)
    G = 1e-3 * rng.uniform(-1, 1, (2, 2))
    if seed == 0:
        G = np.array([[0.0, 2e-3], [0.0, 0.0]])  # pure shear d_x u_y
    if seed == 1:
        G = np.array([[1e-3, 0.0], [0.0, -1e-3]])  # pure extension
    f = chapman_enskog_f(rho, ux, uy, G, s_nu)
    g = np.zeros(5)
    _, _, (r, vx, vy, T) = oracle.collide(prob, f, g)
    assert abs(vx - ux) < 1e-15 and abs(vy - uy) < 1e-15
    # T = sum g + Q/2 with sum g = 0 (Eq. 25): the source is 2T.
    want = dissipation_exact(nu, G)
    assert abs(2.0 * T - want) <= 1e-10 * want


def test_source_needs_no_buoyancy():
    prob = W.cavity(16, Ra=1e4)
    prob["viscous_heating"] = True
    with pytest.raises(oracle.OracleError):
        oracle.Sim(prob)


def test_no_flow_no_extra_source():
    base = W.problem(6, 10, 0.1, 0.1, [W.PERIODIC, W.PERIODIC, W.dirichlet(0.0), W.dirichlet(1.0)],
                     Q=1e-3)
    T0 = W.noise_field(7, 6, 10, 0.1)
    a = oracle.Sim(base, T=T0)
    b = oracle.Sim(dict(base, viscous_heating=True), T=T0)
    a.step(200)
    b.step(200)
    for x, y in zip(a.macros(), b.macros()):
        assert np.array_equal(x, y)


def steady_channel(ny, transpose=False):
    prob = W.viscous_channel(ny, transpose=transpose)
    s = oracle.Sim(prob, nthreads=1)
    s.step(int(6 * ny * ny / prob["alpha"]))
    rho, ux, uy, T = s.macros()
    return (T[0, :] if transpose else T[:, 0]), (uy[0, :] if transpose else ux[:, 0])


def e2(a, b):
    return math.sqrt(float(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def test_poiseuille_second_order():
    errs = []
    for ny in (8, 16, 32):
        T, _ = steady_channel(ny)
        errs.append(e2(T, W.viscous_channel_exact(ny)))
    slopes = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    print("E2", errs, "slopes", slopes)
    assert errs[-1] < 2.5e-3
    assert all(1.9 < s < 2.2 for s in slopes)


def test_poiseuille_turned_channel():
    T1, u1 = steady_channel(16)
    T2, u2 = steady_channel(16, transpose=True)
    scale = float(np.max(np.abs(T1)))
    assert np.max(np.abs(T1 - T2)) < 1e-9 * scale
    assert np.max(np.abs(u1 - u2)) < 1e-9 * float(np.max(np.abs(u1)))


def couette_T_error(U, ny=16, Tc=0.0, Th=0.0, nu=0.1, alpha=0.1):
    """Thermal Couette flow with viscous heating: the uniform shear U/H dissipates
    nu U^2/H^2 everywhere, so the steady temperature is the conduction line plus the
    parabola nu U^2 y (H - y)/(2 alpha H^2) (a closed form of Eq. 1c with a uniform source)."""
    p = W.couette(nx=4, ny=ny, nu=nu, alpha=alpha, U=U, Tc=Tc, Th=Th)
    p["viscous_heating"] = True
    s = oracle.Sim(p, nthreads=1)
    s.step(int(8 * ny * ny / min(nu, alpha)))
    T = s.macros()[3][:, 0]
    y = np.arange(ny) + 0.5
    heat = nu * U * U / (2 * alpha * ny * ny) * y * (ny - y)
    Ta = Tc + (Th - Tc) * y / ny + heat
    return float(np.abs(T - Ta).max() / np.abs(heat).max())


def test_couette_viscous_heating_closed_form():
    e1 = couette_T_error(0.01)
    e2_ = couette_T_error(0.02)
    e_walls = couette_T_error(0.01, Tc=-0.001, Th=0.002)
    print("Couette heating errors", e1, e2_, e_walls)
    # The only departure is the O(Ma^2) compressibility error of the flow, so it is small
    # and grows as U^2.
    assert e1 < 2e-6 and e_walls < 2e-6
    assert 3.5 < e2_ / e1 < 4.5
