"""Pins of the FP64 oracle against closed forms and the paper's stated results (CPU).

Citations refer to Fei & Luo, arXiv:1801.04577. Each test names the fact it pins
and why its tolerance holds:
  * Sec. 3.1: steady diffusion with a uniform source is reproduced exactly by the
    D2Q5 CLBM with half-way general bounce-back when lambda_2 follows Cui's rule
    (the paper's Fig. 2 minimum; round-off exact for quadratic profiles);
  * Sec. 3: the no-slip rule for s_3 makes body-force Poiseuille flow accurate;
  * Eq. (27)-(28) extrapolate quadratics exactly, so Neumann and Robin walls are
    exact in the same steady problem;
  * hydrodynamic limits: shear waves decay at nu k^2, temperature waves at alpha k^2
    and are advected at the fluid speed (Galilean invariance of central moments);
  * momentum and heat bookkeeping in a uniform periodic box is exact.
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def e2(a, b):
    """Global relative error of Sec. 3.1."""
    return math.sqrt(float(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def y_nodes(n):
    """Half-way walls: node j sits at distance j + 1/2 from the wall."""
    return np.arange(n) + 0.5


# --------------------------------------------------------------------------
# Sec. 3.1: time-independent diffusion with a heat source, L = 6
# --------------------------------------------------------------------------

def diffusion_problem(alpha, bottom, top, L=6, dT=1.0, **rates):
    Q = 2.0 * alpha * dT / L ** 2
    return W.problem(1, L, 0.1, alpha, [W.PERIODIC, W.PERIODIC, bottom, top], Q=Q, **rates)


def diffusion_exact(L=6, T0=0.0, dT=1.0):
    y = y_nodes(L)
    return T0 + dT * (y / L) * (2.0 - y / L)


def steady_T(prob, steps=20000):
    s = oracle.Sim(prob)
    s.step(steps)
    return s.macros()[3][:, 0], s


@pytest.mark.parametrize("alpha", [0.1, 1.0 / 3.0])
def test_diffusion_dirichlet_exact(alpha):
    T, _ = steady_T(diffusion_problem(alpha, W.dirichlet(0.0), W.dirichlet(1.0)))
    assert e2(T, diffusion_exact()) < 1e-12


@pytest.mark.parametrize("alpha", [0.1, 1.0 / 3.0])
def test_diffusion_neumann_top_exact(alpha):
    """T_a'(L) = 0, so an adiabatic top wall has the same solution."""
    T, _ = steady_T(diffusion_problem(alpha, W.dirichlet(0.0), W.adiabatic()))
    assert e2(T, diffusion_exact()) < 1e-12


@pytest.mark.parametrize("b1,b2", [(1.0, 0.5), (2.0, 3.0)])
def test_diffusion_robin_exact(b1, b2):
    """Robin data matched to T_a: bottom (outward -y) b3 = -2 dT b1/L + b2 T_0,
    top (outward +y) b3 = b2 T_L."""
    L, dT = 6, 1.0
    bottom = W.robin(b1, b2, -2.0 * dT * b1 / L + b2 * 0.0)
    top = W.robin(b1, b2, b2 * 1.0)
    T, s = steady_T(diffusion_problem(0.1, bottom, top))
    assert e2(T, diffusion_exact()) < 1e-12
    # Eq. (28) gives the exact wall values of the quadratic.
    Tw_b, d_b = s.wall_values(2)
    Tw_t, d_t = s.wall_values(3)
    assert Tw_b[0] == pytest.approx(0.0, abs=1e-12)
    assert Tw_t[0] == pytest.approx(1.0, abs=1e-12)
    assert d_b[0] == pytest.approx(-2.0 * dT / L, abs=1e-12)
    assert d_t[0] == pytest.approx(0.0, abs=1e-12)


@pytest.mark.parametrize("alpha,best", [(0.1, 0.75), (1.0 / 3.0, 4.0 / 3.0)])
def test_lambda2_sweep_minimum(alpha, best):
    """Fig. 2: over lambda_2 in [0.2, 1.8] the error E_2 is smallest at 3/4 (alpha = 1/10)
    and 4/3 (alpha = 1/3)."""
    grid = sorted(set(np.round(np.linspace(0.2, 1.8, 17), 12)) | {0.75, 4.0 / 3.0})
    errs = []
    for l2 in grid:
        T, _ = steady_T(diffusion_problem(alpha, W.dirichlet(0.0), W.dirichlet(1.0), lambda_2=l2),
                        steps=8000)
        errs.append(e2(T, diffusion_exact()))
    k = int(np.argmin(errs))
    assert grid[k] == pytest.approx(best, abs=1e-12)
    assert errs[k] < 1e-12
    assert sorted(errs)[1] > 1e-5


# --------------------------------------------------------------------------
# Body-force channel (Sec. 3.2 flow field, Sec. 3 no-slip rule)
# --------------------------------------------------------------------------

def test_channel_steady_state():
    H, nu, gx, Q = 32, 0.05, 1e-6, 1e-4
    prob = W.channel(nx=1, ny=H, nu=nu, gx=gx, Q=Q)
    s = oracle.Sim(prob)
    s.step(150000)
    rho, ux, uy, T = s.macros()
    y = y_nodes(H)
    u_a = gx * y * (H - y) / (2 * nu)
    T_a = Q * y * (H - y) / (2 * prob["alpha"])
    # Temperature: exact steady state (the quadratic is reproduced to round-off).
    assert e2(T[:, 0], T_a) < 1e-11
    # Velocity: the no-slip rule makes it accurate; the residual is the O(Ma^2)
    # density variation of the weakly compressible scheme.
    assert e2(ux[:, 0], u_a) < 1e-6
    assert np.max(np.abs(uy)) < 1e-13
    # Control run: s_3 = s_nu gives a visible slip error.
    s_nu = oracle.rates(prob)[0]
    c = oracle.Sim(dict(prob, s_3=s_nu))
    c.step(150000)
    assert e2(c.macros()[1][:, 0], u_a) > 1e-4


def test_channel_transposed():
    """Swapping x and y (walls in x, force along y) transposes the solution exactly."""
    a = oracle.Sim(W.problem(3, 10, 0.07, 0.05, [W.PERIODIC] * 2 + [W.dirichlet(0.2), W.dirichlet(-0.1)],
                             Fx=2e-5, Q=3e-4, g_beta=0.0))
    b = oracle.Sim(W.problem(10, 3, 0.07, 0.05, [W.dirichlet(0.2), W.dirichlet(-0.1)] + [W.PERIODIC] * 2,
                             Fy=2e-5, Q=3e-4, g_beta=0.0))
    a.step(400)
    b.step(400)
    ra, uxa, uya, Ta = a.macros()
    rb, uxb, uyb, Tb = b.macros()
    # Equal up to the order of floating-point operations.
    scale = np.max(np.abs(uxa))
    np.testing.assert_allclose(uxa, uyb.T, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(uya, uxb.T, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(Ta, Tb.T, rtol=0, atol=1e-14)


def channel_series(y, t, H, g, nu, nterms=400):
    """Start-up of body-force channel flow from rest (continuum):
    u = g y (H - y)/(2 nu) - sum_{n odd} 4 g H^2/(nu pi^3 n^3) sin(n pi y/H) e^{-nu n^2 pi^2 t/H^2}."""
    u = g * y * (H - y) / (2 * nu)
    for n in range(1, 2 * nterms, 2):
        u -= 4 * g * H ** 2 / (nu * math.pi ** 3 * n ** 3) * np.sin(n * math.pi * y / H) \
            * math.exp(-nu * n * n * math.pi ** 2 * t / H ** 2)
    return u


def test_channel_transient_10000_steps():
    """64x32 channel after 10 000 steps against the continuum start-up series, for u
    (g_x, nu) and T (Q, alpha). The lattice solution differs by the lattice dispersion of
    the decaying modes and by the half-step force and source in the initial state
    (u(0) = F/2, T(0) = Q/2); both are below 1e-3 of the field maximum here."""
    H, nu, gx, Q = 32, 0.05, 1e-6, 1e-4
    prob = W.channel(nx=2, ny=H, nu=nu, gx=gx, Q=Q)
    s = oracle.Sim(prob)
    s.step(10000)
    rho, ux, uy, T = s.macros()
    y = y_nodes(H)
    u_a = channel_series(y, 10000.0, H, gx, nu)
    T_a = channel_series(y, 10000.0, H, Q, prob["alpha"])
    assert np.max(np.abs(ux[:, 0] - u_a)) < 1e-3 * np.max(u_a)
    assert np.max(np.abs(T[:, 0] - T_a)) < 1e-3 * np.max(T_a)


# --------------------------------------------------------------------------
# Thermal Couette flow (moving top wall)
# --------------------------------------------------------------------------

def couette_run(U, Q, H=16, Tc=0.0, Th=1.0, alpha=0.1):
    prob = W.couette(nx=2, ny=H, nu=0.1, alpha=alpha, U=U, Tc=Tc, Th=Th, Q=Q)
    s = oracle.Sim(prob)
    s.step(40000)
    return s.macros()


@pytest.mark.parametrize("Q", [0.0, 2e-4])
def test_thermal_couette(Q):
    """Linear velocity between a resting and a moving wall; linear temperature between
    the wall temperatures plus Q y (H - y)/(2 alpha) with a uniform source. Temperature
    is exact. The velocity carries the O(Ma^2) density variation of the weakly
    compressible scheme: its error must scale as U^2 (ratio 100 for U 0.01 -> 0.001) and
    stay far below Ma^2 = 3 U^2."""
    H, Tc, Th, alpha = 16, 0.0, 1.0, 0.1
    y = y_nodes(H)
    errs = []
    for U in (0.01, 0.001):
        rho, ux, uy, T = couette_run(U, Q, H, Tc, Th, alpha)
        T_a = Tc + (Th - Tc) * y / H + Q * y * (H - y) / (2 * alpha)
        assert e2(T[:, 0], T_a) < 1e-11
        assert np.max(np.abs(uy)) < 1e-14
        errs.append(np.max(np.abs(ux[:, 0] - U * y / H)) / U)
    assert errs[0] < 1e-2 * 3 * 0.01 ** 2
    assert errs[0] / errs[1] == pytest.approx(100.0, rel=0.05)


# --------------------------------------------------------------------------
# Hydrodynamic limits in a periodic box
# --------------------------------------------------------------------------

def _proj(field, mode):
    return float(np.sum(field * mode) / np.sum(mode * mode))


@pytest.mark.parametrize("direction", ["axis", "diagonal"])
def test_shear_wave_decay(direction):
    """A shear wave decays as exp(-nu |k|^2 t). The diagonal wave shears k20 - k02
    (the s+/s- block of Eq. 8); the axis wave shears k11. Lattice dispersion at
    |k| dx = 2 pi/32 is well below 1%."""
    N, nu, A = 32, 0.05, 1e-3
    prob = W.problem(N, N, nu, 0.05, [W.PERIODIC] * 4)
    y, x = np.mgrid[0:N, 0:N].astype(float)
    k = 2 * math.pi / N
    if direction == "axis":
        mode, k2 = np.sin(k * y), k * k
        s = oracle.Sim(prob, ux=A * mode)
    else:
        mode, k2 = np.sin(k * (x + y)), 2 * k * k
        s = oracle.Sim(prob, ux=A * mode / math.sqrt(2), uy=-A * mode / math.sqrt(2))
    s.step(100)
    a1 = _proj(s.macros()[1], mode)
    s.step(1000)
    a2 = _proj(s.macros()[1], mode)
    nu_eff = math.log(a1 / a2) / (1000 * k2)
    assert nu_eff == pytest.approx(nu, rel=1e-2)


@pytest.mark.parametrize("U", [0.05, -0.08])
def test_temperature_wave_advection(U):
    """T = A sin(k(x - U t)) exp(-alpha k^2 t) in a uniform flow: phase speed U and decay
    alpha k^2 (to 1%; the central-moment shift of Eq. 17 makes this frame independent)."""
    N, alpha = 32, 0.05
    prob = W.problem(N, N, 0.05, alpha, [W.PERIODIC] * 4)
    y, x = np.mgrid[0:N, 0:N].astype(float)
    k = 2 * math.pi / N
    s = oracle.Sim(prob, ux=U, uy=0.03, T=1e-2 * np.sin(k * x))
    ph, amp = [], []
    for _ in range(12):
        s.step(50)
        T = s.macros()[3]
        a, b = _proj(T, np.sin(k * x)), _proj(T, np.cos(k * x))
        ph.append(math.atan2(-b, a))
        amp.append(math.hypot(a, b))
    ph = np.unwrap(ph)
    assert (ph[-1] - ph[1]) / (k * 500) == pytest.approx(U, rel=1e-2)
    assert math.log(amp[1] / amp[-1]) / (500 * k * k) == pytest.approx(alpha, rel=1e-2)


def test_uniform_box_bookkeeping():
    """Uniform periodic box: every node sees the same force F(t) = F_v + g beta (T(t) - T0)
    with T(t) = T_init + Q/2 + Q t (Eq. 25), and sum_i f_i e_i gains F(t) each step, so
    u(t) = (rho u_init + sum_{s<t} F(s) + F(t)/2)/rho exactly."""
    gb, T0, Q, Fx, Fy = 1e-3, 0.1, 2e-4, 3e-6, -1e-6
    prob = W.problem(3, 3, 0.1, 0.07, [W.PERIODIC] * 4, g_beta=gb, T0=T0, Fx=Fx, Fy=Fy, Q=Q)
    rho0, ux0, uy0, Ti = 1.02, 0.01, -0.02, 0.3
    s = oracle.Sim(prob, rho=rho0, ux=ux0, uy=uy0, T=Ti)
    jx, jy = rho0 * ux0, rho0 * uy0
    for t in range(60):
        rho, ux, uy, T = s.macros()
        Tt = Ti + Q / 2 + Q * t
        Fyt = Fy + gb * (Tt - T0)
        np.testing.assert_allclose(T, Tt, rtol=0, atol=1e-14)
        np.testing.assert_allclose(rho, rho0, rtol=0, atol=1e-14)
        np.testing.assert_allclose(ux, (jx + Fx / 2) / rho0, rtol=0, atol=1e-15)
        np.testing.assert_allclose(uy, (jy + Fyt / 2) / rho0, rtol=0, atol=1e-15)
        jx += Fx
        jy += Fyt
        s.step(1)


def test_uniform_state_is_stationary():
    prob = W.problem(5, 4, 0.1, 0.07, [W.PERIODIC] * 4)
    s = oracle.Sim(prob, rho=1.01, ux=0.04, uy=-0.03, T=0.2)
    f0, g0 = s.state()
    s.step(50)
    f1, g1 = s.state()
    np.testing.assert_allclose(f1, f0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(g1, g0, rtol=0, atol=1e-15)


@pytest.mark.parametrize("walls", ["dirichlet", "adiabatic", "mixed"])
def test_walled_rest_state_is_stationary(walls):
    """Bounce-back and general bounce-back map the rest equilibrium at the wall
    temperature onto itself."""
    Tw = 0.3
    side = {"dirichlet": [W.dirichlet(Tw)] * 4, "adiabatic": [W.adiabatic()] * 4,
            "mixed": [W.dirichlet(Tw), W.dirichlet(Tw), W.adiabatic(), W.adiabatic()]}[walls]
    prob = W.problem(6, 5, 0.1, 0.07, side)
    s = oracle.Sim(prob, T=Tw)
    f0, g0 = s.state()
    s.step(50)
    f1, g1 = s.state()
    np.testing.assert_allclose(f1, f0, rtol=0, atol=1e-15)
    np.testing.assert_allclose(g1, g0, rtol=0, atol=1e-15)


def test_mass_conservation_cavity():
    """Half-way bounce-back returns every population that hits a wall, so total mass is
    constant (to round-off over 2000 steps)."""
    prob = W.cavity(24, Ra=1e5, Pr=0.71)
    s = oracle.Sim(prob, T=W.cavity_initial_T(prob, seed=3))
    m0 = s.macros()[0].sum()
    s.step(2000)
    m1 = s.macros()[0].sum()
    assert abs(m1 - m0) / m0 < 1e-13


def test_cavity_circulation_direction():
    """Hot wall at x-, cold at x+, gravity along -y: fluid rises along the hot wall
    (Eq. 2 with g pointing to -y gives F_y = +g beta (T - T0))."""
    prob = W.cavity(20, Ra=1e4, Pr=0.71)
    s = oracle.Sim(prob)
    s.step(3000)
    rho, ux, uy, T = s.macros()
    assert uy[10, 2] > 0 and uy[10, -3] < 0
    assert ux[-3, 10] > 0 and ux[2, 10] < 0
