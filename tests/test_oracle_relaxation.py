"""Every relaxation rate of the oracle's collision, pinned mode by mode (CPU only).

Fei & Luo (arXiv:1801.04577), Sec. 2.1 Eq. (7)-(10) and Sec. 2.2-2.3 Eq. (18)-(24): in
central-moment space one collision takes each relaxed moment's departure from its
equilibrium, multiplies it by one minus its rate and adds the force or source term. The
relaxation matrix S of Eq. (8) couples k20 and k02 through the block [[s+, s-], [s-, s+]]
with s+- = (s_b +- s_nu)/2, so the trace k20 + k02 relaxes at s_b and the difference
k20 - k02 at s_nu; k11 relaxes at s_nu, k21 and k12 at s_3, k22 at s_4. The thermal
matrix S_T relaxes the first moments at lambda_1 and the second at lambda_2.

The moments here are taken by brute force from the populations the oracle returns
(sum_i f_i (e_ix - u_x)^m (e_iy - u_y)^n over the velocities of Eq. 3), not through the
oracle's matrices. A last test pins the bulk rate s_b at the level of the hydrodynamics:
a standing sound wave decays at k^2 (nu + nu_b)/2 with nu_b = c_s^2 (1/s_b - 1/2).
"""
import math

import numpy as np
import pytest
from scipy.optimize import curve_fit

import oracle
import workloads as W

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
CS2, CT2 = 1.0 / 3.0, 2.0 / 5.0


def cm(p, ux, uy, m, n):
    """Central moment of order (m, n) of populations p over the first len(p) velocities."""
    q = len(p)
    return float(np.sum(p * (EX[:q] - ux) ** m * (EY[:q] - uy) ** n))


def flow_modes(f, ux, uy):
    rho = float(f.sum())
    k = {mn: cm(f, ux, uy, *mn) for mn in [(2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]}
    return {
        "trace": k[(2, 0)] + k[(0, 2)] - 2.0 * rho * CS2,  # departure from Eq. (9)
        "diff": k[(2, 0)] - k[(0, 2)],
        "k11": k[(1, 1)],
        "k21": k[(2, 1)],
        "k12": k[(1, 2)],
        "k22": k[(2, 2)] - rho * CS2 * CS2,
    }


def thermal_modes(g, ux, uy, T):
    return {
        "t10": cm(g, ux, uy, 1, 0),
        "t01": cm(g, ux, uy, 0, 1),
        "t20": cm(g, ux, uy, 2, 0) - CT2 * T,  # departure from Eq. (19)
        "t02": cm(g, ux, uy, 0, 2) - CT2 * T,
    }


def random_state(rng, zero_velocity):
    """Populations of a node: the rest weights scaled by rho plus a random departure; with
    zero_velocity the departure carries no momentum, so u = 0 when F = 0."""
    w = np.array([4 / 9] + [1 / 9] * 4 + [1 / 36] * 4)
    rho, T = rng.uniform(0.9, 1.1), rng.uniform(-0.5, 0.5)
    f = rho * w + rng.uniform(-0.02, 0.02, 9)
    g = T / 5 + rng.uniform(-0.02, 0.02, 5)
    if zero_velocity:
        jx, jy = f @ EX, f @ EY
        f[1] -= jx / 2
        f[3] += jx / 2
        f[2] -= jy / 2
        f[4] += jy / 2
        tx, ty = g @ EX[:5], g @ EY[:5]
        g[1] -= tx / 2
        g[3] += tx / 2
        g[2] -= ty / 2
        g[4] += ty / 2
    return f, g


def rate_problem(rng, forced, **fixed):
    kw = dict(s_b=rng.uniform(0.3, 1.9), s_4=rng.uniform(0.3, 1.9), s_3=rng.uniform(0.3, 1.9),
              lambda_2=rng.uniform(0.3, 1.9))
    kw.update(fixed)
    kw = {k: v for k, v in kw.items() if v is not None}
    if forced:
        kw.update(g_beta=rng.uniform(0, 1e-2), T0=rng.uniform(-0.2, 0.2),
                  Fx=rng.uniform(-1e-3, 1e-3), Fy=rng.uniform(-1e-3, 1e-3),
                  Q=rng.uniform(-1e-2, 1e-2))
    return W.problem(3, 3, rng.uniform(0.01, 0.3), rng.uniform(0.01, 0.3), [W.PERIODIC] * 4,
                     **kw)


def paper_rates(prob):
    """The rates a problem asks for, from the paper rather than from the oracle: s_nu from
    nu = c_s^2 (1/s_nu - 1/2) (Sec. 2.1), lambda_1 from alpha = c_T^2 (1/lambda_1 - 1/2)
    (Sec. 2.2), s_3 by the no-slip rule of Sec. 3 and lambda_2 by the rule of Sec. 3.1
    unless given, and s_b = s_4 = 1 unless given (the paper leaves them open)."""
    s_nu = 1.0 / (prob["nu"] / CS2 + 0.5)
    l1 = 1.0 / (prob["alpha"] / CT2 + 0.5)
    given = lambda k, default: default if prob.get(k) is None else prob[k]
    return (s_nu, given("s_b", 1.0), given("s_3", (16 - 8 * s_nu) / (8 - s_nu)),
            given("s_4", 1.0), l1, given("lambda_2", 12 * (l1 - 2) / (l1 - 12)))


def expected_factors(prob):
    """(1 - rate) per mode."""
    s_nu, s_b, s_3, s_4, l1, l2 = paper_rates(prob)
    return ({"trace": 1 - s_b, "diff": 1 - s_nu, "k11": 1 - s_nu, "k21": 1 - s_3,
             "k12": 1 - s_3, "k22": 1 - s_4},
            {"t10": 1 - l1, "t01": 1 - l1, "t20": 1 - l2, "t02": 1 - l2},
            (s_3, l2))


def check_relaxation(prob, f, g):
    fp, gp, (rho_o, ux_o, uy_o, T_o) = oracle.collide(prob, f, g)
    # Eq. (25), (2), (12): the macroscopic values the collision is taken at
    Q = prob["Q"]
    T = float(g.sum()) + 0.5 * Q
    Fx = prob["Fx"]
    Fy = prob["Fy"] + prob["g_beta"] * (T - prob["T0"])
    rho = float(f.sum())
    ux, uy = (f @ EX + 0.5 * Fx) / rho, (f @ EY + 0.5 * Fy) / rho
    assert (rho_o, ux_o, uy_o, T_o) == pytest.approx((rho, ux, uy, T), abs=1e-15)
    ff, ft, (s_3, l2) = expected_factors(prob)
    pre, post = flow_modes(f, ux, uy), flow_modes(fp, ux, uy)
    # Eq. (10): the force enters the third-order central moments through (I - S/2) C
    force = {"k21": (1 - 0.5 * s_3) * CS2 * Fy, "k12": (1 - 0.5 * s_3) * CS2 * Fx}
    for k, fac in ff.items():
        want = fac * pre[k] + force.get(k, 0.0)
        assert post[k] == pytest.approx(want, abs=2e-15), (k, post[k], want)
    # conserved and forced moments: rho unchanged, momentum gains F (first central = +F/2)
    assert float(fp.sum()) == pytest.approx(rho, abs=1e-15)
    assert cm(fp, ux, uy, 1, 0) == pytest.approx(0.5 * Fx, abs=1e-15)
    assert cm(fp, ux, uy, 0, 1) == pytest.approx(0.5 * Fy, abs=1e-15)
    # Eq. (23)-(24): the source enters the thermal second moments through (I - S_T/2) R
    tpre, tpost = thermal_modes(g, ux, uy, T), thermal_modes(gp, ux, uy, T)
    src = {"t20": (1 - 0.5 * l2) * CT2 * Q, "t02": (1 - 0.5 * l2) * CT2 * Q}
    for k, fac in ft.items():
        want = fac * tpre[k] + src.get(k, 0.0)
        assert tpost[k] == pytest.approx(want, abs=2e-15), (k, tpost[k], want)
    assert float(gp.sum()) == pytest.approx(float(g.sum()) + Q, abs=1e-15)


@pytest.mark.parametrize("seed", range(6))
def test_rest_node_departures_scale_by_one_minus_rate(seed):
    """u = 0, F = Q = 0: each relaxed moment's departure is multiplied by 1 - its rate."""
    rng = np.random.default_rng(300 + seed)
    prob = rate_problem(rng, forced=False)
    f, g = random_state(rng, zero_velocity=True)
    check_relaxation(prob, f, g)


@pytest.mark.parametrize("seed", range(6))
def test_moving_forced_node_relaxation(seed):
    """Any u, with the force of Eq. (2) and the source of Eq. (24): the same factors in the
    frame of Eq. (12)'s velocity, plus the (I - S/2) C and (I - S_T/2) R terms."""
    rng = np.random.default_rng(400 + seed)
    prob = rate_problem(rng, forced=True)
    f, g = random_state(rng, zero_velocity=False)
    check_relaxation(prob, f, g)


@pytest.mark.parametrize("seed", range(3))
def test_default_rates(seed):
    """With no override: s_b = s_4 = 1 take the trace and k22 to equilibrium in one
    collision, s_3 follows the no-slip rule and lambda_2 the rule of Sec. 3.1."""
    rng = np.random.default_rng(500 + seed)
    prob = rate_problem(rng, forced=seed > 0, s_b=None, s_4=None, s_3=None, lambda_2=None)
    f, g = random_state(rng, zero_velocity=seed == 0)
    check_relaxation(prob, f, g)


def test_rates_enter_their_own_modes_only():
    """Changing one rate changes exactly the modes it relaxes (one at a time)."""
    rng = np.random.default_rng(600)
    base = rate_problem(rng, forced=True)
    f, g = random_state(rng, zero_velocity=False)
    fp0, gp0, (_, ux, uy, T) = oracle.collide(base, f, g)
    touched = {"s_b": {"trace"}, "s_4": {"k22"}, "s_3": {"k21", "k12"},
               "lambda_2": {"t20", "t02"}}
    m0, t0 = flow_modes(fp0, ux, uy), thermal_modes(gp0, ux, uy, T)
    for rate, modes in touched.items():
        prob = dict(base)
        prob[rate] = base[rate] * 0.8
        fp, gp, _ = oracle.collide(prob, f, g)
        m, t = flow_modes(fp, ux, uy), thermal_modes(gp, ux, uy, T)
        both = {**{k: (m[k], m0[k]) for k in m}, **{k: (t[k], t0[k]) for k in t}}
        for k, (a, b) in both.items():
            if k in modes:
                assert abs(a - b) > 1e-8, (rate, k)
            else:
                assert a == pytest.approx(b, abs=2e-15), (rate, k)


# --------------------------------------------------------------------------
# Hydrodynamic pin of the bulk rate: a standing sound wave
# --------------------------------------------------------------------------

def _damped(t, gam, om, a, b):
    return np.exp(-gam * t) * (a * np.cos(om * t) + b * np.sin(om * t))


@pytest.mark.parametrize("s_b", [None, 1.5, 0.7])
def test_sound_wave_decay_sets_bulk_viscosity(s_b):
    """rho = 1 + eps cos(k x), u = 0 in a periodic box. Linearised, the isotropic part of
    the viscous stress carries nu_b = c_s^2 (1/s_b - 1/2) (the trace of the second moments
    relaxes at s_b), the deviatoric part nu, so the density amplitude obeys
    A'' + (nu + nu_b) k^2 A' + c_s^2 k^2 A = 0: it decays at Gamma = k^2 (nu + nu_b)/2 and
    oscillates at omega = sqrt(c_s^2 k^2 - Gamma^2). At k = 2 pi/64 the lattice corrections
    are O(k^2) ~ 1e-2 relative at most (the fit lands within 1e-3); the mode is fitted
    over 12 periods after the first."""
    N, nu, eps = 64, 0.02, 1e-5
    prob = W.problem(N, 2, nu, 0.05, [W.PERIODIC] * 4, s_b=s_b)
    k = 2 * math.pi / N
    x = np.arange(N, dtype=float)
    mode = np.cos(k * x)
    s = oracle.Sim(prob, rho=np.broadcast_to(1.0 + eps * mode, (2, N)))
    period = 2 * math.pi / (math.sqrt(CS2) * k)
    t0 = int(period)
    s.step(t0)
    ts, amp = [], []
    for _ in range(int(12 * period) // 4):
        s.step(4)
        ts.append(s.t - t0)
        amp.append(float(np.sum((s.macros()[0][0] - 1.0) * mode) / np.sum(mode * mode)))
    ts, amp = np.array(ts, dtype=float), np.array(amp)
    s_b_used = 1.0 if s_b is None else s_b
    nu_b = CS2 * (1.0 / s_b_used - 0.5)
    gam = 0.5 * k * k * (nu + nu_b)
    om = math.sqrt(CS2 * k * k - gam * gam)
    popt, _ = curve_fit(_damped, ts, amp, p0=[gam, om, amp[0], 0.0])
    assert popt[0] == pytest.approx(gam, rel=5e-3), (popt[0], gam)
    assert popt[1] == pytest.approx(om, rel=5e-3)
    # a bulk rate equal to the shear rate (plain BGK trace) would give a different decay
    gam_shear = 0.5 * k * k * 2 * nu
    assert abs(popt[0] - gam_shear) > 0.1 * gam
