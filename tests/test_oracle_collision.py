"""Collision invariants of the oracle (CPU only).

Properties fixed by the structure of Eq. (7)-(10) and Eq. (23)-(25) of Fei & Luo
(arXiv:1801.04577), independent of how the oracle evaluates them:
  * density is unchanged by the collision;
  * momentum sum_i f_i e_i gains exactly F (consistent forcing, Eq. 10, 12);
  * sum_i g_i gains exactly Q (Eq. 23-25), whatever lambda_0 is;
  * with F = Q = 0 the equilibrium of Eq. (9), (19) is a fixed point.
"""
import numpy as np
import pytest

import oracle
import workloads as W

EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)


def random_node(rng):
    rho = rng.uniform(0.9, 1.1)
    ux, uy = rng.uniform(-0.1, 0.1, 2)
    T = rng.uniform(-0.5, 0.5)
    f, g = oracle.equilibrium(rho, ux, uy, T)
    f = f + rng.uniform(-0.01, 0.01, 9)
    g = g + rng.uniform(-0.01, 0.01, 5)
    return f, g


def random_problem(rng, **over):
    prob = W.problem(4, 4, rng.uniform(0.01, 0.3), rng.uniform(0.01, 0.3), [W.PERIODIC] * 4,
                     g_beta=rng.uniform(0, 1e-3), T0=rng.uniform(-0.2, 0.2),
                     Fx=rng.uniform(-1e-4, 1e-4), Fy=rng.uniform(-1e-4, 1e-4),
                     Q=rng.uniform(-1e-3, 1e-3), s_b=rng.uniform(0.5, 1.5),
                     s_4=rng.uniform(0.5, 1.5))
    prob.update(over)
    return prob


@pytest.mark.parametrize("seed", range(8))
def test_conservation_and_exact_source(seed):
    rng = np.random.default_rng(seed)
    prob = random_problem(rng)
    f, g = random_node(rng)
    fp, gp, (rho, ux, uy, T) = oracle.collide(prob, f, g)
    Fx = prob["Fx"]
    Fy = prob["Fy"] + prob["g_beta"] * (T - prob["T0"])
    assert fp.sum() == pytest.approx(f.sum(), abs=1e-15)
    assert (fp @ EX) - (f @ EX) == pytest.approx(Fx, abs=1e-15)
    assert (fp @ EY) - (f @ EY) == pytest.approx(Fy, abs=1e-15)
    assert gp.sum() - g.sum() == pytest.approx(prob["Q"], abs=1e-15)
    # Reported macroscopic values (Eq. 12 and Eq. 25).
    assert rho == pytest.approx(f.sum(), abs=1e-15)
    assert T == pytest.approx(g.sum() + prob["Q"] / 2, abs=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_lambda0_does_not_matter(seed):
    """The zeroth thermal moment relaxes to T + Q/2 for any lambda_0."""
    rng = np.random.default_rng(50 + seed)
    prob = random_problem(rng)
    f, g = random_node(rng)
    outs = [oracle.collide(dict(prob, lambda_0=l0), f, g) for l0 in (0.3, 1.0, 1.7)]
    for fp, gp, _ in outs[1:]:
        np.testing.assert_allclose(fp, outs[0][0], atol=1e-15)
        np.testing.assert_allclose(gp, outs[0][1], atol=1e-15)


@pytest.mark.parametrize("seed", range(4))
def test_equilibrium_is_fixed_point(seed):
    rng = np.random.default_rng(70 + seed)
    prob = random_problem(rng, Fx=0.0, Fy=0.0, Q=0.0, g_beta=0.0)
    rho = rng.uniform(0.9, 1.1)
    ux, uy = rng.uniform(-0.1, 0.1, 2)
    T = rng.uniform(-0.5, 0.5)
    f, g = oracle.equilibrium(rho, ux, uy, T)
    fp, gp, _ = oracle.collide(prob, f, g)
    np.testing.assert_allclose(fp, f, atol=2e-16)
    np.testing.assert_allclose(gp, g, atol=2e-16)


def test_rate_validation():
    prob = W.problem(4, 4, 0.1, 0.1, [W.PERIODIC] * 4)
    with pytest.raises(oracle.OracleError):
        oracle.rates(dict(prob, nu=-0.1))
    with pytest.raises(oracle.OracleError):
        oracle.rates(dict(prob, s_3=2.5))
    with pytest.raises(oracle.OracleError):
        oracle.Sim(dict(prob, ny=1, sides=[W.PERIODIC] * 2 + [W.dirichlet(0)] * 2))
