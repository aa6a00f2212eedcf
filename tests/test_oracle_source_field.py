"""Pins of the oracle's spatially variable heat source (CPU only).

Fei & Luo (arXiv:1801.04577) treat a heat source that varies in space in Sec. 3.2 (the
viscous dissipation of a channel flow); the oracle also takes a source given per node,
Q(x) = Q + Q_field(x), in Eq. (23)-(25). Pinned here:
  * a uniform field is the uniform source, bit for bit;
  * steady diffusion between isothermal walls with a source linear across the channel,
    alpha T'' + a + b y = 0: the D2Q5 scheme with the lambda_2 rule of Sec. 3.1 and the
    half-way general bounce-back reproduces the cubic closed form to round-off (the rule
    makes the steady scheme exact for the quadratic of Sec. 3.1; a linear source adds a
    cubic term, which the second-order difference operator the steady scheme reduces to
    also differentiates exactly), while lambda_2 = 1 is off by 4e-3;
  * a quadratic source (quartic T) converges at second order in the grid spacing;
  * a two-dimensional random field gives the transpose of its transposed problem, bit
    for bit (the field is read at the right node in both directions).
"""
import math

import numpy as np
import pytest

import oracle
import workloads as W


def e2(a, b):
    return math.sqrt(float(np.sum((a - b) ** 2) / np.sum(b ** 2)))


def column(L, alpha, q, top=None, **rates):
    prob = W.problem(1, L, 0.1, alpha, [W.PERIODIC, W.PERIODIC, W.dirichlet(0.0), top or W.dirichlet(0.0)],
                     **rates)
    prob["Q_field"] = np.asarray(q, dtype=float)[:, None]
    s = oracle.Sim(prob)
    s.step(int(40 * L * L / alpha) + 2000)
    return s.macros()[3][:, 0]


def test_uniform_field_is_uniform_source():
    prob = W.cavity(20, 16, Ra=1e4, Pr=0.71, Q=3e-4)
    T = W.cavity_initial_T(prob, seed=3)
    a = oracle.Sim(prob, T=T)
    field = dict(prob, Q=0.0, Q_field=np.full((16, 20), 3e-4))
    b = oracle.Sim(field, T=T)
    a.step(200)
    b.step(200)
    for x, y in zip(a.macros(), b.macros()):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("alpha", [0.1, 1.0 / 3.0])
@pytest.mark.parametrize("L", [6, 12])
def test_linear_source_exact(alpha, L):
    a, b = 2e-3, 1e-3
    y = np.arange(L) + 0.5
    T = column(L, alpha, a + b * y)
    exact = (-(a * y ** 2 / 2 + b * y ** 3 / 6) + (a * L / 2 + b * L ** 2 / 6) * y) / alpha
    assert e2(T, exact) < 1e-12
    # the exactness comes from the lambda_2 rule
    assert e2(column(L, alpha, a + b * y, lambda_2=1.0), exact) > 1e-3


def test_quadratic_source_second_order():
    alpha, a, b, c = 0.1, 2e-3, 1e-3, 1e-4
    errs = []
    for L in (6, 12, 24):
        y = np.arange(L) + 0.5
        s = 6.0 / L   # the same continuum problem on a domain of length 6, grid spacing s
        q = (a + b * (y * s) + c * (y * s) ** 2) * s * s
        T = column(L, alpha, q)
        Y = y * s
        exact = (-(a * Y ** 2 / 2 + b * Y ** 3 / 6 + c * Y ** 4 / 12)
                 + (a * 6 / 2 + b * 36 / 6 + c * 216 / 12) * Y) / alpha
        errs.append(e2(T, exact))
    slopes = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert errs[0] > 1e-6 and all(1.8 < sl < 2.2 for sl in slopes), (errs, slopes)


def test_random_field_transposes():
    rng = np.random.default_rng(5)
    nx, ny = 14, 9
    q = rng.uniform(0.0, 2e-4, (ny, nx))
    walls = [W.dirichlet(0.2), W.dirichlet(-0.1)]
    a = W.problem(nx, ny, 0.08, 0.06, [W.PERIODIC, W.PERIODIC] + walls, Q=1e-5)
    a["Q_field"] = q
    b = W.problem(ny, nx, 0.08, 0.06, walls + [W.PERIODIC, W.PERIODIC], Q=1e-5)
    b["Q_field"] = q.T.copy()
    sa, sb = oracle.Sim(a), oracle.Sim(b)
    sa.step(300)
    sb.step(300)
    Ta, Tb = sa.macros()[3], sb.macros()[3]
    np.testing.assert_allclose(Ta, Tb.T, rtol=0, atol=1e-15)
    assert np.abs(Ta - Ta.mean(axis=1, keepdims=True)).max() > 1e-6   # the field made T vary along x
