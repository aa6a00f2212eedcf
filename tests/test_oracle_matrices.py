"""Pins of the oracle's transforms against their definitions (CPU only).

The oracle types in the matrices printed in Eq. (6a), (6b), (16), (17) of Fei &
Luo (arXiv:1801.04577). These tests rebuild them from the definitions of raw and
central moments, Eq. (4) and Eq. (13), over the velocity set of Eq. (3), so a
mistyped entry, sign or index fails here.
"""
import numpy as np
import pytest

import oracle

# Eq. (3), D2Q9; the D2Q5 set is its first five members.
EX = np.array([0, 1, 0, -1, 0, 1, -1, -1, 1], dtype=float)
EY = np.array([0, 0, 1, 0, -1, 1, 1, -1, -1], dtype=float)
# Eq. (5) and Eq. (14): (m, n) exponents of the moment sets.
SET9 = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2), (1, 1), (2, 1), (1, 2), (2, 2)]
SET5 = [(0, 0), (1, 0), (0, 1), (2, 0), (0, 2)]


def raw_moments(f, ex, ey, mset):
    return np.array([np.sum(f * ex ** m * ey ** n) for (m, n) in mset])


def central_moments(f, ex, ey, mset, ux, uy):
    return np.array([np.sum(f * (ex - ux) ** m * (ey - uy) ** n) for (m, n) in mset])


def test_M_is_raw_moment_map():
    M = oracle.matrix_M()
    brute = np.array([[EX[i] ** m * EY[i] ** n for i in range(9)] for (m, n) in SET9])
    assert np.array_equal(M, brute)


def test_MT_is_raw_moment_map():
    MT = oracle.matrix_MT()
    brute = np.array([[EX[i] ** m * EY[i] ** n for i in range(5)] for (m, n) in SET5])
    assert np.array_equal(MT, brute)


@pytest.mark.parametrize("seed", range(5))
def test_N_shifts_raw_to_central(seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.0, 1.0, 9)
    ux, uy = rng.uniform(-0.3, 0.3, 2)
    got = oracle.matrix_N(ux, uy) @ (oracle.matrix_M() @ f)
    want = central_moments(f, EX, EY, SET9, ux, uy)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("seed", range(5))
def test_NT_shifts_raw_to_central(seed):
    rng = np.random.default_rng(100 + seed)
    g = rng.uniform(0.0, 1.0, 5)
    ux, uy = rng.uniform(-0.3, 0.3, 2)
    got = oracle.matrix_NT(ux, uy) @ (oracle.matrix_MT() @ g)
    want = central_moments(g, EX[:5], EY[:5], SET5, ux, uy)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-14)


def test_N_every_entry_is_exercised():
    """Unit vectors in raw-moment space: N e_k is column k, each checked against the
    binomial expansion of the central moment, (e - u)^m = sum_j C(m,j) e^j (-u)^(m-j)."""
    from math import comb
    ux, uy = 0.17, -0.23
    N = oracle.matrix_N(ux, uy)
    for r, (m, n) in enumerate(SET9):
        for c, (a, b) in enumerate(SET9):
            want = 0.0
            if a <= m and b <= n:
                want = comb(m, a) * comb(n, b) * (-ux) ** (m - a) * (-uy) ** (n - b)
            assert N[r, c] == pytest.approx(want, abs=1e-15), (r, c)


def test_inverses():
    M = np.array([[EX[i] ** m * EY[i] ** n for i in range(9)] for (m, n) in SET9])
    MT = M[:5, :5]
    np.testing.assert_allclose(oracle.matrix_Minv() @ M, np.eye(9), atol=1e-15)
    np.testing.assert_allclose(oracle.matrix_MTinv() @ MT, np.eye(5), atol=1e-15)


def test_shift_inverse_is_opposite_shift():
    """A shift by u followed by a shift by -u is the identity (binomial theorem)."""
    ux, uy = 0.21, 0.08
    np.testing.assert_allclose(oracle.matrix_N(-ux, -uy) @ oracle.matrix_N(ux, uy), np.eye(9),
                               atol=1e-15)
    np.testing.assert_allclose(oracle.matrix_NT(-ux, -uy) @ oracle.matrix_NT(ux, uy), np.eye(5),
                               atol=1e-15)


def test_rest_equilibrium_weights():
    """At rest Eq. (9) gives the D2Q9 weights 4/9, 1/9, 1/36; Eq. (19) with c_T^2 = 2/5
    gives 1/5 for every D2Q5 direction."""
    f, g = oracle.equilibrium(1.0, 0.0, 0.0, 1.0)
    np.testing.assert_allclose(f, [4 / 9] + [1 / 9] * 4 + [1 / 36] * 4, atol=1e-16)
    np.testing.assert_allclose(g, [0.2] * 5, atol=1e-16)


@pytest.mark.parametrize("seed", range(4))
def test_equilibrium_product_form(seed):
    """Central moments of Eq. (9) are those of a Maxwellian, so the raw equilibrium
    moments factor as rho m_a(ux) m_b(uy) with m_0 = 1, m_1 = u, m_2 = 1/3 + u^2; on the
    D2Q9 lattice that is f_i = rho phi(e_ix, ux) phi(e_iy, uy), phi(0, u) = 2/3 - u^2,
    phi(+-1, u) = (1/3 + u^2 +- u)/2. For D2Q5, g_0 = T(1 - 2 c_T^2 - |u|^2) and
    g_(+-x) = T(c_T^2 + ux^2 +- ux)/2."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.8, 1.2)
    ux, uy = rng.uniform(-0.2, 0.2, 2)
    T = rng.uniform(-1, 1)

    def phi(e, u):
        return 2.0 / 3.0 - u * u if e == 0 else (1.0 / 3.0 + u * u + e * u) / 2.0

    f, g = oracle.equilibrium(rho, ux, uy, T)
    want_f = np.array([rho * phi(EX[i], ux) * phi(EY[i], uy) for i in range(9)])
    ct2 = 0.4
    want_g = np.array([T * (1 - 2 * ct2 - ux * ux - uy * uy),
                       T * (ct2 + ux * ux + ux) / 2, T * (ct2 + uy * uy + uy) / 2,
                       T * (ct2 + ux * ux - ux) / 2, T * (ct2 + uy * uy - uy) / 2])
    np.testing.assert_allclose(f, want_f, atol=1e-15)
    np.testing.assert_allclose(g, want_g, atol=1e-15)


def test_rates_at_paper_values():
    """Sec. 3.1 prints (lambda_1, lambda_2) = (4/3, 3/4) for alpha = 1/10 and (3/4, 4/3)
    for alpha = 1/3, both of which satisfy lambda_2 = 12(lambda_1 - 2)/(lambda_1 - 12)."""
    import workloads as W
    for alpha, l1, l2 in ((0.1, 4 / 3, 3 / 4), (1 / 3, 3 / 4, 4 / 3)):
        prob = W.problem(1, 6, 0.1, alpha, [W.PERIODIC] * 2 + [W.dirichlet(0)] * 2)
        r = oracle.rates(prob)
        assert r[5] == pytest.approx(l1, rel=1e-14)
        assert r[6] == pytest.approx(l2, rel=1e-14)
    # nu = (1/s_nu - 1/2)/3 inverted, and the no-slip rule's fixed point:
    # s_3 = (16 - 8 s_nu)/(8 - s_nu) gives (1/s_nu - 1/2)(1/s_3 - 1/2) = 3/16.
    prob = W.problem(1, 6, 0.05, 0.05, [W.PERIODIC] * 4)
    s_nu, s_b, s_3 = oracle.rates(prob)[:3]
    assert (1 / s_nu - 0.5) / 3 == pytest.approx(0.05, rel=1e-14)
    assert (1 / s_nu - 0.5) * (1 / s_3 - 0.5) == pytest.approx(3 / 16, rel=1e-13)
