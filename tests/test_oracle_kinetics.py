"""Pins of the oracle's kinetics and linear algebra against independent facts.

* Robertson's right-hand side is checked against its textbook equations.
* Mass conservation: w^T f(y) = 0 for association reactions with w_C = w_A + w_B.
* The analytic Jacobian is checked against central differences, which are exact
  up to round-off because mass-action f is at most quadratic here.
* LU with partial pivoting against numpy.linalg.solve, crafted ties and the
  residual bound; WRMS norm (Sec. 2, Eq. (3)) against hand-computed values.
"""
import numpy as np
import pytest

from paper_2405_01713_amd import workloads as W


def test_robertson_rhs_matches_textbook(oracle):
    m = W.robertson_mechanism()
    kf, kr = oracle.rates(m)
    assert np.allclose(kf, [0.04, 3e7, 1e4], rtol=1e-14)
    assert np.all(kr == 0.0)
    rng = np.random.default_rng(0)
    for _ in range(20):
        y1, y2, y3 = rng.uniform(0, 1, 3)
        f = oracle.rhs(m, kf, kr, [y1, y2, y3])
        ref = [-0.04 * y1 + 1e4 * y2 * y3,
               0.04 * y1 - 1e4 * y2 * y3 - 3e7 * y2 * y2,
               3e7 * y2 * y2]
        assert np.allclose(f, ref, rtol=1e-12, atol=1e-9)


def test_rates_arrhenius_and_detailed_balance(oracle):
    m = W.synthetic_mechanism(21, 84, seed=1)
    T = 1733.0
    kf, kr = oracle.rates(m, T)
    # equilibrium constant K_r = kf/kr = exp(g_A + g_B - g_C)
    g = m["g"]
    a, b, c = m["reac"][:, 0], m["reac"][:, 1], m["prod"][:, 0]
    assert np.allclose(np.log(kf / kr), g[a] + g[b] - g[c], rtol=0, atol=1e-12)
    # ln k_f is affine in 1/T with slope -Ea/R
    kf2, _ = oracle.rates(m, 2 * T)
    assert np.allclose(np.log(kf2) - np.log(kf), m["EaR"] * (1 / T - 1 / (2 * T)), atol=1e-10)


@pytest.mark.parametrize("S,R", [(9, 30), (21, 84), (53, 325)])
def test_mass_conservation(oracle, S, R):
    m = W.synthetic_mechanism(S, R, seed=3)
    rng = np.random.default_rng(S)
    kf, kr = oracle.rates(m, 1500.0)
    for _ in range(10):
        y = rng.uniform(0, 0.1, S)
        f = oracle.rhs(m, kf, kr, y)
        scale = np.sum(np.abs(f) * m["w"])
        assert abs(np.dot(m["w"], f)) <= 1e-13 * scale


@pytest.mark.parametrize("S,R", [(3, 3), (9, 30), (21, 84)])
def test_jacobian_central_difference_exact(oracle, S, R):
    m = W.robertson_mechanism() if S == 3 else W.synthetic_mechanism(S, R, seed=5)
    kf, kr = oracle.rates(m, 1200.0)
    rng = np.random.default_rng(1)
    y = rng.uniform(0.01, 0.2, S)
    J = oracle.jac(m, kf, kr, y)
    Jfd = np.zeros_like(J)
    for j in range(S):
        d = 1e-3 * max(abs(y[j]), 1e-3)
        yp, ym = y.copy(), y.copy()
        yp[j] += d
        ym[j] -= d
        Jfd[:, j] = (oracle.rhs(m, kf, kr, yp) - oracle.rhs(m, kf, kr, ym)) / (2 * d)
    scale = np.abs(J).max()
    assert np.abs(J - Jfd).max() <= 1e-8 * scale


def test_jacobian_three_body_and_forcing(oracle):
    # a three-reactant slot and a repeated species exercise the product rule
    m = dict(n_species=4, n_reactions=2,
             reac=np.array([[0, 0, 1], [2, -1, -1]], dtype=np.int32),
             prod=np.array([[3, -1, -1], [0, 1, -1]], dtype=np.int32),
             lnA=np.log([2.0, 3.0]), EaR=np.zeros(2), lnK=np.log([0.5, 4.0]))
    kf, kr = oracle.rates(m)
    y = np.array([0.3, 0.7, 0.2, 0.9])
    J = oracle.jac(m, kf, kr, y)
    Jfd = np.zeros((4, 4))
    for j in range(4):
        yp, ym = y.copy(), y.copy()
        yp[j] += 1e-4
        ym[j] -= 1e-4
        Jfd[:, j] = (oracle.rhs(m, kf, kr, yp) - oracle.rhs(m, kf, kr, ym)) / 2e-4
    assert np.abs(J - Jfd).max() < 1e-7  # cubic term: O(d^2) FD error
    F = np.array([1.0, -2.0, 0.5, 0.25])
    assert np.allclose(oracle.rhs(m, kf, kr, y, F) - oracle.rhs(m, kf, kr, y), F)


def test_lu_matches_numpy(oracle):
    rng = np.random.default_rng(7)
    for n in (1, 2, 3, 9, 21, 53, 64):
        A = rng.standard_normal((n, n)) + n * np.eye(n) * rng.uniform(0, 1)
        b = rng.standard_normal(n)
        LU, perm, info = oracle.lu_factor(A)
        assert info == 0
        x = oracle.lu_solve(LU, perm, b)
        xr = np.linalg.solve(A, b)
        assert np.allclose(x, xr, rtol=1e-9, atol=1e-12)
        # backward error bound ||Ax - b|| <= c n u ||A|| ||x||
        res = np.linalg.norm(A @ x - b, np.inf)
        assert res <= 10 * n * 2.2e-16 * np.linalg.norm(A, np.inf) * np.linalg.norm(x, np.inf) + 1e-300


def test_lu_pivot_ties_lowest_original_row(oracle):
    # column 0 has |a| = 2 in rows 1 and 3: row 1 must be chosen
    A = np.array([[1.0, 2.0, 0.0, 1.0],
                  [-2.0, 1.0, 1.0, 0.0],
                  [0.5, 0.0, 3.0, 1.0],
                  [2.0, 1.0, 0.0, 4.0]])
    LU, perm, info = oracle.lu_factor(A)
    assert info == 0 and perm[0] == 1
    # after eliminating with row 1, column 1 holds 2.5 (row 0), 0.25 (row 2)
    # and 2 (row 3): row 0 is the second pivot
    assert perm[1] == 0
    b = np.arange(4.0)
    assert np.allclose(oracle.lu_solve(LU, perm, b), np.linalg.solve(A, b))
    # an exact tie in the second column (-3 and 3): original row 1 wins
    B = np.array([[4.0, 1.0, 1.0], [0.0, -3.0, 2.0], [0.0, 3.0, 5.0]])
    LU, perm, info = oracle.lu_factor(B)
    assert list(perm[:2]) == [0, 1]


def test_lu_singular_reports_column(oracle):
    A = np.array([[1.0, 2.0], [2.0, 4.0]])
    _, _, info = oracle.lu_factor(A)
    assert info == 2
    _, _, info = oracle.lu_factor(np.zeros((3, 3)))
    assert info == 1


def test_wrms_hand_values(oracle):
    assert oracle.wrms([3.0, 4.0], [1.0, 1.0]) == pytest.approx(np.sqrt(12.5), rel=1e-15)
    assert oracle.wrms([1.0, -2.0, 2.0], [2.0, 1.0, 0.5]) == pytest.approx(np.sqrt(3.0), rel=1e-15)
    assert oracle.wrms([5.0], [0.2]) == pytest.approx(1.0, rel=1e-15)
