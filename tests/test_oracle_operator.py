"""Pins of the oracle's operator (paper Sec. 2 and Sec. 3).

Structure checks use the paper's stated properties (eqs. (AN), (AxAy), (M); the gamma_0 M-matrix
statement; SPD for constant equal coefficients; real spectrum for equal variable coefficients),
and the consistency check compares against closed-form Riemann-Liouville derivatives.
"""
import numpy as np
import pytest

import workloads
from oracle.operator import Operator, operator_from_problem, paper_A, toeplitz_T
from oracle.weights import wsgd


def _rand_op(rng, n1, n2, alpha=1.7, beta=1.3, tau=0.05, const=None):
    shape = (n2, n1)
    if const is None:
        f = lambda: rng.uniform(0.5, 2.0, size=shape)
        dp, dm, ep, em = f(), f(), f(), f()
    else:
        d, e = const
        dp = dm = np.full(shape, d)
        ep = em = np.full(shape, e)
    return Operator(alpha, beta, n1, n2, 1.0 / (n1 + 1), 1.0 / (n2 + 1), tau, dp, dm, ep, em)


def test_toeplitz_entries_follow_eq_AN():
    n, g = 9, 1.45
    w = wsgd(g, n)
    T = toeplitz_T(g, n)
    for i in range(n):
        for j in range(n):
            k = i - j + 1
            assert T[i, j] == (w[k] if k >= 0 else 0.0)
    np.testing.assert_array_equal(paper_A(g, n), -T)


def test_dense_equals_kronecker_field_form():
    rng = np.random.default_rng(0)
    op = _rand_op(rng, 7, 15)
    U = rng.standard_normal((15, 7))
    np.testing.assert_allclose(op.dense() @ U.ravel(), op.apply(U).ravel(), rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(np.diag(op.dense()).reshape(15, 7), op.diag(), rtol=1e-14)


def test_scaled_form_eq_M_is_system_over_r():
    rng = np.random.default_rng(1)
    op = _rand_op(rng, 7, 7)
    r = op.tau / (2 * op.hx ** op.alpha)
    np.testing.assert_allclose(op.paper_scaled_dense(), op.dense() / r, rtol=1e-12, atol=1e-9)


def test_spd_for_constant_equal_coefficients():
    # Sec. 2: with d+ = d- = d and e+ = e- = e constant, M is symmetric positive definite BTTB.
    op = _rand_op(None, 15, 15, alpha=1.3, beta=1.8, const=(1.3, 0.7))
    A = op.dense()
    np.testing.assert_allclose(A, A.T, atol=1e-12)
    assert np.linalg.eigvalsh(A).min() > 0


@pytest.mark.parametrize("alpha,beta", [(1.6, 1.9), (1.57, 1.57)])
def test_m_matrix_above_gamma0(alpha, beta):
    # Sec. 2: alpha, beta in [gamma_0, 2) gives a strictly diagonally dominant M-matrix.
    rng = np.random.default_rng(2)
    op = _rand_op(rng, 15, 15, alpha=alpha, beta=beta)
    A = op.dense()
    off = A - np.diag(np.diag(A))
    assert np.all(off <= 1e-15)
    assert np.all(np.diag(A) > np.abs(off).sum(axis=1))


def test_not_m_matrix_below_gamma0():
    rng = np.random.default_rng(3)
    op = _rand_op(rng, 15, 15, alpha=1.2, beta=1.3)
    A = op.dense()
    off = A - np.diag(np.diag(A))
    assert off.max() > 0  # w2 < 0 gives positive off-diagonal entries


@pytest.mark.parametrize("g", [1.2, 1.5, 1.9])
def test_symmetric_part_spectrum_bound(g):
    # Szego/Tilli and eq. (10): eig(-(T + T^T)) lies in (0, ||q_g||_inf) with ||q_g|| = (g-1) 2^(g+1).
    T = toeplitz_T(g, 63)
    ev = np.linalg.eigvalsh(-(T + T.T))
    assert ev.min() > 0 and ev.max() < (g - 1) * 2 ** (g + 1)


def test_real_spectrum_for_equal_variable_coefficients():
    # Sec. 3.2: with d+ = d- = e+ = e- (variable) the spectrum is real.
    rng = np.random.default_rng(4)
    n = 15
    X, Y = np.meshgrid(np.arange(1, n + 1) / (n + 1), np.arange(1, n + 1) / (n + 1))
    c = 1 + X + Y ** 2
    op = Operator(1.6, 1.6, n, n, 1 / (n + 1), 1 / (n + 1), 0.05, c, c, c, c)
    ev = np.linalg.eigvals(op.dense())
    assert np.abs(ev.imag).max() < 1e-8 * np.abs(ev).max()


def _consistency_error(n, alpha, beta):
    # u = x^3 (1-x)^4 * y^4 (1-y)^3: asymmetric, so swapping left/right derivatives is detected,
    # and smooth enough at the boundary (zero extension in C^2) for pointwise O(h^2) consistency.
    from numpy.polynomial import Polynomial as Pn

    Xp = Pn([0, 0, 0, 1]) * Pn([1, -1]) ** 4
    Yp = Pn([0, 0, 0, 0, 1]) * Pn([1, -1]) ** 3
    h = 1.0 / (n + 1)
    x = h * np.arange(1, n + 1)
    Yg, Xg = np.meshgrid(x, x, indexing="ij")
    dp, dm, ep, em = 1 + Xg, 2 - Yg, 1.5 + Xg * Yg, 0.5 + Yg
    op = Operator(alpha, beta, n, n, h, h, 1.0, dp, dm, ep, em)
    U = Xp(Xg) * Yp(Yg)
    exact = (dp * workloads.poly_rl_left(Xp, alpha, Xg, 0.0) * Yp(Yg)
             + dm * workloads.poly_rl_right(Xp, alpha, Xg, 1.0) * Yp(Yg)
             + ep * Xp(Xg) * workloads.poly_rl_left(Yp, beta, Yg, 0.0)
             + em * Xp(Xg) * workloads.poly_rl_right(Yp, beta, Yg, 1.0))
    return np.abs(op.L(U) - exact).max()


@pytest.mark.parametrize("alpha,beta", [(1.8, 1.6), (1.2, 1.9)])
def test_wsgd_second_order_consistency(alpha, beta):
    # Sec. 2: the WSGD formula with shifts (1,0) approximates each RL derivative to O(h^2).
    errs = [_consistency_error(n, alpha, beta) for n in (31, 63, 127, 255)]
    ratios = [errs[i] / errs[i + 1] for i in range(3)]
    assert all(3.7 < r < 4.3 for r in ratios[1:]), ratios


# ---- the point-sampled application used at sizes where the full product is too slow ----
@pytest.mark.parametrize("n1,n2", [(63, 63), (31, 63)])
def test_L_points_equal_full_application(n1, n2):
    p = workloads.config_c2(n1, 32)
    p.n2 = n2
    op = operator_from_problem(p, 0.0)
    U = np.random.default_rng(5).standard_normal((n2, n1))
    rng = np.random.default_rng(6)
    js = np.concatenate([[0, 0, n2 - 1, n2 - 1], rng.integers(0, n2, 40)])
    is_ = np.concatenate([[0, n1 - 1, 0, n1 - 1], rng.integers(0, n1, 40)])
    full_L, full_A = op.L(U), op.apply(U)
    np.testing.assert_allclose(op.L_points(U, js, is_), full_L[js, is_], rtol=0,
                               atol=1e-12 * np.abs(full_L).max())
    np.testing.assert_allclose(op.apply_points(U, js, is_), full_A[js, is_], rtol=0,
                               atol=1e-12 * np.abs(full_A).max())
    # and against the dense matrix of eq. (AxAy), row by row
    Ld = op.L_dense()
    rows = js * n1 + is_
    np.testing.assert_allclose(op.L_points(U, js, is_), Ld[rows] @ U.ravel(), rtol=0,
                               atol=1e-12 * np.abs(full_L).max())


# ---- the band (Laplacian) preconditioner P_2 of Sec. 4.3 ----
def test_band_operator_is_r_times_paper_P2():
    from oracle.operator import band_operator, band_P2_scaled_dense

    p = workloads.config_c2(15, 32)
    op = operator_from_problem(p, 0.0)
    r = op.tau / (2.0 * op.hx ** op.alpha)
    B = band_operator(op)
    np.testing.assert_allclose(B.dense(), r * band_P2_scaled_dense(op), rtol=0, atol=1e-13)
    # the field-form application and the pointwise diagonal agree with the assembled matrix
    U = np.random.default_rng(1).standard_normal((15, 15))
    np.testing.assert_allclose(B.apply(U).ravel(), B.dense() @ U.ravel(), atol=1e-12)
    np.testing.assert_allclose(B.diag().ravel(), np.diag(B.dense()), atol=1e-13)


def test_band_P2_has_five_diagonals():
    # Sec. 4.3: "only five nonzero diagonals" (offsets 0, +-1, +-n1 in the lexicographic order)
    from oracle.operator import band_P2_scaled_dense

    n = 15
    op = operator_from_problem(workloads.config_c2(n, 32), 0.0)
    P2 = band_P2_scaled_dense(op)
    offs = {j - i for i, j in zip(*np.nonzero(P2))}
    assert offs == {0, 1, -1, n, -n}


def test_band_P2_equals_system_matrix_at_order_two():
    # With alpha = beta = 2 the WSGD weights are (1, -2, 1) and the system matrix M of eq. (M) is
    # the band preconditioner itself (the "Laplacian preconditioner (alpha = beta = 2)", Sec. 4.3).
    from oracle.operator import band_P2_scaled_dense

    n = 15
    p = workloads.config_c2(n, 32)
    dp, dm, ep, em = workloads.sample(p, 0.0)
    h = 1.0 / (n + 1)
    op2 = Operator(2.0, 2.0, n, n, h, h, p.tau, dp, dm, ep, em)
    np.testing.assert_allclose(band_P2_scaled_dense(op2), op2.paper_scaled_dense(), rtol=1e-13,
                               atol=1e-13 * np.abs(op2.paper_scaled_dense()).max())


def test_band_P2_spd_for_constant_equal_coefficients():
    from oracle.operator import band_P2_scaled_dense

    n = 15
    h = 1.0 / (n + 1)
    one = np.ones((n, n))
    op = Operator(1.6, 1.8, n, n, h, h, 1.0 / 32, one, one, 2 * one, 2 * one)
    P2 = band_P2_scaled_dense(op)
    np.testing.assert_allclose(P2, P2.T, atol=1e-12)
    assert np.linalg.eigvalsh(P2).min() > 0
