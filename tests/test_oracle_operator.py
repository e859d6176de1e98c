"""Pins of the oracle's operator (paper Sec. 2 and Sec. 3).

Structure checks use the paper's stated properties (eqs. (AN), (AxAy), (M); the gamma_0 M-matrix
statement; SPD for constant equal coefficients; real spectrum for equal variable coefficients),
and the consistency check compares against closed-form Riemann-Liouville derivatives.
"""
import numpy as np
import pytest

import workloads
from oracle.operator import Operator, paper_A, toeplitz_T
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
