"""Pins of the oracle's Grunwald coefficients and WSGD weights (paper Sec. 2, Sec. 3.1).

Each check uses something other than the oracle's own formula: a library binomial routine, the
binomial series / generating functions, closed forms printed in the paper, and the g = 2 case.
"""
import numpy as np
import pytest
from scipy.special import binom

from oracle.weights import grunwald, wsgd

GAMMAS = [1.1, 1.2, 1.5, 1.562, 1.6, 1.8, 1.9, 1.99]


@pytest.mark.parametrize("g", GAMMAS)
def test_grunwald_matches_library_binomial(g):
    K = 200
    k = np.arange(K + 1)
    ref = (-1.0) ** k * binom(g, k)
    # the recurrence accumulates ~K ulps; the library routine loses a few digits near g = 2
    np.testing.assert_allclose(grunwald(g, K), ref, rtol=5e-11, atol=1e-300)


@pytest.mark.parametrize("g", GAMMAS)
def test_grunwald_properties(g):
    # Sec. 2: g_0 = 1, g_1 = -g, g_2 > g_3 > ... > 0, partial sums < 0, sum -> 0.
    gk = grunwald(g, 5000)
    assert gk[0] == 1.0 and gk[1] == pytest.approx(-g, abs=1e-15)
    assert np.all(gk[2:] > 0) and np.all(np.diff(gk[2:]) < 0)
    ps = np.cumsum(gk)
    assert np.all(ps[1:] < 0)
    # closed form of the partial sum: sum_{k<=K} (-1)^k C(g,k) = (-1)^K C(g-1,K)
    K = np.arange(len(gk))
    np.testing.assert_allclose(ps, (-1.0) ** K * binom(g - 1, K), rtol=1e-10, atol=1e-14)
    assert abs(ps[-1]) < 5000 ** (-(g - 1)) * 2  # tail decays like K^(1-g)


@pytest.mark.parametrize("g", [1.3, 1.7])
@pytest.mark.parametrize("z", [0.5, -0.7, 0.3 + 0.4j, -0.2 - 0.6j])
def test_grunwald_generating_function(g, z):
    gk = grunwald(g, 400)
    s = np.sum(gk * z ** np.arange(401))
    assert abs(s - (1 - z) ** g) < 1e-13


@pytest.mark.parametrize("g", GAMMAS)
def test_wsgd_closed_forms(g):
    # Proposition (ww): w0 = g/2, w1 = (2-g-g^2)/2 < 0, w2 = g(g^2+g-4)/4,
    # 1 >= w0 >= w3 >= w4 >= ... >= 0, partial sums < 0 for n >= 2, sum = 0.
    w = wsgd(g, 20000)
    assert w[0] == pytest.approx(g / 2, abs=1e-15)
    assert w[1] == pytest.approx((2 - g - g * g) / 2, abs=1e-15) and w[1] < 0
    assert w[2] == pytest.approx(g * (g * g + g - 4) / 4, abs=1e-14)
    assert 1 >= w[0] >= w[3]
    assert np.all(np.diff(w[3:]) <= 0) and np.all(w[3:] >= 0)
    ps = np.cumsum(w)
    assert np.all(ps[2:] < 0)
    assert abs(ps[-1]) < 20000 ** (-(g - 1)) * 2


def test_wsgd_w2_sign_changes_at_gamma0():
    # Sec. 2: w2 >= 0 iff g >= gamma_0 = (sqrt(17) - 1) / 2, the M-matrix threshold.
    g0 = (np.sqrt(17.0) - 1.0) / 2.0
    assert wsgd(g0 - 1e-6, 3)[2] < 0 < wsgd(g0 + 1e-6, 3)[2]


@pytest.mark.parametrize("g", [1.2, 1.5, 1.9])
@pytest.mark.parametrize("z", [0.5, -0.7, 0.3 + 0.4j])
def test_wsgd_generating_function(g, z):
    # From eq. (w): sum_k w_k z^k = (g/2 + (2-g) z / 2) (1 - z)^g.
    w = wsgd(g, 400)
    s = np.sum(w * z ** np.arange(401))
    assert abs(s - (g / 2 + (2 - g) * z / 2) * (1 - z) ** g) < 1e-13


@pytest.mark.parametrize("g", [1.2, 1.5, 1.9])
def test_symbol_closed_form(g):
    # Proposition (pro2), eq. (fgamma): f(xi) = -sum_{k>=-1} w_{k+1} e^{ik xi}
    #                                      = -[(2 - g(1 - e^{-i xi}))/2] (1 + e^{i(xi+pi)})^g.
    K = 200000
    w = wsgd(g, K)
    for xi in [0.3, 1.0, 2.0, np.pi, -1.3]:
        k = np.arange(-1, K)
        trunc = -np.sum(w * np.exp(1j * k * xi))
        closed = -((2 - g * (1 - np.exp(-1j * xi))) / 2) * (1 + np.exp(1j * (xi + np.pi))) ** g
        assert abs(trunc - closed) < 5 * K ** (-g)
    # Proposition (PaPb): q = f(xi) + f(-xi) >= 0 with max (g-1) 2^(g+1) at xi = pi.
    xs = np.linspace(-np.pi, np.pi, 2001)
    f = lambda x: -((2 - g * (1 - np.exp(-1j * x))) / 2) * (1 + np.exp(1j * (x + np.pi))) ** g
    q = (f(xs) + f(-xs)).real
    assert q.min() > -1e-12
    assert q.max() == pytest.approx((g - 1) * 2 ** (g + 1), rel=1e-12)


@pytest.mark.parametrize("g", [1.1, 1.4, 1.6, 1.9])
def test_wsgd_l1_norm_closed_form(g):
    # Proof of Proposition (pro2): sum |w_k| = g^2 + g - 2 + g/4 (|g^2+g-4| - (g^2+g-4)).
    K = 2_000_000
    w = wsgd(g, K)
    closed = g * g + g - 2 + g / 4 * (abs(g * g + g - 4) - (g * g + g - 4))
    # all w_k, k >= 3, are positive; the neglected tail is bounded by C K^-g
    assert np.sum(np.abs(w)) == pytest.approx(closed, abs=4 * K ** (-g))


def test_gamma_two_is_laplacian():
    # The g = 2 weights are (1, -2, 1, 0, ...), so T_2 = tridiag(1, -2, 1) (Sec. 4.3, P_2).
    w = wsgd(2.0, 10)
    np.testing.assert_array_equal(w, [1, -2, 1, 0, 0, 0, 0, 0, 0, 0, 0])
