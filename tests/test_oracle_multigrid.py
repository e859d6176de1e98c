"""Pins of the oracle's multigrid pieces (paper Sec. 4)."""
import numpy as np
import pytest

import workloads
from oracle import multigrid as mg
from oracle.operator import Operator, operator_from_problem, toeplitz_T


def test_prolongation_is_bilinear_stencil():
    # P = T(1 + cos t) K (Sec. 4.1): column J carries 1/2, 1, 1/2 at fine 2J-1, 2J, 2J+1 (1-based).
    n = 15
    P = mg.prolong_1d(n)
    assert P.shape == (15, 7)
    for J in range(1, 8):
        col = np.zeros(n)
        col[2 * J - 2], col[2 * J - 1], col[2 * J] = 0.5, 1.0, 0.5
        np.testing.assert_array_equal(P[:, J - 1], col)


def test_prolongation_reproduces_linear_functions():
    # Remark after Lemma (lemapp): the transfer operator is bilinear interpolation.
    n = 31
    h = 1.0 / (n + 1)
    xf = h * np.arange(1, n + 1)
    xc = 2 * h * np.arange(1, 16)
    f = lambda x, y: 0.3 + 2 * x - 1.5 * y
    Yc, Xc = np.meshgrid(xc, xc, indexing="ij")
    Yf, Xf = np.meshgrid(xf, xf, indexing="ij")
    fine = mg.prolong(f(Xc, Yc), n, n)
    # exact wherever the 4 surrounding coarse nodes are interior (the boundary value is 0, not f)
    np.testing.assert_allclose(fine[1:-1, 1:-1], f(Xf, Yf)[1:-1, 1:-1], atol=1e-13)


def test_even_side_prolongation_follows_the_downsampling_definition():
    # Sec. 4.1: [K]_{i,j} = 1 iff i = 2j - (n+1) mod 2 (1-based), k = (n - n mod 2)/2; for even n the
    # coarse point j is fine point 2j - 1, and P = T(1 + cos t) K puts 1/2, 1, 1/2 at fine 2j-2, 2j-1,
    # 2j (the entry at fine index 0 falls outside the grid).
    n = 16
    P = mg.prolong_1d(n)
    assert P.shape == (16, 8)
    for j in range(1, 9):
        col = np.zeros(n + 2)  # 1-based fine indices 0..n+1
        col[2 * j - 2], col[2 * j - 1], col[2 * j] = 0.5, 1.0, 0.5
        np.testing.assert_array_equal(P[:, j - 1], col[1:n + 1])


def test_even_side_prolongation_reproduces_bilinear_functions():
    # On an even side the coarse points are x_{2j-1} = (2j-1) h (1-based), spacing 2h; the last fine
    # point lies between the last coarse point and the boundary x = 1, where the field is 0.  So
    # bilinear interpolation of a bilinear function that vanishes on x = 1 and y = 1 is exact at
    # every fine point.
    n = 32
    h = 1.0 / (n + 1)
    xf = h * np.arange(1, n + 1)
    xc = h * (2 * np.arange(1, n // 2 + 1) - 1)
    f = lambda x, y: 1.3 * (1.0 - x) * (1.0 - y)
    Yc, Xc = np.meshgrid(xc, xc, indexing="ij")
    Yf, Xf = np.meshgrid(xf, xf, indexing="ij")
    np.testing.assert_allclose(mg.prolong(f(Xc, Yc), n, n), f(Xf, Yf), rtol=0, atol=1e-14)
    # and one that does not vanish there is exact away from the last fine row and column
    g = lambda x, y: 0.3 + 2 * x - 1.5 * y
    np.testing.assert_allclose(mg.prolong(g(Xc, Yc), n, n)[:-1, :-1], g(Xf, Yf)[:-1, :-1], rtol=0, atol=1e-13)


def test_even_side_full_weighting_of_constants():
    # R = P^T/4 of a constant on an even side: unit weights except the first coarse row and column,
    # whose stencil loses its fine index 0 (weight 1/2 of 2): 3/4 per direction.
    n = 16
    w = np.ones(8)
    w[0] = 0.75
    np.testing.assert_allclose(mg.restrict(np.ones((n, n)), n, n), np.outer(w, w), rtol=0, atol=1e-15)


def test_full_weighting_preserves_constants():
    n = 15
    r = mg.restrict(np.ones((n, n)), n, n)
    np.testing.assert_allclose(r, np.ones((7, 7)), atol=1e-15)


def test_laplacian_galerkin_is_rediscretisation_1d():
    # Textbook fact (g = 2 weights, Sec. 4.3): P^T tridiag(1,-2,1)_n P = tridiag(1,-2,1)_k / 2.
    n = 31
    T = toeplitz_T(2.0, n)
    P = mg.prolong_1d(n)
    np.testing.assert_allclose(P.T @ T @ P, toeplitz_T(2.0, 15) / 2, atol=1e-14)


def _c2_op(n, steps=32):
    p = workloads.config_c2(n, steps)
    return operator_from_problem(p, 0.0)


@pytest.mark.parametrize("n", [15, 31])
def test_composed_galerkin_equals_dense_triple_product(n):
    op = _c2_op(n)
    dense = mg.galerkin_hierarchy_dense(op)
    comp = mg.galerkin_hierarchy_composed(op)
    assert len(dense) == len(comp)
    for d, c in zip(dense[1:], comp[1:]):
        Ad, Ac = d.dense(), c.dense()
        np.testing.assert_allclose(Ac, Ad, rtol=1e-12, atol=1e-12 * np.abs(Ad).max())
        np.testing.assert_allclose(c.diag(), d.diag(), rtol=1e-12)


def test_constant_coefficient_galerkin_is_toeplitz():
    # With constant coefficients one level of P^T (I kron T) P is again Toeplitz in x with entries
    # (p * t * p)[2m], p = [1/2, 1, 1/2]  (odd n, coarse points injected: no corner correction).
    n, g = 31, 1.5
    T = toeplitz_T(g, n)
    P = mg.prolong_1d(n)
    C = P.T @ T @ P
    t = np.zeros(2 * n + 1)  # t[m + n] = T[i, j] with m = i - j
    for m in range(-n + 1, n):
        t[m + n] = T[max(m, 0), max(-m, 0)]
    ptp = np.convolve(np.convolve([0.5, 1, 0.5], t), [0.5, 1, 0.5])  # centre index n + 2
    for i in range(15):
        for j in range(15):
            m = i - j
            assert C[i, j] == pytest.approx(ptp[n + 2 + 2 * m], abs=1e-13)


def test_two_grid_contracts_and_is_flat_in_n():
    # Theorem (theorem21bis): for constant equal coefficients (SPD, s/r = O(1)) the TGM with damped
    # Jacobi and bilinear P contracts with a constant independent of N.
    rhos = []
    for n in (15, 31):
        A = operator_from_problem(workloads.config_c1(n), 0.0).dense()
        G = mg.tgm_iteration_matrix(A, mg.prolong_2d_dense(n, n), 0.7, 1)
        rhos.append(np.abs(np.linalg.eigvals(G)).max())
    assert max(rhos) < 0.6 and abs(rhos[1] - rhos[0]) < 0.05, rhos


def test_two_grid_contracts_variable_coefficients():
    # The variable-coefficient extension at the end of Sec. 4.1: still a contraction.
    n = 31
    A = operator_from_problem(workloads.config_c2(n, n + 1), 0.0).dense()
    for nu in (1, 2):
        G = mg.tgm_iteration_matrix(A, mg.prolong_2d_dense(n, n), 0.7, nu)
        assert np.abs(np.linalg.eigvals(G)).max() < 0.9


def test_jacobi_damping_within_lemma_bound():
    # Lemma (lemsmo): 0 < omega < 2 a0 / ||F||_inf, a0 = 1/r - 2(d w1^a + s/r e w1^b).
    from oracle.weights import wsgd

    p = workloads.config_c1(63)
    a, b = p.alpha, p.beta
    r = p.tau / (2 * p.hx ** a)
    s = p.tau / (2 * p.hy ** b)
    a0 = 1 / r - 2 * (wsgd(a, 2)[1] + s / r * wsgd(b, 2)[1])
    Finf = (a - 1) * 2 ** (a + 1) + s / r * (b - 1) * 2 ** (b + 1)
    assert 0.7 < 2 * a0 / Finf


@pytest.mark.parametrize("variant", ["geometric", "galerkin"])
def test_vcycle_contraction_is_mesh_independent(variant):
    # Sec. 4.2 / Sec. 5 protocol (tau = h): the V-cycle contraction factor stays bounded away from 1
    # and its growth with n saturates (power iteration on e <- e - V A e).
    rates = []
    for n in (15, 31, 63):
        op = _c2_op(n, n + 1)
        lv = mg.geometric_hierarchy(op) if variant == "geometric" else mg.galerkin_hierarchy_composed(op)
        vc = mg.VCycle(lv)
        e = np.random.default_rng(n).standard_normal((n, n))
        for _ in range(12):
            e_new = e - vc(op.apply(e))
            rate = np.linalg.norm(e_new) / np.linalg.norm(e)
            e = e_new / np.linalg.norm(e_new)
        rates.append(rate)
    assert max(rates) < 0.75, rates
    assert rates[2] - rates[1] < rates[1] - rates[0], rates


def test_geometric_and_galerkin_iteration_counts_agree():
    # Sec. 5, Example 1 discussion: the geometric and Galerkin preconditioners need the same number
    # of GMRES iterations.
    from oracle.krylov import fgmres

    for n in (31, 63):
        op = _c2_op(n, n + 1)
        b = np.random.default_rng(1).standard_normal((n, n))
        its = [fgmres(op.apply, b, mg.VCycle(lv), rtol=1e-7, restart=20).iters
               for lv in (mg.geometric_hierarchy(op), mg.galerkin_hierarchy_composed(op))]
        assert abs(its[0] - its[1]) <= 1, its


def test_vcycle_matrix_spectral_radius_small_grid():
    # the dense error-propagation matrix I - V A: spectral radius equals the power-iteration rate
    op = _c2_op(15, 16)
    vc = mg.VCycle(mg.geometric_hierarchy(op))
    G = mg.vcycle_iteration_matrix(vc)
    assert np.abs(np.linalg.eigvals(G)).max() < 0.7


def test_geometric_hierarchy_shapes_and_injection():
    op = _c2_op(63)
    lv = mg.geometric_hierarchy(op)
    assert [l.n1 for l in lv] == [63, 31, 15, 7]
    assert lv[1].hx == pytest.approx(2 * op.hx)
    np.testing.assert_array_equal(lv[1].dp, op.dp[1::2, 1::2])
    # injected coefficients equal the coefficient function sampled at the coarse points
    p = workloads.config_c2(31, 32)
    X, Y = np.meshgrid(np.arange(1, 32) / 32, np.arange(1, 32) / 32)
    np.testing.assert_allclose(lv[1].dp, p.dp(X, Y, 0.0), rtol=1e-15)


def test_even_geometric_hierarchy_shapes_and_injection():
    # even sides: 64 -> 32 -> 16 -> 8 (the paper's 8 x 8 coarsest grid), coarse point J at fine 2J
    # (0-based), so the injected coefficients are the coefficient function at x = (2J + 1) h
    p = workloads.config_c2(64, 32)
    op = operator_from_problem(p, 0.0)
    lv = mg.geometric_hierarchy(op)
    assert [l.n1 for l in lv] == [64, 32, 16, 8]
    assert lv[1].hx == pytest.approx(2 * op.hx)
    np.testing.assert_array_equal(lv[1].dp, op.dp[0::2, 0::2])
    xc = (2 * np.arange(32) + 1) / 65.0
    X, Y = np.meshgrid(xc, xc)
    np.testing.assert_allclose(lv[1].dp, p.dp(X, Y, 0.0), rtol=1e-15)
    np.testing.assert_allclose(lv[1].em, p.em(X, Y, 0.0), rtol=1e-15)


def test_standalone_vcycle_iteration_contracts_at_the_spectral_radius():
    # the stand-alone V-cycle iteration propagates the error with I - V A: the residual ratios
    # settle near its spectral radius (in a norm-independent way, so within a margin) and the
    # iteration converges, C1-like problem on a grid small enough for the dense matrix
    import workloads
    from oracle.cn import rhs
    from oracle.operator import operator_from_problem

    p = workloads.config_c1(31)
    op = operator_from_problem(p, 0.0)
    vc = mg.VCycle(mg.geometric_hierarchy(op))
    rho = max(abs(np.linalg.eigvals(mg.vcycle_iteration_matrix(vc))))
    b = rhs(op, workloads.sample_u0(p), workloads.sample_source(p, 0.5 * p.tau))
    x, k, hist = mg.mg_solve(op.apply, b, vc, 1e-10, 200)
    assert hist[-1] <= 1e-10 * hist[0]
    ratios = np.array(hist[1:]) / np.array(hist[:-1])
    tail = ratios[len(ratios) // 2:]
    assert np.all(tail <= rho * 1.5 + 1e-3)
    assert np.exp(np.mean(np.log(tail))) == pytest.approx(rho, rel=0.1)
    # mesh independence of the cycle count (Sec. 4: the V-cycle is optimal for this class)
    p2 = workloads.config_c1(63)
    op2 = operator_from_problem(p2, 0.0)
    b2 = rhs(op2, workloads.sample_u0(p2), workloads.sample_source(p2, 0.5 * p2.tau))
    _, k2, _ = mg.mg_solve(op2.apply, b2, mg.VCycle(mg.geometric_hierarchy(op2)), 1e-10, 200)
    assert abs(k2 - k) <= 2
    # and it solves the system
    from oracle.cn import solve_step
    np.testing.assert_allclose(x, solve_step(op, b), rtol=0, atol=1e-8 * np.abs(x).max())


# ---- the V-cycle against its iteration matrix written out densely (Sec. 4) ----
def _smoother(A, omega):
    return np.eye(A.shape[0]) - omega * (A / np.diag(A)[:, None])


def _cycle_matrix(vc):
    """x = V b for every unit b: the V-cycle as a matrix (it is linear in b)."""
    L0 = vc.levels[0]
    N = L0.n1 * L0.n2
    V = np.empty((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        V[:, c] = vc(e.reshape(L0.n2, L0.n1)).ravel()
    return V


@pytest.mark.parametrize("variant,n", [("geometric", 15), ("galerkin", 15), ("geometric", 16),
                                       ("galerkin", 16)])
def test_two_level_vcycle_equals_two_grid_formula(variant, n):
    # Two levels (15 -> 7 or 16 -> 8, exact coarse solve), one pre- and one post-sweep from a zero
    # guess: the error propagates with S (I - P A_c^-1 R A) S, R = P^T/4, S = I - omega D^-1 A (the
    # two-grid method of Sec. 4 with the pre-smoothing step of the V-cycle paragraph added).  For
    # Galerkin A_c = R A P, which turns the coarse correction into the paper's
    # I - P (P^T A P)^-1 P^T A.  P is T(p) K with K the down-sampling of Sec. 4.1 for either parity.
    op = _c2_op(n)
    cn = mg.default_coarsest(n, n)
    levels = (mg.geometric_hierarchy(op) if variant == "geometric"
              else mg.galerkin_hierarchy_dense(op, cn))
    assert len(levels) == 2
    vc = mg.VCycle(levels, omega=0.7)
    A = op.dense()
    P = mg.prolong_2d_dense(n, n)
    Ac = levels[1].dense()
    S = _smoother(A, 0.7)
    expect = S @ (np.eye(A.shape[0]) - P @ np.linalg.solve(Ac, 0.25 * P.T @ A)) @ S
    got = np.eye(A.shape[0]) - _cycle_matrix(vc) @ A
    np.testing.assert_allclose(got, expect, rtol=0, atol=1e-12)
    if variant == "galerkin":
        tgm = mg.tgm_iteration_matrix(A, P, 0.7, 1) @ S
        np.testing.assert_allclose(got, tgm, rtol=0, atol=1e-12)


def test_three_level_vcycle_follows_the_recursion():
    # Three levels (31 -> 15 -> 7) with two pre- and one post-sweep and omega = 0.6: the coarse
    # problem is solved by the next cycle, whose map is B_1 = (I - E_1) A_1^-1, so
    # E_0 = S^1 (I - P B_1 R A_0) S^2 and E_1 = S_1 (I - P A_2^-1 R A_1) S_1^2.  A dropped or extra
    # smoothing step, a missing correction or a wrong transfer scaling breaks the equality.
    op = _c2_op(31)
    levels = mg.geometric_hierarchy(op)
    assert [L.n1 for L in levels] == [31, 15, 7]
    vc = mg.VCycle(levels, omega=0.6, nu_pre=2, nu_post=1)
    A0, A1, A2 = levels[0].dense(), levels[1].dense(), levels[2].dense()
    P0, P1 = mg.prolong_2d_dense(31, 31), mg.prolong_2d_dense(15, 15)
    S0, S1 = _smoother(A0, 0.6), _smoother(A1, 0.6)
    I0, I1 = np.eye(A0.shape[0]), np.eye(A1.shape[0])
    E1 = S1 @ (I1 - P1 @ np.linalg.solve(A2, 0.25 * P1.T @ A1)) @ S1 @ S1
    B1 = (I1 - E1) @ np.linalg.inv(A1)
    E0 = S0 @ (I0 - P0 @ B1 @ (0.25 * P0.T @ A0)) @ S0 @ S0
    got = I0 - _cycle_matrix(vc) @ A0
    np.testing.assert_allclose(got, E0, rtol=0, atol=1e-11)
