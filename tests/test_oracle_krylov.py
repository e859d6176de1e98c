"""Pins of the oracle's flexible GMRES."""
import numpy as np

import workloads
from oracle import multigrid as mg
from oracle.krylov import fgmres
from oracle.operator import operator_from_problem


def test_fgmres_solves_dense_system_exactly_within_n_steps():
    rng = np.random.default_rng(0)
    N = 40
    A = np.eye(N) * 4 + rng.standard_normal((N, N)) * 0.3
    b = rng.standard_normal((N,))
    res = fgmres(lambda v: A @ v, b, rtol=1e-13, restart=N, maxit=N)
    assert res.converged and res.iters <= N
    np.testing.assert_allclose(res.x, np.linalg.solve(A, b), rtol=1e-11, atol=1e-12)


def test_fgmres_restarted_reports_true_residual():
    rng = np.random.default_rng(1)
    N = 60
    A = np.eye(N) * 3 + rng.standard_normal((N, N)) * 0.3
    b = rng.standard_normal((N,))
    res = fgmres(lambda v: A @ v, b, rtol=1e-12, restart=5, maxit=400)
    assert res.converged and res.cycles > 1
    true = np.linalg.norm(b - A @ res.x) / np.linalg.norm(b)
    assert abs(true - res.relres) < 1e-15 and true <= 1e-12


def test_mg_preconditioned_fgmres_matches_lu():
    p = workloads.config_c2(31, 32)
    op = operator_from_problem(p, 0.0)
    b = np.random.default_rng(2).standard_normal((31, 31))
    vc = mg.VCycle(mg.geometric_hierarchy(op))
    res = fgmres(op.apply, b, vc, rtol=1e-12, restart=20)
    x = np.linalg.solve(op.dense(), b.ravel()).reshape(31, 31)
    assert res.converged and res.iters < 30
    assert np.linalg.norm(res.x - x) <= 1e-10 * np.linalg.norm(x)
