"""Whole-scheme pins of the oracle: the paper's printed Error columns and second-order convergence.

The expected values in tests/golden/paper_error_tables.json are copied from the paper's Tables
(tabel3), (tabel1) and (tabel4) (Sec. 5).  The paper solved each step with GMRES to 1e-7, so the
discretisation error dominates and an exact per-step solve reproduces the printed digits.
"""
import json
import os

import numpy as np
import pytest

import workloads
from oracle.cn import IterativeSolver, DirectSolver, cn_run

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_error_tables.json")


def _final_error(p, **kw):
    r = cn_run(p, **kw)
    X, Y = workloads.grid(p)
    return np.abs(r.u - p.u_exact(X, Y, p.T)).max()


@pytest.mark.parametrize("name,n", [("example1", 16), ("example1", 32), ("example1", 64),
                                    ("example2", 16), ("example2", 32),
                                    ("example3", 16), ("example3", 32), ("example3", 64)])
def test_paper_error_columns(name, n):
    ref = json.load(open(GOLDEN))[name][str(n)]
    p = getattr(workloads, name)(n)
    err = _final_error(p)
    assert err == pytest.approx(ref, rel=5e-3), (err, ref)


def test_second_order_in_h_equals_tau():
    # Sec. 2: truncation error O(hx^2 + hy^2 + tau^2); with tau = h the error ratio tends to 4.
    errs = []
    for n in (15, 31, 63):
        p = workloads.config_c1(n)  # M = n + 1, tau = h
        errs.append(_final_error(p))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert all(3.6 < r < 4.4 for r in ratios), ratios


def test_iterative_oracle_matches_direct():
    # The tight FGMRES + geometric V-cycle oracle reproduces the dense LU time stepping.
    p = workloads.config_c2(31, 4)
    a = cn_run(p, solver=DirectSolver()).u
    b = cn_run(p, solver=IterativeSolver(rtol=1e-13)).u
    assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(a)


@pytest.mark.parametrize("n", [16, 32])
def test_iterative_oracle_on_even_grids_matches_direct(n):
    # The paper's own grids (n = 2^l, Sec. 5): FGMRES with the even-side V-cycle (coarse point j at
    # fine 2j - 1, 1-based, down to 8 x 8) reproduces the dense LU time stepping.
    p = workloads.example1(n)
    p.M = 4
    a = cn_run(p, solver=DirectSolver()).u
    b = cn_run(p, solver=IterativeSolver(rtol=1e-13)).u
    assert np.linalg.norm(a - b) <= 1e-11 * np.linalg.norm(a)
