"""Crank-Nicolson time stepping of the CN-WSGD scheme (paper Sec. 2, eqs. (CNWSGD) and (system)).

Test infrastructure (see the package header).  Pinned by second-order convergence in h = tau on a
manufactured solution and by the paper's printed Error columns of Examples 1-3 (Tables (tabel3),
(tabel1), (tabel4)); see tests/test_oracle_convergence.py.

Step m (m = 1..M):  (I - tau/2 L^(m)) u^(m) = (I + tau/2 L^(m-1)) u^(m-1) + tau v^(m-1/2),
with the coefficients of L^(m) sampled at t^(m) and the source at t^(m-1/2) = (m - 1/2) tau.
The linear system is solved either exactly (dense LU, small grids) or with the oracle's own
flexible GMRES preconditioned by its own geometric V-cycle to a tight tolerance.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.linalg as sla

from .krylov import fgmres
from .multigrid import VCycle, geometric_hierarchy
from .operator import Operator, operator_from_problem


@dataclass
class CNResult:
    u: np.ndarray
    iters: List[int] = field(default_factory=list)


def rhs(op_prev: Operator, u_prev: np.ndarray, v_half: Optional[np.ndarray]) -> np.ndarray:
    """b = (I + tau/2 L^(m-1)) u^(m-1) + tau v^(m-1/2)."""
    b = op_prev.rhs(u_prev)
    if v_half is not None:
        b = b + op_prev.tau * v_half
    return b


class DirectSolver:
    """Dense LU of I - tau/2 L; refactored only when the operator changes."""

    def __init__(self):
        self._key, self._lu = None, None

    def __call__(self, op: Operator, b: np.ndarray, key) -> tuple:
        if key is None or key != self._key:
            self._lu = sla.lu_factor(op.dense())
            self._key = key
        return sla.lu_solve(self._lu, b.ravel()).reshape(b.shape), 0


class IterativeSolver:
    """Oracle FGMRES(restart) + oracle geometric V(1,1) cycle, tight tolerance."""

    def __init__(self, rtol: float = 1e-13, restart: int = 50, omega: float = 0.7,
                 coarsest_n: Optional[int] = None, maxit: int = 1000):
        self.rtol, self.restart, self.omega = rtol, restart, omega
        self.coarsest_n, self.maxit = coarsest_n, maxit
        self._key, self._vc = None, None

    def __call__(self, op: Operator, b: np.ndarray, key) -> tuple:
        if key is None or key != self._key:
            self._vc = VCycle(geometric_hierarchy(op, self.coarsest_n), omega=self.omega)
            self._key = key
        res = fgmres(op.apply, b, self._vc, rtol=self.rtol, restart=self.restart,
                     maxit=self.maxit)
        if not res.converged:
            raise RuntimeError(f"oracle FGMRES did not converge (relres {res.relres:.3e})")
        return res.x, res.iters


def cn_run(p, steps: Optional[int] = None, solver=None, u0: Optional[np.ndarray] = None,
           t0: float = 0.0) -> CNResult:
    """Run `steps` (default p.M) CN steps of problem p from u0 (default the sampled initial data)."""
    from workloads import sample_source, sample_u0

    steps = p.M if steps is None else steps
    if solver is None:
        solver = DirectSolver() if p.N <= 4096 else IterativeSolver()
    u = sample_u0(p) if u0 is None else np.array(u0, dtype=np.float64)
    out = CNResult(u=u)
    tdep = p.coeffs_time_dependent
    op_prev = operator_from_problem(p, t0)
    for m in range(1, steps + 1):
        t_prev, t_now = t0 + (m - 1) * p.tau, t0 + m * p.tau
        op_now = operator_from_problem(p, t_now) if tdep else op_prev
        b = rhs(op_prev, u, sample_source(p, t_prev + 0.5 * p.tau))
        u, its = solver(op_now, b, ("t", t_now) if tdep else "static")
        out.iters.append(its)
        op_prev = op_now
    out.u = u
    return out


def solve_step(op: Operator, b: np.ndarray, solver=None) -> np.ndarray:
    """Solve (I - tau/2 L) x = b once (exact for small N, tight iterative otherwise)."""
    if solver is None:
        solver = DirectSolver() if op.n1 * op.n2 <= 4096 else IterativeSolver()
    x, _ = solver(op, b, None)
    return x
