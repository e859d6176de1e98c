"""Right-preconditioned flexible GMRES (the Krylov solver of paper Sec. 4.3 and Sec. 5).

Test infrastructure (see the package header).  Pinned (tests/test_oracle_krylov.py) by agreement
with a dense LU solve, by the exact solution in at most N iterations on small systems without
preconditioning, and by the minimal-residual property: the residual estimate equals the true
residual of the iterate and never increases.

The paper uses MATLAB's gmres with restart 20 and zero initial guess per time step (Sec. 5).  The
preconditioner is one multigrid cycle, which is a fixed linear map, so plain right preconditioning
would do; the flexible form (storing z_j = M^-1 v_j) is used because it is also valid when the
preconditioner is applied in reduced precision.  Orthogonalisation here is modified Gram-Schmidt
and the small least-squares problem is solved with a library least-squares routine at every step,
so nothing is shared with an implementation that uses classical Gram-Schmidt and Givens rotations.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Callable, Optional

import numpy as np


@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    cycles: int
    converged: bool
    relres: float


def fgmres(apply_A: Callable[[np.ndarray], np.ndarray], b: np.ndarray,
           precond: Optional[Callable[[np.ndarray], np.ndarray]] = None, rtol: float = 1e-10,
           restart: int = 20, maxit: int = 500, x0: Optional[np.ndarray] = None) -> GmresResult:
    """Solve A x = b; stop when the true residual satisfies ||b - A x|| <= rtol ||b||."""
    shape = b.shape
    bv = b.ravel()
    M = precond if precond is not None else (lambda v: v)
    x = np.zeros_like(bv) if x0 is None else x0.ravel().copy()
    bnorm = np.linalg.norm(bv)
    if bnorm == 0.0:
        return GmresResult(x.reshape(shape), 0, 0, True, 0.0)
    total, cycles = 0, 0
    while True:
        r = bv - apply_A(x.reshape(shape)).ravel()
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm or total >= maxit:
            return GmresResult(x.reshape(shape), total, cycles, beta <= rtol * bnorm, beta / bnorm)
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        y = np.zeros(0)
        for j in range(restart):
            z = M(V[j].reshape(shape)).ravel()
            Z.append(z)
            w = apply_A(z.reshape(shape)).ravel()
            for i in range(j + 1):  # modified Gram-Schmidt
                H[i, j] = np.dot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            total += 1
            rhs = np.zeros(j + 2)
            rhs[0] = beta
            y, *_ = np.linalg.lstsq(H[:j + 2, :j + 1], rhs, rcond=None)
            est = np.linalg.norm(rhs - H[:j + 2, :j + 1] @ y)
            if H[j + 1, j] == 0.0 or est <= rtol * bnorm or total >= maxit:
                break
            V.append(w / H[j + 1, j])
        x = x + np.column_stack(Z) @ y
        cycles += 1
