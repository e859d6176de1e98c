"""Multigrid pieces of paper Sec. 4: transfer operators, damped Jacobi, coarse operators, V-cycle.

Test infrastructure (see the package header).  Pins (tests/test_oracle_multigrid.py): the
prolongation equals T(p) K with p = (1+cos t1)(1+cos t2) (Sec. 4.1, Lemma (lemapp)) built from its
Fourier coefficients; bilinear interpolation reproduces linear functions exactly; full weighting
has unit row sums away from the boundary; for the g = 2 (Laplacian) weights the 1-D Galerkin
coarse operator equals the rediscretised one; the two-grid iteration matrix of Sec. 4 has spectral
radius < 1 and the V-cycle contraction stays flat as n grows (Theorem (theorem21bis)); the
composed Galerkin apply equals the dense triple product P^T A P / 4.

Readings of the paper used here (each is listed with its reason in the design notes):
* grid sizes n = 2^l - 1 or n = 2^l with k = (n - n mod 2)/2 coarse points; coarse index j sits at
  fine index i = 2j - (n+1) mod 2 (1-based), i.e. fine 2J + 1 (odd n) or 2J (even n), 0-based
  (Sec. 4.1, the down-sampling matrix K);
* restriction R = P^T / 4 (2-D full weighting: "a proper scaling of the symbol p", Sec. 4.2);
* coarse levels keep the unscaled form I - tau/2 L_l; geometric levels rediscretise with h doubled
  and the coefficient fields injected (sampled at the coarse points), Sec. 4.2;
* Galerkin levels are R A P (TGM step 3, Sec. 4);
* damped Jacobi with the pointwise diagonal of the level matrix, omega = 0.7, one pre- and one
  post-smoothing step, zero initial guess on every coarse level (Sec. 4, V-cycle paragraph;
  Sec. 4.2 settings); the coarsest grid is the paper's 8 x 8: 8 x 8 points when both sides are
  even, 7 x 7 interior points (8 x 8 cells) otherwise, solved exactly.
"""
from __future__ import annotations

from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla

from .operator import Operator


# ----------------------------------------------------------------------------------------------
# Transfer operators
# ----------------------------------------------------------------------------------------------
def coarse_size(n: int) -> int:
    """k = (n - n mod 2) / 2 (Sec. 4.1)."""
    if n < 2:
        raise ValueError("multigrid needs n >= 2")
    return (n - n % 2) // 2


def default_coarsest(n1: int, n2: int) -> int:
    """The paper's 8 x 8 coarsest grid (Sec. 4.2): 8 when both sides are even, else 7."""
    return 8 if (n1 % 2 == 0 and n2 % 2 == 0) else 7


def downsample_1d(n: int) -> np.ndarray:
    """K^k_n of Sec. 4.1: [K]_{i,j} = 1 iff i = 2j - (n+1) mod 2 (1-based); n odd gives i = 2j."""
    k = (n - (n % 2)) // 2
    K = np.zeros((n, k))
    for j in range(1, k + 1):
        i = 2 * j - ((n + 1) % 2)
        K[i - 1, j - 1] = 1.0
    return K


def tau_matrix_p1d(n: int) -> np.ndarray:
    """T_n(1 + cos t): Fourier coefficients 1 (order 0) and 1/2 (orders +-1)."""
    return np.eye(n) + 0.5 * np.eye(n, k=1) + 0.5 * np.eye(n, k=-1)


def prolong_1d(n: int) -> np.ndarray:
    """P_n = T_n(1 + cos t) K^k_n (the 1-D factor of P_N = T_N(p) U_N^k, Sec. 4.1)."""
    return tau_matrix_p1d(n) @ downsample_1d(n)


def prolong_2d_dense(n1: int, n2: int) -> np.ndarray:
    """P_N = P_{n2} kron P_{n1} for the x-fastest ordering (U_N^k = K kron K)."""
    return np.kron(prolong_1d(n2), prolong_1d(n1))


def prolong(E: np.ndarray, n1: int, n2: int) -> np.ndarray:
    """P applied to a coarse field E of shape (k2, k1): fine field (n2, n1)."""
    return prolong_1d(n2) @ E @ prolong_1d(n1).T


def restrict(R: np.ndarray, n1: int, n2: int) -> np.ndarray:
    """R = P^T / 4 applied to a fine field of shape (n2, n1)."""
    return 0.25 * (prolong_1d(n2).T @ R @ prolong_1d(n1))


# ----------------------------------------------------------------------------------------------
# Geometric hierarchy (Sec. 4.2: rediscretisation on the coarser grid)
# ----------------------------------------------------------------------------------------------
def geometric_hierarchy(op0: Operator, coarsest_n: Optional[int] = None) -> List[Operator]:
    if coarsest_n is None:
        coarsest_n = default_coarsest(op0.n1, op0.n2)
    levels = [op0]
    while min(levels[-1].n1, levels[-1].n2) > coarsest_n:
        f = levels[-1]
        k1, k2 = coarse_size(f.n1), coarse_size(f.n2)
        # injection: coarse point j is fine point 2j - (n+1) mod 2 (1-based), i.e. 0-based rows
        # (columns) 1, 3, 5, ... of an odd side and 0, 2, 4, ... of an even one
        o1, o2 = f.n1 % 2, f.n2 % 2
        inj = lambda a: np.ascontiguousarray(a[o2::2, o1::2][:k2, :k1])
        levels.append(Operator(f.alpha, f.beta, k1, k2, 2.0 * f.hx, 2.0 * f.hy, f.tau,
                               inj(f.dp), inj(f.dm), inj(f.ep), inj(f.em)))
    return levels


# ----------------------------------------------------------------------------------------------
# Galerkin hierarchy (TGM step 3: A_k = P^T A P, scaled by the 1/4 of R)
# ----------------------------------------------------------------------------------------------
class DenseLevel:
    """A level given by an explicit matrix (used for the dense Galerkin hierarchy on small grids)."""

    def __init__(self, A: np.ndarray, n1: int, n2: int):
        self.A, self.n1, self.n2 = A, n1, n2

    def apply(self, U):
        return (self.A @ U.ravel()).reshape(self.n2, self.n1)

    def diag(self):
        return np.diag(self.A).reshape(self.n2, self.n1).copy()

    def dense(self):
        return self.A


def galerkin_hierarchy_dense(op0: Operator, coarsest_n: int = 7) -> List:
    """Levels with A_{l+1} = R A_l P, R = P^T/4, computed as dense triple products."""
    levels = [op0]
    A = op0.dense()
    n1, n2 = op0.n1, op0.n2
    while min(n1, n2) > coarsest_n:
        P = prolong_2d_dense(n1, n2)
        A = 0.25 * (P.T @ A @ P)
        n1, n2 = coarse_size(n1), coarse_size(n2)
        levels.append(DenseLevel(A, n1, n2))
    return levels


class ComposedGalerkinLevel:
    """A_l = R_l ... R_1 A_0 P_1 ... P_l applied by composition (any grid size)."""

    def __init__(self, op0: Operator, depth: int):
        self.op0, self.depth = op0, depth
        self.sizes = [(op0.n1, op0.n2)]
        for _ in range(depth):
            a, b = self.sizes[-1]
            self.sizes.append((coarse_size(a), coarse_size(b)))
        self.n1, self.n2 = self.sizes[-1]

    def apply(self, E):
        F = E
        for l in range(self.depth, 0, -1):
            n1, n2 = self.sizes[l - 1]
            F = prolong(F, n1, n2)
        F = self.op0.apply(F)
        for l in range(1, self.depth + 1):
            n1, n2 = self.sizes[l - 1]
            F = restrict(F, n1, n2)
        return F

    def dense(self):
        N = self.n1 * self.n2
        A = np.empty((N, N))
        for c in range(N):
            e = np.zeros(N)
            e[c] = 1.0
            A[:, c] = self.apply(e.reshape(self.n2, self.n1)).ravel()
        return A

    def diag(self):
        """diag_c = e_c^T A_l e_c, evaluated on the support of the composite hat P^ e_c only."""
        op = self.op0
        H = 2 ** self.depth
        hat = 1.0 - np.abs(np.arange(-H + 1, H)) / H  # composite 1-D hat, half-width H
        out = np.empty((self.n2, self.n1))
        for J in range(self.n2):
            fj = H * (J + 1) - 1  # 0-based fine index of coarse point J
            ys = np.arange(fj - H + 1, fj + H)
            for I in range(self.n1):
                fi = H * (I + 1) - 1
                xs = np.arange(fi - H + 1, fi + H)
                Tx = op.Tx[np.ix_(xs, xs)]
                Ty = op.Ty[np.ix_(ys, ys)]
                hx_, hy_ = hat, hat
                P = np.outer(hy_, hx_)
                sub = lambda a: a[np.ix_(ys, xs)]
                LP = (sub(op.dp) * np.outer(hy_, Tx @ hx_) + sub(op.dm) * np.outer(hy_, Tx.T @ hx_)
                      + sub(op.ep) * np.outer(Ty @ hy_, hx_) + sub(op.em) * np.outer(Ty.T @ hy_, hx_))
                AP = P - 0.5 * op.tau * LP
                out[J, I] = np.sum(P * AP) / (4.0 ** self.depth)
        return out


def galerkin_hierarchy_composed(op0: Operator, coarsest_n: int = 7) -> List:
    levels = [op0]
    depth = 0
    n1, n2 = op0.n1, op0.n2
    while min(n1, n2) > coarsest_n:
        depth += 1
        n1, n2 = coarse_size(n1), coarse_size(n2)
        levels.append(ComposedGalerkinLevel(op0, depth))
    return levels


# ----------------------------------------------------------------------------------------------
# Smoother, V-cycle, two-grid
# ----------------------------------------------------------------------------------------------
def jacobi(level, B: np.ndarray, X: np.ndarray, omega: float, Dinv: Optional[np.ndarray] = None):
    """One damped-Jacobi step x <- x + omega D^-1 (b - A x), D = diag(A) (Lemma (lemsmo))."""
    if Dinv is None:
        Dinv = 1.0 / level.diag()
    return X + omega * Dinv * (B - level.apply(X))


class VCycle:
    """One V(nu_pre, nu_post) cycle with zero initial guess on every level (Sec. 4, Sec. 4.2)."""

    def __init__(self, levels: List, omega: float = 0.7, nu_pre: int = 1, nu_post: int = 1):
        self.levels, self.omega, self.nu_pre, self.nu_post = levels, omega, nu_pre, nu_post
        self.Dinv = [1.0 / L.diag() for L in levels[:-1]]
        c = levels[-1]
        self.coarse_lu = sla.lu_factor(c.dense())

    def _solve_coarse(self, B):
        c = self.levels[-1]
        return sla.lu_solve(self.coarse_lu, B.ravel()).reshape(c.n2, c.n1)

    def cycle(self, B: np.ndarray, l: int = 0) -> np.ndarray:
        if l == len(self.levels) - 1:
            return self._solve_coarse(B)
        A, Dinv = self.levels[l], self.Dinv[l]
        X = np.zeros_like(B)
        for _ in range(self.nu_pre):
            X = jacobi(A, B, X, self.omega, Dinv)
        Rr = restrict(B - A.apply(X), A.n1, A.n2)
        E = self.cycle(Rr, l + 1)
        X = X + prolong(E, A.n1, A.n2)
        for _ in range(self.nu_post):
            X = jacobi(A, B, X, self.omega, Dinv)
        return X

    __call__ = cycle


def tgm_iteration_matrix(A: np.ndarray, P: np.ndarray, omega: float, nu: int) -> np.ndarray:
    """S^nu [I - P (P^T A P)^-1 P^T A] with S = I - omega D^-1 A (Sec. 4, TGM iteration matrix)."""
    N = A.shape[0]
    S = np.eye(N) - omega * (A / np.diag(A)[:, None])
    CGC = np.eye(N) - P @ np.linalg.solve(P.T @ A @ P, P.T @ A)
    return np.linalg.matrix_power(S, nu) @ CGC


def vcycle_iteration_matrix(vc: VCycle) -> np.ndarray:
    """I - V A, where V is the (linear) V-cycle map b -> x."""
    L0 = vc.levels[0]
    N = L0.n1 * L0.n2
    A = L0.dense()
    V = np.empty((N, N))
    for c in range(N):
        e = np.zeros(N)
        e[c] = 1.0
        V[:, c] = vc(e.reshape(L0.n2, L0.n1)).ravel()
    return np.eye(N) - V @ A


# ----------------------------------------------------------------------------------------------
# Multigrid as a stand-alone solver (the V-cycle iteration of Sec. 4 without a Krylov method)
# ----------------------------------------------------------------------------------------------
def mg_solve(apply_A, b: np.ndarray, vc: VCycle, rtol: float, max_cycles: int):
    """x_{k+1} = x_k + V(b - A x_k) from x_0 = 0 until ||b - A x||_2 <= rtol ||b||_2.

    Returns (x, cycles, residual norms [||r_0||, ||r_1||, ...]).  The error propagates with the
    iteration matrix I - V A, so the residual ratios approach its spectral radius."""
    x = np.zeros_like(b)
    r = b.copy()
    hist = [float(np.linalg.norm(r))]
    target = rtol * hist[0]
    k = 0
    while k < max_cycles and hist[-1] > target:
        x = x + vc(r)
        r = b - apply_A(x)
        hist.append(float(np.linalg.norm(r)))
        k += 1
    return x, k, hist
