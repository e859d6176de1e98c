"""The CN-WSGD spatial operator and the per-step system (paper Sec. 2).

Test infrastructure (see the package header).  Pins (tests/test_oracle_operator.py): dense
assembly equals the matrix-product (Kronecker) form; the paper's scaled matrix of eq. (M) equals
(1/r) times the unscaled system matrix; symmetric positive definite for constant equal
coefficients; strictly diagonally dominant M-matrix for alpha, beta >= gamma_0; the symbol of
Proposition (pro2) and its bound; O(h^2) consistency of the discrete operator against closed-form
Riemann-Liouville derivatives; second-order convergence of the whole scheme
(tests/test_oracle_convergence.py).

Notation.  Fields are (n2, n1) arrays, x fastest (the lexicographic ordering of Sec. 2).
T_g = [w_{i-j+1}]_{i,j=1..n} with w_k = 0 for k < 0, so the paper's Toeplitz matrix of eq. (AN) is
A^g = -T_g.  The shifted Grunwald sums of Sec. 2 are then

    left  derivative in x:  h^-alpha (I_{n2} kron T_alpha)   u   <->  U @ T_alpha^T / h^alpha
    right derivative in x:  h^-alpha (I_{n2} kron T_alpha^T) u   <->  U @ T_alpha   / h^alpha
    left  derivative in y:  h^-beta  (T_beta kron I_{n1})    u   <->  T_beta   @ U / h^beta
    right derivative in y:  h^-beta  (T_beta^T kron I_{n1})  u   <->  T_beta^T @ U / h^beta

and L u = D+ (left x) + D- (right x) + E+ (left y) + E- (right y), eq. (AxAy) up to the sign of A^g.
The per-step system of eq. (system) is (I - tau/2 L^(m)) u^(m) = (I + tau/2 L^(m-1)) u^(m-1)
+ tau v^(m-1/2); multiplying it by 1/r gives the paper's scaled form M u = b of eqs. (M), (2).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
import scipy.linalg as sla

from .weights import wsgd


def toeplitz_T(g: float, n: int) -> np.ndarray:
    """T_g = [w_{i-j+1}] (n x n): w_1 on the diagonal, w_0 above it, w_{m+1} on the m-th subdiagonal."""
    w = wsgd(g, n)
    first_col = w[1:n + 1]
    first_row = np.zeros(n)
    first_row[0] = w[1]
    if n > 1:
        first_row[1] = w[0]
    return sla.toeplitz(first_col, first_row)


def paper_A(g: float, n: int) -> np.ndarray:
    """The paper's A^g_n of eq. (AN) (= -T_g)."""
    return -toeplitz_T(g, n)


@dataclass
class Operator:
    """One grid level of A = I - tau/2 * L (unscaled form of eq. (system)) with given fields."""

    alpha: float
    beta: float
    n1: int
    n2: int
    hx: float
    hy: float
    tau: float
    dp: np.ndarray
    dm: np.ndarray
    ep: np.ndarray
    em: np.ndarray

    def __post_init__(self):
        self.Tx = toeplitz_T(self.alpha, self.n1) / self.hx ** self.alpha
        self.Ty = toeplitz_T(self.beta, self.n2) / self.hy ** self.beta

    # L u in field form (eq. (AxAy) with A^g = -T_g)
    def L(self, U: np.ndarray) -> np.ndarray:
        return (self.dp * (U @ self.Tx.T) + self.dm * (U @ self.Tx)
                + self.ep * (self.Ty @ U) + self.em * (self.Ty.T @ U))

    def apply(self, U: np.ndarray) -> np.ndarray:
        """A U = U - tau/2 L U."""
        return U - 0.5 * self.tau * self.L(U)

    def rhs(self, U: np.ndarray) -> np.ndarray:
        """(I + tau/2 L) U, the explicit half of the Crank-Nicolson step."""
        return U + 0.5 * self.tau * self.L(U)

    def L_points(self, U: np.ndarray, js, is_) -> np.ndarray:
        """(L U)[j, i] at the listed points only: row j of U against row i of Tx (and Tx^T),
        column i of U against row j of Ty (and Ty^T).  O(n) per point, for very large grids."""
        js, is_ = np.asarray(js), np.asarray(is_)
        out = np.empty(len(js))
        for k, (j, i) in enumerate(zip(js, is_)):
            row, col = U[j, :], U[:, i]
            out[k] = (self.dp[j, i] * (self.Tx[i, :] @ row) + self.dm[j, i] * (self.Tx[:, i] @ row)
                      + self.ep[j, i] * (self.Ty[j, :] @ col) + self.em[j, i] * (self.Ty[:, j] @ col))
        return out

    def apply_points(self, U: np.ndarray, js, is_) -> np.ndarray:
        """(A U)[j, i] = U[j, i] - tau/2 (L U)[j, i] at the listed points."""
        return U[np.asarray(js), np.asarray(is_)] - 0.5 * self.tau * self.L_points(U, js, is_)

    def diag(self) -> np.ndarray:
        """Pointwise diagonal of A: T_g has w_1 on its diagonal."""
        return 1.0 - 0.5 * self.tau * ((self.dp + self.dm) * self.Tx[0, 0]
                                       + (self.ep + self.em) * self.Ty[0, 0])

    def L_dense(self) -> np.ndarray:
        """L as an N x N matrix, N = n1 n2, built with Kronecker products exactly as eq. (AxAy)."""
        I1, I2 = np.eye(self.n1), np.eye(self.n2)
        Lx = (np.diag(self.dp.ravel()) @ np.kron(I2, self.Tx)
              + np.diag(self.dm.ravel()) @ np.kron(I2, self.Tx.T))
        Ly = (np.diag(self.ep.ravel()) @ np.kron(self.Ty, I1)
              + np.diag(self.em.ravel()) @ np.kron(self.Ty.T, I1))
        return Lx + Ly

    def dense(self) -> np.ndarray:
        """A = I - tau/2 L as an N x N matrix."""
        N = self.n1 * self.n2
        return np.eye(N) - 0.5 * self.tau * self.L_dense()

    def paper_scaled_dense(self) -> np.ndarray:
        """The paper's M = 1/r I + A_x + s/r A_y (eq. (M)), assembled from eq. (AN) and (AxAy)."""
        r = self.tau / (2.0 * self.hx ** self.alpha)
        s = self.tau / (2.0 * self.hy ** self.beta)
        I1, I2 = np.eye(self.n1), np.eye(self.n2)
        Aa, Ab = paper_A(self.alpha, self.n1), paper_A(self.beta, self.n2)
        Ax = (np.diag(self.dp.ravel()) @ np.kron(I2, Aa)
              + np.diag(self.dm.ravel()) @ np.kron(I2, Aa.T))
        Ay = (np.diag(self.ep.ravel()) @ np.kron(Ab, I1)
              + np.diag(self.em.ravel()) @ np.kron(Ab.T, I1))
        return np.eye(self.n1 * self.n2) / r + Ax + (s / r) * Ay


def operator_from_problem(p, t: float) -> Operator:
    """The level-0 operator of problem `p` with coefficients sampled at time t."""
    from workloads import sample

    dp, dm, ep, em = sample(p, t)
    return Operator(p.alpha, p.beta, p.n1, p.n2, p.hx, p.hy, p.tau, dp, dm, ep, em)


# ----------------------------------------------------------------------------------------------
# The band (Laplacian) preconditioner of Sec. 4.3
# ----------------------------------------------------------------------------------------------
def laplacian_matrix(n: int) -> np.ndarray:
    """The second-difference matrix tridiag(1, -2, 1) of order n (the Laplacian matrix A^2)."""
    return -2.0 * np.eye(n) + np.eye(n, k=1) + np.eye(n, k=-1)


def band_P2_scaled_dense(op: "Operator") -> np.ndarray:
    """The band preconditioner of Sec. 4.3 assembled as the paper writes it:
    P_x = D+ (I kron A^2) + D- (I kron (A^2)^T), P_y = E+ (A^2 kron I) + E- ((A^2)^T kron I),
    P_2 = (1/r) I - (P_x + (s/r) P_y), with r = tau/(2 hx^alpha), s = tau/(2 hy^beta) the same
    scalings as the system matrix of eq. (M).  Reading: A^2 is the second-difference matrix
    tridiag(1, -2, 1); with that sign P_2 is the alpha = beta = 2 member of the family of eq. (M)
    (whose A^g = -T_g has the positive diagonal -w_1), so it is positive definite like M."""
    r = op.tau / (2.0 * op.hx ** op.alpha)
    s = op.tau / (2.0 * op.hy ** op.beta)
    I1, I2 = np.eye(op.n1), np.eye(op.n2)
    A2x, A2y = laplacian_matrix(op.n1), laplacian_matrix(op.n2)
    Px = np.diag(op.dp.ravel()) @ np.kron(I2, A2x) + np.diag(op.dm.ravel()) @ np.kron(I2, A2x.T)
    Py = np.diag(op.ep.ravel()) @ np.kron(A2y, I1) + np.diag(op.em.ravel()) @ np.kron(A2y.T, I1)
    return np.eye(op.n1 * op.n2) / r - (Px + (s / r) * Py)


class BandOperator(Operator):
    """r P_2 in the unscaled form of the per-step system: I - tau/2 L_2 with L_2 built like L but
    with the Laplacian matrix in place of T_alpha and T_beta and the fractional scalings kept,
    L_2 u = D+ (I kron A^2) u/hx^alpha + D- (I kron (A^2)^T) u/hx^alpha + E+ (A^2 kron I) u/hy^beta
            + E- ((A^2)^T kron I) u/hy^beta.
    Multiplying by r = tau/(2 hx^alpha) turns the paper's P_2 into this matrix, exactly as the
    scaled system matrix M becomes I - tau/2 L (Sec. 4.3, eq. (M))."""

    def __post_init__(self):
        self.Tx = laplacian_matrix(self.n1) / self.hx ** self.alpha
        self.Ty = laplacian_matrix(self.n2) / self.hy ** self.beta


def band_operator(op: "Operator") -> BandOperator:
    """The band preconditioner (unscaled) on the grid and coefficient fields of `op`."""
    return BandOperator(op.alpha, op.beta, op.n1, op.n2, op.hx, op.hy, op.tau,
                        op.dp, op.dm, op.ep, op.em)
