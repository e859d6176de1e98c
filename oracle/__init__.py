"""FP64 CPU oracle for the CN-WSGD / multigrid-preconditioned GMRES solver.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct reference that the
GPU library is checked against.  Only the test suite, the smoke check and the benchmark's CPU
baseline leg may import it; the GPU library never does, and the two share no code (inputs come
from the separate `workloads` package, which holds no solver arithmetic).

Modules, each following the paper (Moghaderi, Dehghan, Donatelli, Mazza, "Spectral analysis and
multigrid preconditioners for two-dimensional space-fractional diffusion equations"):

* `weights`   Grunwald coefficients g_k (eq. (gk)) and WSGD weights w_k (eq. (w)).
* `operator`  the Toeplitz matrix of eq. (AN), the Kronecker operators of eq. (AxAy), the per-step
              system of eq. (system); dense assembly and matrix-product (Kronecker) application.
* `multigrid` bilinear prolongation P = T(p)U (Sec. 4.1, Lemma lemapp), full weighting, damped
              Jacobi (Lemma lemsmo), geometric (rediscretised) and Galerkin (P^T A P) coarse
              operators (Sec. 4.2), the V-cycle, and the two-grid iteration matrix (Sec. 4).
* `krylov`    right-preconditioned flexible GMRES with modified Gram-Schmidt (Sec. 4.3, Sec. 5).
* `cn`        the Crank-Nicolson time loop of eq. (CNWSGD)/(system) with exact or iterative solves.

Parity status of each function is stated in its module header.
"""
