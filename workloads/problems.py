"""Problem descriptions: grids, coefficient fields, manufactured solutions, sources and noise.

The model problem is the 2-D two-sided space-fractional diffusion equation (paper Sec. 2, eq. (1)):

    u_t = d+ D+^alpha u + d- D-^alpha u + e+ D+^beta u + e- D-^beta u + v   on (a1,b1)x(a2,b2),

with zero Dirichlet data and Riemann-Liouville derivatives (Sec. 2, the definitions after eq. (1)).
The grid has n1 x n2 interior points, x_i = a1 + i*hx with hx = (b1-a1)/(n1+1), i = 1..n1 (likewise y),
and M time steps of size tau = T/M (Sec. 2, grid definition).

Every field is returned as a float64 array of shape (n2, n1): row j is y_{j+1}, column i is x_{i+1},
i.e. x varies fastest, which is the lexicographic vector ordering of Sec. 2 (vectors u, d, e, v).

Manufactured solutions are separable, u = phi(t) X(x) Y(y), with X, Y polynomials that vanish to
second order at both ends of the interval.  Their fractional derivatives follow from the power rule
of the Riemann-Liouville operators,

    D+^g (x-a)^p = Gamma(p+1)/Gamma(p+1-g) (x-a)^(p-g),
    D-^g (b-x)^p = Gamma(p+1)/Gamma(p+1-g) (b-x)^(p-g),

applied to the expansion of X in powers of (x-a) and of (b-x).  The source is then
v = u_t - (d+ D+^alpha u + d- D-^alpha u + e+ D+^beta u + e- D-^beta u), which is how the paper's
examples define theirs (Sec. 5: "the source term is such that the solution is ...").
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional, Sequence

import numpy as np
from numpy.polynomial import Polynomial
from scipy.special import gamma as _Gamma

Field3 = Callable[[np.ndarray, np.ndarray, float], np.ndarray]


# ----------------------------------------------------------------------------------------------
# Riemann-Liouville derivatives of polynomials (closed form, Sec. 2 definitions)
# ----------------------------------------------------------------------------------------------
def _rl_power_sum(coef_s: np.ndarray, g: float, s: np.ndarray) -> np.ndarray:
    """sum_p c_p Gamma(p+1)/Gamma(p+1-g) s^(p-g) for s > 0 (the power rule, term by term)."""
    s = np.asarray(s, dtype=np.float64)
    out = np.zeros_like(s)
    for p, c in enumerate(coef_s):
        if c == 0.0:
            continue
        out += c * _Gamma(p + 1.0) / _Gamma(p + 1.0 - g) * np.power(s, p - g)
    return out


def poly_rl_left(poly: Polynomial, g: float, x: np.ndarray, a: float) -> np.ndarray:
    """Left-sided RL derivative of order g of the polynomial `poly` (variable x) on (a, .)."""
    coef = poly(Polynomial([a, 1.0])).coef  # poly(a + s) as a polynomial in s = x - a
    return _rl_power_sum(coef, g, np.asarray(x) - a)


def poly_rl_right(poly: Polynomial, g: float, x: np.ndarray, b: float) -> np.ndarray:
    """Right-sided RL derivative of order g of the polynomial `poly` (variable x) on (., b)."""
    coef = poly(Polynomial([b, -1.0])).coef  # poly(b - s) as a polynomial in s = b - x
    return _rl_power_sum(coef, g, b - np.asarray(x))


# ----------------------------------------------------------------------------------------------
# Problem container
# ----------------------------------------------------------------------------------------------
@dataclass
class Problem:
    name: str
    alpha: float
    beta: float
    n1: int
    n2: int
    a1: float
    b1: float
    a2: float
    b2: float
    T: float
    M: int
    dp: Field3
    dm: Field3
    ep: Field3
    em: Field3
    u0: Callable[[np.ndarray, np.ndarray], np.ndarray]
    source: Field3
    u_exact: Optional[Field3] = None
    coeffs_time_dependent: bool = False
    noise_seed: Optional[int] = None
    # separable description of the source for device-side evaluation:
    # v(x,y,t) = sum_k phi_k(t) * S_k(x,y); S_k sampled on the grid by `source_terms`.
    source_phis: List[Callable[[float], float]] = field(default_factory=list)
    source_fields: List[Callable[[np.ndarray, np.ndarray], np.ndarray]] = field(default_factory=list)

    @property
    def tau(self) -> float:
        return self.T / self.M

    @property
    def hx(self) -> float:
        return (self.b1 - self.a1) / (self.n1 + 1)

    @property
    def hy(self) -> float:
        return (self.b2 - self.a2) / (self.n2 + 1)

    @property
    def N(self) -> int:
        return self.n1 * self.n2


def grid(p: Problem):
    """Interior grid points as (X, Y) arrays of shape (n2, n1)."""
    x = p.a1 + p.hx * np.arange(1, p.n1 + 1, dtype=np.float64)
    y = p.a2 + p.hy * np.arange(1, p.n2 + 1, dtype=np.float64)
    Y, X = np.meshgrid(y, x, indexing="ij")
    return X, Y


def sample(p: Problem, t: float):
    """Coefficient fields (d+, d-, e+, e-) at time t, each (n2, n1) float64, C-contiguous."""
    X, Y = grid(p)
    out = []
    for f in (p.dp, p.dm, p.ep, p.em):
        a = np.ascontiguousarray(np.broadcast_to(f(X, Y, t), X.shape), dtype=np.float64)
        out.append(a)
    return tuple(out)


def sample_u0(p: Problem) -> np.ndarray:
    X, Y = grid(p)
    return np.ascontiguousarray(p.u0(X, Y), dtype=np.float64)


def sample_source(p: Problem, t: float) -> np.ndarray:
    """v(x_i, y_j, t) including the seeded noise field when the problem has one."""
    X, Y = grid(p)
    v = np.ascontiguousarray(p.source(X, Y, t), dtype=np.float64)
    if p.noise_seed is not None:
        v = v + noise_field(p.noise_seed, p.n1, p.n2)
    return v


def source_terms(p: Problem):
    """Separable form v(t) = sum_k phi_k(t) S_k: returns ([phi_k], [S_k sampled]) incl. noise."""
    X, Y = grid(p)
    fields = [np.ascontiguousarray(f(X, Y), dtype=np.float64) for f in p.source_fields]
    phis = list(p.source_phis)
    if p.noise_seed is not None:
        fields.append(noise_field(p.noise_seed, p.n1, p.n2))
        phis.append(lambda t: 1.0)
    return phis, fields


def noise_field(seed: int, n1: int, n2: int) -> np.ndarray:
    """Seeded i.i.d. N(0,1) field, NumPy PCG64, row-major (n2, n1)."""
    return np.random.default_rng(seed).standard_normal((n2, n1))


# ----------------------------------------------------------------------------------------------
# Separable manufactured solution u = phi(t) X(x) Y(y)
# ----------------------------------------------------------------------------------------------
def _manufactured(alpha, beta, a1, b1, a2, b2, Xp: Polynomial, Yp: Polynomial,
                  phi: Callable[[float], float], dphi: Callable[[float], float],
                  dp: Field3, dm: Field3, ep: Field3, em: Field3, coeff_t_dep: bool):
    def u_exact(x, y, t):
        return phi(t) * Xp(x) * Yp(y)

    def u0(x, y):
        return phi(0.0) * Xp(x) * Yp(y)

    def _spatial(x, y, t):
        Xv, Yv = Xp(x), Yp(y)
        dXp = poly_rl_left(Xp, alpha, x, a1)
        dXm = poly_rl_right(Xp, alpha, x, b1)
        dYp = poly_rl_left(Yp, beta, y, a2)
        dYm = poly_rl_right(Yp, beta, y, b2)
        return (dp(x, y, t) * dXp * Yv + dm(x, y, t) * dXm * Yv
                + ep(x, y, t) * Xv * dYp + em(x, y, t) * Xv * dYm)

    def source(x, y, t):
        return dphi(t) * Xp(x) * Yp(y) - phi(t) * _spatial(x, y, t)

    phis: List = []
    fields: List = []
    if not coeff_t_dep:
        # v(t) = phi'(t) X Y - phi(t) * spatial(x, y): two separable terms.
        phis = [dphi, phi]
        fields = [lambda x, y: Xp(x) * Yp(y), lambda x, y: -_spatial(x, y, 0.0)]
    return u_exact, u0, source, phis, fields


def _exp_decay(scale: float = 1.0):
    return (lambda t: scale * np.exp(-t)), (lambda t: -scale * np.exp(-t))


# X(x) = x^2 (1-x)^2 on [0, 1]
_P_X2_1MX2 = Polynomial([0.0, 0.0, 1.0, -2.0, 1.0])
# X(x) = x^3 (1-x)^3 on [0, 1]
_P_X3_1MX3 = Polynomial([0.0, 0.0, 0.0, 1.0, -3.0, 3.0, -1.0])
# X(x) = x^2 (2-x)^2 on [0, 2]
_P_X2_2MX2 = Polynomial([0.0, 0.0, 4.0, -4.0, 1.0])


def _build(name, alpha, beta, n1, n2, dom, T, M, dp, dm, ep, em, Xp, Yp, phi, dphi,
           coeff_t_dep=False, noise_seed=None) -> Problem:
    a1, b1, a2, b2 = dom
    u_exact, u0, source, phis, fields = _manufactured(alpha, beta, a1, b1, a2, b2, Xp, Yp, phi,
                                                      dphi, dp, dm, ep, em, coeff_t_dep)
    return Problem(name=name, alpha=alpha, beta=beta, n1=n1, n2=n2, a1=a1, b1=b1, a2=a2, b2=b2,
                   T=T, M=M, dp=dp, dm=dm, ep=ep, em=em, u0=u0, source=source, u_exact=u_exact,
                   coeffs_time_dependent=coeff_t_dep, noise_seed=noise_seed,
                   source_phis=phis, source_fields=fields)


# ----------------------------------------------------------------------------------------------
# The paper's three examples (Sec. 5), at the paper's even sizes n1 = n2 = M = n
# ----------------------------------------------------------------------------------------------
def example1(n: int, M: Optional[int] = None) -> Problem:
    """Example 1 (Sec. 5.1): alpha=1.8, beta=1.6 on [0,2]^2, u = 16 e^-t x^2(2-x)^2 y^2(2-y)^2.

    The initial condition is taken as u(.,.,0) including the factor 16 (the printed u0 omits it;
    the printed second-order error sequence is only possible with the consistent u0).
    """
    al, be = 1.8, 1.6
    ga, gb = _Gamma(3 - al), _Gamma(3 - be)
    dp = lambda x, y, t: ga * (1 + x) ** al * (1 + y) ** 2
    dm = lambda x, y, t: ga * (3 - x) ** al * (3 - y) ** 2
    ep = lambda x, y, t: gb * (1 + x) ** 2 * (1 + y) ** be
    em = lambda x, y, t: gb * (3 - x) ** 2 * (3 - y) ** be
    phi, dphi = _exp_decay(16.0)
    return _build("example1", al, be, n, n, (0.0, 2.0, 0.0, 2.0), 1.0, M or n, dp, dm, ep, em,
                  _P_X2_2MX2, _P_X2_2MX2, phi, dphi)


def example2(n: int, M: Optional[int] = None) -> Problem:
    """Example 2 (Sec. 5.2): alpha=1.8, beta=1.9, time-dependent coefficients 4(1+t)...."""
    al, be = 1.8, 1.9
    dp = lambda x, y, t: 4 * (1 + t) * x ** al * (1 + y)
    dm = lambda x, y, t: 4 * (1 + t) * (1 - x) ** al * (1 + y)
    ep = lambda x, y, t: 4 * (1 + t) * (1 + x) * y ** be
    em = lambda x, y, t: 4 * (1 + t) * (1 + x) * (1 - y) ** be
    phi, dphi = _exp_decay(1.0)
    return _build("example2", al, be, n, n, (0.0, 1.0, 0.0, 1.0), 1.0, M or n, dp, dm, ep, em,
                  _P_X3_1MX3, _P_X3_1MX3, phi, dphi, coeff_t_dep=True)


def example3(n: int, M: Optional[int] = None) -> Problem:
    """Example 3 (Sec. 5.3): alpha=1.8, beta=1.9, coefficients 6x^alpha, 6(1-x)^alpha, ...."""
    al, be = 1.8, 1.9
    dp = lambda x, y, t: 6 * x ** al + 0 * y
    dm = lambda x, y, t: 6 * (1 - x) ** al + 0 * y
    ep = lambda x, y, t: 6 * y ** be + 0 * x
    em = lambda x, y, t: 6 * (1 - y) ** be + 0 * x
    phi, dphi = _exp_decay(1.0)
    return _build("example3", al, be, n, n, (0.0, 1.0, 0.0, 1.0), 1.0, M or n, dp, dm, ep, em,
                  _P_X3_1MX3, _P_X3_1MX3, phi, dphi)


# ----------------------------------------------------------------------------------------------
# Benchmark workloads (synthetic, shaped like the paper's examples)
# ----------------------------------------------------------------------------------------------
_UNIT = (0.0, 1.0, 0.0, 1.0)


def _const(c):
    return lambda x, y, t: c + 0.0 * x + 0.0 * y


def _c2_coeffs():
    dp = lambda x, y, t: 1 + x + y ** 2
    dm = lambda x, y, t: 2 - x + y
    ep = lambda x, y, t: 1 + x * y
    em = lambda x, y, t: 1.5 + 0.5 * np.sin(np.pi * x) * y
    return dp, dm, ep, em


def config_c1(n: int = 63, M: Optional[int] = None) -> Problem:
    """Constant coefficients d+-=e+-=1, alpha=beta=1.5, unit square, u = x^2(1-x)^2 y^2(1-y)^2 e^-t."""
    phi, dphi = _exp_decay(1.0)
    return _build("c1", 1.5, 1.5, n, n, _UNIT, 1.0, M or (n + 1), _const(1.0), _const(1.0),
                  _const(1.0), _const(1.0), _P_X2_1MX2, _P_X2_1MX2, phi, dphi)


def config_c2(n: int = 511, M: int = 32, seed: Optional[int] = 2) -> Problem:
    """Variable coefficients, alpha=1.8, beta=1.6, n=511, tau=1/32, manufactured + seeded noise."""
    phi, dphi = _exp_decay(1.0)
    dp, dm, ep, em = _c2_coeffs()
    return _build("c2", 1.8, 1.6, n, n, _UNIT, 1.0, M, dp, dm, ep, em, _P_X2_1MX2, _P_X2_1MX2,
                  phi, dphi, noise_seed=seed)


def config_c3(n: int = 2047, M: int = 16, seed: Optional[int] = 3) -> Problem:
    """Large anisotropic instance: alpha=1.2, beta=1.9, C2's coefficients, n=2047, tau=1/16."""
    phi, dphi = _exp_decay(1.0)
    dp, dm, ep, em = _c2_coeffs()
    return _build("c3", 1.2, 1.9, n, n, _UNIT, 1.0, M, dp, dm, ep, em, _P_X2_1MX2, _P_X2_1MX2,
                  phi, dphi, noise_seed=seed)


def _abc_coeff(a, b, c):
    return lambda x, y, t: c * (1 + a * x + b * y ** 2)


def random_instance(rng: np.random.Generator, n_choices: Sequence[int], name: str,
                    M: int, noise_seed: Optional[int]) -> Problem:
    """alpha, beta ~ U[1.1,1.9]; each of d+, d-, e+, e- = c(1 + a x + b y^2), (a,b,c) ~ U[0.5,2]^3."""
    n = int(rng.choice(np.asarray(n_choices)))
    alpha, beta = (float(v) for v in rng.uniform(1.1, 1.9, size=2))
    abc = rng.uniform(0.5, 2.0, size=(4, 3))
    dp, dm, ep, em = (_abc_coeff(*abc[k]) for k in range(4))
    phi, dphi = _exp_decay(1.0)
    return _build(name, alpha, beta, n, n, _UNIT, 1.0, M, dp, dm, ep, em, _P_X2_1MX2, _P_X2_1MX2,
                  phi, dphi, noise_seed=noise_seed)


def config_c4_instances(count: int = 64, seed: int = 4, M: int = 8) -> List[Problem]:
    """Batched workload: `count` instances, n uniform over {127, 255, 511}, tau = 1/8."""
    rng = np.random.default_rng(seed)
    return [random_instance(rng, (127, 255, 511), f"c4_{i}", M, seed + 1000 * i)
            for i in range(count)]


@dataclass
class Request:
    problem: Problem
    arrival: float  # seconds after the start of the run


def config_c5_requests(qps: float, count: int = 220, seed: int = 5,
                       ks: Sequence[int] = (6, 7, 8, 9, 10, 11)) -> List[Request]:
    """Serving workload: Poisson arrivals at `qps`; n = 2^k - 1 with k uniform over `ks`;
    M uniform over the integers 8..128 with tau = 1/M.  Request parameters do not depend on qps."""
    prng = np.random.default_rng(seed)
    arng = np.random.default_rng(seed + 777)
    gaps = arng.exponential(1.0, size=count) / qps
    reqs = []
    t = 0.0
    for i in range(count):
        k = int(prng.choice(np.asarray(ks)))
        M = int(prng.integers(8, 129))
        p = random_instance(prng, (2 ** k - 1,), f"c5_{i}", M, seed + 1000 * i)
        t += float(gaps[i])
        reqs.append(Request(problem=p, arrival=t))
    return reqs
