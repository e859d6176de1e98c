"""Grunwald coefficients and WSGD weights (paper Sec. 2, eqs. (gk) and (w), Proposition (ww)).

Test infrastructure (see the package header).  Pinned by tests/test_oracle_weights.py against the
binomial library routine, the generating functions (1-z)^g and (g/2 + (2-g)z/2)(1-z)^g, the closed
forms of w_0, w_1, w_2 and of sum |w_k| (proof of Proposition (pro2)), and the g = 2 Laplacian case.
"""
from __future__ import annotations

import numpy as np


def grunwald(g: float, K: int) -> np.ndarray:
    """g_k = (-1)^k binom(g, k), k = 0..K  (eq. (gk)).

    The binomial is the product g(g-1)...(g-k+1)/k!, so each coefficient is the previous one times
    -(g-k+1)/k.
    """
    out = np.empty(K + 1, dtype=np.float64)
    out[0] = 1.0
    for k in range(1, K + 1):
        out[k] = out[k - 1] * (-(g - k + 1.0) / k)
    return out


def wsgd(g: float, K: int) -> np.ndarray:
    """WSGD weights with shifts (p, q) = (1, 0), k = 0..K  (eq. (w)).

    w_0 = g/2 * g_0 and w_k = g/2 * g_k + (2-g)/2 * g_{k-1} for k >= 1.
    """
    gk = grunwald(g, K)
    w = np.empty(K + 1, dtype=np.float64)
    w[0] = 0.5 * g * gk[0]
    w[1:] = 0.5 * g * gk[1:] + 0.5 * (2.0 - g) * gk[:-1]
    return w
