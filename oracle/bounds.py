"""Closed-form error bound and success probability of Theorem 4.1
(Shabat et al., arXiv 1310.7202, Section 4, Eq. 4.1 and the probability
formula that follows it; values tabulated in Table 4.1).

TEST INFRASTRUCTURE ONLY: see the package docstring for who may call this.
"""
from __future__ import annotations

import math


def xi(l_minus_k: int, beta: float, gamma: float, n: int) -> float:
    """Success probability of Theorem 4.1 for oversampling l - k, beta > 0,
    gamma > 1 and n columns.  Returns 1 - xi as a float (the table prints
    1 - xi, and 1 - xi is far below the resolution of xi itself)."""
    return one_minus_xi(l_minus_k, beta, gamma, n)


def one_minus_xi(l_minus_k: int, beta: float, gamma: float, n: int) -> float:
    """1 - xi: the first term bounds the chance that the smallest singular
    value of a Gaussian (l-k+1)-column block is too small (controlled by
    beta); the second the chance that ||G|| exceeds sqrt(2n) * gamma
    (controlled by gamma)."""
    if beta <= 0 or gamma <= 1:
        raise ValueError("need beta > 0 and gamma > 1")
    d = l_minus_k + 1
    t1 = (1.0 / math.sqrt(2.0 * math.pi * d)) * (math.e / (d * beta)) ** d
    # second term in log space: (2 g^2 / e^(g^2-1))^n underflows quickly
    g2 = gamma * gamma
    log_base = math.log(2.0 * g2) - (g2 - 1.0)
    log_t2 = n * log_base - math.log(4.0 * (g2 - 1.0) * math.sqrt(math.pi * n * g2))
    t2 = math.exp(log_t2) if log_t2 > -745 else 0.0
    return t1 + t2


def rand_lu_bound(n: int, k: int, l: int, beta: float, gamma: float) -> float:
    """Theorem 4.1: ||L U - P A Q|| <= C * sigma_{k+1}(A); returns C."""
    c1 = 2.0 * math.sqrt(2.0 * n * l * beta ** 2 * gamma ** 2 + 1.0)
    c2 = 2.0 * math.sqrt(2.0 * n * l) * beta * gamma * (k * (n - k) + 1)
    return c1 + c2
