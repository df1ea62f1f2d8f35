"""Exact and approximate bias gap of the maximum over the search tree
(test infrastructure only).

Lemma 3.1 / 3.2 (Appendix A.1-A.2): under the Gaussian leaf-noise model the
maximum over n i.i.d. N(mu, sigma^2) leaves is treated as GEV with location
mu + sigma Phi^-1(1 - 1/n) and scale sigma [Phi^-1(1 - 1/(e n)) -
Phi^-1(1 - 1/n)], so its mean exceeds mu by sigma * Bn(n) with
    Bn(1) = 0,
    Bn(n) = g Phi^-1(1 - 1/(e n)) + (1 - g) Phi^-1(1 - 1/n)   (n > 1),
g the Euler-Mascheroni constant.  The pi_o sub-tree has n = A^(d-1) leaves
and the other sub-trees n = A^d - A^(d-1), giving B_o = sigma_o Bn(A^(d-1))
and B_e = sigma_e Bn(A^d - A^(d-1)).

Lemma 3.4 (Eq. 5) approximates B_e - B_o by
    sqrt(2 log A) (sigma_e sqrt(d) - sigma_o sqrt(d-1)) - (sigma_e - sigma_o)/2,
using Phi^-1(1 - 1/n) ~ sqrt(2 log n) - 0.5.
"""
from __future__ import annotations

import math
from statistics import NormalDist

EULER_GAMMA = 0.57721566490153286060651209008240243

_N = NormalDist()


def probit_upper(n: float) -> float:
    """Phi^-1(1 - 1/n), taken as -Phi^-1(1/n) so that large n keeps its digits."""
    return -_N.inv_cdf(1.0 / n)


def Bn(n: float) -> float:
    if n == 1:
        return 0.0
    g = EULER_GAMMA
    return g * probit_upper(math.e * n) + (1.0 - g) * probit_upper(n)


def exact_gap(sigma_e: float, sigma_o: float, A: int, d: int) -> float:
    """B_e - B_o of Lemma 3.2 (d >= 1)."""
    n_o = A ** (d - 1)
    n_e = A ** d - A ** (d - 1)
    return sigma_e * Bn(n_e) - sigma_o * Bn(n_o)


def approx_gap(sigma_e: float, sigma_o: float, A: int, d: int) -> float:
    """Eq. 5 (natural log)."""
    return (math.sqrt(2.0 * math.log(A)) * (sigma_e * math.sqrt(d) - sigma_o * math.sqrt(d - 1))
            - (sigma_e - sigma_o) / 2.0)
