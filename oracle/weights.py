"""CQ weights as Taylor coefficients of the generating functions.

ORACLE (test infrastructure only).

BE, eqs. (3.3)-(3.4):  ((1 - zeta)/tau)^beta = sum_i d_{1,i} zeta^i.
  (1 - zeta)^beta = sum_i binom(beta, i) (-zeta)^i, and the binomial
  coefficient is the product binom(beta, i) = prod_{k=1..i} (beta - k + 1)/k,
  so (-1)^i binom(beta, i) = prod_{k=1..i} (1 - (1 + beta)/k).

BDF2 (SBD), eqs. (3.11)-(3.12):
  ((1 - zeta) + (1 - zeta)^2/2)^beta / tau^beta
  = (3/2)^beta (1 - zeta)^beta (1 - zeta/3)^beta / tau^beta,
  the Cauchy product of two binomial series.

In the scheme the CQ order is beta = 1 - alpha_k (Section 4).
"""
import numpy as np


def binomial_series(beta: float, n: int) -> np.ndarray:
    """Coefficients of (1 - zeta)^beta up to zeta^n (product form of binom)."""
    k = np.arange(1, n + 1, dtype=np.float64)
    return np.concatenate([[1.0], np.cumprod(1.0 - (1.0 + beta) / k)])


def be_weights(beta: float, tau: float, n: int) -> np.ndarray:
    """d_{1,i}, i = 0..n, eq. (3.4)."""
    return tau ** (-beta) * binomial_series(beta, n)


def bdf2_weights(beta: float, tau: float, n: int) -> np.ndarray:
    """d_{2,i}, i = 0..n, eq. (3.12), as the product of the series of
    (1 - zeta)^beta and (1 - zeta/3)^beta times (3/2)^beta."""
    g = binomial_series(beta, n)
    h = g * (1.0 / 3.0) ** np.arange(n + 1)
    c = np.convolve(g, h)[: n + 1]
    return tau ** (-beta) * 1.5 ** beta * c


def weights(scheme: int, beta: float, tau: float, n: int) -> np.ndarray:
    if scheme == 1:
        return be_weights(beta, tau, n)
    if scheme == 2:
        return bdf2_weights(beta, tau, n)
    raise ValueError("scheme must be 1 (BE) or 2 (BDF2)")


def generating_function(scheme: int, beta: float, tau: float, zeta: complex) -> complex:
    """delta(zeta)^beta in closed form (principal branch), eqs. (3.3), (3.11)."""
    zeta = complex(zeta)
    if scheme == 1:
        delta = (1.0 - zeta) / tau
    else:
        delta = ((1.0 - zeta) + (1.0 - zeta) ** 2 / 2.0) / tau
    return delta ** beta
