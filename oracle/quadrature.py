"""Gauss-Jacobi rules and the fast (sum-of-geometric-sequences) weights.

ORACLE (test infrastructure only). Written in the paper's notation, with
alpha the CQ order (in the schemes alpha -> 1 - alpha_k).

BE, eq. (3.6)-(3.7), i >= 2:
  d_{1,i} = -1/(4 tau^alpha Gamma(1-alpha) Gamma(alpha))
            * int_{-1}^{1} (1-s)^alpha (1+s)^(1-alpha) dbar_{1,i}(s) ds,
  dbar_{1,i}(s) = ((s+1)/2)^(i-2).
  A Gauss-Jacobi rule (nodes s_j, weights lambda_j) for the weight
  (1-s)^alpha (1+s)^(1-alpha) gives w_j = -lambda_j/(4 tau^alpha Gamma Gamma)
  and d_{1,i} ~ sum_j w_j dbar_{1,i}(s_j) + eps_{1,i}.

BDF2, eqs. (3.14)-(3.16), i >= 3:
  d_{2,i} = -(2^(2+2alpha) (-1)^(-alpha))/(tau^alpha Gamma Gamma) int J dbar^1_{2,i}
            - 2^(-alpha-3)/(tau^alpha Gamma Gamma)            int J dbar^2_{2,i},
  J = (1-s)^alpha (1+s)^(2-2alpha),
  dbar^1_{2,i}(s) = (s+5)^(-4) ((s+1)/(s+5))^(i-3),
  dbar^2_{2,i}(s) = (1+3s)^alpha ((s+1)/2)^(i-3).
  Following the remark after (3.16), only real parts are kept:
  Re (-1)^(-alpha) = cos(pi alpha), and Re (1+3s)^alpha = |1+3s|^alpha for
  s >= -1/3, |1+3s|^alpha cos(pi alpha) for s < -1/3.

The Gauss-Jacobi nodes come from scipy.special.roots_jacobi (a library
routine, used as one step), polished by Newton's method; the weights are the
Christoffel numbers of the orthonormal Jacobi polynomials.
"""
from dataclasses import dataclass
from math import gamma, pi, cos

import numpy as np
from scipy import special


def gauss_jacobi(n: int, a: float, b: float):
    """Nodes and weights for int_{-1}^{1} (1-s)^a (1+s)^b f(s) ds.

    Nodes: scipy.special.roots_jacobi, polished by three Newton steps on the
    Jacobi polynomial P_n^(a,b) (scipy.special.eval_jacobi, with
    d/ds P_n^(a,b) = (n+a+b+1)/2 P_{n-1}^(a+1,b+1)). Weights: the Christoffel
    numbers lambda_j = 1 / sum_{k<n} q_k(s_j)^2 of the orthonormal Jacobi
    polynomials, from their three-term recurrence
      sqrt(beta_{k+1}) q_{k+1} = (s - alpha_k) q_k - sqrt(beta_k) q_{k-1},
      q_0 = 1/sqrt(mu_0),  mu_0 = 2^(a+b+1) B(a+1, b+1),
      alpha_k = (b^2 - a^2) / ((2k+a+b)(2k+a+b+2))  (alpha_0 = (b-a)/(a+b+2)),
      beta_k = 4k(k+a)(k+b)(k+a+b) / ((2k+a+b)^2 (2k+a+b+1)(2k+a+b-1)).
    (roots_jacobi's own weights drift by up to ~1e-8 relative at ~1000
    nodes; these keep ~1e-11.)"""
    s, _ = special.roots_jacobi(n, a, b)
    s = np.asarray(s, dtype=np.float64)
    c = 0.5 * (n + a + b + 1.0)
    for _ in range(3):
        s = s - special.eval_jacobi(n, a, b, s) / (c * special.eval_jacobi(n - 1, a + 1.0, b + 1.0, s))

    def alpha(k):
        t = 2.0 * k + a + b
        return (b - a) / (a + b + 2.0) if k == 0 else (b * b - a * a) / (t * (t + 2.0))

    def sqrt_beta(k):
        t = 2.0 * k + a + b
        return np.sqrt(4.0 * k * (k + a) * (k + b) * (k + a + b) / (t * t * (t + 1.0) * (t - 1.0)))

    mu0 = 2.0 ** (a + b + 1.0) * special.beta(a + 1.0, b + 1.0)
    q_prev = np.zeros_like(s)
    q = np.full_like(s, 1.0 / np.sqrt(mu0))
    total = q * q
    for k in range(n - 1):
        q_next = ((s - alpha(k)) * q - (sqrt_beta(k) if k >= 1 else 0.0) * q_prev) / sqrt_beta(k + 1)
        q_prev, q = q, q_next
        total += q * q
    return s, 1.0 / total


@dataclass
class FastRule:
    """One geometric family: d_i ~ sum_j w_j * scale_j * ratio_j^(i - i0)."""
    ratio: np.ndarray   # common ratio of dbar in i
    w: np.ndarray       # integration weights w_j of the paper (with all constants)
    scale: np.ndarray   # the i-independent factor of dbar (1, (s+5)^-4, Re(1+3s)^alpha)
    i0: int             # exponent offset (2 for BE, 3 for BDF2)

    def dbar(self, i: int) -> np.ndarray:
        return self.scale * self.ratio ** (i - self.i0)


def be_rule(alpha: float, tau: float, np_: int) -> FastRule:
    s, lam = gauss_jacobi(np_, alpha, 1.0 - alpha)
    w = -lam / (4.0 * tau ** alpha * gamma(1.0 - alpha) * gamma(alpha))
    return FastRule(ratio=(s + 1.0) / 2.0, w=w, scale=np.ones_like(s), i0=2)


def bdf2_rules(alpha: float, tau: float, np1: int, np2: int):
    gg = gamma(1.0 - alpha) * gamma(alpha)
    s1, lam1 = gauss_jacobi(np1, alpha, 2.0 - 2.0 * alpha)
    w1 = -(2.0 ** (2.0 + 2.0 * alpha)) * cos(pi * alpha) * lam1 / (tau ** alpha * gg)
    r1 = FastRule(ratio=(s1 + 1.0) / (s1 + 5.0), w=w1, scale=(s1 + 5.0) ** -4, i0=3)
    s2, lam2 = gauss_jacobi(np2, alpha, 2.0 - 2.0 * alpha)
    w2 = -(2.0 ** (-alpha - 3.0)) * lam2 / (tau ** alpha * gg)
    re = np.abs(1.0 + 3.0 * s2) ** alpha * np.where(s2 >= -1.0 / 3.0, 1.0, cos(pi * alpha))
    r2 = FastRule(ratio=(s2 + 1.0) / 2.0, w=w2, scale=re, i0=3)
    return r1, r2


def approx_weights(rules, i_from: int, i_to: int) -> np.ndarray:
    """sum over rules and nodes of w_j dbar_i(s_j) for i = i_from..i_to."""
    out = np.zeros(i_to - i_from + 1)
    for k, i in enumerate(range(i_from, i_to + 1)):
        out[k] = sum(float(np.dot(r.w, r.dbar(i))) for r in rules)
    return out


def approx_weights_fast(rules, i_from: int, i_to: int) -> np.ndarray:
    """Same values as approx_weights, vectorised over i (for long ranges)."""
    i = np.arange(i_from, i_to + 1)
    out = np.zeros(len(i))
    for r in rules:
        for wj, sc, rj in zip(r.w, r.scale, r.ratio):
            out += wj * sc * rj ** (i - r.i0)
    return out
