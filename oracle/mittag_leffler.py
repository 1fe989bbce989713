"""Mittag-Leffler function E_alpha(-x), 0 < alpha < 1, x >= 0.

ORACLE (test infrastructure only). Used for closed-form checks: with
alpha1 = alpha2 = alpha, U = G1 + G2 obeys dU/dt + D^{1-alpha} A U = 0, so a
Laplacian mode with eigenvalue lambda evolves as E_alpha(-lambda t^alpha).

Evaluated from the spectral (Laplace-inversion) integral
  E_alpha(-t^alpha) = int_0^inf exp(-r t) K_alpha(r) dr,
  K_alpha(r) = (1/pi) r^(alpha-1) sin(alpha pi) / (r^(2 alpha) + 2 r^alpha cos(alpha pi) + 1),
with x = t^alpha, computed by adaptive quadrature (scipy.integrate.quad).
"""
from math import pi, sin, cos

from scipy import integrate


def ml_neg(alpha: float, x: float) -> float:
    if x == 0.0:
        return 1.0
    t = x ** (1.0 / alpha)

    def k(r):
        ra = r ** alpha
        return (r ** (alpha - 1.0)) * sin(alpha * pi) / (pi * (ra * ra + 2.0 * ra * cos(alpha * pi) + 1.0))

    # split at r = 1 and integrate the exponential tail in the variable r
    f = lambda r: k(r) * __import__("math").exp(-r * t)
    v1 = integrate.quad(f, 0.0, 1.0, epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    v2 = integrate.quad(f, 1.0, float("inf"), epsabs=1e-15, epsrel=1e-13, limit=400)[0]
    return v1 + v2
