"""Pins for the oracle's Gauss-Jacobi rules and fast weights (3.6), (3.14)-(3.16)."""
from math import cos, gamma, pi

import numpy as np
import pytest
from scipy import integrate, special

from oracle import quadrature as Q
from oracle import weights as W


@pytest.mark.parametrize("n", [4, 64, 400, 576, 768, 1024])
@pytest.mark.parametrize("ab", [(0.3, 0.7), (0.8, 0.4), (0.25, 1.5), (0.6, 0.8)])
def test_gauss_jacobi_moments_vs_beta_function(n, ab):
    """Moments up to the rule's exactness degree 2n-1 against Beta values;
    n reaches the node counts the fast rules take (576-1024 at N = 2^16)."""
    a, b = ab
    s, lam = Q.gauss_jacobi(n, a, b)
    for k in sorted(k for k in {0, 1, 2, 10, 100, n, 2 * n - 1} if k <= 2 * n - 1):
        # int (1-s)^a (1+s)^b ((1+s)/2)^k ds = 2^(a+b+1) B(a+1, b+k+1)
        ex = 2.0 ** (a + b + 1) * special.beta(a + 1, b + k + 1)
        got = np.sum(lam * ((1 + s) / 2) ** k)
        # the top moments are carried by the few nodes next to s = 1, whose
        # positions Newton's method fixes to ~1e-15 (measured <= 4e-12
        # relative at n = 1024)
        tol = 1e-13 if k <= 100 else 5e-11
        assert abs(got - ex) <= tol * ex


@pytest.mark.parametrize("alpha", [0.2, 0.6, 0.9])
@pytest.mark.parametrize("np_", [3, 16, 384, 768])
def test_be_rule_exact_up_to_2np_plus_1(alpha, np_):
    """Remark after (3.8): the rule is exact for 2 <= i <= 2 N_p + 1."""
    tau = 0.01
    d = W.be_weights(alpha, tau, 2 * np_ + 5)
    rule = Q.be_rule(alpha, tau, np_)
    for i in range(2, 2 * np_ + 2):
        approx = np.dot(rule.w, rule.dbar(i))
        assert abs(approx - d[i]) <= 1e-13 * abs(d[0])
    # one past the exact range is no longer exact (the quadrature is not trivial)
    i = 2 * np_ + 2
    assert abs(np.dot(rule.w, rule.dbar(i)) - d[i]) > 0.0


@pytest.mark.parametrize("alpha", [0.3, 0.7])
@pytest.mark.parametrize("i", [3, 4, 10, 25])
def test_bdf2_integral_form_with_real_parts(alpha, i):
    """(3.14) with the real-part rule, evaluated by adaptive quadrature
    (no Gauss-Jacobi), equals the Taylor coefficient d_{2,i}."""
    tau = 1.0
    gg = gamma(1 - alpha) * gamma(alpha)
    J = lambda s: (1 - s) ** alpha * (1 + s) ** (2 - 2 * alpha)
    f1 = lambda s: J(s) * (s + 5) ** -4 * ((s + 1) / (s + 5)) ** (i - 3)
    re = lambda s: abs(1 + 3 * s) ** alpha * (1.0 if s >= -1 / 3 else cos(pi * alpha))
    f2 = lambda s: J(s) * re(s) * ((s + 1) / 2) ** (i - 3)
    opts = dict(epsabs=1e-16, epsrel=1e-13, limit=400)
    I1 = integrate.quad(f1, -1, 1, **opts)[0]
    I2 = integrate.quad(f2, -1, -1 / 3, **opts)[0] + integrate.quad(f2, -1 / 3, 1, **opts)[0]
    val = -(2 ** (2 + 2 * alpha)) * cos(pi * alpha) / gg * I1 - 2 ** (-alpha - 3) / gg * I2
    d = W.bdf2_weights(alpha, tau, i)
    assert abs(val - d[i]) <= 1e-10 * abs(d[i])


@pytest.mark.parametrize("alpha", [0.2, 0.6])
def test_bdf2_two_rule_approximation_converges(alpha):
    """(3.16): with N_s = 30 and enough nodes the two-family sum reproduces
    d_{2,i} for every i >= N_s to near rounding."""
    tau, ns, N = 0.001, 30, 3000
    d = W.bdf2_weights(alpha, tau, N)
    r1, r2 = Q.bdf2_rules(alpha, tau, 16, 256)
    approx = Q.approx_weights_fast([r1, r2], ns, N)
    assert np.max(np.abs(approx - d[ns:])) <= 1e-12 * abs(d[0])
    # and the small-i terms are not well approximated (why N_s exists)
    assert abs(Q.approx_weights([r1, r2], 3, 3)[0] - d[3]) > 1e-9 * abs(d[0])
