"""Pins for the oracle's CQ weights (eqs. 3.3-3.4, 3.11-3.12)."""
import mpmath as mp
import numpy as np
import pytest

from oracle import weights as W


@pytest.mark.parametrize("beta", [0.2, 0.5, 0.7, 0.95])
def test_be_weights_vs_high_precision_binomial(beta):
    tau = 0.01
    d = W.be_weights(beta, tau, 5000)
    mp.mp.dps = 40
    for i in [0, 1, 2, 7, 100, 1234, 5000]:
        ex = mp.binomial(mp.mpf(beta), i) * (-1) ** i * mp.mpf(tau) ** (-mp.mpf(beta))
        assert abs(d[i] - float(ex)) <= 1e-13 * abs(float(ex))


@pytest.mark.parametrize("beta", [0.3, 0.8])
def test_bdf2_weights_vs_high_precision_taylor(beta):
    mp.mp.dps = 40
    b = mp.mpf(beta)
    ex = mp.taylor(lambda z: (mp.mpf(3) / 2 - 2 * z + z * z / 2) ** b, 0, 40)
    d = W.bdf2_weights(beta, 1.0, 40)
    for i in range(41):
        assert abs(d[i] - float(ex[i])) <= 1e-14 * max(1e-300, abs(float(ex[i]))) + 1e-17


def test_first_weights_closed_form():
    beta, tau = 0.35, 0.002
    d1 = W.be_weights(beta, tau, 3)
    assert np.isclose(d1[0], tau ** -beta, rtol=1e-15)
    assert np.isclose(d1[1], -beta * tau ** -beta, rtol=1e-15)
    assert np.isclose(d1[2], beta * (beta - 1) / 2 * tau ** -beta, rtol=1e-14)
    d2 = W.bdf2_weights(beta, tau, 3)
    assert np.isclose(d2[0], 1.5 ** beta * tau ** -beta, rtol=1e-15)
    # derivative of (3/2 - 2 z + z^2/2)^beta at 0
    assert np.isclose(d2[1], -2 * beta * 1.5 ** (beta - 1) * tau ** -beta, rtol=1e-14)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("zeta", [0.5, -0.7, 0.3 + 0.4j])
def test_generating_function_at_sample_points(scheme, zeta):
    beta, tau, n = 0.45, 0.05, 400
    d = W.weights(scheme, beta, tau, n)
    s = np.sum(d * np.asarray(zeta, dtype=complex) ** np.arange(n + 1))
    if scheme == 1:
        ex = ((1 - zeta) / tau) ** beta
    else:
        ex = (((1 - zeta) + (1 - zeta) ** 2 / 2) / tau) ** beta
    assert abs(s - ex) <= 1e-13 * abs(ex)
