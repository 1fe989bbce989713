"""Pins of the oracle adjoint (oracle/adjoint.py) against things other than
itself: the duality of a linear map (exact), finite differences of the
forward steppers, a dense space-time transpose solve, mpmath derivatives of
the weights, and the mode-by-mode form."""
import mpmath
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import stepper
from oracle.weights import weights
from paper_1901_05128_amd import workloads as wl

CASES = [
    # dim, nx, ny, alpha1, alpha2, m, N
    (1, 7, 1, 0.3, 0.7, 0.35, 40),
    (2, 5, 4, 0.2, 0.6, 0.55, 36),
]
FAST = dict(np_=12, np1=8, ns=10)


def _setup(case):
    dim, nx, ny, a1, a2, m, N = case
    M = nx * ny
    G0 = wl.g0_random(M, 5).reshape(2, M)
    tgt = np.random.default_rng(11).standard_normal((2, M))
    return dim, nx, ny, a1, a2, m, N, M, G0, tgt


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
def test_g0_gradient_is_the_transpose_of_the_linear_map(case, scheme, method):
    """G^N is linear in G^0, so <g, L d> = <L^T g, d> for every d."""
    dim, nx, ny, a1, a2, m, N, M, G0, tgt = _setup(case)
    rng = np.random.default_rng(3)
    g = rng.standard_normal((2, M))
    gG0 = adj.adjoint_nodal(dim, nx, ny, a1, a2, m, 1.0, N, G0, g, scheme, method, **FAST)[0]
    for _ in range(3):
        dlt = rng.standard_normal((2, M))
        Ld = stepper.solve(dim, nx, ny, a1, a2, m, 1.0, N, dlt, scheme, method, **FAST)
        lhs, rhs = float(np.sum(g * Ld)), float(np.sum(gG0 * dlt))
        assert abs(lhs - rhs) <= 1e-12 * (np.linalg.norm(g) * np.linalg.norm(Ld) + abs(lhs))


def _fd5(f, x, h):
    return (f(x - 2 * h) - 8 * f(x - h) + 8 * f(x + h) - f(x + 2 * h)) / (12 * h)


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
def test_parameter_gradients_match_finite_differences(case, scheme, method):
    """l = 1/2 |G^N - target|^2; fourth-order central differences of the
    stepper in alpha_1, alpha_2 and m (h = 1e-4: truncation and rounding
    both below 1e-11 relative; a(m) has a pole at m = 1/2)."""
    dim, nx, ny, a1, a2, m, N, M, G0, tgt = _setup(case)

    def loss(p):
        GN = stepper.solve(dim, nx, ny, p[0], p[1], p[2], 1.0, N, G0, scheme, method, **FAST)
        return 0.5 * float(np.sum((GN - tgt) ** 2))

    GN = stepper.solve(dim, nx, ny, a1, a2, m, 1.0, N, G0, scheme, method, **FAST)
    _g, ga1, ga2, gm, _ = adj.adjoint_nodal(dim, nx, ny, a1, a2, m, 1.0, N, G0, GN - tgt, scheme, method,
                                            **FAST)
    base = [a1, a2, m]
    for idx, got in enumerate([ga1, ga2, gm]):
        def f(x, idx=idx):
            p = list(base)
            p[idx] = x
            return loss(p)
        fd = _fd5(f, base[idx], 1e-4)
        assert abs(got - fd) <= 1e-8 * abs(fd) + 1e-12, (idx, got, fd)


def _spacetime_dense_K(dim, nx, ny, a1, a2, m, N, scheme):
    """Block lower-triangular space-time matrix of (4.1)/(4.7), rows in the
    paper's scaling (the BDF2 n = 1 row unscaled)."""
    from oracle import grid
    M = nx * ny
    A = grid.laplacian(dim, nx, ny).toarray()
    I = np.eye(M)
    tau = 1.0 / N
    a = (1 - m) / (2 * m - 1)
    d1 = weights(scheme, 1 - a1, tau, N)
    d2 = weights(scheme, 1 - a2, tau, N)

    def D(i, s=1.0):
        return s * np.block([[d1[i] * (a * I + A), -a * d2[i] * I], [-a * d1[i] * I, d2[i] * (a * I + A)]])

    n2 = 2 * M
    K = np.zeros((N * n2, N * n2))
    E = np.eye(n2)
    blk = lambda r, c: (slice(r * n2, (r + 1) * n2), slice(c * n2, (c + 1) * n2))
    for n in range(1, N + 1):
        r = n - 1
        if scheme == 1:
            K[blk(r, r)] += E / tau
            if n >= 2:
                K[blk(r, r - 1)] += -E / tau
            for i in range(0, n):
                K[blk(r, n - i - 1)] += D(i)
        elif n == 1:
            K[blk(0, 0)] += E / tau + D(0, 2 / 3)
        else:
            K[blk(r, r)] += 1.5 * E / tau
            K[blk(r, r - 1)] += -2 * E / tau
            if n >= 3:
                K[blk(r, r - 2)] += 0.5 * E / tau
            for i in range(0, n):
                K[blk(r, n - i - 1)] += D(i)
    return K


@pytest.mark.parametrize("scheme", [1, 2])
def test_multipliers_solve_the_transposed_spacetime_system(scheme):
    """Direct scheme: the multipliers are K^-T [0, .., 0, g] for the dense
    space-time matrix K (its BDF2 first row is the unified row / (3/2))."""
    dim, nx, ny, a1, a2, m, N = 1, 5, 1, 0.4, 0.8, 0.3, 12
    M = nx * ny
    G0 = wl.g0_random(M, 7).reshape(2, M)
    g = np.random.default_rng(2).standard_normal((2, M))
    out = adj.adjoint(stepper.NodalOps(__import__("oracle.grid", fromlist=["x"]).laplacian(dim, nx, ny)),
                      a1, a2, m, 1.0, N, G0, g, scheme, 0, return_mu=True)
    mu = out[5]
    K = _spacetime_dense_K(dim, nx, ny, a1, a2, m, N, scheme)
    rhs = np.zeros(K.shape[0])
    rhs[-2 * M:] = g.reshape(-1)
    mud = np.linalg.solve(K.T, rhs).reshape(N, 2, M)
    if scheme == 2:
        mud[0] = mud[0] / 1.5
    assert np.linalg.norm(mu - mud) <= 1e-11 * np.linalg.norm(mud)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("beta", [0.3, 0.85])
def test_exact_weight_derivatives_match_mpmath(scheme, beta):
    tau, n = 0.01, 24
    got = adj.exact_weights_dbeta(scheme, beta, tau, n)
    mpmath.mp.dps = 30

    def d_i(b, i):
        b = mpmath.mpf(b)
        if scheme == 1:
            return mpmath.mpf(tau) ** (-b) * (-1) ** i * mpmath.binomial(b, i)
        # coefficient of z^i in (3/2 - 2z + z^2/2)^b
        return mpmath.mpf(tau) ** (-b) * mpmath.taylor(lambda z: (mpmath.mpf(3) / 2 - 2 * z + z ** 2 / 2) ** b,
                                                       0, i)[i]

    for i in (0, 1, 2, 5, 13, 24):
        ref = float(mpmath.diff(lambda b: d_i(b, i), beta))
        assert abs(got[i] - ref) <= 1e-12 * max(1.0, abs(ref)), (i, got[i], ref)


@pytest.mark.parametrize("scheme", [1, 2])
def test_fast_weight_derivatives_close_to_exact(scheme):
    """The Gauss-Jacobi sums approximate d_i uniformly in beta, so their beta
    derivative approximates the exact derivative to the rule's accuracy."""
    beta, tau, N = 0.55, 1.0 / 400, 400
    w, dw = adj.scheme_weights(scheme, 1, beta, tau, N, np_=60, np1=16, ns=30)
    d = weights(scheme, beta, tau, N)
    dd = adj.exact_weights_dbeta(scheme, beta, tau, N)
    assert np.max(np.abs(w - d)) <= 1e-9 * abs(d[0])
    assert np.max(np.abs(dw - dd)) <= 1e-7 * np.max(np.abs(dd))


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
def test_modal_adjoint_equals_nodal(scheme, method):
    dim, nx, ny, a1, a2, m, N = 2, 5, 3, 0.25, 0.65, 0.7, 24
    M = nx * ny
    G0 = wl.g0_random(M, 9).reshape(2, M)
    g = np.random.default_rng(4).standard_normal((2, M))
    r1 = adj.adjoint_nodal(dim, nx, ny, a1, a2, m, 1.0, N, G0, g, scheme, method, **FAST)
    r2 = adj.adjoint_reference(dim, nx, ny, a1, a2, m, 1.0, N, G0, g, scheme, method, **FAST)
    assert np.linalg.norm(r1[0] - r2[0]) <= 1e-11 * np.linalg.norm(r1[0])
    for x, y in zip(r1[1:4], r2[1:4]):
        assert abs(x - y) <= 1e-11 * abs(x)
    assert np.linalg.norm(r1[4] - r2[4]) <= 1e-11 * np.linalg.norm(r1[4])
