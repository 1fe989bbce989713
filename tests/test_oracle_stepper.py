"""Pins for the oracle's time steppers: generating-function identities,
brute-force space-time solves, closed forms, convergence rates, and the
fast/direct relations of Section 3."""
from math import gamma

import numpy as np
import pytest

from oracle import grid, modal, stepper
from oracle.mittag_leffler import ml_neg
from oracle.weights import weights
from paper_1901_05128_amd import workloads as wl


def _data_b(n):
    """Paper's data (b): G1 = (1-x) chi_(1/2,1), G2 = x chi_(0,1/2)."""
    x = wl.nodes_1d(n)
    return np.stack([(1 - x) * ((x > 0.5) & (x < 1)), x * ((x > 0) & (x < 0.5))])


CASES = [
    # dim, nx, ny, alpha1, alpha2, m
    (1, 15, 1, 0.3, 0.7, 0.3),
    (2, 4, 3, 0.45, 0.8, 0.62),
]


@pytest.mark.parametrize("case", CASES)
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("zeta", [0.3, -0.25 + 0.2j])
def test_generating_function_identity(case, scheme, zeta):
    """BE: the sequence solves [delta + delta^b1 (a+A), -a delta^b2; ...] G(zeta) = zeta/tau G0
    (proof of Theorem 4.2 / thmO1trareg). BDF2: with V^n = G^n - G^0 it solves the
    system after (4.11) with nu(zeta) = zeta (3 - zeta)/(2 (1 - zeta))."""
    dim, nx, ny, a1, a2, m = case
    T, N = 0.7, 160
    tau = T / N
    a = (1 - m) / (2 * m - 1)
    b1, b2 = 1 - a1, 1 - a2
    G0 = wl.g0_random(nx * ny, 11)
    G = stepper.solve(dim, nx, ny, a1, a2, m, T, N, G0, scheme, 0, keep=True)
    A = grid.laplacian(dim, nx, ny).toarray()
    z = complex(zeta)
    pw = z ** np.arange(N + 1)
    if scheme == 1:
        dl = (1 - z) / tau
        X = np.tensordot(pw[1:], G[1:], axes=(0, 0))
        rhs = [z / tau * G0[0], z / tau * G0[1]]
    else:
        dl = (1 - z) * (3 - z) / (2 * tau)
        nu = z * (3 - z) / (2 * (1 - z))
        X = np.tensordot(pw[1:], G[1:] - G0[None], axes=(0, 0))
        rhs = [-(a * G0[0] + A @ G0[0]) * dl ** b1 * nu + a * dl ** b2 * nu * G0[1],
               -(a * G0[1] + A @ G0[1]) * dl ** b2 * nu + a * dl ** b1 * nu * G0[0]]
    p1, p2 = dl ** b1, dl ** b2
    R1 = dl * X[0] + p1 * (a * X[0] + A @ X[0]) - a * p2 * X[1] - rhs[0]
    R2 = dl * X[1] + p2 * (a * X[1] + A @ X[1]) - a * p1 * X[0] - rhs[1]
    scale = max(np.abs(p1 * (A @ X[0])).max(), np.abs(p2 * (A @ X[1])).max(), np.abs(rhs[0]).max())
    assert np.abs(R1).max() <= 1e-11 * scale
    assert np.abs(R2).max() <= 1e-11 * scale


def _spacetime_dense(dim, nx, ny, a1, a2, m, T, N, G0, scheme):
    """All steps at once: assemble the block lower-triangular space-time matrix
    of (4.1) / (4.7) and solve it densely."""
    M = nx * ny
    A = grid.laplacian(dim, nx, ny).toarray()
    I = np.eye(M)
    tau = T / N
    a = (1 - m) / (2 * m - 1)
    d1 = weights(scheme, 1 - a1, tau, N)
    d2 = weights(scheme, 1 - a2, tau, N)

    def D(i, s=1.0):
        return s * np.block([[d1[i] * (a * I + A), -a * d2[i] * I], [-a * d1[i] * I, d2[i] * (a * I + A)]])

    n2 = 2 * M
    K = np.zeros((N * n2, N * n2))
    f = np.zeros(N * n2)
    g0 = G0.reshape(-1)
    E = np.eye(n2)
    blk = lambda r, c: (slice(r * n2, (r + 1) * n2), slice(c * n2, (c + 1) * n2))
    for n in range(1, N + 1):
        r = n - 1
        if scheme == 1:
            K[blk(r, r)] += E / tau
            if n >= 2:
                K[blk(r, r - 1)] += -E / tau
            else:
                f[r * n2:(r + 1) * n2] += g0 / tau
            for i in range(0, n):
                K[blk(r, n - i - 1)] += D(i)
        elif n == 1:
            K[blk(0, 0)] += E / tau + D(0, 2 / 3)
            f[:n2] += g0 / tau - D(0, 1 / 3) @ g0
        else:
            K[blk(r, r)] += 1.5 * E / tau
            K[blk(r, r - 1)] += -2 * E / tau
            if n >= 3:
                K[blk(r, r - 2)] += 0.5 * E / tau
            else:
                f[r * n2:(r + 1) * n2] += -0.5 * g0 / tau
            for i in range(0, n):
                K[blk(r, n - i - 1)] += D(i)
            f[r * n2:(r + 1) * n2] += -0.5 * D(n - 1) @ g0
    X = np.linalg.solve(K, f)
    return X[-n2:].reshape(2, M)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("case", [(1, 5, 1, 0.3, 0.7, 0.3), (2, 3, 3, 0.2, 0.6, 0.55), (1, 4, 1, 0.5, 0.5, 0.0)])
def test_marching_equals_bruteforce_spacetime_solve(case, scheme):
    dim, nx, ny, a1, a2, m = case
    T, N = 1.0, 9
    G0 = wl.g0_random(nx * ny, 5)
    ref = _spacetime_dense(dim, nx, ny, a1, a2, m, T, N, G0, scheme)
    got = stepper.solve(dim, nx, ny, a1, a2, m, T, N, G0, scheme, 0)
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(ref)


@pytest.mark.parametrize("beta", [0.3, 0.8])
def test_cq_of_constant_converges_at_scheme_order(beta):
    """D^beta 1 = t^(-beta)/Gamma(1-beta). BE: sum_{i<n} d_i is first order.
    BDF2 with the starting correction (0, 3/2, 1, 1, ...) of Section 4.2:
    sum_{i<n} d_i + d_{n-1}/2 is second order."""
    ex = 1.0 / gamma(1 - beta)
    errs = {1: [], 2: []}
    Ns = [64, 128, 256, 512]
    for N in Ns:
        tau = 1.0 / N
        d1 = weights(1, beta, tau, N)
        errs[1].append(abs(d1[:N].sum() - ex))
        d2 = weights(2, beta, tau, N)
        errs[2].append(abs(d2[:N].sum() + 0.5 * d2[N - 1] - ex))
    r1 = np.log2(np.array(errs[1][:-1]) / np.array(errs[1][1:]))
    r2 = np.log2(np.array(errs[2][:-1]) / np.array(errs[2][1:]))
    assert np.all(np.abs(r1 - 1.0) < 0.05), r1
    assert np.all(np.abs(r2 - 2.0) < 0.1), r2


@pytest.mark.parametrize("scheme,m,order", [(1, 0.6, 1.0), (2, 0.0, 2.0)])
def test_nonsmooth_data_rates(scheme, m, order):
    """Theorems of Section 4: first order (BE) and second order (corrected BDF2)
    for nonsmooth data; differences of successive refinements, data (b)."""
    nx = 31
    G0 = _data_b(nx)
    Ns = [20, 40, 80, 160, 320]
    sols = [stepper.solve(1, nx, 1, 0.3, 0.7, m, 1.0, N, G0, scheme, 0) for N in Ns]
    e = [np.linalg.norm(sols[i] - sols[i + 1]) for i in range(len(Ns) - 1)]
    rates = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert np.all(np.abs(rates - order) < 0.12), rates


@pytest.mark.parametrize("scheme,order", [(1, 1.0), (2, 2.0)])
def test_equal_orders_reduce_to_mittag_leffler(scheme, order):
    """alpha1 = alpha2 = alpha: U = G1 + G2 solves dU/dt + D^{1-alpha} A U = 0 and
    W = G1 - G2 solves dW/dt + D^{1-alpha}(A + 2a) W = 0, so a mode with
    eigenvalue lambda decays as E_alpha(-lambda t^alpha), resp. E_alpha(-(lambda+2a) t^alpha)."""
    alpha, m, T = 0.5, 0.7, 1.0
    a = (1 - m) / (2 * m - 1)
    lam = 9.0
    ops = stepper.ModalOps(np.array([lam]))
    g0 = np.array([[1.0], [0.25]])
    exU = ml_neg(alpha, lam * T ** alpha) * 1.25
    exW = ml_neg(alpha, (lam + 2 * a) * T ** alpha) * 0.75
    eU, eW = [], []
    for N in [40, 80, 160, 320]:
        g = stepper.run(ops, alpha, alpha, m, T, N, g0, scheme, 0)
        eU.append(abs(g[0, 0] + g[1, 0] - exU))
        eW.append(abs(g[0, 0] - g[1, 0] - exW))
    for e in (eU, eW):
        r = np.log2(np.array(e[:-1]) / np.array(e[1:]))
        assert np.all(np.abs(r - order) < 0.15), r


def test_decoupled_case_m_equals_one():
    """m = 1 gives a = 0: each component solves its own scalar equation."""
    T, N = 1.0, 40
    G0 = wl.g0_random(9, 3)
    both = stepper.solve(1, 9, 1, 0.3, 0.6, 1.0, T, N, G0, 2, 0)
    G0a = G0.copy()
    G0a[1] = 0.0
    only1 = stepper.solve(1, 9, 1, 0.3, 0.6, 1.0, T, N, G0a, 2, 0)
    assert np.allclose(both[0], only1[0], rtol=0, atol=1e-14)
    assert np.allclose(only1[1], 0.0, atol=0)


def test_fast_be_is_exact_when_rule_covers_all_lags():
    """Gauss-Jacobi exactness for 2 <= i <= 2 N_p + 1 makes fast BE equal
    direct BE (up to rounding) for N <= 2 N_p + 1."""
    N, Np = 61, 30
    G0 = wl.g0_intervals(25, 7)
    d = stepper.solve(1, 25, 1, 0.35, 0.75, 0.4, 1.0, N, G0, 1, 0)
    f = stepper.solve(1, 25, 1, 0.35, 0.75, 0.4, 1.0, N, G0, 1, 1, np_=Np)
    assert np.linalg.norm(f - d) <= 1e-13 * np.linalg.norm(d)
    f2 = stepper.solve(1, 25, 1, 0.35, 0.75, 0.4, 1.0, N, G0, 1, 1, np_=8)
    assert np.linalg.norm(f2 - d) > 1e-10 * np.linalg.norm(d)


def test_fast_bdf2_window_and_accuracy():
    N = 200
    G0 = wl.g0_intervals(25, 8)
    d = stepper.solve(1, 25, 1, 0.35, 0.75, 0.4, 1.0, N, G0, 2, 0)
    # window longer than the run: no quadrature at all
    f0 = stepper.solve(1, 25, 1, 0.35, 0.75, 0.4, 1.0, N, G0, 2, 1, np_=4, ns=N + 1)
    assert np.linalg.norm(f0 - d) <= 1e-14 * np.linalg.norm(d)
    f = stepper.solve(1, 25, 1, 0.35, 0.75, 0.4, 1.0, N, G0, 2, 1, np_=192, ns=30)
    assert np.linalg.norm(f - d) <= 1e-12 * np.linalg.norm(d)


@pytest.mark.parametrize("scheme,method", [(1, 0), (1, 1), (2, 0), (2, 1)])
@pytest.mark.parametrize("case", [(1, 15, 1), (2, 7, 5)])
def test_modal_equals_nodal(case, scheme, method):
    dim, nx, ny = case
    N = 40
    G0 = wl.g0_random(nx * ny, 9)
    modes = [(1, 1), (2, 1), (nx, ny), (3, 2)] if dim == 2 else [(1, 0), (2, 0), (7, 0), (15, 0)]
    kw = dict(np_=12, ns=10)
    full = stepper.solve(dim, nx, ny, 0.25, 0.65, 0.58, 1.0, N, G0, scheme, method, **kw)
    ref = modal.project(full, dim, nx, ny, modes)
    got = modal.run_modes(dim, nx, ny, modes, 0.25, 0.65, 0.58, 1.0, N, G0, scheme, method, **kw)
    assert np.max(np.abs(got - ref)) <= 1e-12 * np.max(np.abs(ref))
