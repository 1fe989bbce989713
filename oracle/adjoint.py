"""Gradient of a loss of G^N for the schemes of the stepper module.

ORACLE (test infrastructure only). Not part of the paper: reverse-mode
differentiation (a discrete adjoint) of the BE scheme (4.1)/(4.3) and the
BDF2 scheme (4.7)/(4.8), direct or fast, with respect to G^0, alpha_1,
alpha_2 and m.

Every step of the stepper's schemes has the form, n = 1..N,

    c G^n - E^n + Dm X^n = 0,
    X^n = sum_{i=0}^{n-1} W_i G^{n-i} + [BDF2] 1/2 V_{n-1} G^0,

with
    Dm  = [[a + A, -a], [-a, a + A]]           (symmetric, as A is),
    W_i = diag(w_{1,i}, w_{2,i})                weights of the CQ sum as the
          scheme uses them: the exact d_{k,i} for the direct scheme; for the
          fast scheme the exact d_{k,i} below the lag (2 for BE, N_s for BDF2)
          and the Gauss-Jacobi sums of (3.6)/(3.14) from the lag on,
    V_i = diag(d_{1,i}, d_{2,i})                exact weights (the starting
          correction of (4.7)/(4.8) keeps them),
    c   = 1/tau, E^n = G^{n-1}/tau                                  (BE),
    c   = 3/(2 tau), E^n = (2 G^{n-1} - G^{n-2}/2)/tau, G^{-1} := G^0 (BDF2;
          the n = 1 step of (4.7) is this form divided by 3/2).

For a loss l with g = dl/dG^N, the Lagrange multipliers mu^n solve, for
n = N, N-1, .., 1 (mu^{N+1} = mu^{N+2} = 0),

    (c I + W_0 Dm) mu^n = [n = N] g + F^n - sum_{i=1}^{N-n} W_i Dm mu^{n+i},
    F^n = mu^{n+1}/tau (BE),  (2 mu^{n+1} - mu^{n+2}/2)/tau (BDF2),

(the transpose of the step operator, and the CQ sum run backwards in time
with the same weights), and

    dl/dG^0     = mu^1/tau                                              (BE)
                = (3 mu^1 - mu^2)/(2 tau) - 1/2 sum_n V_{n-1} Dm mu^n  (BDF2)
    dl/da       = -sum_n mu^n . [[1, -1], [-1, 1]] X^n
    dl/dm       = dl/da * da/dm,        da/dm = -1/(2m - 1)^2
    dl/dbeta_k  = -sum_n (Dm mu^n)_k . Y_k^n,
    Y_k^n       = sum_{i=0}^{n-1} (d w_{k,i}/d beta_k) G_k^{n-i}
                  + [BDF2] 1/2 (d d_{k,n-1}/d beta_k) G_k^0,
    dl/dalpha_k = -dl/dbeta_k          (beta_k = 1 - alpha_k).

Weight derivatives: for the exact weights, the recurrence of the weights
module differentiated term by term (BE: g_i = g_{i-1}(1 - (1+beta)/i), so
g'_i = g'_{i-1}(1 - (1+beta)/i) - g_{i-1}/i; BDF2: the product rule through
the Cauchy product), times tau^-beta with its own derivative. For the
Gauss-Jacobi sums, the factor tau^-beta exactly and the rest by a five-point
central difference in beta of the whole rule (nodes and weights recomputed),
step h_rule; its error is of order h_rule^4 times the fifth derivative
(below 1e-11 relative at the default).
"""
from __future__ import annotations

import numpy as np

from . import grid, modal
from .quadrature import approx_weights_fast, be_rule, bdf2_rules
from .stepper import ModalOps, NodalOps, default_np, run
from .weights import binomial_series, weights


def _binomial_series_dbeta(beta, n):
    """d/dbeta of binomial_series(beta, n), by differentiating its product."""
    g = binomial_series(beta, n)
    dg = np.zeros(n + 1)
    for i in range(1, n + 1):
        dg[i] = dg[i - 1] * (1.0 - (1.0 + beta) / i) - g[i - 1] / i
    return dg


def exact_weights_dbeta(scheme, beta, tau, n):
    """d/dbeta of the exact weights d_i, i = 0..n."""
    g = binomial_series(beta, n)
    dg = _binomial_series_dbeta(beta, n)
    lt = np.log(tau)
    if scheme == 1:
        return tau ** (-beta) * (dg - lt * g)
    p3 = (1.0 / 3.0) ** np.arange(n + 1)
    h, dh = g * p3, dg * p3
    c = np.convolve(g, h)[: n + 1]
    dc = np.convolve(dg, h)[: n + 1] + np.convolve(g, dh)[: n + 1]
    f = tau ** (-beta) * 1.5 ** beta
    return f * (dc + (np.log(1.5) - lt) * c)


def _rule_tail(scheme, beta, tau, N, np_, np1, lag):
    """Gauss-Jacobi sums for i = lag..N (the fast scheme's weights there)."""
    rules = [be_rule(beta, tau, np_)] if scheme == 1 else list(bdf2_rules(beta, tau, np1, np_))
    return approx_weights_fast(rules, lag, N)


def scheme_weights(scheme, method, beta, tau, N, np_=None, np1=16, ns=30, h_rule=1e-3):
    """(w, dw/dbeta) of the CQ sum as the scheme uses it, i = 0..N.

    The Gauss-Jacobi sums carry the factor tau^-beta of (3.6)/(3.14); it is
    differentiated exactly, w = tau^-beta q(beta) with q the sums at tau = 1,
    and only q' comes from the five-point difference (its high derivatives
    in beta stay small, where those of tau^-beta grow like ln(1/tau)^5)."""
    d = weights(scheme, beta, tau, N)
    dd = exact_weights_dbeta(scheme, beta, tau, N)
    if method == 0:
        return d, dd
    if np_ is None:
        np_ = default_np(N)
    lag = 2 if scheme == 1 else ns
    w, dw = d.copy(), dd.copy()
    if lag <= N:
        q = lambda b: _rule_tail(scheme, b, 1.0, N, np_, np1, lag)
        h = h_rule
        dq = (q(beta - 2 * h) - 8 * q(beta - h) + 8 * q(beta + h) - q(beta + 2 * h)) / (12 * h)
        tb = tau ** (-beta)
        w[lag:] = tb * q(beta)
        dw[lag:] = tb * (dq - np.log(tau) * q(beta))
    return w, dw


def adjoint(ops, alpha1, alpha2, m, T, N, G0, gN, scheme, method, np_=None, np1=16, ns=30,
            return_mu=False):
    """Gradient of l(G^N) with dl/dG^N = gN ([2][n]).

    Returns (dl/dG0 [2][n], dl/dalpha1, dl/dalpha2, dl/dm, G^N), and the
    multipliers mu^1..mu^N ([N][2][n]) after them when return_mu is true."""
    tau = T / N
    a = (1.0 - m) / (2.0 * m - 1.0)
    beta = (1.0 - alpha1, 1.0 - alpha2)
    n_sp = ops.n
    A = ops.apply
    G = run(ops, alpha1, alpha2, m, T, N, G0, scheme, method, np_, np1, ns, keep=True)
    W, dW, V, dV = [], [], [], []
    for k in range(2):
        w, dw = scheme_weights(scheme, method, beta[k], tau, N, np_, np1, ns)
        W.append(w)
        dW.append(dw)
        V.append(weights(scheme, beta[k], tau, N))
        dV.append(exact_weights_dbeta(scheme, beta[k], tau, N))
    c = 1.0 / tau if scheme == 1 else 1.5 / tau

    def Dm(v):
        return np.stack([a * v[0] + A(v[0]) - a * v[1], a * v[1] + A(v[1]) - a * v[0]])

    # transpose of the step operator: c I + W_0 Dm
    w10, w20 = W[0][0], W[1][0]
    solve_t = ops.factor(c + w10 * a, w10, -a * w10, -a * w20, c + w20 * a, w20)

    gN = np.asarray(gN, dtype=np.float64).reshape(2, n_sp)
    mu = np.zeros((N + 3, 2, n_sp))     # mu[N+1] = mu[N+2] = 0
    psi = np.zeros((N + 3, 2, n_sp))    # psi^n = Dm mu^n
    for n in range(N, 0, -1):
        rhs = gN.copy() if n == N else np.zeros((2, n_sp))
        if scheme == 1:
            rhs += mu[n + 1] / tau
        else:
            rhs += (2.0 * mu[n + 1] - 0.5 * mu[n + 2]) / tau
        for k in range(2):
            if N - n >= 1:
                rhs[k] -= W[k][1:N - n + 1] @ psi[n + 1:N + 1, k]
        mu[n, 0], mu[n, 1] = solve_t(rhs[0], rhs[1])
        psi[n] = Dm(mu[n])

    # dl/dG^0
    if scheme == 1:
        gG0 = mu[1] / tau
    else:
        gG0 = (3.0 * mu[1] - mu[2]) / (2.0 * tau)
        for k in range(2):
            gG0[k] = gG0[k] - 0.5 * (V[k][0:N] @ psi[1:N + 1, k])

    # dl/da and dl/dbeta_k
    ga = 0.0
    gb = [0.0, 0.0]
    for n in range(1, N + 1):
        X = np.zeros((2, n_sp))
        Y = np.zeros((2, n_sp))
        for k in range(2):
            X[k] = W[k][0:n] @ G[n:0:-1, k]
            Y[k] = dW[k][0:n] @ G[n:0:-1, k]
            if scheme == 2:
                X[k] += 0.5 * V[k][n - 1] * G[0, k]
                Y[k] += 0.5 * dV[k][n - 1] * G[0, k]
        dX = X[0] - X[1]
        ga -= float(np.dot(mu[n, 0] - mu[n, 1], dX))
        for k in range(2):
            gb[k] -= float(np.dot(psi[n, k], Y[k]))
    gm = ga * (-1.0 / (2.0 * m - 1.0) ** 2)
    if return_mu:
        return gG0, -gb[0], -gb[1], gm, G[N].copy(), mu[1:N + 1].copy()
    return gG0, -gb[0], -gb[1], gm, G[N].copy()


def adjoint_nodal(dim, nx, ny, alpha1, alpha2, m, T, N, G0, gN, scheme, method, np_=None, np1=16, ns=30,
                  nz=1):
    """adjoint() on the finite-difference grid (sparse nodal operators)."""
    ops = NodalOps(grid.laplacian(dim, nx, ny, nz))
    return adjoint(ops, alpha1, alpha2, m, T, N, G0, gN, scheme, method, np_, np1, ns)


def adjoint_reference(dim, nx, ny, alpha1, alpha2, m, T, N, G0, gN, scheme, method, np_=None, np1=16,
                      ns=30, nz=1):
    """adjoint() mode by mode over every sine mode: the same numbers as
    adjoint_nodal in exact arithmetic. G0 enters through the coefficient
    map c0 = P G0 (modal.to_modes) and G^N = Q cN (modal.from_modes); both
    matrices are symmetric, so dl/dcN = Q gN and dl/dG0 = P dl/dc0."""
    lam = modal.all_eigenvalues(dim, nx, ny, nz)
    c0 = modal.to_modes(G0, dim, nx, ny, nz)
    gc = modal.from_modes(gN, dim, nx, ny, nz)
    g0c, ga1, ga2, gm, cN = adjoint(ModalOps(lam), alpha1, alpha2, m, T, N, c0, gc, scheme, method, np_,
                                    np1, ns)
    return modal.to_modes(g0c, dim, nx, ny, nz), ga1, ga2, gm, modal.from_modes(cN, dim, nx, ny, nz)
