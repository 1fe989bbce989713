"""Direct and fast CQ time steppers for the two-state system (2.1).

ORACLE (test infrastructure only).

System (2.1), with a = (1-m)/(2m-1), A = -Delta (Dirichlet):
  dG1/dt + a D^{1-a1} G1 + D^{1-a1} A G1 = a D^{1-a2} G2,
  dG2/dt + a D^{1-a2} G2 + D^{1-a2} A G2 = a D^{1-a1} G1.
Write d_k,i for the CQ weights of order beta_k = 1 - alpha_k.

Schemes, in the paper's form:
  BE (4.1), n >= 1:
    (G1^n - G1^{n-1})/tau + sum_{i=0}^{n-1} d1_i (a + A) G1^{n-i}
        = a sum_{i=0}^{n-1} d2_i G2^{n-i}           (and 1 <-> 2).
    The CQ sums omit G^0 (remark after (4.3)).
  fast BE (4.2)/(4.3): the same with d_i, i >= 2, replaced by the
    Gauss-Jacobi sums, evaluated through the history parts
    Gh_j(t_n) = r_j Gh_j(t_{n-1}) + w_j G^{n-2}   (n >= 3, Gh_j(t_2) = 0).
  BDF2 (4.7):
    n = 1: (G1^1 - G1^0)/tau + d1_0 (a + A)(2/3 G1^1 + 1/3 G1^0)
               = a d2_0 (2/3 G2^1 + 1/3 G2^0),
    n >= 2: (3/2 G1^n - 2 G1^{n-1} + 1/2 G1^{n-2})/tau
               + (a + A) [sum_{i=0}^{n-1} d1_i G1^{n-i} + 1/2 d1_{n-1} G1^0]
               = a [sum_{i=0}^{n-1} d2_i G2^{n-i} + 1/2 d2_{n-1} G2^0].
  fast BDF2 (4.8): the same, with d_i for i >= N_s replaced by the two
    Gauss-Jacobi families; history parts (remark after (4.8)) over
    i = N_s..n-1 with
    Gh^{2,l}_j(t_n) = r_j Gh^{2,l}_j(t_{n-1}) + w_{l,j} dbar^l_{2,N_s}(s_j) G^{n-N_s}.
    The correction term keeps the exact d_{n-1}.

The spatial operator is abstract: NodalOps applies the sparse A_h and solves
the coupled 2M x 2M system with a sparse LU; ModalOps does the same for a set
of Laplacian eigenvalues (A -> lambda), where the system is 2x2 per mode.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import grid
from .quadrature import be_rule, bdf2_rules
from .weights import weights


class NodalOps:
    def __init__(self, A: sp.csr_matrix):
        self.Amat = A.tocsr()
        self.n = A.shape[0]

    def apply(self, v):
        return self.Amat @ v

    def factor(self, e1, f1, o12, o21, e2, f2):
        """LU of [[e1 I + f1 A, o12 I], [o21 I, e2 I + f2 A]]."""
        I = sp.identity(self.n, format="csr")
        K = sp.bmat([[e1 * I + f1 * self.Amat, o12 * I], [o21 * I, e2 * I + f2 * self.Amat]], format="csc")
        lu = spla.splu(K)
        n = self.n

        def solve(r1, r2):
            x = lu.solve(np.concatenate([r1, r2]))
            return x[:n], x[n:]
        return solve


class ModalOps:
    def __init__(self, lam):
        self.lam = np.asarray(lam, dtype=np.float64)
        self.n = self.lam.shape[0]

    def apply(self, v):
        return self.lam * v

    def factor(self, e1, f1, o12, o21, e2, f2):
        p = e1 + f1 * self.lam
        q = e2 + f2 * self.lam
        det = p * q - o12 * o21

        def solve(r1, r2):
            return (q * r1 - o12 * r2) / det, (p * r2 - o21 * r1) / det
        return solve


def default_np(N: int) -> int:
    """Placeholder rule size when the caller gives none: 3 sqrt(N), at least 16."""
    return max(16, int(np.ceil(3.0 * np.sqrt(N))))


def run(ops, alpha1, alpha2, m, T, N, G0, scheme, method, np_=None, np1=16, ns=30,
        keep=False):
    """Advance G0 ([2][n]) by N steps of size tau = T/N. Returns G^N, or the
    whole trajectory [N+1][2][n] when keep is true."""
    if scheme not in (1, 2) or method not in (0, 1):
        raise ValueError("bad scheme/method")
    tau = T / N
    a = (1.0 - m) / (2.0 * m - 1.0)
    beta = (1.0 - alpha1, 1.0 - alpha2)
    d = [weights(scheme, beta[k], tau, N) for k in range(2)]
    n_sp = ops.n
    G = np.zeros((N + 1, 2, n_sp))
    G[0] = np.asarray(G0, dtype=np.float64).reshape(2, n_sp)
    A = ops.apply

    # implicit operator of the n-th step
    if scheme == 1:
        c = 1.0 / tau
        solve_n = ops.factor(c + d[0][0] * a, d[0][0], -a * d[1][0], -a * d[0][0], c + d[1][0] * a, d[1][0])
    else:
        c = 1.5 / tau
        solve_n = ops.factor(c + d[0][0] * a, d[0][0], -a * d[1][0], -a * d[0][0], c + d[1][0] * a, d[1][0])
        t = 2.0 / 3.0
        solve_1 = ops.factor(1.0 / tau + t * d[0][0] * a, t * d[0][0], -t * a * d[1][0], -t * a * d[0][0],
                             1.0 / tau + t * d[1][0] * a, t * d[1][0])

    # fast history parts
    if method == 1:
        if np_ is None:
            np_ = default_np(N)
        rules = []
        for k in range(2):
            if scheme == 1:
                rk = [be_rule(beta[k], tau, np_)]
                lag = 2
            else:
                rk = list(bdf2_rules(beta[k], tau, np1, np_))
                lag = ns
            rules.append(rk)
        # source coefficient of G^{n-lag}: w_j * dbar_lag(s_j)
        src = [[r.w * r.dbar(lag) for r in rules[k]] for k in range(2)]
        hist = [[np.zeros((len(r.w), n_sp)) for r in rules[k]] for k in range(2)]

    for n in range(1, N + 1):
        S = [np.zeros(n_sp), np.zeros(n_sp)]
        if method == 0:
            if n >= 2:
                for k in range(2):
                    S[k] = d[k][1:n] @ G[n - 1:0:-1, k]
        else:
            for k in range(2):
                top = min(lag - 1, n - 1)           # exact weights d_1..d_top
                if top >= 1:
                    S[k] = d[k][1:top + 1] @ G[n - 1:n - top - 1:-1, k]
                if n >= lag + 1:
                    g = G[n - lag, k]
                    for l, r in enumerate(rules[k]):
                        hist[k][l] = r.ratio[:, None] * hist[k][l] + src[k][l][:, None] * g[None, :]
                        S[k] = S[k] + hist[k][l].sum(axis=0)

        if scheme == 1:
            r1 = G[n - 1, 0] / tau - (a * S[0] + A(S[0])) + a * S[1]
            r2 = G[n - 1, 1] / tau - (a * S[1] + A(S[1])) + a * S[0]
            G[n, 0], G[n, 1] = solve_n(r1, r2)
        elif n == 1:
            g1, g2 = G[0, 0], G[0, 1]
            t = 1.0 / 3.0
            r1 = g1 / tau - t * d[0][0] * (a * g1 + A(g1)) + t * a * d[1][0] * g2
            r2 = g2 / tau - t * d[1][0] * (a * g2 + A(g2)) + t * a * d[0][0] * g1
            G[1, 0], G[1, 1] = solve_1(r1, r2)
        else:
            corr = [0.5 * d[k][n - 1] * G[0, k] for k in range(2)]
            T1 = S[0] + corr[0]
            T2 = S[1] + corr[1]
            r1 = (2.0 * G[n - 1, 0] - 0.5 * G[n - 2, 0]) / tau - (a * T1 + A(T1)) + a * T2
            r2 = (2.0 * G[n - 1, 1] - 0.5 * G[n - 2, 1]) / tau - (a * T2 + A(T2)) + a * T1
            G[n, 0], G[n, 1] = solve_n(r1, r2)
        if not keep and n >= 2 and method == 0:
            pass
    return G if keep else G[N].copy()


def solve(dim, nx, ny, alpha1, alpha2, m, T, N, G0, scheme, method, np_=None, np1=16, ns=30,
          keep=False, nz=1):
    """Nodal solve on the FD grid; G0 is [2][nx*ny*nz] (x fastest)."""
    ops = NodalOps(grid.laplacian(dim, nx, ny, nz))
    return run(ops, alpha1, alpha2, m, T, N, G0, scheme, method, np_, np1, ns, keep)


def cq_history(d, G_hist):
    """S = sum_{i=1}^{n-1} d_i G^{n-i} for G_hist = [G^0..G^{n-1}] ([n][M])
    (the CQ sum without G^0, (3.8) as used in (4.1))."""
    n = G_hist.shape[0]
    if n < 2:
        return np.zeros(G_hist.shape[1])
    return d[1:n] @ G_hist[n - 1:0:-1]
