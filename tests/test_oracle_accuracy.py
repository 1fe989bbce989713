"""Numerical accuracy of the oracle's two evaluations of the same scheme.

Not a pin of the formulas (those are in test_oracle_stepper): this shows that
on a 1023-node grid the per-mode evaluation (oracle.modal.reference) stays at
rounding level against a long-double evaluation of the same per-mode
recurrences, while the nodal fp64 form loses digits to the conditioning of
its stencil and sparse solve. The GPU parity tests therefore use the per-mode
evaluation as their reference."""
import numpy as np
import pytest

from oracle import modal, stepper
from paper_1901_05128_amd import workloads as wl

LD = np.longdouble


def _modal_longdouble(nx, a1, a2, m, T, N, G0, scheme):
    k = np.arange(1, nx + 1)
    S = np.sin(np.pi * np.outer(k, k).astype(LD) / LD(nx + 1))
    h = LD(1) / LD(nx + 1)
    lam = LD(4) / h ** 2 * np.sin(k.astype(LD) * np.pi / (LD(2) * (nx + 1))) ** 2
    tau = LD(T) / LD(N)
    a = (LD(1) - LD(m)) / (LD(2) * LD(m) - LD(1))

    def w(beta):
        kk = np.arange(1, N + 1).astype(LD)
        g = np.concatenate([[LD(1)], np.cumprod(LD(1) - (LD(1) + LD(beta)) / kk)])
        if scheme == 1:
            return tau ** (-LD(beta)) * g
        hh = g * (LD(1) / LD(3)) ** np.arange(N + 1).astype(LD)
        c = np.array([np.sum(g[:i + 1] * hh[i::-1]) for i in range(N + 1)])
        return tau ** (-LD(beta)) * LD(1.5) ** LD(beta) * c

    d = [w(1 - a1), w(1 - a2)]
    G = np.zeros((N + 1, 2, nx), dtype=LD)
    G[0] = (LD(2) / LD(nx + 1)) * (G0.astype(LD) @ S)
    c = LD(1) / tau if scheme == 1 else LD(1.5) / tau
    for n in range(1, N + 1):
        Sh = [np.zeros(nx, dtype=LD), np.zeros(nx, dtype=LD)]
        if n >= 2:
            for q in range(2):
                Sh[q] = d[q][1:n] @ G[n - 1:0:-1, q]
        if scheme == 1:
            E, Tt = [G[n - 1, 0] / tau, G[n - 1, 1] / tau], Sh
        else:
            g2 = G[n - 2] if n >= 2 else G[0]
            E = [(2 * G[n - 1, q] - g2[q] / 2) / tau for q in range(2)]
            Tt = [Sh[q] + d[q][n - 1] / 2 * G[0, q] for q in range(2)]
        r1 = E[0] - (a + lam) * Tt[0] + a * Tt[1]
        r2 = E[1] - (a + lam) * Tt[1] + a * Tt[0]
        p = c + d[0][0] * (a + lam)
        qq = c + d[1][0] * (a + lam)
        o12, o21 = -a * d[1][0], -a * d[0][0]
        det = p * qq - o12 * o21
        G[n, 0] = (qq * r1 - o12 * r2) / det
        G[n, 1] = (p * r2 - o21 * r1) / det
    return (G[N] @ S).astype(np.float64)


@pytest.mark.parametrize("scheme", [1, 2])
def test_modal_reference_is_rounding_accurate_on_1023_nodes(scheme):
    nx, N, T = 1023, 60, 60 / 16384
    G0 = wl.g0_intervals(nx, 2)
    ref = _modal_longdouble(nx, 0.4, 0.8, 0.45, T, N, G0, scheme)
    mod = modal.reference(1, nx, 1, 0.4, 0.8, 0.45, T, N, G0, scheme, 0)
    nod = stepper.solve(1, nx, 1, 0.4, 0.8, 0.45, T, N, G0, scheme, 0)
    e_mod = np.linalg.norm(mod - ref) / np.linalg.norm(ref)
    e_nod = np.linalg.norm(nod - ref) / np.linalg.norm(ref)
    assert e_mod <= 5e-14, e_mod
    assert e_nod > 10 * e_mod  # the conditioning the per-mode form avoids
