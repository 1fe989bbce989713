"""Seeded synthetic workloads: grids, parameters and initial data G0.

This module only draws inputs. It holds none of the method's arithmetic (no
weights, no quadrature, no stepping), so both the GPU path's tests and the
CPU oracle may take their inputs from it.

Domain and data follow the paper's experiments (Section 5): Omega is the unit
interval or the unit square, the Laplacian carries zero Dirichlet data, and the
initial values are nonsmooth indicator functions (the paper's data (b) family),
the paper's smooth data (a) for the Table 5 workload, or, for the smallest
case, an indicator plus smooth data with seeded noise.
Grid nodes are x_i = i*h, h = 1/(n+1), i = 1..n (interior nodes only).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass(frozen=True)
class Problem:
    """One solve of the two-state system.

    dim, nx, ny : grid (ny = 1 for dim = 1); interior nodes per component.
    alpha1, alpha2 : fractional orders in (0, 1); the CQ acts with order 1 - alpha_k.
    m : transition-matrix parameter, m in [0, 1] minus {1/2}; a = (1-m)/(2m-1).
    T, N : final time and number of steps (tau = T/N).
    scheme : 1 = backward Euler CQ, 2 = BDF2 (SBD) CQ with the starting correction.
    method : 0 = direct O(N^2) history, 1 = fast sum-of-geometric-sequences history.
    """
    name: str
    dim: int
    nx: int
    ny: int
    alpha1: float
    alpha2: float
    m: float
    T: float
    N: int
    scheme: int
    method: int
    seed: int
    np_: int = 0          # fast rule size (0 = chosen by the error scan)
    ns: int = 0           # BDF2 local window (0 = default)
    g0_kind: str = "indicator"

    @property
    def M(self) -> int:
        return self.nx * self.ny

    @property
    def a(self) -> float:
        return (1.0 - self.m) / (2.0 * self.m - 1.0)

    def with_(self, **kw) -> "Problem":
        d = dict(self.__dict__)
        d.update(kw)
        return Problem(**d)


def nodes_1d(n: int) -> np.ndarray:
    h = 1.0 / (n + 1)
    return h * np.arange(1, n + 1, dtype=np.float64)


def g0_c1(nx: int, seed: int) -> np.ndarray:
    """G1 = indicator(x < 1/2) (strict, so the node x = 1/2 gets 0);
    G2 = x(1-x) + U(0, 0.1) noise drawn with the given seed."""
    rng = np.random.default_rng(seed)
    x = nodes_1d(nx)
    g1 = (x < 0.5).astype(np.float64)
    g2 = x * (1.0 - x) + rng.uniform(0.0, 0.1, size=nx)
    return np.stack([g1, g2])


def g0_intervals(nx: int, seed: int) -> np.ndarray:
    """G_k = indicator of the closed interval [u_k, v_k] with (u_k, v_k) the
    sorted pair of two U(0,1) draws; one interval per component."""
    rng = np.random.default_rng(seed)
    x = nodes_1d(nx)
    out = []
    for _ in range(2):
        u, v = np.sort(rng.uniform(0.0, 1.0, size=2))
        out.append(((x >= u) & (x <= v)).astype(np.float64))
    return np.stack(out)


def g0_rectangle(nx: int, ny: int, seed: int) -> np.ndarray:
    """G1 = G2 = indicator of one closed rectangle [u1,v1] x [u2,v2] drawn from
    sorted U(0,1) pairs; a rectangle that covers no grid node is drawn again
    from the same stream. Layout [2][ny][nx] flattened to [2][ny*nx] (x fastest)."""
    rng = np.random.default_rng(seed)
    x = nodes_1d(nx)
    y = nodes_1d(ny)
    while True:
        ux, vx = np.sort(rng.uniform(0.0, 1.0, size=2))
        uy, vy = np.sort(rng.uniform(0.0, 1.0, size=2))
        ind = ((y[:, None] >= uy) & (y[:, None] <= vy) & (x[None, :] >= ux) & (x[None, :] <= vx))
        if ind.any():
            break
    f = ind.astype(np.float64).reshape(-1)
    return np.stack([f, f.copy()])


def g0_smooth(nx: int, ny: int = 1) -> np.ndarray:
    """The paper's smooth initial data (a) of Section 5: G1 = x(1-x),
    G2 = sin(x) at the interior nodes (1D). In 2D (not in the paper) the
    same profiles in x times y(1-y)."""
    x = nodes_1d(nx)
    g1, g2 = x * (1.0 - x), np.sin(x)
    if ny > 1:
        y = nodes_1d(ny)
        f = y * (1.0 - y)
        g1 = (f[:, None] * g1[None, :]).reshape(-1)
        g2 = (f[:, None] * g2[None, :]).reshape(-1)
    return np.stack([g1, g2])


def g0_nonsmooth_b(nx: int) -> np.ndarray:
    """The paper's nonsmooth data (b) of Section 5 (1D): G1 = (1-x) on (1/2, 1),
    G2 = x on (0, 1/2), zero elsewhere (open intervals: the node x = 1/2 is 0)."""
    x = nodes_1d(nx)
    return np.stack([np.where(x > 0.5, 1.0 - x, 0.0), np.where(x < 0.5, x, 0.0)])


def g0_box(nx: int, ny: int, nz: int, seed: int) -> np.ndarray:
    """G1 = G2 = indicator of one closed box [u1,v1] x [u2,v2] x [u3,v3] from
    sorted U(0,1) pairs (drawn again until it covers a grid node). Layout
    [2][nz][ny][nx] flattened (x fastest)."""
    rng = np.random.default_rng(seed)
    x, y, z = nodes_1d(nx), nodes_1d(ny), nodes_1d(nz)
    while True:
        b = [np.sort(rng.uniform(0.0, 1.0, size=2)) for _ in range(3)]
        ind = ((z[:, None, None] >= b[2][0]) & (z[:, None, None] <= b[2][1])
               & (y[None, :, None] >= b[1][0]) & (y[None, :, None] <= b[1][1])
               & (x[None, None, :] >= b[0][0]) & (x[None, None, :] <= b[0][1]))
        if ind.any():
            break
    f = ind.astype(np.float64).reshape(-1)
    return np.stack([f, f.copy()])


def g0_random(M: int, seed: int) -> np.ndarray:
    """Plain seeded U(-1,1) data on every node (for operator-level tests)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(2, M))


def g0_for(p: Problem) -> np.ndarray:
    if p.g0_kind == "c1":
        return g0_c1(p.nx, p.seed)
    if p.g0_kind == "random":
        return g0_random(p.M, p.seed)
    if p.g0_kind == "smooth":
        return g0_smooth(p.nx, p.ny)
    if p.dim == 1:
        return g0_intervals(p.nx, p.seed)
    return g0_rectangle(p.nx, p.ny, p.seed)


# The five workloads: small 1D BE direct; 1D 1023 nodes; 2D 255^2; batched; adjoint.
C1 = Problem("c1_1d127_be_direct", 1, 127, 1, 0.3, 0.7, 0.3, 1.0, 1000, 1, 0, 1, g0_kind="c1")
C2 = Problem("c2_1d1023", 1, 1023, 1, 0.4, 0.8, 0.45, 1.0, 2 ** 14, 1, 1, 2)
C3 = Problem("c3_2d255", 2, 255, 255, 0.2, 0.6, 0.55, 1.0, 2 ** 16, 2, 1, 3)
C5 = Problem("c5_adjoint_2d127", 2, 127, 127, 0.2, 0.6, 0.55, 1.0, 4096, 2, 1, 5, np_=192, ns=30)
# The paper's Table 5 problem: 1D h = 1/1024, T = 10, tau = 1/2000 (N = 20000),
# a = -1 (m = 0), BDF2 (SBD) direct and fast, smooth data (a); the three order
# pairs of the table.
T5 = Problem("t5_1d1023_T10", 1, 1023, 1, 0.3, 0.8, 0.0, 10.0, 20000, 2, 1, 0, g0_kind="smooth")
T5_ORDERS = [(0.3, 0.8), (0.4, 0.7), (0.5, 0.6)]


def batched_instances(count: int = 256, seed: int = 4, scale: float = 1.0):
    """Seeded mix of fast-BDF2 instances: 1D or 2D with probability 1/2 each;
    1D nodes 2^k - 1 with k in U{7..12}; 2D sides 2^k - 1 with k in U{6,7,8};
    N = 2^k with k in U{10..15}; alpha_k ~ U(0.1, 0.9);
    m ~ U((0.05, 0.45) U (0.55, 0.95)). `scale` < 1 shrinks N for quick tests."""
    rng = np.random.default_rng(seed)
    out = []
    for b in range(count):
        is2d = rng.uniform() < 0.5
        if is2d:
            k = int(rng.integers(6, 9))
            nx = ny = 2 ** k - 1
        else:
            k = int(rng.integers(7, 13))
            nx, ny = 2 ** k - 1, 1
        N = 2 ** int(rng.integers(10, 16))
        N = max(8, int(N * scale))
        a1, a2 = rng.uniform(0.1, 0.9, size=2)
        lo = rng.uniform() < 0.5
        m = rng.uniform(0.05, 0.45) if lo else rng.uniform(0.55, 0.95)
        out.append(Problem(f"batch{b}", 2 if is2d else 1, nx, ny, float(a1), float(a2), float(m),
                           1.0, N, 2, 1, 1000 + b))
    return out
