"""The schemes of the stepper module for selected Laplacian eigenmodes.

ORACLE (test infrastructure only).

On the uniform grid, the discrete Dirichlet Laplacian is diagonalised by the
sine basis: A_h phi_p = lambda_p phi_p with phi_p(i) = sin(p pi i/(n+1)) and
lambda_p = (4/h^2) sin^2(p pi/(2(n+1))); in 2D phi_pq = phi_p(x) phi_q(y) and
lambda_pq = lambda_p + lambda_q. Every scheme is linear and applies A only as
a multiplication, so the coefficient of G^n on phi_p evolves by the same
scheme with A replaced by lambda_p: a 2x2 system per step. This gives
full-length reference values for a few modes of a large grid.
"""
import numpy as np

from . import grid
from .stepper import ModalOps, run


def mode_eigenvalues(dim, nx, ny, modes):
    lx = grid.eigenvalues_1d(nx)
    if dim == 1:
        return np.array([lx[p - 1] for (p, _q) in modes])
    ly = grid.eigenvalues_1d(ny)
    return np.array([lx[p - 1] + ly[q - 1] for (p, q) in modes])


def mode_vectors(dim, nx, ny, modes):
    """[K][nx*ny] sine modes (x fastest)."""
    out = []
    for (p, q) in modes:
        vx = grid.sine_mode_1d(nx, p)
        if dim == 1:
            out.append(vx)
        else:
            vy = grid.sine_mode_1d(ny, q)
            out.append((vy[:, None] * vx[None, :]).reshape(-1))
    return np.array(out)


def project(G, dim, nx, ny, modes):
    """Coefficients of G ([2][M]) on the given modes: G = sum c_p phi_p."""
    V = mode_vectors(dim, nx, ny, modes)
    scale = 2.0 / (nx + 1) if dim == 1 else 4.0 / ((nx + 1) * (ny + 1))
    return scale * (np.asarray(G).reshape(2, -1) @ V.T)


def run_modes(dim, nx, ny, modes, alpha1, alpha2, m, T, N, G0, scheme, method,
              np_=None, np1=16, ns=30):
    """Mode coefficients [2][K] of G^N, started from the projection of G0."""
    lam = mode_eigenvalues(dim, nx, ny, modes)
    c0 = project(G0, dim, nx, ny, modes)
    return run(ModalOps(lam), alpha1, alpha2, m, T, N, c0, scheme, method, np_, np1, ns)


def sine_matrix(n):
    """S[p-1][i-1] = sin(p pi i/(n+1)); symmetric, S S = (n+1)/2 I."""
    k = np.arange(1, n + 1)
    return np.sin(np.pi * np.outer(k, k) / (n + 1))


def to_modes(G, dim, nx, ny):
    """All sine-mode coefficients of G ([2][M]); layout [2][ny][nx] flattened
    (row = y-mode, column = x-mode), so that G = sum c phi exactly."""
    G = np.asarray(G, dtype=np.float64).reshape(2, -1)
    Sx = sine_matrix(nx)
    if dim == 1:
        return (2.0 / (nx + 1)) * (G @ Sx)
    Sy = sine_matrix(ny)
    out = np.empty_like(G)
    for k in range(2):
        out[k] = ((4.0 / ((nx + 1) * (ny + 1))) * (Sy @ G[k].reshape(ny, nx) @ Sx)).reshape(-1)
    return out


def from_modes(c, dim, nx, ny):
    c = np.asarray(c).reshape(2, -1)
    Sx = sine_matrix(nx)
    if dim == 1:
        return c @ Sx
    Sy = sine_matrix(ny)
    return np.stack([(Sy @ c[k].reshape(ny, nx) @ Sx).reshape(-1) for k in range(2)])


def all_eigenvalues(dim, nx, ny):
    lx = grid.eigenvalues_1d(nx)
    if dim == 1:
        return lx
    ly = grid.eigenvalues_1d(ny)
    return (ly[:, None] + lx[None, :]).reshape(-1)


def reference(dim, nx, ny, alpha1, alpha2, m, T, N, G0, scheme, method, np_=None, np1=16, ns=30):
    """G^N of the nodal scheme, computed mode by mode over every mode.

    The same numbers as stepper.solve in exact arithmetic; in fp64 the per-mode
    form avoids the conditioning kappa = lambda_max/(lambda_min + theta) of the
    nodal stencil and sparse solve, so it is the reference on large grids."""
    lam = all_eigenvalues(dim, nx, ny)
    c0 = to_modes(G0, dim, nx, ny)
    cN = run(ModalOps(lam), alpha1, alpha2, m, T, N, c0, scheme, method, np_, np1, ns)
    return from_modes(cN, dim, nx, ny)
