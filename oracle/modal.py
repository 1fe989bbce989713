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
