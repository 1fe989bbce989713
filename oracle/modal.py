"""The schemes of the stepper module for selected Laplacian eigenmodes.

ORACLE (test infrastructure only).

On the uniform grid, the discrete Dirichlet Laplacian is diagonalised by the
sine basis: A_h phi_p = lambda_p phi_p with phi_p(i) = sin(p pi i/(n+1)) and
lambda_p = (4/h^2) sin^2(p pi/(2(n+1))); in 2D phi_pq = phi_p(x) phi_q(y) and
lambda_pq = lambda_p + lambda_q, in 3D phi_pqr = phi_p(x) phi_q(y) phi_r(z) and
lambda_pqr = lambda_p + lambda_q + lambda_r. Modes are (p, q) pairs (q ignored
in 1D) or (p, q, r) triples in 3D; flattened mode and node layouts run x
fastest, then y, then z. Every scheme is linear and applies A only as
a multiplication, so the coefficient of G^n on phi_p evolves by the same
scheme with A replaced by lambda_p: a 2x2 system per step. This gives
full-length reference values for a few modes of a large grid.
"""
import numpy as np

from . import grid
from .stepper import ModalOps, run


def _mode3(mode):
    p, q = mode[0], mode[1]
    r = mode[2] if len(mode) > 2 else 1
    return p, q, r


def mode_eigenvalues(dim, nx, ny, modes, nz=1):
    lx = grid.eigenvalues_1d(nx)
    if dim == 1:
        return np.array([lx[m[0] - 1] for m in modes])
    ly = grid.eigenvalues_1d(ny)
    if dim == 2:
        return np.array([lx[m[0] - 1] + ly[m[1] - 1] for m in modes])
    lz = grid.eigenvalues_1d(nz)
    return np.array([lx[p - 1] + ly[q - 1] + lz[r - 1] for (p, q, r) in map(_mode3, modes)])


def mode_vectors(dim, nx, ny, modes, nz=1):
    """[K][nx*ny*nz] sine modes (x fastest)."""
    out = []
    for mode in modes:
        p, q, r = _mode3(mode)
        vx = grid.sine_mode_1d(nx, p)
        if dim == 1:
            out.append(vx)
            continue
        vy = grid.sine_mode_1d(ny, q)
        v = (vy[:, None] * vx[None, :]).reshape(-1)
        if dim == 3:
            vz = grid.sine_mode_1d(nz, r)
            v = (vz[:, None] * v[None, :]).reshape(-1)
        out.append(v)
    return np.array(out)


def _scale(dim, nx, ny, nz):
    s = 2.0 / (nx + 1)
    if dim >= 2:
        s *= 2.0 / (ny + 1)
    if dim == 3:
        s *= 2.0 / (nz + 1)
    return s


def project(G, dim, nx, ny, modes, nz=1):
    """Coefficients of G ([2][M]) on the given modes: G = sum c_p phi_p."""
    V = mode_vectors(dim, nx, ny, modes, nz)
    return _scale(dim, nx, ny, nz) * (np.asarray(G).reshape(2, -1) @ V.T)


def run_modes(dim, nx, ny, modes, alpha1, alpha2, m, T, N, G0, scheme, method,
              np_=None, np1=16, ns=30, nz=1):
    """Mode coefficients [2][K] of G^N, started from the projection of G0."""
    lam = mode_eigenvalues(dim, nx, ny, modes, nz)
    c0 = project(G0, dim, nx, ny, modes, nz)
    return run(ModalOps(lam), alpha1, alpha2, m, T, N, c0, scheme, method, np_, np1, ns)


def sine_matrix(n):
    """S[p-1][i-1] = sin(p pi i/(n+1)); symmetric, S S = (n+1)/2 I."""
    k = np.arange(1, n + 1)
    return np.sin(np.pi * np.outer(k, k) / (n + 1))


def to_modes(G, dim, nx, ny, nz=1):
    """All sine-mode coefficients of G ([2][M]); layout [2][nz][ny][nx]
    flattened (x-mode fastest), so that G = sum c phi exactly."""
    G = np.asarray(G, dtype=np.float64).reshape(2, -1)
    Sx = sine_matrix(nx)
    if dim == 1:
        return (2.0 / (nx + 1)) * (G @ Sx)
    Sy = sine_matrix(ny)
    out = np.empty_like(G)
    if dim == 2:
        for k in range(2):
            out[k] = ((4.0 / ((nx + 1) * (ny + 1))) * (Sy @ G[k].reshape(ny, nx) @ Sx)).reshape(-1)
        return out
    Sz = sine_matrix(nz)
    for k in range(2):
        c = np.einsum("rk,qj,pi,kji->rqp", Sz, Sy, Sx, G[k].reshape(nz, ny, nx), optimize=True)
        out[k] = (_scale(3, nx, ny, nz) * c).reshape(-1)
    return out


def from_modes(c, dim, nx, ny, nz=1):
    c = np.asarray(c).reshape(2, -1)
    Sx = sine_matrix(nx)
    if dim == 1:
        return c @ Sx
    Sy = sine_matrix(ny)
    if dim == 2:
        return np.stack([(Sy @ c[k].reshape(ny, nx) @ Sx).reshape(-1) for k in range(2)])
    Sz = sine_matrix(nz)
    return np.stack([np.einsum("rk,qj,pi,rqp->kji", Sz, Sy, Sx, c[k].reshape(nz, ny, nx),
                               optimize=True).reshape(-1) for k in range(2)])


def all_eigenvalues(dim, nx, ny, nz=1):
    lx = grid.eigenvalues_1d(nx)
    if dim == 1:
        return lx
    ly = grid.eigenvalues_1d(ny)
    l2 = (ly[:, None] + lx[None, :]).reshape(-1)
    if dim == 2:
        return l2
    lz = grid.eigenvalues_1d(nz)
    return (lz[:, None] + l2[None, :]).reshape(-1)


def reference(dim, nx, ny, alpha1, alpha2, m, T, N, G0, scheme, method, np_=None, np1=16, ns=30, nz=1):
    """G^N of the nodal scheme, computed mode by mode over every mode.

    The same numbers as stepper.solve in exact arithmetic; in fp64 the per-mode
    form avoids the conditioning kappa = lambda_max/(lambda_min + theta) of the
    nodal stencil and sparse solve, so it is the reference on large grids."""
    lam = all_eigenvalues(dim, nx, ny, nz)
    c0 = to_modes(G0, dim, nx, ny, nz)
    cN = run(ModalOps(lam), alpha1, alpha2, m, T, N, c0, scheme, method, np_, np1, ns)
    return from_modes(cN, dim, nx, ny, nz)
