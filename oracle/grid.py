"""Finite-difference Dirichlet Laplacian on the unit interval / square / cube.

ORACLE (test infrastructure only).

A = -Delta with zero Dirichlet data (Section 2); the spatial discretisation of
the experiments is not stated in the paper, so the standard 3-point (1D),
5-point (2D) and 7-point (3D; the problem statement allows d = 1, 2, 3)
stencils on a uniform grid of interior nodes are used, h = 1/(n+1). Unknowns
are ordered x fastest, then y, then z.
"""
import numpy as np
import scipy.sparse as sp


def laplacian_1d(n: int, length: float = 1.0) -> sp.csr_matrix:
    h = length / (n + 1)
    main = np.full(n, 2.0 / h ** 2)
    off = np.full(n - 1, -1.0 / h ** 2)
    return sp.diags([off, main, off], [-1, 0, 1], format="csr")


def laplacian(dim: int, nx: int, ny: int = 1, nz: int = 1) -> sp.csr_matrix:
    if dim == 1:
        return laplacian_1d(nx)
    ax = laplacian_1d(nx)
    ay = laplacian_1d(ny)
    a2 = (sp.kron(sp.identity(ny), ax) + sp.kron(ay, sp.identity(nx))).tocsr()
    if dim == 2:
        return a2
    az = laplacian_1d(nz)
    return (sp.kron(sp.identity(nz), a2) + sp.kron(az, sp.identity(nx * ny))).tocsr()


def eigenvalues_1d(n: int, length: float = 1.0) -> np.ndarray:
    """Eigenvalues of the 3-point Dirichlet Laplacian, p = 1..n:
    (4/h^2) sin^2(p pi / (2(n+1)))."""
    h = length / (n + 1)
    p = np.arange(1, n + 1)
    return 4.0 / h ** 2 * np.sin(p * np.pi / (2 * (n + 1))) ** 2


def sine_mode_1d(n: int, p: int) -> np.ndarray:
    """Eigenvector sin(p pi i/(n+1)), i = 1..n (unnormalised)."""
    i = np.arange(1, n + 1)
    return np.sin(p * np.pi * i / (n + 1))
