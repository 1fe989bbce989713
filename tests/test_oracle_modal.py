"""Pins of the oracle's per-mode evaluations against its nodal steppers.

Every GPU parity test compares with oracle.modal.reference (and the adjoint
tests with oracle.adjoint.adjoint_reference): the scheme evaluated mode by
mode after a sine transform. Here they are held to the nodal evaluations
(oracle.stepper.solve, oracle.adjoint.adjoint_nodal: sparse A_h, sparse LU of
the coupled 2M x 2M step operator of (4.1)/(4.7)) on grids small enough that
the nodal form is well conditioned. A slip in the transform's scale or
orientation, in the mode eigenvalues, or in the mode ordering of the 2D
layout fails these."""
import numpy as np
import pytest

from oracle import adjoint as adj
from oracle import modal, stepper
from paper_1901_05128_amd import workloads as wl

FAST = dict(np_=12, np1=8, ns=10)
GEOMS = [(1, 15, 1), (2, 7, 5)]


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("m", [0.3, 0.7, 0.0, 1.0])
def test_modal_reference_equals_nodal_stepper(geom, scheme, method, m):
    dim, nx, ny = geom
    M = nx * ny
    N = 60
    G0 = wl.g0_random(M, 21).reshape(2, M)
    ref = modal.reference(dim, nx, ny, 0.35, 0.75, m, 1.0, N, G0, scheme, method, **FAST)
    nod = stepper.solve(dim, nx, ny, 0.35, 0.75, m, 1.0, N, G0, scheme, method, **FAST)
    err = np.linalg.norm(ref - nod) / np.linalg.norm(nod)
    assert err <= 1e-12, err


@pytest.mark.parametrize("geom", GEOMS)
def test_sine_transform_round_trip_and_modes(geom):
    """to_modes inverts from_modes, and a single sine mode maps to a unit
    coefficient at its (row = y-mode, column = x-mode) slot."""
    dim, nx, ny = geom
    M = nx * ny
    rng = np.random.default_rng(4)
    G = rng.standard_normal((2, M))
    assert np.allclose(modal.from_modes(modal.to_modes(G, dim, nx, ny), dim, nx, ny), G, rtol=0, atol=1e-13)
    p, q = (3, 1) if dim == 1 else (3, 2)
    v = modal.mode_vectors(dim, nx, ny, [(p, q)])[0]
    c = modal.to_modes(np.stack([v, 2 * v]), dim, nx, ny)
    slot = (q - 1) * nx + (p - 1)
    e = np.zeros(M)
    e[slot] = 1.0
    assert np.allclose(c, np.stack([e, 2 * e]), rtol=0, atol=1e-13)
    # and A_h v = lambda v with the eigenvalue the reference assigns to that slot
    from oracle import grid
    A = grid.laplacian(dim, nx, ny)
    lam = modal.all_eigenvalues(dim, nx, ny)[slot]
    assert np.allclose(A @ v, lam * v, rtol=1e-13, atol=1e-10)


@pytest.mark.parametrize("geom", GEOMS)
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
def test_adjoint_reference_equals_nodal_adjoint(geom, scheme, method):
    dim, nx, ny = geom
    M = nx * ny
    N = 40
    G0 = wl.g0_random(M, 5).reshape(2, M)
    gN = np.random.default_rng(12).standard_normal((2, M))
    m = 0.35 if dim == 1 else 0.55
    r = adj.adjoint_reference(dim, nx, ny, 0.3, 0.7, m, 1.0, N, G0, gN, scheme, method, **FAST)
    n = adj.adjoint_nodal(dim, nx, ny, 0.3, 0.7, m, 1.0, N, G0, gN, scheme, method, **FAST)
    e0 = np.linalg.norm(r[0] - n[0]) / np.linalg.norm(n[0])
    assert e0 <= 1e-12, e0
    for k in (1, 2, 3):
        assert abs(r[k] - n[k]) <= 1e-11 * abs(n[k]), (k, r[k], n[k])
    eN = np.linalg.norm(r[4] - n[4]) / np.linalg.norm(n[4])
    assert eN <= 1e-12, eN
