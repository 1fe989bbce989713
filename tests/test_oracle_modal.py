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


# ------------------------------------------------------------------ 3D (d = 3)
GEOM3 = (3, 5, 4, 3)   # dim, nx, ny, nz


def test_laplacian_3d_is_the_seven_point_stencil():
    """A_h of the 3D grid applied to a random field equals the 7-point
    stencil written out node by node (zero Dirichlet data outside)."""
    from oracle import grid
    _, nx, ny, nz = GEOM3
    rng = np.random.default_rng(8)
    u = rng.standard_normal((nz, ny, nx))
    A = grid.laplacian(3, nx, ny, nz)
    hx, hy, hz = 1.0 / (nx + 1), 1.0 / (ny + 1), 1.0 / (nz + 1)
    pad = np.zeros((nz + 2, ny + 2, nx + 2))
    pad[1:-1, 1:-1, 1:-1] = u
    ref = np.empty_like(u)
    for k in range(nz):
        for j in range(ny):
            for i in range(nx):
                c = pad[k + 1, j + 1, i + 1]
                ref[k, j, i] = ((2 * c - pad[k + 1, j + 1, i] - pad[k + 1, j + 1, i + 2]) / hx ** 2
                                + (2 * c - pad[k + 1, j, i + 1] - pad[k + 1, j + 2, i + 1]) / hy ** 2
                                + (2 * c - pad[k, j + 1, i + 1] - pad[k + 2, j + 1, i + 1]) / hz ** 2)
    assert np.allclose(A @ u.reshape(-1), ref.reshape(-1), rtol=1e-13, atol=1e-9)


def test_sine_transform_3d_round_trip_and_modes():
    from oracle import grid
    dim, nx, ny, nz = GEOM3
    M = nx * ny * nz
    G = np.random.default_rng(9).standard_normal((2, M))
    assert np.allclose(modal.from_modes(modal.to_modes(G, dim, nx, ny, nz), dim, nx, ny, nz), G, rtol=0,
                       atol=1e-13)
    p, q, r = 4, 2, 3
    v = modal.mode_vectors(dim, nx, ny, [(p, q, r)], nz)[0]
    c = modal.to_modes(np.stack([v, -v]), dim, nx, ny, nz)
    slot = (r - 1) * nx * ny + (q - 1) * nx + (p - 1)
    e = np.zeros(M)
    e[slot] = 1.0
    assert np.allclose(c, np.stack([e, -e]), rtol=0, atol=1e-13)
    lam = modal.all_eigenvalues(dim, nx, ny, nz)[slot]
    assert np.allclose(grid.laplacian(3, nx, ny, nz) @ v, lam * v, rtol=1e-13, atol=1e-10)
    assert lam == pytest.approx(modal.mode_eigenvalues(dim, nx, ny, [(p, q, r)], nz)[0], rel=1e-15)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("m", [0.3, 0.7])
def test_modal_reference_equals_nodal_stepper_3d(scheme, method, m):
    dim, nx, ny, nz = GEOM3
    M = nx * ny * nz
    N = 40
    G0 = wl.g0_random(M, 22).reshape(2, M)
    ref = modal.reference(dim, nx, ny, 0.35, 0.75, m, 1.0, N, G0, scheme, method, nz=nz, **FAST)
    nod = stepper.solve(dim, nx, ny, 0.35, 0.75, m, 1.0, N, G0, scheme, method, nz=nz, **FAST)
    err = np.linalg.norm(ref - nod) / np.linalg.norm(nod)
    assert err <= 1e-12, err


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
def test_adjoint_reference_equals_nodal_adjoint_3d(scheme, method):
    dim, nx, ny, nz = GEOM3
    M = nx * ny * nz
    N = 30
    G0 = wl.g0_random(M, 6).reshape(2, M)
    gN = np.random.default_rng(13).standard_normal((2, M))
    r = adj.adjoint_reference(dim, nx, ny, 0.3, 0.7, 0.6, 1.0, N, G0, gN, scheme, method, nz=nz, **FAST)
    n = adj.adjoint_nodal(dim, nx, ny, 0.3, 0.7, 0.6, 1.0, N, G0, gN, scheme, method, nz=nz, **FAST)
    assert np.linalg.norm(r[0] - n[0]) <= 1e-12 * np.linalg.norm(n[0])
    for k in (1, 2, 3):
        assert abs(r[k] - n[k]) <= 1e-11 * abs(n[k]), (k, r[k], n[k])


# ------------------------------------------- long-double per-mode reference
@pytest.mark.parametrize("geom", [(1, 63, 1, 1), (2, 15, 13, 1), (3, 7, 5, 4)])
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("m", [0.45, 0.8, 0.0])
def test_long_double_modes_equal_fp64_modes(geom, scheme, m):
    """oracle.modal_ld (the direct schemes per mode in extended precision,
    plain C) equals the fp64 per-mode oracle, which the tests above pin to
    the nodal steppers, to the fp64 side's rounding over a few hundred
    steps."""
    from oracle import modal_ld
    dim, nx, ny, nz = geom
    M = nx * ny * nz
    G0 = wl.g0_random(M, 17).reshape(2, M)
    if dim == 1:
        modes = [(1, 1), (2, 1), (17, 1), (63, 1)]
    elif dim == 2:
        modes = [(1, 1), (3, 2), (15, 13), (7, 1)]
    else:
        modes = [(1, 1, 1), (3, 2, 4), (7, 5, 4), (2, 5, 1)]
    a = modal_ld.run_modes_ld(dim, nx, ny, modes, 0.4, 0.8, m, 1.0, 300, G0, scheme, nz=nz)
    b = modal.run_modes(dim, nx, ny, modes, 0.4, 0.8, m, 1.0, 300, G0, scheme, 0, nz=nz)
    assert np.max(np.abs(a - b)) <= 5e-13 * np.max(np.abs(b)), np.max(np.abs(a - b))
