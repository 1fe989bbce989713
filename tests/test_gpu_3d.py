"""GPU parity in 3D (the problem (1.1) is posed for d = 1, 2, 3): 7-point
Laplacian on the unit cube, nodal solver (sine transforms along x, y and z
with the 2x2 solve per mode, every step) and modal solver, direct and fast,
BE and BDF2, against the oracle's per-mode evaluation over every mode
(oracle.modal.reference, pinned to the nodal 3D stepper on the CPU).
Bars as in 1D and 2D: direct 1e-12, fast 1e-8 against the direct scheme
and 1e-11 against the oracle's fast scheme with the same node counts. A
3D problem in a batch, the 3D adjoint, and a 63^3 grid at N = 2^12 on
sampled modes against the long-double direct scheme complete the set."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1901_05128_amd as cq  # noqa: E402
from oracle import adjoint as adj  # noqa: E402
from oracle import modal, modal_ld  # noqa: E402
from paper_1901_05128_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cq.lib()


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


CASES = [
    # nx, ny, nz, alpha1, alpha2, m, T, N
    (9, 7, 5, 0.3, 0.7, 0.35, 1.0, 120),      # ragged GEMM tiles, a < 0
    (31, 17, 13, 0.2, 0.6, 0.55, 1.0, 100),   # 6851 modes
    (33, 33, 33, 0.4, 0.8, 0.0, 1.0, 90),     # 35937 modes (time-blocked modal fast form), a = -1
    (1, 1, 1, 0.5, 0.5, 0.7, 1.0, 9),         # one node
    (1, 6, 3, 0.35, 0.65, 0.8, 1.0, 70),      # degenerate x
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}N{c[7]}")
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("solver", [0, 1], ids=["nodal", "modal"])
def test_3d_solve_matches_oracle(case, scheme, method, solver):
    nx, ny, nz, a1, a2, m, T, N = case
    print(f"3d case={case} scheme={scheme} method={method} solver={solver}", flush=True)
    M = nx * ny * nz
    G0 = wl.g0_box(nx, ny, nz, 7) if M > 8 else wl.g0_random(M, 7)
    g = cq.make_grid(3, nx, ny, nz=nz)
    p = cq.make_params(a1, a2, m, T, N, scheme, method, solver=solver)
    with cq.Solver(g, p, dev(G0)) as s:
        info = s.info()
        s.step(N)
        out, n = s.current()
        out = out.cpu().numpy()
    assert n == N
    ref = modal.reference(3, nx, ny, a1, a2, m, T, N, G0, scheme, 0, nz=nz)
    e = rel(out, ref)
    print(f"  rel_l2 vs direct reference {e:.3e}", flush=True)
    if method == 0:
        assert e <= 1e-12, e
        return
    assert e <= 1e-8, e
    if N > info.lag:
        np_ = info.np_total - info.np1
        ref_f = modal.reference(3, nx, ny, a1, a2, m, T, N, G0, scheme, 1, np_=np_, np1=info.np1 or 16,
                                ns=info.lag, nz=nz)
        ef = rel(out, ref_f)
        print(f"  rel_l2 vs fast reference {ef:.3e}", flush=True)
        assert ef <= 1e-11, ef


def test_3d_rejects_bad_grids():
    p = cq.make_params(0.3, 0.7, 0.3, 1.0, 10, 1, 0, solver=1)
    G0 = dev(np.zeros((2, 8)))
    for g in (cq.make_grid(3, 2, 2, nz=0), cq._lib.Grid(2, 2, 2, 1.0, 1.0, 2, 1.0),
              cq._lib.Grid(3, 2, 2, 1.0, 1.0, 2, 0.0)):
        with pytest.raises(cq.CQError):
            cq.Solver(g, p, G0)


@pytest.mark.parametrize("scheme", [1, 2])
def test_3d_whole_run_on_the_mfma_kernel(scheme):
    """fast_kernel 1 on a 3D grid (ragged 16-mode tiles over x, y and z):
    the whole run in one launch of the 16-mode MFMA kernel, within 1e-13 of
    the streamed run and within the fast scheme's bar of the oracle."""
    nx, ny, nz, N = 9, 7, 6, 100
    M = nx * ny * nz
    G0 = wl.g0_random(M, 88)
    g = cq.make_grid(3, nx, ny, nz=nz)
    kw = dict(np_=24, ns=30) if scheme == 2 else dict(np_=24)
    outs = []
    for fk in (0, 1):
        p = cq.make_params(0.25, 0.7, 0.65, 1.0, N, scheme, 1, solver=cq.SOLVER_MODAL, fast_kernel=fk, **kw)
        outs.append(cq.fp_solve(g, p, dev(G0)).cpu().numpy())
    ref = modal.reference(3, nx, ny, 0.25, 0.7, 0.65, 1.0, N, G0, scheme, 1, np1=16, nz=nz, **kw)
    e, e2 = rel(outs[1], outs[0]), rel(outs[1], ref)
    print(f"  3d whole run scheme={scheme}: vs streamed {e:.2e}, vs oracle fast {e2:.2e}", flush=True)
    assert e <= 1e-13
    assert e2 <= 1e-11


@pytest.mark.parametrize("kernel", [cq.BATCH_DEFAULT, cq.BATCH_TIME_BLOCKED])
def test_3d_in_a_batch(kernel):
    """A 3D problem solved by fp_solve_batched next to 1D and 2D ones, by the
    default choice (the 16-mode MFMA kernel for these problems) and by the
    time-blocked kernel."""
    probs = [(3, 15, 11, 7, 0.3, 0.7, 0.4, 300), (1, 127, 1, 1, 0.6, 0.2, 0.8, 500),
             (2, 31, 29, 1, 0.45, 0.55, 0.3, 400)]
    grids, params, g0s, refs = [], [], [], []
    for i, (dim, nx, ny, nz, a1, a2, m, N) in enumerate(probs):
        M = nx * ny * nz
        G0 = wl.g0_random(M, 70 + i)
        grids.append(cq.make_grid(dim, nx, ny, nz=nz))
        params.append(cq.make_params(a1, a2, m, 1.0, N, 2, 1, np_=24))
        g0s.append(dev(G0))
        refs.append(modal.reference(dim, nx, ny, a1, a2, m, 1.0, N, G0, 2, 1, np_=24, ns=30, nz=nz))
    outs, rep = cq.fp_solve_batched(grids, params, g0s, autotune=kernel)
    assert all(x == (2 if kernel == cq.BATCH_DEFAULT else 1) for x in list(rep.class_blocked)[:rep.classes])
    for (dim, nx, ny, nz, *_r), out, ref in zip(probs, outs, refs):
        e = rel(out.cpu().numpy(), ref)
        print(f"  batch {dim}d {nx}x{ny}x{nz}: rel_l2 vs oracle fast {e:.3e}", flush=True)
        assert e <= 1e-11, e


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
def test_3d_adjoint_matches_oracle(scheme, method):
    nx, ny, nz, N = 9, 7, 6, 80
    M = nx * ny * nz
    G0 = wl.g0_random(M, 81).reshape(2, M)
    gN = np.random.default_rng(82).standard_normal((2, M))
    kw = dict(np_=12, np1=8, ns=10)
    p = cq.make_params(0.3, 0.7, 0.6, 1.0, N, scheme, method, solver=cq.SOLVER_MODAL, **kw)
    gG0, grads = cq.fp_adjoint(cq.make_grid(3, nx, ny, nz=nz), p, dev(G0), dev(gN))
    ref = adj.adjoint_reference(3, nx, ny, 0.3, 0.7, 0.6, 1.0, N, G0, gN, scheme, method, nz=nz, **kw)
    e0 = rel(gG0.cpu().numpy(), ref[0])
    print(f"  3d adjoint scheme={scheme} method={method}: dG0 {e0:.3e}", flush=True)
    assert e0 <= 1e-10
    for k in range(3):
        tol = 1e-8 if (method == 1 and k < 2) else 1e-9
        assert abs(grads[k] - ref[k + 1]) <= tol * abs(ref[k + 1]), (k, grads[k], ref[k + 1])


@pytest.mark.parametrize("scheme,method", [(2, 0), (2, 1), (1, 0)])
def test_3d_63_cubed_sampled_modes(scheme, method):
    """63^3 nodes (250047 modes, 2 x 250047 DOF), N = 2^12, modal solver:
    sampled sine modes (first, last, tile boundaries, extremes per axis)
    against the long-double direct scheme: direct relative L2 1e-12, fast
    1e-8."""
    n, N = 63, 2 ** 12
    G0 = wl.g0_box(n, n, n, 9)
    # flat index (r-1) 63^2 + (q-1) 63 + (p-1): 0 .. 250046; (2, 5, 3) and
    # (3, 5, 3) are 8191 and 8192
    modes = [(1, 1, 1), (2, 3, 5), (63, 63, 63), (1, 1, 63), (63, 1, 1), (32, 32, 32), (17, 40, 9),
             (2, 5, 3), (3, 5, 3)]
    g = cq.make_grid(3, n, n, nz=n)
    p = cq.make_params(0.25, 0.75, 0.6, 1.0, N, scheme, method, solver=cq.SOLVER_MODAL)
    out = cq.fp_solve(g, p, dev(G0)).cpu().numpy()
    coef = modal.to_modes(out, 3, n, n, n)
    idx = [(r - 1) * n * n + (q - 1) * n + (pp - 1) for (pp, q, r) in modes]
    got = coef[:, idx]
    ref = modal_ld.run_modes_ld(3, n, n, modes, 0.25, 0.75, 0.6, 1.0, N, G0, scheme, nz=n)
    e = rel(got, ref)
    print(f"  63^3 scheme={scheme} method={method}: rel L2 on {len(modes)} modes {e:.3e}", flush=True)
    assert e <= (1e-12 if method == 0 else 1e-8), e
