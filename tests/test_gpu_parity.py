"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

The reference is the oracle's scheme evaluated mode by mode over every sine
mode (oracle.modal.reference): the same numbers as the nodal oracle in exact
arithmetic, but free of the nodal form's fp64 conditioning (on 1023 nodes the
nodal fp64 oracle itself drifts by 1e-12..1e-9 from a long-double evaluation).
Tolerances: direct CQ relative L2 <= 1e-12; fast CQ <= 1e-8 against the
direct reference (the fast algorithm's stated accuracy) and <= 1e-11 against
the oracle's fast scheme with the same node counts (the two Gauss-Jacobi rules
are computed independently)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1901_05128_amd as cq  # noqa: E402
from oracle import modal, stepper  # noqa: E402
from oracle.weights import weights  # noqa: E402
from paper_1901_05128_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cq.lib()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device="cuda")


# ---------------------------------------------------------------- cq_history
@pytest.mark.parametrize("n,M", [(1, 7), (2, 5), (5, 1), (64, 63), (65, 65), (333, 1000), (1000, 129),
                                 (4097, 64)])
@pytest.mark.parametrize("scheme", [1, 2])
def test_cq_history_matches_oracle(n, M, scheme):
    print(f"cq_history n={n} M={M} scheme={scheme}", flush=True)
    rng = np.random.default_rng(n * 7 + M)
    G = rng.uniform(-1, 1, size=(n, M))
    beta, tau = 0.35, 1.0 / 1000
    S = cq.cq_history(scheme, beta, tau, dev(G)).cpu().numpy()
    d = weights(scheme, beta, tau, n)
    ref = stepper.cq_history(d, G)
    if n == 1:
        assert np.all(S == 0.0)
    else:
        assert np.max(np.abs(S - ref)) <= 1e-13 * np.max(np.abs(d[1:])) * n


# ---------------------------------------------------------------- small solves
SMALL = [
    # dim, nx, ny, alpha1, alpha2, m, T, N
    (1, 127, 1, 0.3, 0.7, 0.3, 1.0, 1000),      # configuration 1 in full
    (1, 1023, 1, 0.4, 0.8, 0.45, 1.0 / 32, 512),  # configuration 2's grid and tau, 512 steps
    (1, 100, 1, 0.25, 0.55, 0.7, 1.0, 150),     # ragged tiles and blocks
    (1, 1, 1, 0.5, 0.5, 0.2, 1.0, 7),
    (2, 31, 17, 0.2, 0.6, 0.55, 1.0, 100),      # ragged 2D tiles
    (2, 63, 63, 0.35, 0.65, 0.0, 1.0, 160),     # a = -1
    (2, 97, 85, 0.3, 0.6, 0.6, 1.0, 100),       # >= 8192 modes: blocked modal fast form
]


@pytest.mark.parametrize("case", SMALL, ids=lambda c: f"{c[0]}d{c[1]}x{c[2]}N{c[7]}")
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("solver", [0, 1], ids=["nodal", "modal"])
def test_solve_matches_oracle(case, scheme, method, solver):
    dim, nx, ny, a1, a2, m, T, N = case
    print(f"solve case={case} scheme={scheme} method={method} solver={solver}", flush=True)
    G0 = wl.g0_intervals(nx, 2) if dim == 1 else wl.g0_rectangle(nx, ny, 3)
    if nx == 1:
        G0 = np.array([[1.0], [0.5]])
    g = cq.make_grid(dim, nx, ny)
    p = cq.make_params(a1, a2, m, T, N, scheme, method, solver=solver)
    with cq.Solver(g, p, dev(G0)) as s:
        info = s.info()
        s.step(N)
        out, n = s.current()
        out = out.cpu().numpy()
    assert n == N
    ref = modal.reference(dim, nx, ny, a1, a2, m, T, N, G0, scheme, 0)
    e = rel(out, ref)
    print(f"  rel_l2 vs direct reference {e:.3e}", flush=True)
    if method == 0:
        assert e <= 1e-12, e
    else:
        assert e <= 1e-8, e
        if N > info.lag:
            np_ = info.np_total - info.np1
            ref_f = modal.reference(dim, nx, ny, a1, a2, m, T, N, G0, scheme, 1, np_=np_, np1=info.np1 or 16,
                                    ns=info.lag)
            ef = rel(out, ref_f)
            print(f"  rel_l2 vs fast reference {ef:.3e}", flush=True)
            assert ef <= 1e-11


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("solver", [0, 1], ids=["nodal", "modal"])
def test_one_step_and_block_boundaries(method, dim, solver):
    """N = 1, and N straddling direct blocks (B = 64) step by step."""
    nx, ny = (40, 1) if dim == 1 else (20, 9)
    G0 = wl.g0_random(nx * ny, 4)
    for N in (1, 2, 64, 65, 129):
        print(f"blocks dim={dim} method={method} solver={solver} N={N}", flush=True)
        p = cq.make_params(0.45, 0.55, 0.65, 0.5, N, 2, method, block_B=64, solver=solver)
        out = cq.fp_solve(cq.make_grid(dim, nx, ny), p, dev(G0)).cpu().numpy()
        ref = modal.reference(dim, nx, ny, 0.45, 0.55, 0.65, 0.5, N, G0, 2, 0)
        assert rel(out, ref) <= (1e-12 if method == 0 else 1e-8)


@pytest.mark.parametrize("block_B", [64, 128, 192, 256])
def test_direct_block_sizes(block_B):
    nx, N = 70, 300
    G0 = wl.g0_random(nx, 8)
    p = cq.make_params(0.3, 0.6, 0.8, 1.0, N, 1, 0, block_B=block_B)
    out = cq.fp_solve(cq.make_grid(1, nx), p, dev(G0)).cpu().numpy()
    ref = modal.reference(1, nx, 1, 0.3, 0.6, 0.8, 1.0, N, G0, 1, 0)
    assert rel(out, ref) <= 1e-12


@pytest.mark.parametrize("block_B", [64, 256], ids=["B64", "B256"])
@pytest.mark.parametrize("scheme", [1, 2])
def test_modal_direct_far_passes(block_B, scheme):
    """Modal direct form with one far-field pass per block_B/64 near blocks
    (the later blocks of a pass add the levels since the pass separately),
    over several passes and a ragged last block, against the oracle."""
    nx, N = 45, 700
    G0 = wl.g0_random(nx, 31)
    p = cq.make_params(0.35, 0.65, 0.7, 1.0, N, scheme, 0, block_B=block_B, solver=1)
    out = cq.fp_solve(cq.make_grid(1, nx), p, dev(G0)).cpu().numpy()
    ref = modal.reference(1, nx, 1, 0.35, 0.65, 0.7, 1.0, N, G0, scheme, 0)
    assert rel(out, ref) <= 1e-12


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("dim", [1, 2])
@pytest.mark.parametrize("solver,block_B,k", [(0, 64, 77), (1, 64, 77), (1, 0, 77), (1, 0, 128), (1, 192, 200)],
                         ids=["nodal", "modal", "modal-pass128-k77", "modal-pass128-k128", "modal-pass192-k200"])
def test_state_roundtrip_is_bitwise(method, dim, solver, block_B, k):
    """Stop after k steps, move the state to a new handle, finish: the levels
    equal those of one uninterrupted run bit for bit (for the modal direct
    form also when k falls inside a far-field pass or inside a block)."""
    if method == 1 and block_B != 64:
        pytest.skip("block_B only changes the direct form")
    nx, ny = (50, 1) if dim == 1 else (12, 10)
    N = 260
    G0 = wl.g0_random(nx * ny, 12)
    g, p = cq.make_grid(dim, nx, ny), cq.make_params(0.3, 0.7, 0.6, 1.0, N, 2, method, block_B=block_B,
                                                     solver=solver)
    with cq.Solver(g, p, dev(G0)) as s:
        s.step(N)
        full = s.current()[0].cpu().numpy()
    with cq.Solver(g, p, dev(G0)) as s:
        s.step(k)
        state = s.get_state()
    with cq.Solver(g, p, dev(np.zeros_like(G0))) as s2:
        s2.set_state(state)
        s2.step(N - k)
        resumed = s2.current()[0].cpu().numpy()
    assert np.array_equal(full, resumed)


def test_nonfinite_g0_rejected():
    G0 = np.zeros((2, 9))
    G0[1, 3] = np.nan
    with pytest.raises(cq.CQError) as e:
        cq.Solver(cq.make_grid(1, 9), cq.make_params(0.3, 0.7, 0.3, 1.0, 4, 1, 0), dev(G0))
    assert e.value.code == -6


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("dim", [1, 2])
def test_modal_and_nodal_agree_stepwise(method, dim):
    """Read out after every few steps: both solvers give the same levels."""
    nx, ny = (33, 1) if dim == 1 else (17, 15)
    N = 90
    G0 = wl.g0_random(nx * ny, 21)
    g = cq.make_grid(dim, nx, ny)
    outs = []
    for solver in (0, 1):
        with cq.Solver(g, cq.make_params(0.25, 0.75, 0.7, 1.0, N, 1, method, solver=solver), dev(G0)) as s:
            seq = []
            for chunk in (1, 2, 29, 58):
                s.step(chunk)
                seq.append(s.current()[0].cpu().numpy())
            outs.append(seq)
    for a, b in zip(*outs):
        assert rel(a, b) <= 1e-12


def test_step_past_end_rejected():
    with cq.Solver(cq.make_grid(1, 9), cq.make_params(0.3, 0.7, 0.3, 1.0, 4, 1, 0), dev(np.ones((2, 9)))) as s:
        s.step(3)
        with pytest.raises(cq.CQError):
            s.step(2)


@pytest.mark.parametrize("dim,nx,ny", [(1, 1, 1), (2, 1, 1), (2, 1, 7), (2, 7, 1), (1, 2, 1)])
@pytest.mark.parametrize("m", [1.0, 0.0, 0.7])
@pytest.mark.parametrize("solver", [0, 1], ids=["nodal", "modal"])
def test_degenerate_grids_and_coupling(dim, nx, ny, m, solver):
    """One-node and one-row grids, the decoupled case m = 1 (a = 0) and
    m = 0 (a = -1), orders near the ends of (0,1), every scheme and method,
    against the oracle."""
    N = 70
    G0 = wl.g0_random(nx * ny, 3)
    for scheme in (1, 2):
        ref = modal.reference(dim, nx, ny, 0.05, 0.95, m, 1.0, N, G0, scheme, 0)
        for method in (0, 1):
            p = cq.make_params(0.05, 0.95, m, 1.0, N, scheme, method, solver=solver)
            out = cq.fp_solve(cq.make_grid(dim, nx, ny), p, dev(G0)).cpu().numpy()
            assert rel(out, ref) <= (1e-12 if method == 0 else 1e-8), (scheme, method, rel(out, ref))


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("dim,nx,ny", [(1, 77, 1), (2, 95, 91)], ids=["1d-77", "2d-8645"])
def test_whole_run_on_the_mfma_kernel(scheme, dim, nx, ny):
    """fast_kernel 1: one fp_step over all N steps runs on the 16-mode MFMA
    kernel (few modes: the final level into the ring; from 8192 modes: into
    the level store), the same scheme as the streamed run within 1e-13, and
    against the oracle's fast scheme with the same rule; fp_solve takes the
    same path; chunked calls keep the streamed path (bit for bit the same
    chunks with fast_kernel 0); the state of the finished run moves to a new
    handle."""
    N = 150
    M = nx * ny
    G0 = wl.g0_random(M, 77)
    g = cq.make_grid(dim, nx, ny)
    kw = dict(np_=40, ns=30) if scheme == 2 else dict(np_=40)
    p0 = cq.make_params(0.3, 0.75, 0.7, 1.0, N, scheme, 1, solver=cq.SOLVER_MODAL, **kw)
    p1 = cq.make_params(0.3, 0.75, 0.7, 1.0, N, scheme, 1, solver=cq.SOLVER_MODAL, fast_kernel=1, **kw)
    with cq.Solver(g, p0, dev(G0)) as s:
        assert s.info().whole_run_kernel == 0
        s.step(N)
        streamed = s.current()[0].cpu().numpy()
    with cq.Solver(g, p1, dev(G0)) as s:
        assert s.info().whole_run_kernel == 1
        s.step(N)
        whole = s.current()[0].cpu().numpy()
        state = s.get_state()
        s.reset(dev(G0))
        s.step(N)
        assert np.array_equal(s.current()[0].cpu().numpy(), whole)
    with cq.Solver(g, p1, dev(np.zeros_like(G0))) as s2:
        s2.set_state(state)
        assert np.array_equal(s2.current()[0].cpu().numpy(), whole)
    solved = cq.fp_solve(g, p1, dev(G0)).cpu().numpy()
    assert np.array_equal(solved, whole)
    chunked = []
    for p in (p0, p1):
        with cq.Solver(g, p, dev(G0)) as s:
            for c in (1, 31, 29, 89):
                s.step(c)
            chunked.append(s.current()[0].cpu().numpy())
    assert np.array_equal(chunked[0], chunked[1])
    e = rel(whole, streamed)
    ref = modal.reference(dim, nx, ny, 0.3, 0.75, 0.7, 1.0, N, G0, scheme, 1, np1=16, **kw)
    e2 = rel(whole, ref)
    print(f"  whole run vs streamed {e:.2e}, vs oracle fast {e2:.2e}", flush=True)
    assert e <= 1e-13
    assert e2 <= 1e-11


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("dim", [1, 2])
def test_modal_steps_in_uneven_chunks_bitwise(method, scheme, dim):
    """fp_step in chunks that start and end inside the time blocks (direct:
    64-step blocks and 128-step far passes; fast: L-step blocks) gives the
    same levels, bit for bit, as one call."""
    nx, ny = (40, 1) if dim == 1 else (9, 7)
    N = 190
    G0 = wl.g0_random(nx * ny, 41)
    g = cq.make_grid(dim, nx, ny)
    p = cq.make_params(0.35, 0.7, 0.6, 1.0, N, scheme, method, solver=cq.SOLVER_MODAL)
    with cq.Solver(g, p, dev(G0)) as s:
        s.step(N)
        one = s.current()[0].cpu().numpy()
    with cq.Solver(g, p, dev(G0)) as s:
        for c in (1, 2, 29, 30, 31, 7, 64, 26):
            s.step(c)
        many = s.current()[0].cpu().numpy()
    assert np.array_equal(one, many)


# ------------------------------------------------------------ maximum sizes
@pytest.mark.parametrize("nx", [1024, 1025, 4096], ids=["1024-one-row-per-thread", "1025-two-rows", "4096-max"])
@pytest.mark.parametrize("method", [0, 1])
def test_nodal_1d_row_count_limits(nx, method):
    """The 1D nodal step at the edges of its row-per-thread variants (1024
    nodes: one row per thread, multipliers in registers; 1025: two rows per
    thread; 4096: the largest 1D grid) against the per-mode reference."""
    N = 40
    print(f"nodal 1D nx={nx} method={method}", flush=True)
    G0 = wl.g0_intervals(nx, 7)
    g = cq.make_grid(1, nx, 1)
    p = cq.make_params(0.3, 0.7, 0.6, 0.05, N, 2, method, solver=cq.SOLVER_NODAL)
    with cq.Solver(g, p, dev(G0)) as s:
        info = s.info()
        s.step(N)
        out = s.current()[0].cpu().numpy()
    ref = modal.reference(1, nx, 1, 0.3, 0.7, 0.6, 0.05, N, G0, 2, 0)
    e = rel(out, ref)
    print(f"  rel_l2 vs direct reference {e:.3e}", flush=True)
    assert e <= (1e-12 if method == 0 else 1e-8), e
    if method == 1:
        ref_f = modal.reference(1, nx, 1, 0.3, 0.7, 0.6, 0.05, N, G0, 2, 1, np_=info.np_total - info.np1,
                                np1=info.np1 or 16, ns=info.lag)
        assert rel(out, ref_f) <= 1e-11


@pytest.mark.parametrize("scheme,np_,np1", [(1, 1024, 0), (2, 1008, 16)], ids=["BE-1024", "BDF2-16+1008"])
@pytest.mark.parametrize("solver", [0, 1], ids=["nodal", "modal"])
def test_fast_rule_at_the_node_limit(scheme, np_, np1, solver):
    """The fast form with the most nodes a solver keeps per component (1024:
    N_p = 1024 for BE, N_{p,1} + N_{p,2} = 16 + 1008 for BDF2), against the
    oracle's fast scheme with the same node counts and the direct reference."""
    dim, nx, ny, N = 2, 15, 9, 120
    print(f"fast rule limit scheme={scheme} np={np_} np1={np1} solver={solver}", flush=True)
    G0 = wl.g0_rectangle(nx, ny, 3)
    g = cq.make_grid(dim, nx, ny)
    p = cq.make_params(0.3, 0.6, 0.6, 1.0, N, scheme, 1, np_=np_, np1=np1, ns=30 if scheme == 2 else 0,
                       solver=solver)
    with cq.Solver(g, p, dev(G0)) as s:
        info = s.info()
        s.step(N)
        out = s.current()[0].cpu().numpy()
    assert info.np_total == 1024
    ref = modal.reference(dim, nx, ny, 0.3, 0.6, 0.6, 1.0, N, G0, scheme, 0)
    assert rel(out, ref) <= 1e-8
    ref_f = modal.reference(dim, nx, ny, 0.3, 0.6, 0.6, 1.0, N, G0, scheme, 1, np_=np_, np1=np1 or 16, ns=info.lag)
    ef = rel(out, ref_f)
    print(f"  rel_l2 vs fast reference {ef:.3e}", flush=True)
    assert ef <= 1e-11
