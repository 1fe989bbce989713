"""Batched fast solves (fp_solve_batched): uneven problems in one captured
graph, checked against the per-mode oracle and against single solves."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1901_05128_amd as cq  # noqa: E402
from oracle import modal  # noqa: E402
from paper_1901_05128_amd import workloads as wl  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cq.lib()


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _mixed(count, seed, nmax=300):
    rng = np.random.default_rng(seed)
    probs = []
    for b in range(count):
        if rng.uniform() < 0.5:
            dim, nx, ny = 1, int(rng.choice([7, 31, 100, 127, 255])), 1
        else:
            dim, nx, ny = 2, int(rng.choice([7, 15, 31])), int(rng.choice([9, 15, 33]))
        N = int(rng.integers(40, nmax))
        scheme = int(rng.integers(1, 3))
        a1, a2 = (float(v) for v in rng.uniform(0.1, 0.9, size=2))
        m = float(rng.uniform(0.55, 0.95))
        np_ = max(8, int(math.ceil(3 * math.sqrt(N))))
        probs.append((dim, nx, ny, a1, a2, m, 1.0, N, scheme, np_))
    return probs


def _run(probs, autotune=True, seed=0):
    grids, params, g0s = [], [], []
    for i, (dim, nx, ny, a1, a2, m, T, N, scheme, np_) in enumerate(probs):
        grids.append(cq.make_grid(dim, nx, ny))
        params.append(cq.make_params(a1, a2, m, T, N, scheme, 1, np_=np_))
        g0s.append(torch.tensor(wl.g0_random(nx * ny, seed + i), device="cuda"))
    outs, rep = cq.fp_solve_batched(grids, params, g0s, autotune=autotune)
    return [o.cpu().numpy() for o in outs], [g.cpu().numpy() for g in g0s], rep


def test_batched_matches_oracle_mixed():
    probs = _mixed(14, 3)
    outs, g0s, rep = _run(probs)
    print(f"batch classes={rep.classes} lanes={list(rep.class_lanes)[:rep.classes]} "
          f"run_s={rep.run_s:.3f}", flush=True)
    assert rep.problems == len(probs)
    assert rep.modes == sum(p[1] * p[2] for p in probs)
    for (dim, nx, ny, a1, a2, m, T, N, scheme, np_), out, g0 in zip(probs, outs, g0s):
        ref_f = modal.reference(dim, nx, ny, a1, a2, m, T, N, g0, scheme, 1, np_=np_, np1=16, ns=30)
        ref_d = modal.reference(dim, nx, ny, a1, a2, m, T, N, g0, scheme, 0)
        ef, ed = rel(out, ref_f), rel(out, ref_d)
        print(f"  {dim}d {nx}x{ny} N={N} scheme={scheme} np={np_}: vs fast {ef:.2e} vs direct {ed:.2e}",
              flush=True)
        assert ef <= 1e-11
        assert ed <= 1e-8


def test_batched_equals_single_solves_and_tiles_agree():
    """Autotuned, default and time-blocked batches against single modal
    solves: the time-blocked kernel runs the single solve's arithmetic
    (1e-13); the kernel choices of the other two may sum in another order
    (the fast scheme's 1e-11)."""
    probs = _mixed(10, 8)
    a, g0s, rep_a = _run(probs, autotune=True, seed=50)
    b, _, rep_b = _run(probs, autotune=False, seed=50)
    c, _, rep_c = _run(probs, autotune=cq.BATCH_TIME_BLOCKED, seed=50)
    for (dim, nx, ny, a1, a2, m, T, N, scheme, np_), oa, ob, oc, g0 in zip(probs, a, b, c, g0s):
        single = cq.fp_solve(cq.make_grid(dim, nx, ny),
                             cq.make_params(a1, a2, m, T, N, scheme, 1, np_=np_, solver=cq.SOLVER_MODAL),
                             torch.tensor(g0, device="cuda")).cpu().numpy()
        assert rel(oa, single) <= 1e-11
        assert rel(ob, single) <= 1e-11
        assert rel(oc, single) <= 1e-13
    assert all(x in (32, 64) for x in list(rep_a.class_lanes)[:rep_a.classes])
    assert all(x in (1, 2) for x in list(rep_b.class_blocked)[:rep_b.classes])
    assert all(x == 1 for x in list(rep_c.class_blocked)[:rep_c.classes])


@pytest.mark.parametrize("np_", [None, 200, 380, 500, 700])
def test_time_blocked_kernel(np_):
    """BDF2 problems (lag 30) with the time-blocked kernel forced:
    blocks of 30 steps, a ragged last block, runs shorter than one block or
    one half-block, and node counts up to 768 (every register class of the
    kernel), against the oracle and against single modal solves."""
    rng = np.random.default_rng(17)
    probs = []
    for N in (7, 16, 29, 31, 45, 61, 90, 151):
        dim, nx, ny = (1, int(rng.choice([31, 63])), 1) if N % 2 else (2, 9, 11)
        a1, a2 = (float(v) for v in rng.uniform(0.1, 0.9, size=2))
        m = float(rng.uniform(0.55, 0.95))
        probs.append((dim, nx, ny, a1, a2, m, 1.0, N, 2, np_ or max(8, int(math.ceil(3 * math.sqrt(N))))))
    outs, g0s, rep = _run(probs, autotune=cq.BATCH_TIME_BLOCKED, seed=300)
    print(f"batch classes={rep.classes} blocked={list(rep.class_blocked)[:rep.classes]}", flush=True)
    assert all(x == 1 for x in list(rep.class_blocked)[:rep.classes])
    for (dim, nx, ny, a1, a2, m, T, N, scheme, npn), out, g0 in zip(probs, outs, g0s):
        single = cq.fp_solve(cq.make_grid(dim, nx, ny),
                             cq.make_params(a1, a2, m, T, N, scheme, 1, np_=npn, solver=cq.SOLVER_MODAL),
                             torch.tensor(g0, device="cuda")).cpu().numpy()
        ref = modal.reference(dim, nx, ny, a1, a2, m, T, N, g0, scheme, 1, np_=npn, np1=16, ns=30)
        e1, e2 = rel(out, single), rel(out, ref)
        print(f"  {dim}d {nx}x{ny} N={N} np={npn}: vs single {e1:.2e} vs oracle {e2:.2e}", flush=True)
        assert e1 <= 1e-13
        assert e2 <= 1e-11


@pytest.mark.parametrize("np_", [None, 100, 200, 380, 560])
def test_mfma_tile_kernel(np_):
    """The 16-mode MFMA kernel (forced): BDF2 problems (lag 30) and BE
    problems (exact window of 2 np + 2 <= 32 lags) in blocks of 16 steps,
    runs shorter than one block, a ragged last block, ragged 16-mode tiles
    (31 and 63 modes in 1D, 99 in 2D) and node counts up to 576 per
    component (every tile count of the kernel's templates up to 18 per
    wave), against the oracle's fast scheme and against single modal solves
    (the same rule; the kernel sums in another order)."""
    rng = np.random.default_rng(29)
    probs = []
    for N, scheme in ((5, 2), (16, 2), (17, 1), (31, 2), (33, 1), (64, 2), (90, 1), (151, 2)):
        dim, nx, ny = (1, int(rng.choice([31, 63])), 1) if N % 2 else (2, 9, 11)
        a1, a2 = (float(v) for v in rng.uniform(0.1, 0.9, size=2))
        m = float(rng.uniform(0.55, 0.95))
        npn = np_ or max(8, int(math.ceil(3 * math.sqrt(N))))
        probs.append((dim, nx, ny, a1, a2, m, 1.0, N, scheme, npn))
    outs, g0s, rep = _run(probs, autotune=cq.BATCH_MFMA_TILE, seed=400)
    print(f"batch classes={rep.classes} blocked={list(rep.class_blocked)[:rep.classes]}", flush=True)
    assert all(x == 2 for x in list(rep.class_blocked)[:rep.classes])
    for (dim, nx, ny, a1, a2, m, T, N, scheme, npn), out, g0 in zip(probs, outs, g0s):
        single = cq.fp_solve(cq.make_grid(dim, nx, ny),
                             cq.make_params(a1, a2, m, T, N, scheme, 1, np_=npn, solver=cq.SOLVER_MODAL),
                             torch.tensor(g0, device="cuda")).cpu().numpy()
        ref = modal.reference(dim, nx, ny, a1, a2, m, T, N, g0, scheme, 1, np_=npn, np1=16, ns=30)
        e1, e2 = rel(out, single), rel(out, ref)
        print(f"  {dim}d {nx}x{ny} N={N} scheme={scheme} np={npn}: vs single {e1:.2e} vs oracle {e2:.2e}",
              flush=True)
        assert e1 <= 1e-11
        assert e2 <= 1e-11


@pytest.mark.parametrize("ns", [16, 33])
def test_mfma_tile_kernel_lag_limits_and_tiny_tiles(ns):
    """The MFMA kernel at the ends of its lag range (N_s = 16: blocks as long
    as the lag; N_s = 33: the earlier-level window reaching 32 lags back),
    with a single mode (15 idle columns of the 16-mode tile) and exactly one
    full tile, against the oracle's fast scheme with the same rule."""
    probs = [(1, 1, 1, 0.3, 0.7, 0.8, 1.0, 47, 2, 40), (1, 16, 1, 0.55, 0.25, 0.7, 1.0, 64, 2, 40),
             (2, 3, 5, 0.8, 0.4, 0.9, 1.0, 35, 2, 40)]
    grids, params, g0s = [], [], []
    for i, (dim, nx, ny, a1, a2, m, T, N, scheme, npn) in enumerate(probs):
        grids.append(cq.make_grid(dim, nx, ny))
        params.append(cq.make_params(a1, a2, m, T, N, scheme, 1, np_=npn, ns=ns))
        g0s.append(torch.tensor(wl.g0_random(nx * ny, 600 + i), device="cuda"))
    outs, rep = cq.fp_solve_batched(grids, params, g0s, autotune=cq.BATCH_MFMA_TILE)
    assert all(x == 2 for x in list(rep.class_blocked)[:rep.classes])
    for (dim, nx, ny, a1, a2, m, T, N, scheme, npn), out, g0 in zip(probs, outs, g0s):
        g0n = g0.cpu().numpy()
        ref = modal.reference(dim, nx, ny, a1, a2, m, T, N, g0n, scheme, 1, np_=npn, np1=16, ns=ns)
        e = rel(out.cpu().numpy(), ref)
        print(f"  ns={ns} {dim}d {nx}x{ny} N={N}: vs oracle {e:.2e}", flush=True)
        assert e <= 1e-11


def test_mfma_tile_kernel_falls_back_where_it_does_not_apply():
    """Forcing the MFMA kernel leaves a class it cannot take (700 nodes per
    component) on the time-blocked kernel, with the same results as that
    kernel forced."""
    probs = [(1, 31, 1, 0.3, 0.7, 0.8, 1.0, 40, 2, 700), (2, 9, 11, 0.6, 0.2, 0.7, 1.0, 37, 2, 700)]
    a, _, rep_a = _run(probs, autotune=cq.BATCH_MFMA_TILE, seed=500)
    b, _, rep_b = _run(probs, autotune=cq.BATCH_TIME_BLOCKED, seed=500)
    assert all(x == 1 for x in list(rep_a.class_blocked)[:rep_a.classes])
    for oa, ob in zip(a, b):
        assert np.array_equal(oa, ob)


def test_batched_rejects_direct_method_and_bad_lag():
    g = [cq.make_grid(1, 15)]
    G0 = [torch.zeros((2, 15), dtype=torch.float64, device="cuda")]
    with pytest.raises(cq.CQError):
        cq.fp_solve_batched(g, [cq.make_params(0.3, 0.6, 0.7, 1.0, 10, 2, 0)], G0)
    with pytest.raises(cq.CQError):
        cq.fp_solve_batched(g, [cq.make_params(0.3, 0.6, 0.7, 1.0, 10, 2, 1, ns=80)], G0)


def test_batched_reduced_c4_mix():
    """The seeded 256-instance mix of the batched workload, 24 of them with N
    scaled by 1/32 and grids capped, autotuned, against single modal solves
    (the fast scheme's 1e-11: the kernel chosen may sum in another order)."""
    inst = wl.batched_instances(24, seed=4, scale=1 / 32)
    probs = []
    for p in inst:
        nx = min(p.nx, 511) if p.dim == 1 else min(p.nx, 63)
        ny = 1 if p.dim == 1 else nx
        np_ = max(8, int(math.ceil(3 * math.sqrt(p.N))))
        probs.append((p.dim, nx, ny, p.alpha1, p.alpha2, p.m, p.T, p.N, 2, np_))
    outs, g0s, rep = _run(probs, seed=200)
    for (dim, nx, ny, a1, a2, m, T, N, scheme, np_), out, g0 in zip(probs, outs, g0s):
        single = cq.fp_solve(cq.make_grid(dim, nx, ny),
                             cq.make_params(a1, a2, m, T, N, scheme, 1, np_=np_, solver=cq.SOLVER_MODAL),
                             torch.tensor(g0, device="cuda")).cpu().numpy()
        e = rel(out, single)
        print(f"  {dim}d {nx}x{ny} N={N} np={np_}: vs single {e:.2e}", flush=True)
        assert e <= 1e-11
