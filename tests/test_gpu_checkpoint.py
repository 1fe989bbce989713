"""The checkpointed gradient (fast method): the forward recomputed segment by
segment from saved states on a binomial schedule instead of kept whole.

Against the kept-whole form on the same handle parameters with the streamed
forward (forward_kernel 1): G^N, dl/dG0 and dl/dm bit for bit (the same
arithmetic in the same order); dl/dalpha_k to
relative 1e-10 (the contraction is summed as Toeplitz products per segment
instead of the near-field + block-DFT form; its terms cancel across modes,
so the difference is rounding of the terms' scale, not of the sum). Against the oracle adjoint at
its usual bars. Schedules from one saved state (every segment advanced to
from the start) to one per segment; segments of one chunk; a run at the
adjoint workload's size; and a gradient on the 2D 255^2 grid at N = 2^16
under a budget that the kept-whole form exceeds (checked by duality with
the GPU forward)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1901_05128_amd as cq  # noqa: E402
from oracle import adjoint as adj  # noqa: E402
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


def _grad(g, p, G0, gN, **kw):
    with cq.Adjoint(g, p, **kw) as h:
        info = h.info()
        GN = torch.empty_like(G0)
        gG0, grads = h.run(G0, gN, GN=GN)
        # a second run on the same handle gives the same numbers
        gG0b, gradsb = h.run(G0, gN)
        assert torch.equal(gG0, gG0b) and list(grads) == list(gradsb)
    return GN.cpu().numpy(), gG0.cpu().numpy(), list(grads), info


def _compare(whole, ck):
    GN0, g00, gr0, _ = whole
    GN1, g01, gr1, info = ck
    assert info.mode == 2
    assert np.array_equal(GN0, GN1)
    assert np.array_equal(g00, g01)
    assert gr0[2] == gr1[2], (gr0[2], gr1[2])
    for k in range(2):
        assert abs(gr0[k] - gr1[k]) <= 1e-10 * abs(gr0[k]), (k, gr0[k], gr1[k])


CASES = [
    # dim, nx, ny, alpha1, alpha2, m, N, scheme, np
    (1, 31, 1, 0.3, 0.7, 0.35, 300, 2, 12),
    (2, 9, 7, 0.2, 0.6, 0.55, 250, 2, 12),
    (1, 20, 1, 0.45, 0.55, 0.8, 200, 1, 10),
    (2, 97, 85, 0.25, 0.65, 0.6, 130, 2, 12),   # 8245 modes
    (1, 7, 1, 0.4, 0.8, 0.45, 1001, 2, 16),     # a one-step last chunk
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0]}d{c[1]}x{c[2]}N{c[6]}s{c[7]}")
@pytest.mark.parametrize("slots,segment_steps", [(1, 1), (2, 1), (3, 1), (0, 1), (0, 0), (2, 0)])
def test_checkpointed_equals_kept_whole(case, slots, segment_steps):
    dim, nx, ny, a1, a2, m, N, scheme, npn = case
    print(f"ckpt case={case} slots={slots} seg={segment_steps}", flush=True)
    M = nx * ny
    G0 = dev(wl.g0_random(M, 91).reshape(2, M))
    gN = dev(np.random.default_rng(92).standard_normal((2, M)))
    g = cq.make_grid(dim, nx, ny)
    kw = dict(np_=npn, np1=8, ns=10) if scheme == 2 else dict(np_=npn)
    p = cq.make_params(a1, a2, m, 1.0, N, scheme, 1, solver=cq.SOLVER_MODAL, **kw)
    whole = _grad(g, p, G0, gN, mode=1, forward_kernel=1)
    ck = _grad(g, p, G0, gN, mode=2, slots=slots, segment_steps=segment_steps)
    info = ck[3]
    print(f"  segments {info.segments} x {info.segment_steps} steps, {info.slots} states, "
          f"{info.forward_steps} forward steps", flush=True)
    if slots:
        assert info.slots == slots
    _compare(whole, ck)
    if M <= 300:
        ref = adj.adjoint_reference(dim, nx, ny, a1, a2, m, 1.0, N, G0.cpu().numpy(), gN.cpu().numpy(), scheme, 1,
                                    **kw)
        assert rel(ck[1], ref[0]) <= 1e-10
        for k in range(3):
            assert abs(ck[2][k] - ref[k + 1]) <= (1e-8 if k < 2 else 1e-10) * abs(ref[k + 1])


def test_checkpoint_schedule_costs():
    """One saved state: every segment is advanced to from the start
    (forward steps N + seg * S (S - 1) / 2); one per segment: N + seg (S - 1)."""
    nx, N = 15, 600
    g = cq.make_grid(1, nx)
    p = cq.make_params(0.3, 0.7, 0.35, 1.0, N, 2, 1, np_=12, np1=8, ns=10, solver=cq.SOLVER_MODAL)
    with cq.Adjoint(g, p, mode=2, slots=1, segment_steps=1) as h:
        inf = h.info()
        S, seg = inf.segments, inf.segment_steps
        assert inf.forward_steps == N + seg * S * (S - 1) // 2
    with cq.Adjoint(g, p, mode=2, slots=S, segment_steps=1) as h:
        inf = h.info()
        assert inf.forward_steps == N + seg * (S - 1)


def test_checkpointed_rejects_direct_and_small_budgets():
    g = cq.make_grid(1, 15)
    pd = cq.make_params(0.3, 0.7, 0.35, 1.0, 100, 2, 0, solver=cq.SOLVER_MODAL)
    with pytest.raises(cq.CQError):
        cq.Adjoint(g, pd, mode=2)
    pf = cq.make_params(0.3, 0.7, 0.35, 1.0, 100, 2, 1, np_=12, np1=8, ns=10, solver=cq.SOLVER_MODAL)
    with pytest.raises(cq.CQError):
        cq.Adjoint(g, pf, mode=1, max_device_bytes=4096)
    with pytest.raises(cq.CQError):
        cq.Adjoint(g, pf, mode=2, max_device_bytes=4096)


def test_checkpointed_at_adjoint_workload_size():
    """2D 127^2, BDF2 fast (16 + 192 nodes, N_s = 30), N = 4096: four saved
    states against the kept-whole form."""
    nx = ny = 127
    M = nx * ny
    G0 = dev(wl.g0_rectangle(nx, ny, 5))
    gN = dev(np.random.default_rng(93).standard_normal((2, M)))
    g = cq.make_grid(2, nx, ny)
    p = cq.make_params(0.2, 0.6, 0.55, 1.0, 4096, 2, 1, np_=192, np1=16, ns=30, solver=cq.SOLVER_MODAL)
    whole = _grad(g, p, G0, gN, mode=1, forward_kernel=1)
    ck = _grad(g, p, G0, gN, mode=2, slots=4)
    inf = ck[3]
    print(f"  127^2: {inf.segments} segments of {inf.segment_steps}, {inf.slots} states, "
          f"{inf.forward_steps} forward steps, {inf.device_bytes / 2**30:.2f} GiB "
          f"(kept whole {whole[3].device_bytes / 2**30:.2f} GiB)", flush=True)
    _compare(whole, ck)


def test_gradient_on_255_squared_at_2_16_steps_under_a_budget():
    """2D 255^2, BDF2 fast, N = 2^16 (the 2D workload's grid and steps): the
    kept-whole form needs about 273 GB and is refused under a 150 GB budget;
    the checkpointed form runs in it. dl/dG0 is checked by duality with the
    GPU forward map G0 -> G^N (linear): <gN, L d> = <dl/dG0, d>."""
    nx = ny = 255
    M = nx * ny
    N = 2 ** 16
    g = cq.make_grid(2, nx, ny)
    p = cq.make_params(0.2, 0.6, 0.55, 1.0, N, 2, 1, solver=cq.SOLVER_MODAL)
    budget = 150 * 10 ** 9
    with pytest.raises(cq.CQError) as ei:
        cq.Adjoint(g, p, mode=1, max_device_bytes=budget)
    assert ei.value.code == cq._lib.CQ_ENOMEM
    G0 = dev(wl.g0_rectangle(nx, ny, 3))
    rng = np.random.default_rng(94)
    gN = dev(rng.standard_normal((2, M)))
    with cq.Adjoint(g, p, max_device_bytes=budget) as h:
        inf = h.info()
        print(f"  255^2 N=2^16: mode {inf.mode}, {inf.segments} segments of {inf.segment_steps}, {inf.slots} "
              f"states, {inf.forward_steps} forward steps, {inf.device_bytes / 1e9:.1f} GB", flush=True)
        assert inf.mode == 2 and inf.device_bytes <= budget
        gG0, grads = h.run(G0, gN)
    assert all(np.isfinite(grads))
    d = rng.standard_normal((2, M))
    Ld = cq.fp_solve(g, p, dev(d)).cpu().numpy()
    gNh = gN.cpu().numpy()
    lhs, rhs = float(np.sum(gNh * Ld)), float(np.sum(gG0.cpu().numpy() * d))
    print(f"  duality {lhs:.12e} {rhs:.12e}", flush=True)
    assert abs(lhs - rhs) <= 1e-11 * np.linalg.norm(gNh) * np.linalg.norm(Ld)
