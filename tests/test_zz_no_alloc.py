"""The allocation-free history row (cq_history_noalloc) against cq_history,
through the C ABI: the same sum (weights computed on the device instead of
the host, so the two agree to rounding: relative L2 1e-12, the direct-sum
bar), on two calls in a row, the second with a smaller input, and under the
oracle's sum as well."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_1901_05128_amd as cq  # noqa: E402
from oracle import stepper  # noqa: E402
from oracle.weights import weights  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    cq.lib()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("scheme", [1, 2])
def test_noalloc_history_matches_allocating_entry_point(scheme):
    beta, tau = 0.35, 1.0 / 4096
    # (n, M): a large call (several slices, partial sums in the workspace),
    # then a smaller one that must not see the first call's contents; then a
    # row wider than the partial-sum region (one slice, written directly)
    shapes = [(4097, 1023), (300, 65), (20, (1 << 20) + 7)]
    for i, (n, M) in enumerate(shapes):
        print(f"noalloc scheme={scheme} call={i} n={n} M={M}", flush=True)
        rng = np.random.default_rng(100 * scheme + i)
        G = torch.tensor(rng.uniform(-1, 1, size=(n, M)), dtype=torch.float64, device="cuda")
        S_ref = cq.cq_history(scheme, beta, tau, G).cpu().numpy()
        S = torch.full((M,), np.nan, dtype=torch.float64, device="cuda")
        cq.cq_history_noalloc(scheme, beta, tau, G, S)
        torch.cuda.synchronize()
        S = S.cpu().numpy()
        assert np.all(np.isfinite(S))
        assert _rel(S, S_ref) <= 1e-12, (i, _rel(S, S_ref))
        if n * M <= 4097 * 1023:
            d = weights(scheme, beta, tau, n)
            ref = stepper.cq_history(d, G.cpu().numpy())
            assert _rel(S, ref) <= 1e-12, (i, _rel(S, ref))
        del G


def test_noalloc_history_edge_sizes():
    beta, tau = 0.6, 1e-3
    for n, M in [(1, 5), (2, 1), (17, 3)]:
        G = torch.tensor(np.random.default_rng(n).uniform(-1, 1, size=(n, M)), dtype=torch.float64, device="cuda")
        S = torch.full((M,), np.nan, dtype=torch.float64, device="cuda")
        cq.cq_history_noalloc(2, beta, tau, G, S)
        torch.cuda.synchronize()
        ref = stepper.cq_history(weights(2, beta, tau, n), G.cpu().numpy()) if n > 1 else np.zeros(M)
        got = S.cpu().numpy()
        if n == 1:
            assert np.all(got == 0.0)
        else:
            assert np.max(np.abs(got - ref)) <= 1e-13 * np.max(np.abs(ref)) * n
