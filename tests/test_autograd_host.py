"""Host logic of the torch.autograd wrapper, with the two library calls
replaced by stand-ins (no GPU): which inputs receive a gradient, and with
which dtype and device."""
import pytest

torch = pytest.importorskip("torch")

from paper_1901_05128_amd import _lib, autograd as ag  # noqa: E402


@pytest.fixture
def fake_lib(monkeypatch):
    calls = []

    def fp_solve(grid, prm, G0):
        return G0 * 2.0

    def fp_adjoint(grid, prm, G0, gN):
        calls.append((prm.alpha1, prm.alpha2, prm.m))
        return gN * 3.0, (1.5, -2.5, 4.0)

    monkeypatch.setattr(_lib, "fp_solve", fp_solve)
    monkeypatch.setattr(_lib, "fp_adjoint", fp_adjoint)
    return calls


def test_numbers_get_no_gradient(fake_lib):
    G0 = torch.ones(2, 3, dtype=torch.float64, requires_grad=True)
    GN = ag.solve(G0, 0.3, 0.7, 0.35, 1, 3, N=4)
    GN.sum().backward()
    assert torch.equal(G0.grad, torch.full((2, 3), 3.0, dtype=torch.float64))
    assert fake_lib == [(0.3, 0.7, 0.35)]


def test_scalar_gradients_follow_their_inputs(fake_lib):
    G0 = torch.ones(2, 3, dtype=torch.float64)
    a1 = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    m = torch.tensor(0.35, dtype=torch.float32, requires_grad=True)
    a2 = torch.tensor(0.7, dtype=torch.float64)          # a tensor without grad
    GN = ag.solve(G0, a1, a2, m, 1, 3, N=4)
    GN.sum().backward()
    assert a1.grad.dtype == torch.float64 and a1.grad.item() == 1.5
    assert m.grad.dtype == torch.float32 and m.grad.item() == 4.0
    assert a2.grad is None and G0.grad is None


def test_no_adjoint_when_nothing_needs_a_gradient(fake_lib):
    G0 = torch.ones(2, 3, dtype=torch.float64)
    a1 = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    GN = ag.solve(G0, a1, 0.7, 0.35, 1, 3, N=4)
    GN.sum().backward()
    assert len(fake_lib) == 1
