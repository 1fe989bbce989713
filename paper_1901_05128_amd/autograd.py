"""torch.autograd wrapper: G^N as a differentiable function of G^0, alpha_1,
alpha_2 and m (modal solver). The forward pass calls fp_solve; the backward
pass calls fp_adjoint with the incoming gradient as dl/dG^N (which re-runs
the forward with its trajectory kept, then the adjoint sweep)."""
import torch

from . import _lib


class _Solve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, G0, alpha1, alpha2, m, grid_args, prm_args):
        dim, nx, ny = grid_args
        a1, a2, mm = float(alpha1), float(alpha2), float(m)
        grid = _lib.make_grid(dim, nx, ny)
        prm = _lib.make_params(a1, a2, mm, *prm_args)
        G0c = G0.detach().contiguous()
        GN = _lib.fp_solve(grid, prm, G0c)
        ctx.save_for_backward(G0c)
        ctx.grid, ctx.prm = grid, prm
        return GN

    @staticmethod
    def backward(ctx, gN):
        (G0c,) = ctx.saved_tensors
        gG0, (da1, da2, dm) = _lib.fp_adjoint(ctx.grid, ctx.prm, G0c, gN.detach().contiguous())
        dev, dt = G0c.device, G0c.dtype
        return (gG0, torch.tensor(da1, device=dev, dtype=dt), torch.tensor(da2, device=dev, dtype=dt),
                torch.tensor(dm, device=dev, dtype=dt), None, None)


def solve(G0, alpha1, alpha2, m, dim, nx, ny=1, T=1.0, N=1, scheme=2, method=1, np_=0, np1=0, ns=0):
    """G^N of the scheme (BE = 1 / BDF2 = 2, direct = 0 / fast = 1) from G0
    ([2][M] float64 on the GPU); alpha1, alpha2, m may be 0-dim tensors that
    require gradients."""
    prm_args = (T, N, scheme, method, 0.0, np_, np1, ns, 0, 0, _lib.SOLVER_MODAL)
    return _Solve.apply(G0, alpha1, alpha2, m, (dim, nx, ny), prm_args)
