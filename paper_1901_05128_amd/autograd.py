"""torch.autograd wrapper: G^N as a differentiable function of G^0, alpha_1,
alpha_2 and m (modal solver). The forward pass calls fp_solve; the backward
pass calls fp_adjoint with the incoming gradient as dl/dG^N (which re-runs
the forward with its trajectory kept, then the adjoint sweep)."""
import torch

from . import _lib


def _scalar_spec(x):
    """(dtype, device) of a scalar argument's gradient: its own, for a tensor;
    None for a Python number (no gradient is returned for it)."""
    if isinstance(x, torch.Tensor):
        return (x.dtype, x.device)
    return None


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
        ctx.specs = (_scalar_spec(alpha1), _scalar_spec(alpha2), _scalar_spec(m))
        return GN

    @staticmethod
    def backward(ctx, gN):
        (G0c,) = ctx.saved_tensors
        need = ctx.needs_input_grad
        if not any(need[:4]):
            return (None,) * 6
        gG0, scal = _lib.fp_adjoint(ctx.grid, ctx.prm, G0c, gN.detach().contiguous())
        out = [gG0 if need[0] else None]
        for k in range(3):
            spec = ctx.specs[k]
            if need[k + 1] and spec is not None:
                out.append(torch.tensor(scal[k], dtype=spec[0], device=spec[1]))
            else:
                out.append(None)
        return tuple(out) + (None, None)


def solve(G0, alpha1, alpha2, m, dim, nx, ny=1, T=1.0, N=1, scheme=2, method=1, np_=0, np1=0, ns=0):
    """G^N of the scheme (BE = 1 / BDF2 = 2, direct = 0 / fast = 1) from G0
    ([2][M] float64 on the GPU). alpha1, alpha2 and m are Python numbers or
    0-dim tensors (any device); a tensor that requires grad receives its
    gradient with its own dtype and device, a number receives none."""
    prm_args = (T, N, scheme, method, 0.0, np_, np1, ns, 0, 0, _lib.SOLVER_MODAL)
    return _Solve.apply(G0, alpha1, alpha2, m, (dim, nx, ny), prm_args)
