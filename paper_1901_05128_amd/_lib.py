"""ctypes binding of libcqfp.so (the C ABI in include/cqfp.h).

Argument marshalling only: every step of the solver runs in the HIP library.
Device arrays are torch tensors (fp64, contiguous, on the current HIP device)
and the stream is torch's current stream. If the library is not built, every
call raises; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcqfp.so")

CQ_OK, CQ_EINVAL, CQ_ESINGULAR, CQ_ENOMEM, CQ_EHIP, CQ_ETOL, CQ_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "CQ_OK", -1: "CQ_EINVAL", -2: "CQ_ESINGULAR", -3: "CQ_ENOMEM", -4: "CQ_EHIP",
                -5: "CQ_ETOL", -6: "CQ_ENONFINITE"}

# every entry point the header declares
EXPORTS = ["cq_weights", "cq_fast_rule", "cq_history", "cq_history_noalloc", "fp_create", "fp_step", "fp_current", "fp_info",
           "fp_get_state", "fp_set_state", "fp_reset", "fp_destroy", "fp_solve", "fp_solve_batched",
           "fp_adjoint", "fp_adjoint_create", "fp_adjoint_create_opts", "fp_adjoint_info", "fp_adjoint_run", "cq_prof_enable", "cq_prof_read",
           "cq_last_error"]
PROF_KINDS = {"hist_fast": 0, "hist_direct": 1, "far_toeplitz": 2, "solve_1d": 3, "prep_2d": 4, "dst_gemm": 5,
              "reduce_row": 6, "modal_fast": 7, "modal_near": 8, "batched": 9, "reduce_far": 10,
              "transpose": 11, "beta_spec": 12}


class CQError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


class Grid(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("lx", C.c_double), ("ly", C.c_double),
                ("nz", C.c_int32), ("lz", C.c_double)]


class Params(C.Structure):
    _fields_ = [("alpha1", C.c_double), ("alpha2", C.c_double), ("m", C.c_double), ("T", C.c_double),
                ("N", C.c_int64), ("scheme", C.c_int32), ("method", C.c_int32), ("fast_tol", C.c_double),
                ("np", C.c_int32), ("np1", C.c_int32), ("ns", C.c_int32), ("np_max", C.c_int32),
                ("block_B", C.c_int32), ("solver", C.c_int32), ("fast_kernel", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("n", C.c_int64), ("N", C.c_int64), ("np_total", C.c_int32), ("lag", C.c_int32),
                ("max_eps", C.c_double), ("theta", C.c_double * 2), ("block_B", C.c_int32),
                ("ksplit", C.c_int32), ("device_bytes", C.c_size_t), ("state_bytes", C.c_size_t),
                ("np1", C.c_int32), ("whole_run_kernel", C.c_int32)]


class AdjointOpts(C.Structure):
    _fields_ = [("max_device_bytes", C.c_size_t), ("mode", C.c_int32), ("segment_steps", C.c_int32),
                ("slots", C.c_int32), ("forward_kernel", C.c_int32)]


class AdjointInfo(C.Structure):
    _fields_ = [("mode", C.c_int32), ("segment_steps", C.c_int64), ("segments", C.c_int32), ("slots", C.c_int32),
                ("forward_steps", C.c_int64), ("device_bytes", C.c_size_t), ("forward_kernel", C.c_int32)]


class BatchReport(C.Structure):
    _fields_ = [("problems", C.c_int32), ("modes", C.c_int64), ("classes", C.c_int32),
                ("class_npl64", C.c_int32 * 8), ("class_lanes", C.c_int32 * 8), ("class_problems", C.c_int32 * 8),
                ("class_blocked", C.c_int32 * 8),
                ("setup_s", C.c_double), ("autotune_s", C.c_double), ("run_s", C.c_double)]


_lib: Optional[C.CDLL] = None


def lib() -> C.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run paper_1901_05128_amd/build.py "
                           "(or __graft_entry__.build())")
    try:  # share the HIP runtime torch already loaded (same SONAME)
        import torch  # noqa: F401
    except Exception:
        pass
    L = C.CDLL(LIB_PATH)
    P, D, I32, I64, VP = C.POINTER, C.c_double, C.c_int32, C.c_int64, C.c_void_p
    L.cq_weights.argtypes = [I32, D, D, I64, P(D)]
    L.cq_fast_rule.argtypes = [I32, D, D, I64, D, I32, I32, I32, I32, I32, P(D), P(D), P(I32), P(I32), P(D)]
    L.cq_history.argtypes = [I32, D, D, VP, I64, I64, VP, VP]
    L.cq_history_noalloc.argtypes = [I32, D, D, VP, I64, I64, VP, VP]
    L.fp_create.argtypes = [P(Grid), P(Params), VP, VP, P(VP)]
    L.fp_step.argtypes = [VP, I64]
    L.fp_current.argtypes = [VP, VP, P(I64)]
    L.fp_info.argtypes = [VP, P(Info)]
    L.fp_get_state.argtypes = [VP, VP, P(C.c_size_t)]
    L.fp_set_state.argtypes = [VP, VP, C.c_size_t]
    L.fp_reset.argtypes = [VP, VP]
    L.fp_destroy.argtypes = [VP]
    L.cq_prof_enable.argtypes = [I32]
    L.cq_prof_read.argtypes = [I32, P(I64), P(D)]
    L.fp_solve.argtypes = [P(Grid), P(Params), VP, VP, VP]
    L.fp_solve_batched.argtypes = [I32, P(Grid), P(Params), P(VP), P(VP), VP, I32, P(BatchReport)]
    L.fp_adjoint.argtypes = [P(Grid), P(Params), VP, VP, VP, P(D), VP, VP]
    L.fp_adjoint_create.argtypes = [P(Grid), P(Params), VP, P(VP)]
    L.fp_adjoint_create_opts.argtypes = [P(Grid), P(Params), P(AdjointOpts), VP, P(VP)]
    L.fp_adjoint_info.argtypes = [VP, P(AdjointInfo)]
    L.fp_adjoint_run.argtypes = [VP, VP, VP, VP, P(D), VP]
    L.cq_last_error.argtypes = []
    L.cq_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name != "cq_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != CQ_OK:
        raise CQError(rc, lib().cq_last_error().decode())


def make_grid(dim: int, nx: int, ny: int = 1, lx: float = 1.0, ly: float = 1.0, nz: int = 1,
              lz: float = 1.0) -> Grid:
    return Grid(dim, nx, ny if dim >= 2 else 1, lx, ly, nz if dim == 3 else 1, lz)


def grid_nodes(grid: Grid) -> int:
    return grid.nx * (grid.ny if grid.dim >= 2 else 1) * (grid.nz if grid.dim == 3 else 1)


SOLVER_NODAL, SOLVER_MODAL = 0, 1


def make_params(alpha1, alpha2, m, T, N, scheme, method, fast_tol=0.0, np_=0, np1=0, ns=0, np_max=0,
                block_B=0, solver=SOLVER_NODAL, fast_kernel=0) -> Params:
    return Params(alpha1, alpha2, m, T, int(N), scheme, method, fast_tol, np_, np1, ns, np_max, block_B, solver,
                  fast_kernel)


def params_of(p) -> tuple:
    """(Grid, Params) of a workloads.Problem."""
    return (make_grid(p.dim, p.nx, p.ny),
            make_params(p.alpha1, p.alpha2, p.m, p.T, p.N, p.scheme, p.method, np_=p.np_, ns=p.ns))


# ---- host entry points ----
def cq_weights(scheme: int, beta: float, tau: float, n: int) -> np.ndarray:
    out = np.empty(n + 1, dtype=np.float64)
    _check(lib().cq_weights(scheme, beta, tau, n, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def cq_fast_rule(scheme, beta, tau, N, tol=0.0, np_=0, np1=0, ns=0, np_max=0, cap=8192):
    r = np.empty(cap)
    c = np.empty(cap)
    cnt, lag, me = C.c_int32(), C.c_int32(), C.c_double()
    dp = C.POINTER(C.c_double)
    _check(lib().cq_fast_rule(scheme, beta, tau, N, tol, np_, np1, ns, np_max, cap, r.ctypes.data_as(dp),
                              c.ctypes.data_as(dp), C.byref(cnt), C.byref(lag), C.byref(me)))
    return r[:cnt.value].copy(), c[:cnt.value].copy(), lag.value, me.value


# ---- device entry points (torch tensors) ----
def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t, name):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()):
        raise CQError(CQ_EINVAL, f"{name} must be a contiguous float64 device tensor")
    return C.c_void_p(t.data_ptr())


def cq_history(scheme, beta, tau, G_hist, S_out=None):
    """S = sum_{i=1}^{n-1} d_i G^{n-i} for G_hist = [G^0..G^{n-1}] ([n][M])."""
    import torch
    n, M = G_hist.shape
    if S_out is None:
        S_out = torch.empty(M, dtype=torch.float64, device=G_hist.device)
    _check(lib().cq_history(scheme, beta, tau, _dev(G_hist, "G_hist"), n, M, _dev(S_out, "S_out"), _stream()))
    return S_out


def cq_history_noalloc(scheme, beta, tau, G_hist, S_out):
    """cq_history without device allocation (S_out is required); enqueued on
    torch's current stream without synchronising it."""
    n, M = G_hist.shape
    _check(lib().cq_history_noalloc(scheme, beta, tau, _dev(G_hist, "G_hist"), n, M, _dev(S_out, "S_out"),
                                    _stream()))
    return S_out


class Solver:
    """A solver handle (fp_create ... fp_destroy)."""

    def __init__(self, grid: Grid, params: Params, G0):
        self._h = C.c_void_p()
        self.grid, self.params = grid, params
        self.M = grid_nodes(grid)
        if tuple(G0.shape) not in ((2, self.M), (2 * self.M,)):
            raise CQError(CQ_EINVAL, f"G0 must have shape [2][{self.M}]")
        _check(lib().fp_create(C.byref(grid), C.byref(params), _dev(G0, "G0"), _stream(), C.byref(self._h)))

    def step(self, nsteps: int):
        _check(lib().fp_step(self._h, nsteps))

    def current(self, out=None):
        import torch
        if out is None:
            out = torch.empty((2, self.M), dtype=torch.float64, device="cuda")
        n = C.c_int64()
        _check(lib().fp_current(self._h, _dev(out, "out"), C.byref(n)))
        return out, n.value

    def info(self) -> Info:
        inf = Info()
        _check(lib().fp_info(self._h, C.byref(inf)))
        return inf

    def get_state(self) -> bytes:
        nb = C.c_size_t(0)
        _check(lib().fp_get_state(self._h, None, C.byref(nb)))
        buf = C.create_string_buffer(nb.value)
        _check(lib().fp_get_state(self._h, buf, C.byref(nb)))
        return buf.raw[: nb.value]

    def set_state(self, state: bytes):
        buf = C.create_string_buffer(state, len(state))
        _check(lib().fp_set_state(self._h, buf, len(state)))

    def reset(self, G0):
        _check(lib().fp_reset(self._h, _dev(G0, "G0")))

    def close(self):
        if self._h:
            _check(lib().fp_destroy(self._h))
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def prof_enable(on: bool = True):
    _check(lib().cq_prof_enable(1 if on else 0))


def prof_read(kind) -> tuple:
    """(launches, total_ms) for a kernel kind (name or number)."""
    k = PROF_KINDS[kind] if isinstance(kind, str) else int(kind)
    n, ms = C.c_int64(), C.c_double()
    _check(lib().cq_prof_read(k, C.byref(n), C.byref(ms)))
    return n.value, ms.value


def fp_solve(grid: Grid, params: Params, G0, GN=None):
    import torch
    M = grid_nodes(grid)
    if GN is None:
        GN = torch.empty((2, M), dtype=torch.float64, device=G0.device)
    _check(lib().fp_solve(C.byref(grid), C.byref(params), _dev(G0, "G0"), _dev(GN, "GN"), _stream()))
    return GN


def fp_adjoint(grid: Grid, params: Params, G0, gN, gG0=None, GN=None):
    """Gradient of a loss of G^N (modal solver): given gN = dl/dG^N, returns
    (dl/dG0 tensor, (dl/dalpha1, dl/dalpha2, dl/dm)); G^N is written to GN
    when given."""
    import torch
    if gG0 is None:
        gG0 = torch.empty_like(G0)
    g = (C.c_double * 3)()
    _check(lib().fp_adjoint(C.byref(grid), C.byref(params), _dev(G0, "G0"), _dev(gN, "gN"), _dev(gG0, "gG0"), g,
                            _dev(GN, "GN") if GN is not None else None, _stream()))
    return gG0, (g[0], g[1], g[2])


class Adjoint:
    """Gradient handle (fp_adjoint_create): set-up and device arrays once,
    then run(G0, gN) per gradient."""

    def __init__(self, grid: Grid, params: Params, mode: int = 0, max_device_bytes: int = 0,
                 segment_steps: int = 0, slots: int = 0, forward_kernel: int = 0):
        """mode 0 automatic, 1 keep the trajectory whole, 2 checkpointed
        (fast method); forward_kernel 0 automatic, 1 streamed state, 2 the
        16-mode MFMA kernel; see cq_adjoint_opts."""
        self._h = C.c_void_p()
        self.M = grid_nodes(grid)
        opts = AdjointOpts(max_device_bytes, mode, segment_steps, slots, forward_kernel)
        _check(lib().fp_adjoint_create_opts(C.byref(grid), C.byref(params), C.byref(opts), _stream(),
                                            C.byref(self._h)))

    def info(self) -> AdjointInfo:
        inf = AdjointInfo()
        _check(lib().fp_adjoint_info(self._h, C.byref(inf)))
        return inf

    def run(self, G0, gN, gG0=None, GN=None):
        import torch
        if gG0 is None:
            gG0 = torch.empty_like(G0)
        g = (C.c_double * 3)()
        _check(lib().fp_adjoint_run(self._h, _dev(G0, "G0"), _dev(gN, "gN"), _dev(gG0, "gG0"), g,
                                    _dev(GN, "GN") if GN is not None else None))
        return gG0, (g[0], g[1], g[2])

    def close(self):
        if self._h:
            _check(lib().fp_destroy(self._h))
            self._h = C.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


BATCH_DEFAULT, BATCH_AUTOTUNE, BATCH_TIME_BLOCKED, BATCH_MFMA_TILE, BATCH_PER_STEP = 0, 1, 2, 3, 4


def fp_solve_batched(grids, params, G0s, GNs=None, autotune=True):
    """Solve len(grids) independent fast problems in one batched launch.
    autotune: True (time the kernels per class), False (the default choice),
    or one of the BATCH_* kernel choices. Returns (list of GN tensors,
    BatchReport)."""
    import torch
    n = len(grids)
    if not (len(params) == n == len(G0s)):
        raise CQError(CQ_EINVAL, "grids, params and G0s must have the same length")
    if GNs is None:
        GNs = [torch.empty_like(g) for g in G0s]
    ga = (Grid * n)(*grids)
    pa = (Params * n)(*params)
    g0 = (C.c_void_p * n)(*[_dev(g, "G0").value for g in G0s])
    gn = (C.c_void_p * n)(*[_dev(g, "GN").value for g in GNs])
    rep = BatchReport()
    mode = int(autotune) if not isinstance(autotune, bool) else (1 if autotune else 0)
    _check(lib().fp_solve_batched(n, ga, pa, g0, gn, _stream(), mode, C.byref(rep)))
    return GNs, rep
