"""Long-double per-mode reference of the direct schemes (modal_ld.c).

ORACLE (test infrastructure only). A second evaluation of the per-mode
recurrence of oracle.modal (the direct BE (4.1) and BDF2 (4.7) schemes with
A -> lambda_p), in x87 extended precision, for measuring full-length fp64
runs (N = 2^14..2^16 steps) against the scheme's exact value. The C source
is compiled to oracle/libmodal_ld.so by the repository's build step, or here
with gcc on first use."""
import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "modal_ld.c")
LIB = os.path.join(HERE, "libmodal_ld.so")
CMD = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]

_lib = None


def build():
    subprocess.run(CMD, check=True, capture_output=True)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        L = C.CDLL(LIB)
        I, D, P = C.c_int, C.c_double, C.POINTER
        L.modal_direct_ld.argtypes = [I, I, I, I, I, P(I), P(I), P(I), D, D, D, D, C.c_long, P(D), I, P(D)]
        L.modal_direct_ld.restype = I
        _lib = L
    return _lib


def run_modes_ld(dim, nx, ny, modes, alpha1, alpha2, m, T, N, G0, scheme, nz=1):
    """Coefficients [2][K] of G^N of the direct scheme on the given modes
    ((p, q) pairs, q ignored in 1D, or (p, q, r) triples in 3D), from the
    nodal G0 ([2][nx*ny*nz])."""
    K = len(modes)
    mp = (C.c_int * K)(*[int(md[0]) for md in modes])
    mq = (C.c_int * K)(*[int(md[1]) if len(md) > 1 else 1 for md in modes])
    mr = (C.c_int * K)(*[int(md[2]) if len(md) > 2 else 1 for md in modes])
    G0 = np.ascontiguousarray(np.asarray(G0, dtype=np.float64).reshape(-1))
    out = np.zeros(2 * K)
    dp = C.POINTER(C.c_double)
    rc = lib().modal_direct_ld(dim, nx, ny if dim >= 2 else 1, nz if dim == 3 else 1, K, mp, mq, mr, alpha1, alpha2,
                               m, T, int(N), G0.ctypes.data_as(dp), scheme, out.ctypes.data_as(dp))
    if rc != 0:
        raise RuntimeError(f"modal_direct_ld returned {rc}")
    return out.reshape(2, K)
