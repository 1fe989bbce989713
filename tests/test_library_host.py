"""CPU tests of the C-ABI library: it loads, exports every declared entry
point, and its host-side math (weights, fast rules, argument checks, step
operator check) agrees with the oracle. No device compute is called."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_1901_05128_amd as cq
from paper_1901_05128_amd import _lib
from oracle import quadrature as Q
from oracle import weights as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "cqfp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    names = _declared_functions()
    assert len(names) >= 12
    L = cq.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTS)


@pytest.mark.parametrize("scheme", [1, 2])
@pytest.mark.parametrize("beta", [0.1, 0.4, 0.8, 0.99])
def test_weights_match_oracle(scheme, beta):
    tau, n = 1.0 / 3000, 20000
    d = cq.cq_weights(scheme, beta, tau, n)
    o = W.weights(scheme, beta, tau, n)
    assert np.max(np.abs(d - o)) <= 1e-14 * abs(o[0])
    assert np.max(np.abs(d - o) / np.abs(o)) <= 2e-11


@pytest.mark.parametrize("beta", [0.2, 0.7])
@pytest.mark.parametrize("np_", [5, 64, 384])
def test_be_fast_rule_matches_oracle(beta, np_):
    tau = 1e-3
    r, c, lag, _ = cq.cq_fast_rule(1, beta, tau, 4000, np_=np_)
    o = Q.be_rule(beta, tau, np_)
    assert lag == 2 and len(r) == np_
    i = np.argsort(r)
    oi = np.argsort(o.ratio)
    assert np.allclose(r[i], o.ratio[oi], rtol=0, atol=2e-15)
    ocoef = (o.w * o.dbar(2))[oi]
    assert np.max(np.abs(c[i] - ocoef)) <= 1e-12 * np.max(np.abs(ocoef))


@pytest.mark.parametrize("beta", [0.3, 0.8])
def test_bdf2_fast_rule_matches_oracle(beta):
    tau, ns = 1e-3, 30
    r, c, lag, _ = cq.cq_fast_rule(2, beta, tau, 4000, np_=96, np1=16, ns=ns)
    r1, r2 = Q.bdf2_rules(beta, tau, 16, 96)
    assert lag == ns and len(r) == 112
    ref_r = np.concatenate([r1.ratio, r2.ratio])
    ref_c = np.concatenate([r1.w * r1.dbar(ns), r2.w * r2.dbar(ns)])
    # compare as approximations of d_i (node order may differ)
    i = np.arange(ns, 600)
    got = (c[None, :] * r[None, :] ** (i[:, None] - ns)).sum(axis=1)
    ref = (ref_c[None, :] * ref_r[None, :] ** (i[:, None] - ns)).sum(axis=1)
    assert np.max(np.abs(got - ref)) <= 1e-13 * abs(W.bdf2_weights(beta, tau, 0)[0])


@pytest.mark.parametrize("scheme,N", [(1, 1000), (1, 16384), (2, 16384), (2, 300)])
def test_fast_rule_scan_meets_target(scheme, N):
    beta, tol = 0.6, 1e-8
    r, c, lag, me = cq.cq_fast_rule(scheme, beta, 1.0 / N, N, tol=tol)
    d = W.weights(scheme, beta, 1.0 / N, N)
    i = np.arange(lag, N + 1)
    approx = np.zeros(len(i))
    for rj, cj in zip(r, c):
        approx += cj * rj ** (i - lag)
    eps = np.max(np.abs(approx - d[lag:])) / abs(d[0])
    assert eps <= tol / (10 * N) * 1.01
    assert abs(eps - me) <= 1e-3 * max(me, 1e-30) + 1e-18


def test_fast_rule_reports_etol():
    with pytest.raises(cq.CQError) as e:
        cq.cq_fast_rule(1, 0.3, 1.0 / 65536, 65536, tol=1e-8, np_max=32)
    assert e.value.code == _lib.CQ_ETOL


@pytest.mark.parametrize("args", [(3, 0.5, 0.1, 10), (1, 0.0, 0.1, 10), (1, 1.0, 0.1, 10), (1, 0.5, -1.0, 10),
                                  (2, 0.5, 0.1, -1)])
def test_weights_reject_bad_arguments(args):
    with pytest.raises(cq.CQError) as e:
        cq.cq_weights(*args)
    assert e.value.code == _lib.CQ_EINVAL


def _create(grid, prm):
    h = C.c_void_p()
    dummy = C.c_void_p(0x1000)  # never dereferenced: checks fail first
    rc = cq.lib().fp_create(C.byref(grid), C.byref(prm), dummy, None, C.byref(h))
    return rc, h


@pytest.mark.parametrize("bad", [
    dict(alpha1=0.0), dict(alpha2=1.0), dict(m=0.5), dict(m=1.2), dict(T=0.0), dict(N=0), dict(scheme=3),
    dict(method=2), dict(ns=2, scheme=2), dict(block_B=100), dict(np_=-1)])
def test_fp_create_rejects_bad_params(bad):
    kw = dict(alpha1=0.3, alpha2=0.7, m=0.3, T=1.0, N=10, scheme=1, method=0)
    kw.update(bad)
    prm = cq.make_params(**kw)
    rc, h = _create(cq.make_grid(1, 31), prm)
    assert rc == _lib.CQ_EINVAL and not h.value


@pytest.mark.parametrize("grid", [cq.make_grid(4, 4), cq.make_grid(1, 0), cq.make_grid(1, 5000),
                                  cq.Grid(1, 4, 2, 1.0, 1.0), cq.make_grid(2, 4, 4, lx=0.0),
                                  cq.Grid(3, 2, 2, 1.0, 1.0, 0, 1.0), cq.Grid(2, 2, 2, 1.0, 1.0, 3, 1.0),
                                  cq.Grid(3, 2, 2, 1.0, 1.0, 2, 0.0), cq.Grid(3, 2, 2048, 1.0, 1.0, 1024, 1.0)])
def test_fp_create_rejects_bad_grid(grid):
    rc, h = _create(grid, cq.make_params(0.3, 0.7, 0.3, 1.0, 10, 1, 0))
    assert rc == _lib.CQ_EINVAL


def test_fp_create_reports_singular_step_operator():
    """alpha1 = alpha2 = 0.1, m = 0.45 (a = -5.5), T = 1, N = 1 on the 127-node
    grid: the coupling eigenvalue theta = c/d_0 + a - |a| = 1 - 11 = -10 lies
    below -lambda_min = -(4/h^2) sin^2(pi h/2) = -9.869..."""
    rc, h = _create(cq.make_grid(1, 127), cq.make_params(0.1, 0.1, 0.45, 1.0, 1, 1, 0))
    assert rc == _lib.CQ_ESINGULAR
    assert "positive definite" in cq.lib().cq_last_error().decode()
    # a smaller step is fine (fails later, at the device, on a CPU-only machine)
    rc2, _ = _create(cq.make_grid(1, 127), cq.make_params(0.1, 0.1, 0.45, 1.0, 1024, 1, 0))
    assert rc2 != _lib.CQ_ESINGULAR


def test_fast_create_reports_etol_before_device():
    prm = cq.make_params(0.3, 0.7, 0.3, 1.0, 65536, 1, 1, fast_tol=1e-8, np_max=16)
    rc, _ = _create(cq.make_grid(1, 31), prm)
    assert rc == _lib.CQ_ETOL


def _adjoint_create(grid, prm):
    h = C.c_void_p()
    rc = cq.lib().fp_adjoint_create(C.byref(grid), C.byref(prm), None, C.byref(h))
    return rc, h


def test_adjoint_create_host_checks():
    """The gradient handle's argument checks come before any device call:
    the nodal solver, bad parameters and a fast window above 32 levels are
    rejected with CQ_EINVAL; a singular step operator with CQ_ESINGULAR."""
    g = cq.make_grid(1, 31)
    rc, h = _adjoint_create(g, cq.make_params(0.3, 0.7, 0.3, 1.0, 10, 1, 0, solver=cq.SOLVER_NODAL))
    assert rc == _lib.CQ_EINVAL and not h.value
    assert "modal" in cq.lib().cq_last_error().decode()
    rc, h = _adjoint_create(g, cq.make_params(0.0, 0.7, 0.3, 1.0, 10, 1, 0, solver=cq.SOLVER_MODAL))
    assert rc == _lib.CQ_EINVAL
    rc, h = _adjoint_create(g, cq.make_params(0.3, 0.7, 0.3, 1.0, 100, 2, 1, np_=16, ns=40,
                                              solver=cq.SOLVER_MODAL))
    assert rc == _lib.CQ_EINVAL and "32" in cq.lib().cq_last_error().decode()
    rc, h = _adjoint_create(cq.make_grid(1, 127), cq.make_params(0.1, 0.1, 0.45, 1.0, 1, 1, 0,
                                                                 solver=cq.SOLVER_MODAL))
    assert rc == _lib.CQ_ESINGULAR


def test_adjoint_opts_host_checks():
    """The memory form's checks come before any device call: an unknown mode,
    negative counts, and the checkpointed form for the direct method."""
    g = cq.make_grid(1, 31)
    fast = cq.make_params(0.3, 0.7, 0.3, 1.0, 100, 2, 1, np_=12, np1=8, ns=10, solver=cq.SOLVER_MODAL)
    direct = cq.make_params(0.3, 0.7, 0.3, 1.0, 100, 2, 0, solver=cq.SOLVER_MODAL)
    L = cq.lib()
    for prm, opts in [(fast, _lib.AdjointOpts(0, 3, 0, 0)), (fast, _lib.AdjointOpts(0, 2, -1, 0)),
                      (fast, _lib.AdjointOpts(0, 2, 0, -2)), (direct, _lib.AdjointOpts(0, 2, 0, 0))]:
        h = C.c_void_p()
        rc = L.fp_adjoint_create_opts(C.byref(g), C.byref(prm), C.byref(opts), None, C.byref(h))
        assert rc == _lib.CQ_EINVAL and not h.value, (opts.mode, rc)
    assert "fast method" in L.cq_last_error().decode()
    assert L.fp_adjoint_info(None, None) == _lib.CQ_EINVAL


def test_handle_calls_reject_null():
    L = cq.lib()
    assert L.fp_step(None, 1) == _lib.CQ_EINVAL
    assert L.fp_adjoint_run(None, None, None, None, None, None) == _lib.CQ_EINVAL
    assert L.fp_destroy(None) == _lib.CQ_OK


def test_history_noalloc_host_checks():
    """The allocation-free history row rejects sizes beyond its static
    workspace (2^20 levels) and bad arguments before any device call."""
    L = cq.lib()
    fake = C.c_void_p(16)  # never dereferenced: every case fails its checks first
    assert L.cq_history_noalloc(1, 0.4, 1e-3, fake, (1 << 20) + 1, 10, fake, None) == _lib.CQ_EINVAL
    assert "2^20" in cq.lib().cq_last_error().decode() or "1048576" in cq.lib().cq_last_error().decode()
    assert L.cq_history_noalloc(3, 0.4, 1e-3, fake, 10, 10, fake, None) == _lib.CQ_EINVAL
    assert L.cq_history_noalloc(1, 1.0, 1e-3, fake, 10, 10, fake, None) == _lib.CQ_EINVAL
    assert L.cq_history_noalloc(1, 0.4, 1e-3, fake, 0, 10, fake, None) == _lib.CQ_EINVAL
    assert L.cq_history_noalloc(1, 0.4, 1e-3, None, 10, 10, fake, None) == _lib.CQ_EINVAL
