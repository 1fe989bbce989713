#!/usr/bin/env python3
"""Throughput of the CQ Fokker-Planck solver on one MI355X.

One bench step = full solves (all N time steps, inputs resident in HBM) of
the workload's timed variants. For the 2D 255^2, N = 2^16 workload (the
default) that is the BDF2 scheme with the fast history and with the direct
(blocked Toeplitz) history, one after the other on one stream; for the 1D
workloads it is BE and BDF2, each fast and direct, run concurrently, one
stream each. The value is whole-job
DOF*steps/s (DOF = 2 components x grid nodes) over the timed variants. Every
variant (BE included) then runs once more, serially and outside the timed
region, with HIP events around every kernel launch: that pass gives the
per-variant times, the fast-vs-direct difference of both schemes and the
dominant kernel's roofline. The CPU oracle's rate is reported beside it
(timed on a prefix of the same workload, extrapolated to N steps). With the
default workload the line also carries the adjoint rate ("adjoint": gradients
per second of the 127^2, N = 4096 adjoint workload, measured afterwards).

Usage: python bench.py [--steps K] [--warmup W] [--workload c3|c2|c1|c4|c5|t5]
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6        # MI355X dense FP64 (vector and MFMA)

WORKLOADS = {
    # name: (description, dim, nx, ny, alpha1, alpha2, m, T, N, seed)
    "c1": ("1D 127 nodes, N=1000", 1, 127, 1, 0.3, 0.7, 0.3, 1.0, 1000, 1),
    "c2": ("1D 1023 nodes, N=2^14", 1, 1023, 1, 0.4, 0.8, 0.45, 1.0, 2 ** 14, 2),
    "c3": ("2D 255x255 nodes, N=2^16", 2, 255, 255, 0.2, 0.6, 0.55, 1.0, 2 ** 16, 3),
    # the paper's Table 5 problem (Section 5): h = 1/1024, T = 10, tau = 1/2000,
    # a = -1 (m = 0), BDF2 (SBD) direct and fast, smooth data (a)
    "t5": ("1D 1023 nodes, T=10, tau=1/2000 (N=20000), data (a), the paper's Table 5", 1, 1023, 1, 0.3, 0.8, 0.0,
           10.0, 20000, None),
}
VARIANTS = [(1, 1), (1, 0), (2, 1), (2, 0)]  # (scheme, method)
# variants inside the timed step (the rest run in the serial pass only)
TIMED = {"c3": [(2, 1), (2, 0)], "t5": [(2, 1), (2, 0)]}
# variants of the serial pass (default: all four)
SERIAL = {"t5": [(2, 1), (2, 0)]}
# workloads whose timed variants run one after another on one stream: at c3 the
# far-field passes fill the chip, and the fast solve's kernels between them on a
# second stream made the step 5.6% slower (9.04 s against 8.55 s)
ONE_STREAM = {"c3"}
# Table 5's CPU times (seconds, BDF2 direct / fast, order pairs (0.3,0.8),
# (0.4,0.7), (0.5,0.6); the paper names no machine) and its L2 errors
# E_1, E_2 against a tau/2 run
T5_PAPER = {"direct_s": [870.13, 883.70, 882.48], "fast_s": [209.44, 210.83, 211.36],
            "direct_E": [[2.628e-10, 7.571e-09], [4.019e-10, 3.471e-09], [7.399e-10, 1.561e-09]],
            "fast_E": [[3.543e-10, 1.321e-08], [4.862e-10, 5.697e-09], [1.008e-09, 2.375e-09]]}
VNAME = {(1, 1): "be_fast", (1, 0): "be_direct", (2, 1): "bdf2_fast", (2, 0): "bdf2_direct"}
SOLVERS = {"nodal": 0, "modal": 1}


def g0_for(w):
    from paper_1901_05128_amd import workloads as wl
    _, dim, nx, ny, *_rest, seed = w
    if seed is None:
        return wl.g0_smooth(nx, ny)
    if nx == 127 and dim == 1:
        return wl.g0_c1(nx, seed)
    return wl.g0_intervals(nx, seed) if dim == 1 else wl.g0_rectangle(nx, ny, seed)


def kernel_work(kind, w, scheme, method, info, M, solver=1):
    """Algorithmic (bytes, flops) summed over the launches of one solve."""
    N = w[8]
    twoM = 2 * M
    if method == 1 and kind in ("hist_direct", "far_toeplitz", "modal_near"):
        return 0, 0
    if method == 0 and kind in ("hist_fast", "modal_fast"):
        return 0, 0
    if kind == "hist_fast":
        # one launch per block of bt steps: state read + write once, the bt
        # levels entering the state, bt history values out; 2 FMAs per node
        # per step
        L, npn, Bt = info.lag, info.np_total, info.block_B
        b, f = 0, 0
        for n in range(1, N + 1, Bt):
            bt = min(Bt, N - n + 1)
            b += twoM * 8 * (2 * npn + 2 * bt)
            f += twoM * 4 * npn * bt
        return b, f
    if kind == "far_toeplitz":
        # nodal: one pass per block of B steps over the levels before it.
        # modal: one pass of Bf rows per Bf steps, and for each later 64-step
        # block of the pass the levels since the pass. Rows past N are not
        # counted; bytes = levels read once + rows written once.
        Bf = info.block_B
        Bn = 64 if solver == 1 else Bf
        fl, by = 0, 0
        for n0 in range(Bn, N, Bn):
            base = (n0 // Bf) * Bf
            rows_pass = min(Bf, N - n0)
            if base == n0:
                fl += 2 * rows_pass * n0 * twoM
                by += (n0 + rows_pass) * twoM * 8
            else:
                rows, lv = min(Bn, N - n0), n0 - base
                fl += 2 * rows * lv * twoM
                by += (lv + rows) * twoM * 8
        return by, fl
    if kind == "hist_direct":
        B = info.block_B
        by = 0
        for n in range(1, N + 1):
            n0 = ((n - 1) // B) * B
            by += twoM * 8 * ((n - 1 - n0) + 1 + (1 if n0 >= 1 else 0))
        return by, 0
    if kind == "dst_gemm":
        nx, ny = w[2], w[3]
        return 0, N * 2 * (2 * ny * nx * nx + 2 * ny * ny * nx) * 2
    if kind == "modal_fast":
        # wave-per-mode (few modes) or blocked (many modes: the window steps;
        # the state pass is counted under hist_fast): 2 FMAs per node and
        # component per step, plus the exact-weight window
        L, npn = info.lag, info.np_total
        if M >= 8192:
            return N * twoM * 8 * 3, N * twoM * 2 * (L - 1)
        return 0, N * twoM * (4 * npn + 2 * (L - 1))
    if kind == "modal_near":
        # in-block near field (b terms at block offset b) + far-field read + level write
        B = 64
        f = 0
        for n in range(1, N + 1):
            f += twoM * 2 * ((n - 1) % B)
        return N * twoM * 8 * 2, f
    if kind in ("solve_1d", "prep_2d"):
        # window of exact weights (fast) or the partial sums, G^{n-1}, G^{n-2}, G0, output
        win = (info.lag - 1) if method == 1 else 1
        return N * twoM * 8 * (win + 5), 0
    return 0, 0


def cpu_baseline(w, variants):
    """The oracle (oracle.stepper: nodal direct and fast steppers) timed on
    prefixes of the same workload (same grid, tau and G0) and extrapolated
    to all N steps. The direct stepper's step n costs c1 + c2 (n - 1): c2
    (one history level of both components) is the oracle's own history sum
    over a block of stored levels, timed with all BLAS threads and with one;
    c1 comes from two prefix runs (their difference cancels the set-up, the
    history share of the extra steps taken out). The fast stepper's step
    costs a constant once its state is live (steps beyond the lag): the
    difference of two prefix runs past the lag. Elementwise numpy and the
    sparse LU solves run on one thread, so only c2 depends on the core
    count; the faster of the two thread counts is the reported value."""
    import numpy as np
    from oracle import stepper
    from oracle.weights import weights
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        cores = os.cpu_count() or 1
    desc, dim, nx, ny, a1, a2, m, T, N, seed = w
    G0 = g0_for(w)
    tau = T / N
    M = nx * ny
    t_start = time.perf_counter()

    def run(scheme, method, n):
        t0 = time.perf_counter()
        stepper.solve(dim, nx, ny, a1, a2, m, n * tau, n, G0, scheme, method,
                      np_=(None if method == 0 else max(16, int(np.ceil(3 * N ** 0.5)))), ns=30)
        return time.perf_counter() - t0

    # c2: the history sum over nh stored levels of [2][M] (about 256 MB)
    nh = int(max(16, min(N, 256e6 // (16 * M))))
    rng = np.random.default_rng(0)
    Gh = rng.standard_normal((nh, 2 * M))
    d = weights(2, 1.0 - a1, tau, nh)

    def t_hist():
        best = 1e30
        for _ in range(3):
            t0 = time.perf_counter()
            stepper.cq_history(d, Gh)
            best = min(best, time.perf_counter() - t0)
        return best / (nh - 1)

    c2_all = t_hist()
    c2_one = c2_all
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            c2_one = t_hist()
    del Gh
    na, nb = (64, 256) if dim == 1 else (8, 24)
    full = {"all": 0.0, "one": 0.0}
    parts = []
    for scheme, method in variants:
        if method == 0:
            ta, tb = run(scheme, 0, na), run(scheme, 0, nb)
            hist_steps = sum(k - 1 for k in range(na + 1, nb + 1))
            c1 = max(0.0, (tb - ta - c2_all * hist_steps) / (nb - na))
            tot = N * (N - 1) / 2
            full["all"] += c1 * N + c2_all * tot
            full["one"] += c1 * N + c2_one * tot
            parts.append(f"{VNAME[(scheme, 0)]}: prefixes {na}/{nb} steps {ta:.3f}/{tb:.3f} s, "
                         f"c1 {c1 * 1e3:.2f} ms/step")
        else:
            lag = 3 if scheme == 1 else 31
            fa, fb = (max(na, lag), max(na, lag) + (nb - na)) if dim == 1 else (lag, lag + 4)
            ta, tb = run(scheme, 1, fa), run(scheme, 1, fb)
            per = (tb - ta) / (fb - fa)
            full["all"] += per * N
            full["one"] += per * N
            parts.append(f"{VNAME[(scheme, 1)]}: prefixes {fa}/{fb} steps {ta:.3f}/{tb:.3f} s, "
                         f"{per * 1e3:.3f} ms/step")
    work = len(variants) * 2 * M * N
    spent = time.perf_counter() - t_start
    # the oracle's faster configuration is the baseline (on a shared host the
    # threaded history sum can be the slower one)
    best, used = (full["all"], int(cores)) if full["all"] <= full["one"] else (full["one"], 1)
    return {"value": work / best, "unit": "DOF*steps/s", "cores": used, "kind": "oracle",
            "extrapolated": True, "value_all_threads": work / full["all"], "all_threads": int(cores),
            "value_1core": work / full["one"],
            "est_full_run_s": best, "est_full_run_s_all_threads": full["all"], "est_full_run_s_1core": full["one"],
            "sample": f"{desc}, the timed variants ({', '.join(VNAME[v] for v in variants)}) of the oracle "
                      f"(numpy/scipy fp64 nodal steppers) on prefixes of the workload, extrapolated to N = {N}: "
                      + "; ".join(parts)
                      + f"; history sum c2 {c2_all * 1e3:.3f} ms per level ({cores} threads), "
                        f"{c2_one * 1e3:.3f} ms (1 thread), timed over {nh} levels; {spent:.1f} s of CPU work"}


# source file of each kernel family whose traffic profiles/traffic.json holds
KERNEL_SOURCE = {"far_toeplitz": "far.hip", "hist_fast": "kernels.hip", "batched": "batch_mx.hip"}


def copy_probe(mib):
    """Four copies of a mib-MiB device buffer (a plain copy kernel of known
    size) after the measured work: rocprofv3's FETCH_SIZE and WRITE_SIZE of
    these calibrate the counters. Returns the bytes copied each way."""
    import torch

    nel = mib * (1 << 20) // 8
    src = torch.ones(nel, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(4):
        dst.copy_(src)
    torch.cuda.synchronize()
    return nel * 8


def load_traffic(kernel_name, workload):
    """HBM traffic per launch from the committed rocprofv3 --pmc summary for
    this kernel and workload, or None when it is missing or the kernel's
    source file changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        src = os.path.join(ROOT, "paper_1901_05128_amd", "csrc", KERNEL_SOURCE[kernel_name])
        rec = json.load(open(path))
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
        ent = rec.get(f"{kernel_name}@{workload}")
        if not ent or ent.get("source_sha256") != sha:
            return None
        return ent.get("bytes_per_launch")
    except Exception:
        return None


def bench_batched(args):
    """One step = one batched solve of the 256 seeded fast-BDF2 problems
    (1D 127..4095 nodes and 2D 63^2..255^2, N = 2^10..2^15, np = ceil(3 sqrt N))."""
    import math

    import torch

    import paper_1901_05128_amd as cq
    from paper_1901_05128_amd import workloads as wl
    torch.cuda.set_device(0)
    inst = wl.batched_instances(256, seed=4)
    grids, params, g0s = [], [], []
    for i, p in enumerate(inst):
        grids.append(cq.make_grid(p.dim, p.nx, p.ny))
        params.append(cq.make_params(p.alpha1, p.alpha2, p.m, p.T, p.N, 2, 1,
                                     np_=int(math.ceil(3 * math.sqrt(p.N)))))
        g0 = wl.g0_intervals(p.nx, 1000 + i) if p.dim == 1 else wl.g0_rectangle(p.nx, p.ny, 1000 + i)
        g0s.append(torch.tensor(g0, dtype=torch.float64, device="cuda"))
    outs = [torch.empty_like(g) for g in g0s]
    kern = {"auto": cq.BATCH_AUTOTUNE, "default": cq.BATCH_DEFAULT, "time_blocked": cq.BATCH_TIME_BLOCKED,
            "mfma_tile": cq.BATCH_MFMA_TILE, "per_step": cq.BATCH_PER_STEP}[args.batch_kernel]
    for _ in range(args.warmup):
        cq.fp_solve_batched(grids, params, g0s, outs, autotune=kern)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = []
    for _ in range(args.steps):
        reps.append(cq.fp_solve_batched(grids, params, g0s, outs, autotune=kern)[1])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    dofsteps = args.steps * sum(2 * p.nx * p.ny * p.N for p in inst)
    rep = reps[-1]
    # the time loops' work: per mode, component and step, the state update and
    # its weighting (4 flops per node, 16 + ceil(3 sqrt N) nodes) and the
    # exact-weight window (2 flops per lag below N_s = 30); FP64 vector bound
    flops = sum(2 * p.nx * p.ny * p.N * (4 * (16 + int(math.ceil(3 * math.sqrt(p.N)))) + 2 * 29) for p in inst)
    ach = flops / rep.run_s / 1e12
    kinds = list(rep.class_blocked)[:rep.classes]
    mx = sum(1 for x in kinds if x == 2)
    # FP64 matrix and vector peaks are the same figure on this GPU
    roofline = {"bound": "mfma" if 2 * mx > len(kinds) else "alu", "achieved": ach, "peak": FP64_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
                "kernel": "k_modal_batch_mx / k_modal_batch_tb / k_modal_batch (all classes)",
                "timed": "graph run time of the last step (the kernels run inside one captured graph)",
                "traffic": None}
    rec = {
        "metric": "DOF*steps/s (batched fast BDF2 solves)", "value": dofsteps / (t1 - t0), "unit": "DOF*steps/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": (t1 - t0) / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded indicator initial data)",
        "config": {"workload": "c4: 256 seeded fast-BDF2 problems, 1D 127-4095 nodes / 2D 63^2-255^2, "
                               "N=2^10..2^15, np=ceil(3 sqrt N), one captured graph",
                   "modes": rep.modes, "classes": rep.classes,
                   "lanes_per_mode": list(rep.class_lanes)[:rep.classes],
                   "class_kernel": [{0: "per_step", 1: "time_blocked", 2: "mfma_tile"}[x] for x in kinds],
                   "kernel_choice": args.batch_kernel},
        "breakdown": {"setup_s": rep.setup_s, "autotune_s": rep.autotune_s, "graph_run_s": rep.run_s},
        "roofline": roofline,
    }
    print(json.dumps(rec), flush=True)


def bench_adjoint(args, emit=True):
    """One step = one gradient of l = 1/2 |G^N - target|^2 on the adjoint
    workload (2D 127^2, BDF2 fast, N = 4096, np = 16 + 192, ns = 30): the
    forward solve with the trajectory kept, the reversed-time adjoint sweep
    and the gradient passes (dl/dG0 and the three scalars)."""
    import numpy as np
    import torch

    import paper_1901_05128_amd as cq
    from paper_1901_05128_amd import workloads as wl
    torch.cuda.set_device(0)
    nx = ny = 127
    N = 4096
    g = cq.make_grid(2, nx, ny)

    def prm(a1, a2, m):
        return cq.make_params(a1, a2, m, 1.0, N, 2, 1, np_=192, np1=16, ns=30, solver=cq.SOLVER_MODAL)

    G0 = torch.tensor(wl.g0_rectangle(nx, ny, 5), dtype=torch.float64, device="cuda")
    target = cq.fp_solve(g, prm(0.25, 0.55, 0.55), torch.tensor(wl.g0_rectangle(nx, ny, 6), dtype=torch.float64,
                                                               device="cuda"))
    p = prm(0.2, 0.6, 0.55)
    GN = cq.fp_solve(g, p, G0)
    gN = GN - target
    gG0 = torch.empty_like(G0)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    h = cq.Adjoint(g, p)      # host set-up (weights, rules, derivatives) and device arrays, once
    setup_s = time.perf_counter() - ts
    for _ in range(args.warmup):
        h.run(G0, gN, gG0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        _, grads = h.run(G0, gN, gG0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = (t1 - t0) / args.steps
    ts = time.perf_counter()
    cq.fp_adjoint(g, p, G0, gN, gG0)
    oneshot_s = time.perf_counter() - ts
    M = nx * ny
    # kernel timing: one more gradient outside the timed region
    kinds = ["hist_fast", "far_toeplitz", "reduce_far", "modal_fast", "dst_gemm", "transpose", "beta_spec", "batched"]
    ktime = {}
    roofline = None
    if not args.no_prof:
        cq.prof_enable(True)
        h.run(G0, gN, gG0)
        torch.cuda.synchronize()
        for k in kinds:
            n_l, ms = cq.prof_read(k)
            if n_l:
                ktime[k] = (n_l, ms)
        cq.prof_enable(False)
        twoM = 2 * M
        npn, L, Bt = 16 + 192, 30, 30
        work = {}
        b_h, f_h = 0, 0
        for n in range(1, N + 1, Bt):
            bt = min(Bt, N - n + 1)
            b_h += twoM * 8 * (2 * npn + 2 * bt)
            f_h += twoM * 4 * npn * bt
        # with forward_kernel 2 both sweeps run on the 16-mode MFMA kernel,
        # else on the state pass and the window steps
        mxf = h.info().forward_kernel == 2
        sweeps = 0 if mxf else 2
        work["hist_fast"] = (sweeps * b_h, sweeps * f_h)  # forward and adjoint sweeps
        # up to 448 nodes the MFMA sweeps also write their levels as the block
        # DFTs' time series (the bench's handle has the memory for them)
        cols = mxf and npn <= 448
        if mxf:
            # per sweep: state update and weighting (4 flops per node), window
            # (2 per lag below L); two arrays written per step (level and
            # history sum, or psi and mu), three with the time series
            work["batched"] = (2 * (3 if cols else 2) * N * twoM * 8, 2 * N * twoM * (4 * npn + 2 * (L - 1)))
        # the d/dalpha contraction's near field: blocks of Bk steps (the power
        # of two nearest 2.25 sqrt(N), 128 here), each step n of block i
        # summing dw_{n-l} g^l over the levels l of blocks i-1 and i up to n
        # (2 flops per product, mode and component); a block reads those
        # levels once and writes its rows
        Bk = 1 << min(8, max(3, round(math.log2(2.25 * math.sqrt(N)))))
        f_far, b_far = 0, 0
        for n0 in range(0, N, Bk):
            bt = min(Bk, N - n0)
            l0 = max(1, n0 - Bk + 1)
            f_far += sum(2 * (n - l0 + 1) * twoM for n in range(n0 + 1, n0 + bt + 1))
            b_far += (n0 + bt - l0 + 1) * twoM * 8 + bt * twoM * 8
        work["far_toeplitz"] = (b_far, f_far)
        # its farther block pairs: per mode and component nb FFTs of P = 2 Bk
        # points (5 P log2 P flops each) and (nb-2)(nb-1)/2 block products of
        # Bk + 1 frequencies (8 flops each), reading psi and g (N doubles each)
        nb, P = -(-N // Bk), 2 * Bk
        work["beta_spec"] = (twoM * 2 * N * 8, twoM * (nb * 5 * P * int(math.log2(P)) +
                                                      (nb - 2) * (nb - 1) // 2 * (Bk + 1) * 8))
        if not cols:
            work["transpose"] = (2 * 2 * N * twoM * 8, 0)
        # window steps, both sweeps (none with the MFMA kernel): 2 flops per
        # lag below L, Sf read, level and S (forward) or mu (adjoint) written
        work["modal_fast"] = (sweeps * N * twoM * 8 * 3, sweeps * N * twoM * 2 * (L - 1))
        dom = max(ktime, key=lambda k: ktime[k][1])
        if dom in work:
            n_l, ms = ktime[dom]
            avg = ms / 1e3 / n_l
            b, f = work[dom]
            ff = f / n_l / avg / 1e12 / FP64_PEAK_TFLOPS
            bf = b / n_l / avg / 1e9 / HBM_PEAK_GBS
            if ff >= bf:
                roofline = {"bound": "mfma" if dom in ("far_toeplitz", "batched") else "alu",
                            "achieved": ff * FP64_PEAK_TFLOPS,
                            "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ff, "hbm_frac": bf}
            else:
                roofline = {"bound": "hbm", "achieved": bf * HBM_PEAK_GBS, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                            "frac": bf, "fp64_frac": ff}
            roofline.update({"kernel": dom, "avg_launch_us": avg * 1e6, "launches": n_l,
                             "timed": "one extra gradient after the timed region, HIP events per launch",
                             "traffic": load_traffic(dom, "c5")})
    rec = {
        "metric": "gradients/s (dl/dG0 and dl/dalpha_1, dl/dalpha_2, dl/dm)", "value": 1.0 / per,
        "unit": "grads/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": per * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic (seeded rectangle indicators)",
        "config": {"workload": "c5: adjoint, 2D 127x127 nodes, BDF2 fast (np 16+192, ns 30), N=4096, "
                               "alpha=(0.2,0.6), m=0.55, target from alpha=(0.25,0.55)",
                   "dof": 2 * M, "N": N,
                   "sweeps": "16-mode MFMA kernel" if h.info().forward_kernel == 2 else "streamed state"},
        "grads": list(grads),
        "breakdown": {"handle_setup_s": setup_s, "one_shot_fp_adjoint_s": oneshot_s,
                      "note": "value times fp_adjoint_run on a handle made once (fixed grid and parameters)"},
        "kernels_ms": {k: {"launches": v[0], "total_ms": v[1]} for k, v in ktime.items()},
        "roofline": roofline,
    }
    h.close()
    if emit and args.copy_probe:
        rec["copy_probe_bytes_each_way"] = copy_probe(args.copy_probe)
    if emit:
        print(json.dumps(rec), flush=True)
    return rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default 5; 2 for c3, 1 for c4)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default 2; 1 for c3 and c4)")
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS) + ["c4", "c5"])
    ap.add_argument("--t5-errors", action="store_true",
                    help="t5: also run tau/2 (N = 40000) and report the L2 errors of Table 5's protocol")
    ap.add_argument("--t5-data", default="a", choices=["a", "b"],
                    help="t5: the paper's smooth data (a) or nonsmooth data (b)")
    ap.add_argument("--variants", default="default",
                    help="comma list of be_fast,be_direct,bdf2_fast,bdf2_direct timed in a step "
                         "(default: bdf2_fast,bdf2_direct for c3, all four otherwise)")
    ap.add_argument("--solver", default="modal", choices=sorted(SOLVERS),
                    help="modal: sine transform once, per-mode recurrences; nodal: per-step grid solve")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--fast-kernel", default="auto", choices=["auto", "mfma", "streamed"],
                    help="modal fast runs: one launch of the 16-mode MFMA kernel per whole run where it "
                         "applies (mfma), the state streamed in time blocks (streamed), or the first from "
                         "8192 modes (auto: fewer modes leave the kernel's 16-mode workgroups too few)")
    ap.add_argument("--batch-kernel", default="auto",
                    choices=["auto", "default", "time_blocked", "mfma_tile", "per_step"],
                    help="c4: the batched kernel per class (auto: timed per class)")
    ap.add_argument("--no-adjoint", action="store_true",
                    help="c3: skip the adjoint rate (gradients/s on the 127^2, N = 4096 workload) added to the line")
    ap.add_argument("--no-prof", action="store_true",
                    help="skip the serial pass (kernel timings, the untimed variants)")
    ap.add_argument("--serial", action="store_true",
                    help="run the timed variants one after another (default: one stream each, concurrently; c3 always one stream)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, copy a MIB-sized device buffer 4 times (a plain copy kernel of "
                         "known size that scales the rocprofv3 FETCH_SIZE/WRITE_SIZE counters)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = {"c3": 2, "c4": 1}.get(args.workload, 5)
    if args.warmup is None:
        args.warmup = 1 if args.workload in ("c3", "c4") else 2
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: this solver has no multi-GPU path (the modal solver would "
              "shard by sine mode with no per-step exchange); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1901_05128_amd as cq

    if args.workload == "c4":
        return bench_batched(args)
    if args.workload == "c5":
        return bench_adjoint(args)
    w = WORKLOADS[args.workload]
    desc, dim, nx, ny, a1, a2, m, T, N, seed = w
    M = nx * ny
    if args.variants == "default":
        timed = TIMED.get(args.workload, VARIANTS)
    else:
        timed = [v for v in VARIANTS if VNAME[v] in args.variants.split(",")]
    # the serial pass runs every variant of the workload unless it is skipped
    variants = SERIAL.get(args.workload, VARIANTS) if not args.no_prof else timed
    variants = variants + [v for v in timed if v not in variants]
    serial = args.serial or args.workload in ONE_STREAM
    torch.cuda.set_device(0)
    g0 = g0_for(w)
    if args.workload == "t5" and args.t5_data == "b":
        from paper_1901_05128_amd import workloads as wl
        g0 = wl.g0_nonsmooth_b(nx)
        desc = desc.replace("data (a)", "data (b)")
    G0 = torch.tensor(g0, dtype=torch.float64, device="cuda")
    grid = cq.make_grid(dim, nx, ny)
    solvers, streams = {}, {}
    fast_k = 1 if args.fast_kernel == "mfma" or (args.fast_kernel == "auto" and M >= 8192) else 0
    for v in variants:
        # each timed variant on its own stream (default priority) unless serial
        streams[v] = torch.cuda.Stream() if (v in timed and not serial) else torch.cuda.current_stream()
        with torch.cuda.stream(streams[v]):
            solvers[v] = cq.Solver(grid, cq.make_params(a1, a2, m, T, N, v[0], v[1],
                                                        solver=SOLVERS[args.solver],
                                                        fast_kernel=fast_k), G0)
    torch.cuda.synchronize()
    outs = {v: torch.empty((2, M), dtype=torch.float64, device="cuda") for v in variants}

    # the nodal solver launches kernels every step: enqueued whole, one
    # variant's N steps would fill its queue and hold the host until they ran,
    # so the variants go round-robin in chunks of steps, which keeps every
    # stream fed (the modal solver enqueues a whole run in a few hundred
    # launches)
    chunk = 256 if args.solver == "nodal" and not serial else N

    def one_step(events=None):
        if chunk == N:
            for v in timed:
                s = solvers[v]
                with torch.cuda.stream(streams[v]):
                    if events is not None:
                        events[v][0].record()
                    s.reset(G0)
                    s.step(N)
                    s.current(outs[v])
                    if events is not None:
                        events[v][1].record()
            return
        for v in timed:
            with torch.cuda.stream(streams[v]):
                if events is not None:
                    events[v][0].record()
                solvers[v].reset(G0)
        for n0 in range(0, N, chunk):
            for v in timed:
                with torch.cuda.stream(streams[v]):
                    solvers[v].step(min(chunk, N - n0))
        for v in timed:
            with torch.cuda.stream(streams[v]):
                solvers[v].current(outs[v])
                if events is not None:
                    events[v][1].record()

    for k in range(args.warmup):
        one_step()
        torch.cuda.synchronize()
        print(f"# warmup step {k + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    ev = {v: [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)] for v in timed}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        one_step({v: ev[v][k] for v in timed})
        if args.workload == "c3":
            # a progress line per step (each takes seconds); the wait only
            # follows work already queued, so the timed work is unchanged
            ev[timed[-1]][k][1].synchronize()
            print(f"# timed step {k + 1}/{args.steps}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_var_ms = {v: sum(a.elapsed_time(b) for a, b in ev[v]) / args.steps for v in timed}
    elapsed = t1 - t0
    dofsteps = args.steps * len(timed) * 2 * M * N
    value = dofsteps / elapsed

    # Serial pass outside the timed region: every variant once, one after
    # another on one stream, with HIP events around every kernel launch, so
    # that each launch's duration is its own and not stretched by kernels of
    # other variants sharing the GPU.
    kinds = ["hist_fast", "hist_direct", "far_toeplitz", "solve_1d", "prep_2d", "dst_gemm", "modal_fast",
             "modal_near", "reduce_far"]
    ktime = {}
    serial_ms = {}
    if not args.no_prof:
        torch.cuda.synchronize()
        cq.prof_enable(True)
        for v in variants:
            s = solvers[v]
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            with torch.cuda.stream(streams[v]):
                e0.record()
                s.reset(G0)
                s.step(N)
                s.current(outs[v])
                e1.record()
            torch.cuda.synchronize()
            serial_ms[v] = e0.elapsed_time(e1)
            print(f"# serial pass {VNAME[v]} {serial_ms[v]:.1f} ms", file=sys.stderr, flush=True)
        for kname in kinds:
            n_l, ms = cq.prof_read(kname)
            if n_l:
                ktime[kname] = (n_l, ms)
        cq.prof_enable(False)
    roofline = None
    if ktime:
        dom = max(ktime, key=lambda k: ktime[k][1])
        n_l, ms = ktime[dom]
        tot_b, tot_f = 0, 0
        for v in variants:
            info = solvers[v].info()
            b, f = kernel_work(dom, w, v[0], v[1], info, M, SOLVERS[args.solver])
            tot_b += b
            tot_f += f
        avg_s = ms / 1e3 / n_l
        f_frac = (tot_f / n_l / avg_s / 1e12) / FP64_PEAK_TFLOPS if tot_f else 0.0
        b_frac = (tot_b / n_l / avg_s / 1e9) / HBM_PEAK_GBS if tot_b else 0.0
        if f_frac >= b_frac:
            ach = tot_f / n_l / avg_s / 1e12
            roofline = {"bound": "mfma" if dom in ("far_toeplitz", "dst_gemm") else "alu", "achieved": ach,
                        "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": ach / FP64_PEAK_TFLOPS,
                        "hbm_frac": b_frac}
        else:
            ach = tot_b / n_l / avg_s / 1e9
            roofline = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": ach / HBM_PEAK_GBS, "fp64_frac": f_frac}
        roofline["kernel"] = dom
        roofline["avg_launch_us"] = avg_s * 1e6
        roofline["launches"] = n_l
        roofline["algorithmic_per_launch"] = (tot_f if f_frac >= b_frac else tot_b) / n_l
        roofline["timed"] = ("serial pass after the timed region (variants " +
                             ", ".join(VNAME[v] for v in variants) + "), HIP events per launch")
        roofline["traffic"] = load_traffic(dom, args.workload)

    # fast vs direct on the GPU (the metric's accuracy side)
    fvd = {}
    for scheme in (1, 2):
        if (scheme, 1) in outs and (scheme, 0) in outs:
            f, d = outs[(scheme, 1)], outs[(scheme, 0)]
            fvd[f"scheme{scheme}"] = float(torch.linalg.norm(f - d) / torch.linalg.norm(d))

    info_np = {VNAME[v]: solvers[v].info().np_total for v in variants if v[1] == 1}
    fast_kern = {VNAME[v]: ("16-mode MFMA kernel, one launch" if solvers[v].info().whole_run_kernel else "streamed state")
                 for v in variants if v[1] == 1}
    breakdown = {VNAME[v]: {"ms": per_var_ms[v], "dofsteps_per_s": 2 * M * N / (per_var_ms[v] / 1e3),
                            "where": "timed step (one stream)" if serial else "timed step (concurrent)"}
                 for v in timed}
    for v, ms in serial_ms.items():
        ent = breakdown.setdefault(VNAME[v], {})
        ent["serial_ms"] = ms
        ent["serial_dofsteps_per_s"] = 2 * M * N / (ms / 1e3)
    for s in solvers.values():
        s.close()

    rec = {
        "metric": "DOF*steps/s (fast and direct CQ solves)",
        "value": value,
        "unit": "DOF*steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": (("synthetic (the paper's nonsmooth initial data (b))" if args.t5_data == "b" else
                  "synthetic (the paper's smooth initial data (a))") if seed is None
                 else "synthetic (seeded indicator initial data)"),
        "config": {"workload": f"{args.workload}: {desc}, alpha=({a1},{a2}), m={m}, T={T}",
                   "solver": args.solver, "streams": "serial" if serial else "one per variant",
                   "timed_variants": [VNAME[v] for v in timed], "dof": 2 * M, "N": N,
                   "fast_nodes": info_np, "fast_kernel": fast_kern},
        "breakdown": breakdown,
        "fast_vs_direct_rel_l2": fvd,
        "kernels_ms": {k: {"launches": v[0], "total_ms": v[1]} for k, v in ktime.items()},
        "roofline": roofline,
    }
    if args.workload == "t5":
        # vs_baseline: the paper's Table 5 CPU times for the same workload and
        # step (BDF2 direct + fast at (0.3, 0.8)) as DOF*steps/s
        paper_rate = 2 * 2 * M * N / (T5_PAPER["direct_s"][0] + T5_PAPER["fast_s"][0])
        rec["vs_baseline"] = value / paper_rate
        rec["baseline"] = {"value": paper_rate, "unit": "DOF*steps/s",
                           "source": "Table 5 CPU times 870.13 s (SBD) + 209.44 s (FSBD) at (0.3, 0.8), "
                                     "2 x 1023 DOF x 20000 steps each; the paper names no machine"}
        if args.t5_errors:
            # the paper's protocol: E_k = ||G_k^N(tau) - G_k^N(tau/2)||_L2, h = 1/1024
            ref = cq.fp_solve(grid, cq.make_params(a1, a2, m, T, 2 * N, 2, 0, solver=SOLVERS[args.solver]), G0)
            h = 1.0 / (nx + 1)
            errs = {}
            for v in timed:
                dlt = (outs[v] - ref).cpu()
                errs[VNAME[v]] = [float((h * (dlt[k] ** 2).sum()) ** 0.5) for k in range(2)]
            rec["t5_errors"] = {"ours": errs, "paper": {"bdf2_direct": T5_PAPER["direct_E"][0],
                                                          "bdf2_fast": T5_PAPER["fast_E"][0]},
                                "note": "reference run at tau/2 (the paper used tau = 1/4000 too); "
                                        "the paper's spatial scheme is unstated"}
    if args.copy_probe:
        rec["copy_probe_bytes_each_way"] = copy_probe(args.copy_probe)
    if args.workload == "c3" and not args.no_adjoint:
        # the metric's second half, the adjoint rate, on its own workload (the
        # 127^2 grid, N = 4096), measured after the timed region above (the
        # solvers above are closed by now)
        torch.cuda.empty_cache()
        adj = bench_adjoint(argparse.Namespace(steps=10, warmup=2, no_prof=args.no_prof), emit=False)
        rec["adjoint"] = {k: adj[k] for k in ("metric", "value", "unit", "steps", "warmup", "ms_per_step", "config",
                                              "roofline")}
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w, timed)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
