#!/usr/bin/env python3
"""Benchmark of blocked randomized QRCP on one MI355X.

One step = one full factorization A P = Q R (every block: sketch, pivoted QR
of the sketch, column moves, panel QR, T factor, trailing update) of the
headline workload: m = n = 8192, FP64, b = 256, p = 10, permutation pivoting,
A = U diag(s) V^T with Haar U, V and s_j = 10^(-6 (j-1)/8191) (synthetic,
seeded).  The input is resident in HBM before the timed region; each step
restores A from a resident copy (a device-to-device copy outside the timed
events) and factors it.

Prints ONE JSON line (rank 0).  value = normalised GFLOP/s, i.e.
(2 m n^2 - 2 n^3/3) / time, the Householder-QR flop count (4/3 n^3 for a
square matrix), which is the metric's normalisation.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GFLOP/s (4/3·n³-normalised) randQRCP n=8192 FP64 vs mixed; bwd/fwd ratio"
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 (matrix and vector)
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="H1")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision run (profiling)")
    ap.add_argument("--no-residual", action="store_true", help="skip the residual check (profiling)")
    ap.add_argument("--cpu-blocks", type=int, default=0,
                    help="oracle: leading blocks factored on the CPU (0: the whole factorization)")
    ap.add_argument("--no-bwd", action="store_true", help="skip the bwd/fwd ratio measurement (C5)")
    ap.add_argument("--no-c4", action="store_true", help="skip the C4 (16384 x 8192) mixed vs FP64 timing")
    ap.add_argument("--no-c3", action="store_true", help="skip the C3 (8192^2 orthonormal pivoting) timing")
    ap.add_argument("--power", type=int, default=1,
                    help="also time the workload with this many power-iteration steps (Section 6.3); 0 skips")
    ap.add_argument("--no-panel-pivot", action="store_true",
                    help="skip timing the workload with Fig. 3's in-block pivot P-hat")
    ap.add_argument("--calibrate", action="store_true",
                    help="also run one plain copy-like kernel (torch.neg) over 2^26 doubles, to scale HBM counters")
    return ap.parse_args()


GEMM_SOURCES = ("paper_1505_08115_amd/csrc/gemm.hip",)   # the file that defines the GEMM kernels
PMC_SUMMARY = "profiles/trailing_update_H1_pmc.txt"
# the trailing update of a block (Section 5.1): T^T W, W = V^T C, C -= V (T^T W)
UPDATE_CLASSES = ("vt_gemm", "w_gemm", "update_gemm")


def gemm_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in GEMM_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload):
    """HBM bytes per block's trailing update from the committed counter summary,
    or None when there is none for this workload or the GEMM sources have
    changed since the counters were taken."""
    path = os.path.join(ROOT, PMC_SUMMARY)
    if workload != "H1" or not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("gemm_source_sha256") != gemm_source_hash():
        return None
    try:
        return float(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(A_host, w, nblocks):
    """The oracle, as it stands, on the same factorization (nblocks = 0), or
    on its first `nblocks` blocks (rank = nblocks * b) when a shorter run is
    wanted; at H1 the whole factorization takes about half a minute on 16
    host cores."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import workloads as W
    from oracle import rqrcp as O
    full = nblocks <= 0 or nblocks * w.b >= w.n
    k = w.n if full else nblocks * w.b
    t0 = time.perf_counter()
    O.rqrcp(A_host, w.b, w.p, seed=w.seed, rank=0 if full else k)
    dt = time.perf_counter() - t0
    flops = W.flops_normalised(w.m, w.n) if full else W.flops_normalised_prefix(w.m, w.n, k)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    what = (f"the whole {w.name} factorization (the same input, sketches and block size)" if full else
            f"first {nblocks} blocks (rank {k}) of the {w.name} factorization, normalised by the Householder-QR "
            f"flops of those {k} columns")
    # classical column-pivoted QR (LAPACK dgeqp3 through scipy, threaded BLAS)
    # as context on the host, at C2's 4096^2 size (it is BLAS-2 bound and
    # would take minutes at 8192^2); not a parity reference for the
    # randomized pivots
    import scipy.linalg
    Ac = np.array(W.workload_matrix(W.WORKLOADS["C2"]).numpy(), order="F")
    t1 = time.perf_counter()
    scipy.linalg.qr(Ac, pivoting=True, mode="r", overwrite_a=True, check_finite=False)
    dq = time.perf_counter() - t1
    geqp3 = {"workload": f"classical QRCP (LAPACK dgeqp3 via scipy) of C2's {Ac.shape[0]}x{Ac.shape[1]} FP64 "
                         f"matrix on the host", "seconds": dq,
             "value": W.flops_normalised(*Ac.shape) / dq / 1e9, "unit": "GFLOP/s"}
    return {"value": flops / dt / 1e9, "unit": "GFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"{what}, {dt:.1f} s wall", "seconds": dt, "context_classical_qrcp": geqp3}


def bwd_fwd_ratio(reps=5, dtype=None):
    """bwd/fwd of the truncated factorization on C5 (4096^2 FP64, b = 128,
    p = 10, k = 256): fwd = factor(rank = k) + lowrank; bwd = lowrank_backward
    with the forward's factors kept, or with recompute (a fixed-pivot
    refactorization, no sketch, then lowrank_backward).  Medians of `reps`
    HIP-event timings; the Python wrappers allocate their outputs and
    workspaces through torch's caching allocator inside the timed calls."""
    import numpy as np
    import torch

    import paper_1505_08115_amd as R
    import workloads as W
    w = W.WORKLOADS["C5"]
    dev = torch.device("cuda:0")
    dtype = dtype or torch.float64
    A = R.colmajor(W.workload_matrix(w, device=dev).to(dtype))
    k = w.rank
    g = torch.Generator(device="cpu").manual_seed(55)
    Gbar = R.colmajor(torch.randn(w.m, w.n, generator=g, dtype=torch.float64).to(dev).to(dtype))

    def timed(fn):
        out = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            out.append(e0.elapsed_time(e1))
        return float(np.median(out[1:]))          # the first call warms up

    state = {}

    def fwd():
        state["Fz"] = R.factor(A, block=w.b, oversample=w.p, seed=w.seed, rank=k)
        state["Ak"] = R.lowrank(state["Fz"], k)

    def bwd():
        state["dA"] = R.lowrank_backward(A, state["Fz"], Gbar, k)

    def bwd_recompute():
        Fz2 = R.factor(A, block=w.b, oversample=0, rank=k, jpvt=state["Fz"].jpvt)
        state["dA2"] = R.lowrank_backward(A, Fz2, Gbar, k)

    tf = timed(fwd)
    tb = timed(bwd)
    tr = timed(bwd_recompute)
    agree = float(torch.linalg.norm(state["dA2"] - state["dA"]) / torch.linalg.norm(state["dA"]))
    name = "FP64" if dtype == torch.float64 else ("FP32 storage (FP32 factorization; truncation and backward on FP32 matrix "
                                                 "cores, their small factors Q_k, R_k, R_11^-1 in FP64)")
    return {"workload": f"C5: {w.m}x{w.n} {name}, b={w.b}, p={w.p}, k={k}", "fwd_ms": tf, "bwd_ms": tb,
            "bwd_recompute_ms": tr, "ratio": tb / tf, "ratio_recompute": tr / tf,
            "recompute_vs_kept_rel_diff": agree, "dtype": "f64" if dtype == torch.float64 else "f32"}


def methods_123(reps=3):
    """Section 7's three methods on the 1024^2 matrix with a spectral gap
    (C3's subcase): Method 1 (permutation, p = 10), Method 2 (orthonormal
    pivoting, p = b/2) and blockRRQR (Method 3: orthonormal pivoting, q = 2
    power steps, diagonalised blocks, p = b/2), b = 64; and Method 3 at the
    configured block size b = 256 (the cooperative Jacobi SVD of each
    256 x 256 triangle).  Median HIP-event times and how closely |R_kk|
    follows sigma_k (median |log|)."""
    import numpy as np
    import torch

    import paper_1505_08115_amd as R
    import workloads as W
    w = W.WORKLOADS["C3s"]
    dev = torch.device("cuda:0")
    A = R.colmajor(W.workload_matrix(w, device=dev))
    s = np.asarray(w.sigma(), dtype=np.float64)
    b = 64
    out = {"workload": f"C3s: {w.m}x{w.n} FP64, sigma with a 1e-6 gap after 256, b={b} (method3_b256: b=256)"}
    for name, kw in (("method1", dict(block=b, pivot="perm", oversample=10)),
                     ("method2", dict(block=b, pivot="ortho", oversample=b // 2)),
                     ("method3", dict(block=b, pivot="ortho", oversample=b // 2, power=2, diagonalize=True)),
                     ("method3_b256", dict(block=256, pivot="ortho", oversample=w.p, power=2, diagonalize=True))):
        ts = []
        for _ in range(reps + 1):
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            Fz = R.factor(A, seed=w.seed, **kw)
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        d = np.abs(np.diag(Fz.F.cpu().numpy()))
        out[name] = {"ms": float(np.median(ts[1:])),
                     "median_abs_log_rkk_over_sigma": float(np.median(np.abs(np.log(d / s))))}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; multi-GPU execution is not implemented, "
                                   "run with --gpus 1"}))
        sys.exit(2)
    import numpy as np
    import torch

    import paper_1505_08115_amd as R
    import workloads as W

    w = W.WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    A = W.workload_matrix(w, device=dev)
    m, n = A.shape

    def run(wl, Ain, steps, warmup, profile, check=True, power=0, panel_pivot=False, fixed=None):
        """Time `steps` factorizations of Ain (already resident) with HIP events.

        Inside the timed steps only the launches of the trailing update (T^T W,
        W = V^T C, the update) are bracketed by the library's events (the
        roofline is measured live); with `profile`, `steps` further
        factorizations bracket every kernel class for the breakdown, outside
        the timed region.  fixed: a jpvt to refactor with (fixed pivots, no
        sketch; the blocks run one after the other)."""
        dtype = torch.float32 if wl.precision == "mixed" else torch.float64
        m, n = Ain.shape
        A0 = R.colmajor(Ain.to(dtype))
        F = torch.empty_like(A0)
        sizes = R.factor_sizes(m, n, dtype, block=wl.b, oversample=wl.p, pivot=wl.pivot, rank=wl.rank,
                               precision="mixed" if wl.precision == "mixed" else "plain", power=power,
                               panel_pivot=panel_pivot, fixed_pivots=fixed is not None)
        jp = torch.empty(n, dtype=torch.int32, device=dev) if fixed is None else fixed.clone()
        tau = torch.empty(max(1, sizes[0]), dtype=torch.float64, device=dev)
        T = torch.empty(max(1, sizes[1]), dtype=torch.float64, device=dev)
        S = torch.empty(sizes[2], dtype=torch.float64, device=dev) if wl.pivot == "ortho" else None
        work = torch.empty(sizes[3], dtype=torch.uint8, device=dev)
        info = torch.zeros(4, dtype=torch.int32, device=dev)
        kw = dict(block=wl.b, oversample=wl.p, seed=wl.seed, pivot=wl.pivot, rank=wl.rank, info=info,
                  precision="mixed" if wl.precision == "mixed" else "plain", power=power, panel_pivot=panel_pivot,
                  fixed_pivots=fixed is not None)
        for _ in range(warmup):
            F.copy_(A0)
            R.factor_into(F, jp, tau, T, S, work, **kw)
        torch.cuda.synchronize()
        if profile:
            R.timing_classes(list(UPDATE_CLASSES))
            R.timing_enable(True)
            R.timing_read()
        times = []
        for _ in range(steps):
            F.copy_(A0)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            R.factor_into(F, jp, tau, T, S, work, **kw)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        prof = R.timing_read() if profile else {}
        every = {}
        if profile:
            R.timing_classes(None)
            for _ in range(steps):
                F.copy_(A0)
                R.factor_into(F, jp, tau, T, S, work, **kw)
            torch.cuda.synchronize()
            every = R.timing_read()
        R.timing_enable(False)
        prof = (prof, every)
        run.last_jpvt = jp.clone()
        if not check:
            return times, prof, None, info.tolist()
        # correctness of the timed factorization, against the matrix it saw;
        # Q rebuilt independently by torch (LAPACK orgqr semantics)
        Ad = A0.double()
        Fd = F.double()
        Q = torch.linalg.householder_product(Fd.contiguous(), tau.contiguous())
        res = float(torch.linalg.norm(Ad[:, jp.long()] - Q @ torch.triu(Fd[:n])) / torch.linalg.norm(Ad)) \
            if wl.pivot == "perm" else None
        del Q, Fd, Ad, work
        return times, prof, res, info.tolist()

    times, (prof, prof_all), res, info = run(w, A, args.steps, args.warmup, True, check=not args.no_residual)
    jp_main = run.last_jpvt
    ms = float(np.mean(times))
    flops = W.flops_normalised(m, n)
    value = flops / (ms * 1e-3) / 1e9

    # the mixed-precision form of the same factorization (BF16 sketch, FP32
    # update, FP64 panel/T/pivoted QR of the sketch), on the FP32-rounded input
    mixed = None
    mname = {"H1": "H2"}.get(w.name)
    if mname and not args.no_mixed:
        wm = W.WORKLOADS[mname]
        mt, (_, mprof), mres, minfo = run(wm, A, args.steps, args.warmup, True, check=not args.no_residual)
        mms = float(np.mean(mt))
        mixed = {"workload": f"{wm.name}: FP32 storage, BF16 sketch, FP32 update, b={wm.b}, p={wm.p}",
                 "value": flops / (mms * 1e-3) / 1e9, "ms_per_step": mms, "residual": mres, "info": minfo,
                 "speedup_vs_fp64": ms / mms,
                 "breakdown": {k: v[1] / args.steps for k, v in mprof.items()}}

    # C4: the tall mixed-precision workload (16384 x 8192, FP32 storage, BF16
    # sketch, b = 256, p = 16) beside the plain FP64 factorization of the same
    # matrix with the same block sizes
    c4 = None
    if w.name == "H1" and not args.no_c4:
        w4 = W.WORKLOADS["C4"]
        A4 = W.workload_matrix(w4, device=dev)
        f4 = W.flops_normalised(w4.m, w4.n)
        t4m, (_, p4m), r4m, i4m = run(w4, A4, args.steps, args.warmup, True, check=not args.no_residual)
        w4p = W.Workload("C4 plain", w4.m, w4.n, w4.b, w4.p, "perm", "f64", w4.profile, w4.seed)
        t4p, (_, p4p), r4p, i4p = run(w4p, A4, args.steps, args.warmup, True, check=not args.no_residual)
        del A4
        m4, p4 = float(np.mean(t4m)), float(np.mean(t4p))
        c4 = {"workload": f"C4: {w4.m}x{w4.n}, b={w4.b}, p={w4.p}; mixed (FP32 storage, BF16 sketch, FP32 update) "
                          f"and plain FP64 on the same matrix",
              "mixed": {"ms_per_step": m4, "value": f4 / (m4 * 1e-3) / 1e9, "residual": r4m, "info": i4m,
                        "breakdown": {k: v[1] / args.steps for k, v in p4m.items()}},
              "fp64": {"ms_per_step": p4, "value": f4 / (p4 * 1e-3) / 1e9, "residual": r4p, "info": i4p,
                       "breakdown": {k: v[1] / args.steps for k, v in p4p.items()}},
              "speedup_mixed_vs_fp64": p4 / m4}

    # C3: the orthonormal-pivoting form (Section 4.2, eq. Ycols) at 8192^2,
    # b = 256, p = 10 (its parity and invariants are a GPU test of their own)
    c3 = None
    if w.name == "H1" and not args.no_c3:
        w3 = W.WORKLOADS["C3"]
        A3 = W.workload_matrix(w3, device=dev)
        t3, (_, p3), _, i3 = run(w3, A3, min(args.steps, 3), 1, True, check=False)
        del A3
        m3 = float(np.mean(t3))
        c3 = {"workload": f"C3: {w3.m}x{w3.n} FP64, orthonormal pivoting, b={w3.b}, p={w3.p}, sigma 1/j with a "
                          f"1e-6 gap after 2048",
              "ms_per_step": m3, "value": W.flops_normalised(w3.m, w3.n) / (m3 * 1e-3) / 1e9, "info": i3,
              "slowdown_vs_permutation": m3 / ms,
              "breakdown": {k: v[1] / min(args.steps, 3) for k, v in p3.items()}}

    # the same factorization with q steps of the power iteration on every
    # sketch (Section 6.3): two more products per block, serial schedule
    power = None
    if args.power > 0 and w.precision != "mixed":
        pt, (_, pprof), pres, pinfo = run(w, A, args.steps, args.warmup, True, check=not args.no_residual,
                                          power=args.power)
        pms = float(np.mean(pt))
        power = {"workload": f"{w.name} with q={args.power} power-iteration steps per sketch",
                 "ms_per_step": pms, "value": flops / (pms * 1e-3) / 1e9, "slowdown_vs_q0": pms / ms,
                 "residual": pres, "info": pinfo,
                 "breakdown": {k: v[1] / args.steps for k, v in pprof.items()}}

    # the same factorization with Fig. 3's in-block pivot P-hat (a QRCP of
    # every panel's R', the panel restored, permuted and factored again)
    phat = None
    if not args.no_panel_pivot and w.precision != "mixed" and w.pivot == "perm":
        ht, (_, hprof), hres, hinfo = run(w, A, args.steps, args.warmup, True, check=not args.no_residual,
                                          panel_pivot=True)
        hms = float(np.mean(ht))
        phat = {"workload": f"{w.name} with the in-block pivot P-hat", "ms_per_step": hms,
                "value": flops / (hms * 1e-3) / 1e9, "slowdown_vs_identity": hms / ms, "residual": hres,
                "info": hinfo, "breakdown": {k: v[1] / args.steps for k, v in hprof.items()}}

    # roofline of the trailing update, the matrix-core work of every block
    # (Section 5.1): T^T W, W = V^T C and C -= V (T^T W), measured live inside
    # the timed steps with HIP events on the streams they run on (the update
    # itself on the auxiliary stream, capped at half the CUs, beside the next
    # block's pivoted QR); one "launch" = one block's three products
    nb_upd = prof.get("w_gemm", (0,))[0]
    tfl = sum(prof.get(c, (0, 0.0, 0.0, 0.0))[2] for c in UPDATE_CLASSES)
    tms = sum(prof.get(c, (0, 0.0, 0.0, 0.0))[1] for c in UPDATE_CLASSES)
    tby = sum(prof.get(c, (0, 0.0, 0.0, 0.0))[3] for c in UPDATE_CLASSES)
    achieved = tfl / (tms * 1e-3) / 1e12 if tms > 0 else 0.0
    parts = {}
    for c in UPDATE_CLASSES:
        n_, ms_, fl_, _ = prof.get(c, (0, 0.0, 0.0, 0.0))
        parts[c] = {"avg_launch_ms": ms_ / max(1, n_), "tflops": fl_ / (ms_ * 1e-3) / 1e12 if ms_ > 0 else 0.0,
                    "launches_per_step": n_ / max(1, args.steps)}
    roof = {"kernel": "trailing update per block: T^T W + W = V^T C + C -= V (T^T W) (FP64 MFMA; the last "
                      "on the auxiliary stream at half the CUs)", "bound": "mfma",
            "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
            "traffic": measured_traffic(w.name), "launches_per_step": nb_upd / max(1, args.steps),
            "avg_launch_ms": tms / max(1, nb_upd), "flops_per_launch": tfl / max(1, nb_upd),
            "algorithmic_bytes_per_launch": tby / max(1, nb_upd), "parts": parts}
    # the dominant kernel of the factorization: the pivoted QR of the sketch,
    # one grid-wide exchange per pivot decision (latency-bound)
    qn, qms, qfl, _ = prof_all.get("qrcp", (0, 0.0, 0.0, 0.0))
    qsteps_all = sum(min(w.b, n - i * w.b) for i in range(-(-n // w.b))) if w.rank == 0 else w.rank
    dominant = {"kernel": "qrcp_reg_kernel (pivoted QR of the sketch, Section 4.1 eq. Yrows)", "bound": "latency",
                "achieved": qfl / (qms * 1e-3) / 1e12 if qms > 0 else 0.0, "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": (qfl / (qms * 1e-3) / 1e12) / PEAK_FP64_TFLOPS if qms > 0 else 0.0,
                "ms_per_step": qms / args.steps, "share_of_step": qms / args.steps / ms,
                "us_per_pivot_step": qms / args.steps / qsteps_all * 1e3}
    # the trailing update alone on the whole chip: a fixed-pivot
    # refactorization runs the blocks one after the other, the update uncapped
    uncapped = None
    if w.pivot == "perm" and w.precision != "mixed":
        _, (uprof, _), _, _ = run(w, A, args.steps, 1, True, check=False, fixed=jp_main)
        un, ums, ufl, _ = uprof.get("update_gemm", (0, 0.0, 0.0, 0.0))
        uncapped = {"kernel": "C -= V (T^T W) uncapped on the whole chip (fixed-pivot refactorization, "
                              "blocks one after the other)",
                    "avg_launch_ms": ums / max(1, un), "achieved_tflops": ufl / (ums * 1e-3) / 1e12 if ums else 0.0,
                    "frac": (ufl / (ums * 1e-3) / 1e12) / PEAK_FP64_TFLOPS if ums else 0.0}
    # the latency-bound cooperative kernels: one grid-wide exchange per pivot
    # decision (pivoted QR of the sketch) and per panel column
    qsteps = sum(min(w.b, n - i * w.b) for i in range(-(-n // w.b))) if w.rank == 0 else w.rank
    latency = {"qrcp_us_per_pivot_step": prof_all.get("qrcp", (0, 0.0))[1] / args.steps / qsteps * 1e3,
               "panel_us_per_column": prof_all.get("panel", (0, 0.0))[1] / args.steps / qsteps * 1e3,
               "pivot_steps_per_factorization": qsteps}
    breakdown = {k: {"ms_per_step": v[1] / args.steps, "launches_per_step": v[0] / args.steps,
                     "tflops": (v[2] / (v[1] * 1e-3) / 1e12) if v[1] > 0 and v[2] > 0 else None,
                     "gbs": (v[3] / (v[1] * 1e-3) / 1e9) if v[1] > 0 and v[3] > 0 else None}
                 for k, v in prof_all.items()}

    out = {
        "metric": METRIC, "value": value, "unit": "GFLOP/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{w.name}: randomized blocked QRCP, m={m} n={n}, {w.precision}, b={w.b}, "
                               f"p={w.p}, {w.pivot} pivoting, A = U diag(s) V^T, Haar U,V, seed {w.seed}",
                   "m": m, "n": n, "block": w.b, "oversample": w.p, "pivot": w.pivot},
        "roofline": roof,
        "roofline_dominant": dominant,
        "extra": {"residual": res, "info": info, "step_ms": times, "breakdown": breakdown, "latency": latency,
                  "update_uncapped": uncapped,
                  "mixed": mixed, "c4": c4, "c3": c3, "power_iteration": power, "panel_pivot": phat},
    }
    if not args.no_bwd:
        out["extra"]["methods_123"] = methods_123()
        out["extra"]["bwd_fwd"] = bwd_fwd_ratio()
        out["extra"]["bwd_fwd_fp32"] = bwd_fwd_ratio(dtype=torch.float32)
    if args.calibrate:
        # 512 MiB read + 512 MiB written by one elementwise kernel
        x = torch.rand(1 << 26, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.neg(x, out=y)
        torch.cuda.synchronize()
        out["extra"]["calibration"] = {"kernel": "torch.neg", "read_bytes": 1 << 29, "write_bytes": 1 << 29}
        del x, y
    if not args.no_cpu_baseline and w.n <= 8192:
        A_host = A.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(A_host, w, args.cpu_blocks)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
