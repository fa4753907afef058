#!/usr/bin/env python3
"""Benchmark: LU with partial pivoting, FP64, n = 32768, on one MI355X.

One step = one blocked right-looking factorization P*A = L*U of the whole
n x n matrix (column-block factorization, interchanges, triangular solve and
trailing update for every block of columns) through the C ABI.  The input is
the seeded synthetic matrix A with iid U(-1,1) entries (the paper evaluates on
randomly generated dense matrices); it is resident in HBM before timing, and
each step first restores it with a device-to-device copy (inside the step, so
the reported rate is slightly pessimistic).

The JSON line carries:
  value       2/3 n^3 / (mean step time), TFLOP/s
  roofline    the trailing-update GEMM (128x128-tile kernel): its algorithmic
              flops 2*M*N*K summed over its launches in the timed steps,
              divided by the summed launch durations from HIP events recorded
              on the library's stream, against MI355X's FP64 MFMA peak; traffic
              = the HBM/algorithmic byte ratio from the committed counter summary
              (measured at n = 24576, labelled) times this run's algorithmic
              bytes per launch
  cpu_baseline  the CPU oracle (unblocked FP64 LUPP) on the host cores: n = 512
              (median of 3) and n = 4096, each with 1 thread and with all cores,
              the input copy outside the timer; value = all cores at n = 4096.
              The same leg solves the kappa systems of the kappa leg (n = 4096)
              with the oracle: their FP64 reference solutions
  check       info and a random-probe residual of the last step, and the
              closed-form pivots of A = Pi*D (D column diagonally dominant) at
              the same n, compared bit for bit
  c2          FP64 and FP32 factorizations at n = 4096, 8192, 16384 (and FP32 at
              32768): median of 3, TFLOP/s against the FP64 / FP32 peaks, probe
              residual, Pi*D closed-form pivots at every n
  mixed       the mixed-precision solve (lupp_dgesv_mixed) at n = 32768 and
              16384: FP32 factorization with BF16 / FP16 / FP8 trailing
              updates, then FP64 classical or GMRES refinement to backward
              error <= 1e-14, on the diagonally dominant matrix (U(-0.5,0.5),
              then a_ii := sum_j |a_ij|), b iid U(-1,1); effective rate 2/3 n^3
              over the wall time; forward errors against the GPU FP64 solve and
              (second, untimed call with b = A x_true) against x_true
  kappa       n = 4096, A = U diag(sigma) V^T with geometric sigma from 1 to
              1/kappa, kappa in {1e2, 1e4, 1e6}, b = A x_true: iterations, eta and
              forward errors (vs the CPU oracle's FP64 solve, the GPU FP64 solve
              and x_true) per (precision, kappa, refinement)
  batched     20000 independent systems, n_i iid uniform on [8, 128], A_i and
              b_i iid U(-1,1), packed column-major (lupp_xgesv_batched: LU with
              partial pivoting and solve): factorizations per second from the
              median of 20 replays of a captured HIP graph (inputs restored
              between replays, outside the timed interval), against the HBM
              roofline of the call's algorithmic bytes (A and b read, the factors and x
              written, pivots written, sizes and offsets read); the size-class
              schedule is the one the library's autotuner chooses live on this
              GPU (recorded, with the initial schedule's time for comparison)
  dataflow    the headline factorization by the dataflow (algorithm-by-blocks)
              runtime at lookahead depth 2 and 4: time, pivots against the
              headline run's
  qr          Householder QR (lupp_dgeqrf, compact WY) at n = 4096, 8192,
              16384: TFLOP/s on 4/3 n^3, column-block and update time, probe
              residual of Q R x against A x
  randutv     randUTV (lupp_drandutv, block 64) at n = 2048, 4096, 8192 and
              q = 0, 1, 2 (and q = 1 with U and V formed): times; at n = 2048
              the identity A = U T V^T, orthogonality and diag(T) against the
              singular values; the vendor SVD's time at n = 2048 as labelled
              context (the paper's comparison point)
  large       n = 65536 (diagonally dominant recipe drawn on the device): plain FP64
              factorization + solve against the FP8-update GMRES-IR solve (wall
              times, effective TFLOP/s, backward errors, forward error against
              the FP64 solve, a long-double host check of 64 sampled rows)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6
FP32_PEAK_TFLOPS = 157.3
TRAFFIC_RATIO_FP64_GEMM = 1.808  # HBM bytes / algorithmic bytes, k_dgemm_sub_16 role 0, n = 24576 counters


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def probe_residual(torch, A0, LU, ipiv, nprobe=8, seed=5):
    """||P A X - L (U X)||_1 / (n u ||A||_1 ||X||_1) with an FP64 random probe
    X (n x nprobe); products formed with torch.matmul (rocBLAS), independent
    of the library."""
    n = A0.shape[0]
    g = torch.Generator(device="cuda").manual_seed(seed)
    X = torch.rand((n, nprobe), generator=g, dtype=torch.float64, device="cuda") * 2 - 1
    perm = torch.arange(n, device="cuda")
    piv = (ipiv.long() - 1).cpu().numpy()
    p = np.arange(n)
    for k, v in enumerate(piv):
        if v != k:
            p[k], p[v] = p[v], p[k]
    perm = torch.from_numpy(p).cuda()
    PAX = A0[perm, :] @ X
    U = torch.triu(LU)
    UX = U @ X
    del U
    L = torch.tril(LU, -1)
    L.diagonal().fill_(1.0)
    LUX = L @ UX
    del L
    r = (PAX - LUX).abs().sum(0).max().item()
    na = A0.abs().sum(0).max().item()
    nx = X.abs().sum(0).max().item()
    return r / (n * 2.0 ** -53 * na * nx)


def closed_form_ipiv(perm) -> np.ndarray:
    """Pivots of A = Pi*D with D's pivot order the identity: row perm[d] of A
    holds row d of D; partial pivoting picks D's row k at step k, wherever the
    earlier interchanges have moved it."""
    perm = np.asarray(perm)
    m = len(perm)
    where = np.array(perm, copy=True)      # current row of D-row d
    content = np.empty(m, dtype=np.int64)  # D-row at current row r
    content[perm] = np.arange(m)
    ipiv = np.empty(m, dtype=np.int32)
    for k in range(m):
        r = int(where[k])
        ipiv[k] = r + 1
        if r != k:
            dk = int(content[k])
            content[k], content[r] = k, dk
            where[k], where[dk] = k, r
    return ipiv


def host_backward_error(A, x, b) -> float:
    r = b - A @ x
    den = np.abs(A).sum(axis=1).max() * np.abs(x).max() + np.abs(b).max()
    return float(np.abs(r).max() / den) if den > 0 else 0.0


def rel_err(x, ref) -> float:
    """||x - ref||_inf / ||ref||_inf (device or host vectors)."""
    d = (x - ref).abs().max() if hasattr(x, "abs") else np.abs(x - ref).max()
    r = ref.abs().max() if hasattr(ref, "abs") else np.abs(ref).max()
    return float(d / r)


def pi_d_matrix(torch, n, seed, tdt):
    """A = Pi*D on the device, D strictly column diagonally dominant by an
    absolute margin of 1 (off-diagonal iid U(-1,1) from torch's seeded
    generator, d_jj = 1 + sum_{i != j} |d_ij|), row i of D placed at row perm[i]
    of A.  Returns (A column-major, perm)."""
    g = torch.Generator(device="cuda").manual_seed(seed)
    D = torch.empty((n, n), dtype=tdt, device="cuda").t()
    D.uniform_(-1.0, 1.0, generator=g)
    D.diagonal().zero_()
    colsum = D.abs().sum(dim=0, dtype=torch.float64)
    D.diagonal().copy_((1.0 + colsum).to(tdt))
    del colsum
    perm = torch.randperm(n, generator=torch.Generator().manual_seed(seed + 1))
    A = torch.empty_like(D.t()).t()
    A[perm.cuda()] = D
    del D
    return A, perm.numpy()


def factor_dev(lupp, h, A, tdt):
    import torch
    n = A.shape[1]
    ipiv = torch.empty(max(1, min(A.shape)), dtype=torch.int32, device="cuda")
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    (lupp.lupp_dgetrf if tdt == torch.float64 else lupp.lupp_sgetrf)(A, ipiv, info, handle=h)
    return ipiv[:min(A.shape[0], n)], info


def pid_pivot_check(torch, lupp, n, seed, tdt):
    """Closed-form pivots of a Pi*D factorization, bit for bit."""
    A, perm = pi_d_matrix(torch, n, seed, tdt)
    h = lupp.Handle()
    ipiv, info = factor_dev(lupp, h, A, tdt)
    h.sync()
    got = ipiv.cpu().numpy()
    want = closed_form_ipiv(perm)
    bad = np.nonzero(got != want)[0]
    h.close()
    del A
    torch.cuda.empty_cache()
    return {"n": n, "pivots_equal_closed_form": bool(len(bad) == 0), "mismatches": int(len(bad)),
            "first_mismatch": int(bad[0]) if len(bad) else -1, "info": int(info.item())}


def c2_leg(torch, lupp, seed, sizes=(4096, 8192, 16384), extra_f32=(32768,), reps=3):
    """Plain blocked LUPP FP64 and FP32 over a range of n (A iid U(-1,1) drawn
    on the device with torch's seeded generator): median of reps timed calls
    after one warmup (the input restored outside the timed interval, HIP events
    around the factorization on the handle's stream)."""
    out = []
    for dname, tdt, peak in (("f64", torch.float64, FP64_PEAK_TFLOPS), ("f32", torch.float32, FP32_PEAK_TFLOPS)):
        ns = list(sizes) + (list(extra_f32) if dname == "f32" else [])
        for n in ns:
            g = torch.Generator(device="cuda").manual_seed(seed + n)
            A0 = torch.empty((n, n), dtype=tdt, device="cuda").t()
            A0.uniform_(-1.0, 1.0, generator=g)
            A = torch.empty_like(A0.t()).t()
            h = lupp.Handle()
            times = []
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            for r in range(reps + 1):
                A.copy_(A0)
                torch.cuda.synchronize()
                e0.record()
                ipiv, info = factor_dev(lupp, h, A, tdt)
                e1.record()
                h.sync()
                torch.cuda.synchronize()
                if r > 0:
                    times.append(e0.elapsed_time(e1))
            ms = float(np.median(times))
            flops = 2.0 / 3.0 * float(n) ** 3
            tf = flops / (ms * 1e-3) / 1e12
            u = 2.0 ** -53 if dname == "f64" else 2.0 ** -24
            res = probe_residual(torch, A0.double(), A.double(), ipiv) * (2.0 ** -53 / u)
            h.close()
            del A, A0
            torch.cuda.empty_cache()
            pid = pid_pivot_check(torch, lupp, n, seed + 7 * n, tdt)
            rec = {"dtype": dname, "n": n, "ms": round(ms, 3), "tflops": round(tf, 3), "peak": peak,
                   "frac": round(tf / peak, 4), "info": int(info.item()), "probe_scaled_residual": res,
                   "pi_d": pid}
            log("c2: %s" % rec)
            out.append(rec)
    return {"workload": "plain blocked LUPP, A iid U(-1,1) (device-drawn, seed + n), 1 warmup + median of %d" % reps,
            "runs": out}


def cpu_baseline(seed, kappa_systems=None):
    """The oracle (unblocked right-looking FP64 LUPP) on the host cores: n = 512
    (median of 3) and n = 4096 (one run), each with 1 thread and with all the
    cores of the affinity mask; the input copy is made before the timer.  Then
    the FP64 reference solutions of the kappa systems (all cores)."""
    import oracle
    import synth
    cores = oracle.host_cores()
    runs = []
    for n, reps in ((512, 3), (4096, 1)):
        A = synth.uniform(seed, 0, n, n)
        for th in (1, cores):
            ts = []
            for _ in range(reps):
                W = np.array(A, order="F", copy=True)
                t = time.perf_counter()
                oracle.getrf(W, nthreads=th, overwrite=True)
                ts.append(time.perf_counter() - t)
            dt = float(np.median(ts))
            runs.append({"n": n, "threads": th, "seconds": round(dt, 4),
                         "tflops": 2.0 / 3.0 * n ** 3 / dt / 1e12})
            log("cpu oracle n=%d threads=%d: %.3f s" % (n, th, dt))
    refs = {}
    for key, (A, b) in (kappa_systems or {}).items():
        W = np.array(A, order="F", copy=True)
        t = time.perf_counter()
        LU, ipiv, info = oracle.getrf(W, nthreads=cores, overwrite=True)
        x, st = oracle.getrs(LU, ipiv, b)
        refs[key] = x
        log("cpu oracle reference solve %s: %.2f s" % (key, time.perf_counter() - t))
    best = [r for r in runs if r["n"] == 4096 and r["threads"] == cores][0]
    return {"value": best["tflops"], "unit": "TFLOP/s", "cores": cores, "kind": "oracle",
            "sample": "whole FP64 factorization at n=4096 (A iid U(-1,1), seed %d), all %d cores; also n=512 "
                      "(median of 3) and 1 thread, in runs" % (seed, cores),
            "runs": runs}, refs


def fp64_solve(torch, lupp, A0, B):
    """GPU FP64 LUPP + solve of A0 X = B (A0 not modified)."""
    A = torch.empty_like(A0.t()).t()
    A.copy_(A0)
    X = torch.empty_like(B.t()).t()
    X.copy_(B)
    h = lupp.Handle()
    ipiv, info = factor_dev(lupp, h, A, torch.float64)
    lupp.lupp_dgetrs(A, ipiv, X, handle=h)
    h.sync()
    h.close()
    del A
    return X


def mixed_runs(torch, lupp, A0, b, runs, fp64_ms=None, x_fp64=None, x_true=None, x_ref=None, b_true=None):
    """Timed mixed solves of A0 x = b (one right-hand side each); forward
    errors against the references given.  b_true = A0 x_true (an untimed
    second call per run) when b itself is not A0 x_true."""
    n = A0.shape[0]
    X = torch.empty((1, n), dtype=torch.float64, device="cuda").t()
    h = lupp.Handle()
    flops = 2.0 / 3.0 * float(n) ** 3
    out = []
    # first call allocates the workspace (FP32 copy of A): untimed
    lupp.lupp_dgesv_mixed(A0, b, X, lupp.ir_opts(runs[0][1], factor_prec=runs[0][0]), handle=h)
    for prec, solver in runs:
        torch.cuda.synchronize()
        t = time.perf_counter()
        rep = lupp.lupp_dgesv_mixed(A0, b, X, lupp.ir_opts(solver, factor_prec=prec), handle=h)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t) * 1e3
        r = {"factor_prec": prec, "solver": solver, "status": rep["status_name"], "iters": rep["iters"],
             "inner_iters": rep["inner_iters"], "backward_error": rep["backward_error"],
             "factor_ms": round(rep["factor_ms"], 2), "refine_ms": round(rep["refine_ms"], 2),
             "wall_ms": round(ms, 2), "effective_tflops": round(flops / (ms * 1e-3) / 1e12, 3)}
        if fp64_ms:
            r["speedup_vs_fp64_factor"] = round(fp64_ms / ms, 3)
        if x_fp64 is not None:
            r["forward_error_vs_gpu_fp64"] = rel_err(X[:, 0], x_fp64)
        if x_ref is not None:
            r["forward_error_vs_cpu_oracle"] = rel_err(X[:, 0].cpu().numpy(), x_ref)
        if x_true is not None:
            if b_true is None:
                r["forward_error_vs_x_true"] = rel_err(X[:, 0], x_true)
            else:
                Xt = torch.empty_like(X.t()).t()
                lupp.lupp_dgesv_mixed(A0, b_true, Xt, lupp.ir_opts(solver, factor_prec=prec), handle=h)
                r["forward_error_vs_x_true"] = rel_err(Xt[:, 0], x_true)
        log("mixed n=%d: %s" % (n, r))
        out.append(r)
    h.close()
    return out


def diag_dominant_dev(torch, A0):
    """In place: U(-1,1) -> U(-0.5,0.5) (exact), then a_ii := sum_j |a_ij|."""
    A0.mul_(0.5)
    d = A0.abs().sum(dim=1)
    A0.diagonal().copy_(d)
    del d


def mixed_leg(torch, lupp, A0, n, seed, fp64_ms, runs):
    """Mixed-precision solves on the diagonally dominant matrix built in place
    from A0 (A0 is overwritten)."""
    import synth
    diag_dominant_dev(torch, A0)
    b = torch.from_numpy(synth.uniform(seed, 1, n, 1)).cuda()  # (n, 1), column-major
    g = torch.Generator(device="cuda").manual_seed(seed + 3)
    x_true = torch.empty(n, dtype=torch.float64, device="cuda").uniform_(-1.0, 1.0, generator=g)
    b_true = (A0 @ x_true).view(n, 1)
    x64 = fp64_solve(torch, lupp, A0, b)[:, 0]
    out = mixed_runs(torch, lupp, A0, b, runs, fp64_ms, x_fp64=x64, x_true=x_true, b_true=b_true)
    conv = [r for r in out if r["status"] == "converged"]
    best = max(conv, key=lambda r: r["effective_tflops"]) if conv else None
    return {"workload": "diag-dominant n=%d (a_ii = row abs-sum of U(-0.5,0.5)), b iid U(-1,1), tol 1e-14; forward "
                        "errors vs the GPU FP64 LUPP solve and, from a second untimed call with b = A x_true "
                        "(x_true iid U(-1,1)), vs x_true" % n,
            "runs": out, "best_converged": best}


def mixed16_leg(torch, lupp, seed, n=16384):
    """Config C3a at n = 16384: the diagonally dominant recipe drawn on the
    device (torch's seeded generator)."""
    g = torch.Generator(device="cuda").manual_seed(seed + n)
    A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    A0.uniform_(-1.0, 1.0, generator=g)
    diag_dominant_dev(torch, A0)
    b = torch.empty((n, 1), dtype=torch.float64, device="cuda").uniform_(-1.0, 1.0, generator=g)
    x_true = torch.empty(n, dtype=torch.float64, device="cuda").uniform_(-1.0, 1.0, generator=g)
    b_true = (A0 @ x_true).view(n, 1)
    x64 = fp64_solve(torch, lupp, A0, b)[:, 0]
    runs = [("fp16", "gmres"), ("bf16", "gmres"), ("fp16", "classical"), ("bf16", "classical")]
    out = mixed_runs(torch, lupp, A0, b, runs, x_fp64=x64, x_true=x_true, b_true=b_true)
    del A0
    torch.cuda.empty_cache()
    return {"workload": "diag-dominant n=%d drawn on the device (seed %d), b iid U(-1,1); forward errors vs the "
                        "GPU FP64 solve and vs x_true (b = A x_true, untimed second call)" % (n, seed + n),
            "runs": out}


def kappa_systems(seed, n=4096, kappas=(1e2, 1e4, 1e6)):
    """A = U diag(sigma) V^T, sigma_i = kappa^(-(i-1)/(n-1)), U and V the Q
    factors of QR of iid Gaussian matrices (Philox streams 2 and 3, signs fixed
    so diag(R) > 0); b = A x_true with x_true iid U(-1,1) (stream 4)."""
    import synth
    t = time.time()

    def haar(sid):  # the same construction as synth.kappa_matrix, its factors shared over kappa
        q, r = np.linalg.qr(synth.gaussian(seed, sid, n, n))
        return q * np.sign(np.diag(r))[None, :]
    U = haar(2)
    V = haar(3)
    x_true = synth.uniform(seed, 4, n, 1)[:, 0]
    out = {}
    for k in kappas:
        sig = k ** (-(np.arange(n) / max(n - 1, 1)))
        A = np.asfortranarray((U * sig[None, :]) @ V.T)
        out["%g" % k] = (A, A @ x_true)
    log("kappa systems built in %.1f s" % (time.time() - t))
    return out, x_true


def kappa_leg(torch, lupp, systems, x_true, refs):
    res = []
    xt = torch.from_numpy(x_true).cuda()
    for key, (A, b) in systems.items():
        A0 = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
        bd = torch.from_numpy(b.copy()).cuda().view(-1, 1)
        x64 = fp64_solve(torch, lupp, A0, bd)[:, 0]
        runs = [(p, s) for p in ("bf16", "fp16") for s in ("classical", "gmres")]
        out = mixed_runs(torch, lupp, A0, bd, runs, x_fp64=x64, x_true=xt, x_ref=refs.get(key))
        for r in out:
            r["kappa"] = float(key)
        res.extend(out)
        del A0
    return {"workload": "n=4096, A = U diag(sigma) V^T (Haar U, V from QR of Philox Gaussians, geometric sigma "
                        "1..1/kappa), b = A x_true; forward errors vs the CPU oracle's FP64 solve (when the CPU leg "
                        "ran), the GPU FP64 solve and x_true",
            "runs": res}


def dataflow_leg(torch, lupp, A0, A, fn, ref_ipiv, nb, depths=(2, 4)):
    """The same factorization by the dataflow (algorithm-by-blocks) runtime,
    lookahead depth d: one untimed and one timed call per depth; pivots
    compared with the headline run's."""
    n = A0.shape[0]
    runs = []
    for d in depths:
        hd = lupp.Handle()
        hd.set_option(4, d)
        if nb:
            hd.set_option(1, nb)
        ipd = torch.empty_like(ref_ipiv)
        infd = torch.empty(1, dtype=torch.int32, device="cuda")
        ms = None
        for r in range(2):
            A.copy_(A0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn(A, ipd, infd, handle=hd)
            hd.sync()
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
        hd.close()
        runs.append({"depth": d, "ms": round(ms, 3), "tflops": round(2.0 / 3.0 * n ** 3 / (ms * 1e-3) / 1e12, 3),
                     "info": int(infd.item()), "ipiv_equal_to_headline": bool(torch.equal(ipd, ref_ipiv))})
    out = {"workload": "the headline factorization (n=%d) by the dataflow runtime, lookahead depth d "
                       "(one call after one untimed call, input restored outside the timer)" % n, "runs": runs}
    log("dataflow: %s" % out)
    return out


def qr_leg(torch, lupp, seed, sizes=(4096, 8192, 16384)):
    """Householder QR (lupp_dgeqrf) of A iid U(-1,1) drawn on the device:
    best of two calls after one untimed call; TFLOP/s on 4/3 n^3; the
    column-block and update shares from the library's phase events; a
    probe of ||A x - Q (R x)|| with Q applied on the device by torch."""
    runs = []
    for n in sizes:
        g = torch.Generator(device="cuda").manual_seed(seed + n)
        A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").t().uniform_(-1.0, 1.0, generator=g)
        A = torch.empty_like(A0.t()).t()
        tau = torch.empty(n, dtype=torch.float64, device="cuda")
        h = lupp.Handle()
        ts = []
        for r in range(3):
            A.copy_(A0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            lupp.lupp_dgeqrf(A, tau, h)
            h.sync()
            torch.cuda.synchronize()
            if r:
                ts.append(time.perf_counter() - t0)
        h.set_option(3, 1)
        A.copy_(A0)
        lupp.lupp_dgeqrf(A, tau, h)
        h.sync()
        pc, pms, _ = h.timing_summary("panel")
        uc, ums, ufl = h.timing_summary("update", reset=True)
        h.close()
        # probe: x random, y = R x, then Q y by the reflectors in reverse order
        x = torch.rand((n, 4), generator=g, dtype=torch.float64, device="cuda") * 2 - 1
        y = torch.triu(A) @ x
        for j in range(n - 1, -1, -1):
            v = A[j:, j].clone()
            v[0] = 1.0
            y[j:] -= tau[j] * torch.outer(v, v @ y[j:])
            if j % 2048 == 0:
                torch.cuda.synchronize()
        res = float((A0 @ x - y).abs().max() / (n * 2.0 ** -53 * A0.abs().sum(0).max() * x.abs().max()))
        ms = min(ts) * 1e3
        runs.append({"n": n, "ms": round(ms, 3), "tflops": round(4.0 / 3.0 * n ** 3 / (ms * 1e-3) / 1e12, 3),
                     "frac_fp64_peak": round(4.0 / 3.0 * n ** 3 / (ms * 1e-3) / 1e12 / FP64_PEAK_TFLOPS, 4),
                     "panel_ms": round(pms, 2), "panel_launches": pc, "update_ms": round(ums, 2),
                     "update_tflops": round(ufl / (ums * 1e-3) / 1e12, 3) if ums > 0 else None,
                     "probe_scaled_residual": res})
        del A, A0
        torch.cuda.empty_cache()
    out = {"workload": "Householder QR, A iid U(-1,1) (device-drawn, seed + n), best of 2 after 1 warmup; "
                       "flops 4/3 n^3", "runs": runs}
    log("qr: %s" % out)
    return out


def utv_leg(torch, lupp, seed, sizes=(2048, 4096, 8192), qs=(0, 1, 2)):
    """randUTV (lupp_drandutv, b = 64) of A iid U(-1,1) drawn on the device,
    Gaussian draws G from torch's generator: best of two calls per (n, q),
    T only and (q = 1) with U and V formed; at n = 2048 the diagonal of T
    against the singular values from torch.linalg.svdvals (rocSOLVER, a
    labelled run-only comparison) and the identity A = U T V^T."""
    runs = []
    for n in sizes:
        g = torch.Generator(device="cuda").manual_seed(seed + 7 * n)
        A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").t().uniform_(-1.0, 1.0, generator=g)
        G = torch.empty((n, n), dtype=torch.float64, device="cuda").t().normal_(generator=g)
        A = torch.empty_like(A0.t()).t()
        U = torch.empty_like(A0.t()).t()
        V = torch.empty_like(A0.t()).t()
        h = lupp.Handle()
        for q, uv in [(q, False) for q in qs] + [(1, True)]:
            ts = []
            for r in range(2):
                A.copy_(A0)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                lupp.lupp_drandutv(A, G, q, U if uv else None, V if uv else None, h)
                h.sync()
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            rec = {"n": n, "q": q, "uv": uv, "ms": round(min(ts) * 1e3, 2)}
            if uv and n <= 2048:
                s_ref = torch.linalg.svdvals(A0)
                d = torch.diagonal(A)
                rec["identity_scaled_residual"] = float((U @ A @ V.t() - A0).abs().max() /
                                                        (n * 2.0 ** -53 * A0.abs().sum(0).max()))
                rec["orthogonality_U"] = float((U.t() @ U - torch.eye(n, dtype=torch.float64, device="cuda")).abs().max())
                rec["diag_T_vs_svdvals_max_rel_first_64"] = float(((d[:64] - s_ref[:64]).abs() / s_ref[:64]).max())
                rec["diag_T_vs_svdvals_max_rel_all"] = float(((d - s_ref).abs() / s_ref).max())
            runs.append(rec)
        h.close()
        del A, A0, G, U, V
        torch.cuda.empty_cache()
    # the vendor SVD at the smallest size, as labelled context (the paper's comparison point)
    n = sizes[0]
    g = torch.Generator(device="cuda").manual_seed(seed)
    A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").uniform_(-1.0, 1.0, generator=g)
    torch.linalg.svdvals(A0[:256, :256])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    torch.linalg.svd(A0)
    torch.cuda.synchronize()
    svd_ms = (time.perf_counter() - t0) * 1e3
    out = {"workload": "randUTV, block 64, A iid U(-1,1) (device-drawn), G iid N(0,1); best of 2", "runs": runs,
           "context_torch_linalg_svd_ms": {"n": n, "ms": round(svd_ms, 1),
                                            "note": "rocSOLVER through torch, U S V^T formed; run only"}}
    log("randutv: %s" % out)
    return out


def large_leg(torch, lupp, n, seed):
    """FP8-update GMRES-IR solve against plain FP64 LUPP + solve at a large n,
    on the diagonally dominant recipe drawn on the device (torch's seeded
    generator: U(-0.5,0.5), then a_ii := sum_j |a_ij|), b iid U(-1,1)."""
    g = torch.Generator(device="cuda").manual_seed(seed + 65536)
    A0 = torch.empty((n, n), dtype=torch.float64, device="cuda").t()
    A0.uniform_(-0.5, 0.5, generator=g)
    d = A0.abs().sum(dim=1)
    A0.diagonal().copy_(d)
    del d
    b = torch.empty((n, 1), dtype=torch.float64, device="cuda").uniform_(-1.0, 1.0, generator=g)
    flops = 2.0 / 3.0 * float(n) ** 3

    def eta(x):
        r = b[:, 0] - torch.mv(A0, x)
        den = A0.abs().sum(dim=1).max() * x.abs().max() + b.abs().max()
        return float(r.abs().max() / den)

    # plain FP64: factorization, then the solve (workspace set up by a small call first)
    h = lupp.Handle()
    small = torch.eye(64, dtype=torch.float64, device="cuda").t()  # column-major
    ip_s = torch.empty(64, dtype=torch.int32, device="cuda")
    in_s = torch.empty(1, dtype=torch.int32, device="cuda")
    lupp.lupp_dgetrf(small, ip_s, in_s, handle=h)
    A = torch.empty_like(A0.t()).t()  # column-major working copy
    A.copy_(A0)
    ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    x = b.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lupp.lupp_dgetrf(A, ipiv, info, handle=h)
    h.sync()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lupp.lupp_dgetrs(A, ipiv, x, handle=h)
    h.sync()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    fp64 = {"factor_ms": round((t1 - t0) * 1e3, 2), "solve_ms": round((t2 - t1) * 1e3, 2),
            "wall_ms": round((t2 - t0) * 1e3, 2), "tflops": round(flops / (t1 - t0) / 1e12, 3),
            "info": int(info.item()), "backward_error": eta(x[:, 0])}
    log("large FP64: %s" % fp64)
    h.close()
    x64 = x
    del A, ipiv, info
    torch.cuda.empty_cache()

    X = torch.empty((1, n), dtype=torch.float64, device="cuda").t()
    h = lupp.Handle()
    opts = lupp.ir_opts("gmres", factor_prec="fp8")
    lupp.lupp_dgesv_mixed(A0, b, X, opts, handle=h)  # allocates the FP32 workspace: untimed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = lupp.lupp_dgesv_mixed(A0, b, X, opts, handle=h)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    h.close()
    mixed = {"factor_prec": "fp8", "solver": "gmres", "status": rep["status_name"], "iters": rep["iters"],
             "inner_iters": rep["inner_iters"], "backward_error": rep["backward_error"],
             "backward_error_check": eta(X[:, 0]), "factor_ms": round(rep["factor_ms"], 2),
             "refine_ms": round(rep["refine_ms"], 2), "wall_ms": round(ms, 2),
             "effective_tflops": round(flops / (ms * 1e-3) / 1e12, 3),
             "speedup_vs_fp64_solve": round(fp64["wall_ms"] / ms, 3)}
    mixed["forward_error_vs_gpu_fp64"] = rel_err(X[:, 0], x64[:, 0])
    # 64 sampled rows of the residual in long double on the host
    rows = torch.randperm(n, generator=torch.Generator().manual_seed(seed + 64))[:64]
    Ar = A0[rows.cuda()].cpu().numpy().astype(np.longdouble)
    xr = X[:, 0].cpu().numpy().astype(np.longdouble)
    br = b[rows.cuda(), 0].cpu().numpy().astype(np.longdouble)
    rr = np.abs(br - Ar @ xr).max()
    den = float(A0.abs().sum(dim=1).max()) * float(np.abs(xr).max()) + float(b.abs().max())
    mixed["sampled_rows_backward_error_longdouble"] = float(rr / np.longdouble(den))
    log("large mixed: %s" % mixed)
    del A0, b, X, x64
    torch.cuda.empty_cache()
    return {"workload": "diag-dominant n=%d (U(-0.5,0.5), a_ii = row abs-sum, drawn on the device from seed %d), "
                        "b iid U(-1,1); FP8 (e4m3, per-block power-of-two scales) updates + FP64 GMRES-IR to 1e-14 "
                        "vs plain FP64 LUPP + solve" % (n, seed + 65536),
            "n": n, "fp64": fp64, "mixed": mixed}


def batched_leg(torch, lupp, seed, count=20000, replays=20, dtype="f64", graph=True):
    import synth
    npdt = np.float64 if dtype == "f64" else np.float32
    sizes = synth.batch_sizes(seed, count)
    A, a_off, B, b_off = synth.batch_uniform(seed, sizes, npdt)
    dn = torch.from_numpy(sizes).cuda()
    dao = torch.from_numpy(a_off).cuda()
    dbo = torch.from_numpy(b_off).cuda()
    A0 = torch.from_numpy(A).cuda()
    B0 = torch.from_numpy(B).cuda()
    dA, dB = A0.clone(), B0.clone()
    n64 = dn.to(torch.int64)
    p_off = torch.zeros_like(n64)
    p_off[1:] = torch.cumsum(n64, 0)[:-1]
    ipiv = torch.zeros(int(n64.sum()), dtype=torch.int32, device="cuda")
    info = torch.zeros(count, dtype=torch.int32, device="cuda")
    h = lupp.Handle(tuned=False)
    lupp.lupp_xgesv_batched(dn, dA, dao, ipiv, p_off, dB, dbo, info, handle=h)  # workspace
    torch.cuda.synchronize()

    def timed(nrep):
        g = None
        if graph:
            g = torch.cuda.CUDAGraph()
            dA.copy_(A0)
            dB.copy_(B0)
            torch.cuda.synchronize()
            with torch.cuda.graph(g):
                lupp.lupp_xgesv_batched(dn, dA, dao, ipiv, p_off, dB, dbo, info, handle=h)
        ts = []
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for r in range(nrep + 2):
            dA.copy_(A0)
            dB.copy_(B0)
            torch.cuda.synchronize()
            e0.record()
            if g is not None:
                g.replay()
            else:
                lupp.lupp_xgesv_batched(dn, dA, dao, ipiv, p_off, dB, dbo, info, handle=h)
            e1.record()
            torch.cuda.synchronize()
            if r >= 2:
                ts.append(e0.elapsed_time(e1))
        return ts

    # the library's initial schedule, then the autotuner's choice made live on
    # this GPU (the timed result); the committed cache's choice is recorded
    initial_ms = float(np.median(timed(max(3, replays // 4))))
    from paper_2104_05782_amd import autotune as _at
    tune = _at.sweep(h, dtype, 2500) if graph else None
    cached = _at.load().get(_at.device_arch(), {}).get(dtype, {}).get("schedule")
    times = timed(replays)
    ms = float(np.median(times))
    bad = int((info != 0).sum().item())
    # algorithmic bytes: A read + L\U written (n^2 each), b read + x written,
    # ipiv written (4 B), n and three offsets read (4 + 24 B)
    isz = 8 if dtype == "f64" else 4
    s64 = sizes.astype(np.float64)
    nbytes = float((2 * s64 * s64 * isz + 2 * s64 * isz + 4 * s64 + 28).sum())
    flops = float((2.0 / 3.0 * s64 ** 3 + 2 * s64 ** 2).sum())
    # a sampled backward-error check of the last replay
    X = dB.cpu().numpy()
    u = 2.0 ** -53 if dtype == "f64" else 2.0 ** -24
    worst = 0.0
    for i in range(0, count, max(1, count // 200)):
        n = int(sizes[i])
        Ai = A[a_off[i]:a_off[i] + n * n].reshape(n, n, order="F").astype(np.float64)
        eta = host_backward_error(Ai, X[b_off[i]:b_off[i] + n].astype(np.float64),
                                  B[b_off[i]:b_off[i] + n].astype(np.float64))
        worst = max(worst, eta / (n * u))
    h.close()
    gbs = nbytes / (ms * 1e-3) / 1e9
    out = {"workload": "%d systems, n_i ~ U{8..128}, A_i and b_i iid U(-1,1), %s, LU + solve" % (count, dtype),
           "value": round(count / (ms * 1e-3), 1), "unit": "factorizations/s", "ms": round(ms, 4),
           "replays": replays, "graph": bool(graph), "min_ms": round(min(times), 4), "gflops": round(flops / (ms * 1e-3) / 1e9, 1),
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": 8000.0, "unit": "GB/s",
                        "frac": round(gbs / 8000.0, 4), "traffic": None, "bytes": nbytes},
           "check": {"nonzero_info": bad, "max_backward_error_over_n_u_sampled": worst},
           "schedule": {"autotuned": tune, "initial_schedule_ms": round(initial_ms, 4), "cached": cached,
                        "shapes": lupp.batched_shapes()}}
    log("batched: %s" % out)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=32768)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--nb", type=int, default=0)
    ap.add_argument("--block", type=int, default=0, help="widest cooperative column block (multiple of 16)")
    ap.add_argument("--seed", type=int, default=20210513)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-lookahead", action="store_true")
    ap.add_argument("--no-split", action="store_true",
                    help="no share of the remaining-columns update on the panel's CUs (every launch shape then follows "
                         "from n and nb alone)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision solve leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched small-systems leg")
    ap.add_argument("--no-large", action="store_true", help="skip the large mixed-precision leg")
    ap.add_argument("--no-dataflow", action="store_true", help="skip the dataflow-runtime leg")
    ap.add_argument("--no-qr", action="store_true", help="skip the Householder QR leg")
    ap.add_argument("--no-utv", action="store_true", help="skip the randUTV leg")
    ap.add_argument("--no-c2", action="store_true", help="skip the FP64/FP32 size sweep")
    ap.add_argument("--no-kappa", action="store_true", help="skip the kappa (n=4096) mixed-precision leg")
    ap.add_argument("--large-n", type=int, default=65536)
    ap.add_argument("--profile-once", action="store_true",
                    help="counter runs: factor once without a pristine device copy, after a 1 GiB "
                         "device-to-device copy that calibrates the byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    import paper_2104_05782_amd as lupp

    n = args.n
    npdt = np.float64 if args.dtype == "f64" else np.float32
    tdt = torch.float64 if args.dtype == "f64" else torch.float32
    A0 = torch.empty((n, n), dtype=tdt, device="cuda").t()
    if args.profile_once:
        # counter runs only: the profiler's counter mode does not survive the
        # host-to-device upload of a matrix this size, so the input is drawn on
        # the device (iid U(-1,1) from torch's generator; same shape and
        # distribution, different values)
        g = torch.Generator(device="cuda").manual_seed(args.seed)
        A0.uniform_(-1.0, 1.0, generator=g)
        A_host = None
    else:
        log("generating A (n=%d, seed=%d)" % (n, args.seed))
        t = time.time()
        A_host = synth.uniform(args.seed, 0, n, n)
        if npdt != np.float64:
            A_host = np.asfortranarray(A_host.astype(npdt))
        log("generated in %.1f s; uploading" % (time.time() - t))
        # column-major pristine copy, uploaded in 256 MiB column chunks
        At = A_host.T  # C-ordered view: row c of At is column c of A
        step = max(1, (256 << 20) // (n * At.itemsize))
        for c0 in range(0, n, step):
            A0.t()[c0:c0 + step].copy_(torch.from_numpy(At[c0:c0 + step]))
        A_host = At = None  # the host copy is not needed again
    if args.profile_once:
        if args.steps != 1 or args.warmup != 0:
            sys.exit("--profile-once needs --steps 1 --warmup 0")
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)  # calibration: 1 GiB read, 1 GiB written
        torch.cuda.synchronize()
        del src, dst
        A = A0
    else:
        A = torch.empty_like(A0.t()).t()
    ipiv = torch.empty(n, dtype=torch.int32, device="cuda")
    info = torch.empty(1, dtype=torch.int32, device="cuda")
    h = lupp.Handle()
    if args.nb:
        h.set_option(1, args.nb)
    if args.block:
        h.set_option(2, args.block)
    if args.no_lookahead:
        h.set_option(4, 0)
    if args.no_split:
        h.set_option(7, 0)
    fn = lupp.lupp_dgetrf if args.dtype == "f64" else lupp.lupp_sgetrf

    def step():
        if A is not A0:
            A.copy_(A0)
        fn(A, ipiv, info, handle=h)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log("warmup %d done" % w)
    # events around the trailing updates during the timed steps (the roofline
    # kernel's launch durations); the column-block chain stays uninstrumented
    h.set_option(3, 2)
    h.timing_summary("panel", reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    h.sync()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    flops = 2.0 / 3.0 * float(n) ** 3
    value = flops / (ms_per_step * 1e-3) / 1e12
    log("timed %d steps: %.2f ms/step, %.2f TFLOP/s" % (args.steps, ms_per_step, value))
    alg_bytes = h.timing_bytes("update_big")
    c, ms, fl = h.timing_summary("update_big", reset=True)
    peak = FP64_PEAK_TFLOPS if args.dtype == "f64" else FP32_PEAK_TFLOPS
    achieved = (fl / (ms * 1e-3) / 1e12) if ms > 0 else 0.0
    # HBM traffic of this kernel: the calibrated FETCH_SIZE + WRITE_SIZE of its
    # launches over their algorithmic bytes, 1.808 at n = 24576 (the largest
    # size at which the profiler's counter mode has run; profiles/
    # lupp_n24576_counters.md), applied to this run's algorithmic bytes per launch
    traffic = None
    if args.dtype == "f64" and c > 0:
        traffic = round(TRAFFIC_RATIO_FP64_GEMM * alg_bytes / c, 1)
    roofline = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": "TFLOP/s",
                "frac": round(achieved / peak, 4), "traffic": traffic,
                "traffic_note": ("bytes per launch: %.3f x the algorithmic bytes (C read and written, A and B read once; "
                                 "%.4g per launch here), the ratio measured at n = 24576" %
                                 (TRAFFIC_RATIO_FP64_GEMM, alg_bytes / max(1, c))) if traffic else None,
                "kernel": ("k_dgemm_sub_16<128,128,8,2,4,4,0>" if args.dtype == "f64" else "k_sgemm_sub_16<128,128,16,2,2,2,0>"),
                "launches_per_step": c // max(1, args.steps),
                "avg_launch_ms": round(ms / max(1, c), 4),
                "flops_per_launch": fl / max(1, c)}
    # the phase breakdown, from one more step with every phase instrumented
    # (after the timed region: its events slow the column-block chain by ~3%)
    phases = {}
    if not args.profile_once:
        h.set_option(3, 1)
        step()
        for ph in ("panel", "laswp", "trsm", "update", "update_big", "panel_leaf", "panel_swap", "panel_trsm",
                   "panel_gemm"):
            pc, pms, pfl = h.timing_summary(ph)
            phases[ph] = {"launches": pc, "ms_per_step": pms, "flops": pfl}
        h.timing_summary("panel", reset=True)
        phases["note"] = "one step after the timed region, every phase bracketed by HIP events"
    h.set_option(3, 0)

    dataflow = None
    if not args.no_dataflow and not args.profile_once:
        dataflow = dataflow_leg(torch, lupp, A0, A, fn, ipiv.clone(), args.nb)

    check = None
    if not args.no_check:
        inf = int(info.item())
        res = probe_residual(torch, A0.double(), A.double(), ipiv) if n <= 32768 else None
        check = {"info": inf, "probe_scaled_residual": res}
        if not args.profile_once:
            del A
            A = None
            torch.cuda.empty_cache()
            check["pi_d"] = pid_pivot_check(torch, lupp, n, args.seed + 11, tdt)
        log("check: %s" % check)

    c2 = None
    if not args.no_c2 and not args.profile_once:
        log("c2 sweep")
        c2 = c2_leg(torch, lupp, args.seed)

    ksys = xk_true = None
    if not args.no_kappa and not args.profile_once:
        ksys, xk_true = kappa_systems(args.seed)

    cpu = None
    krefs = {}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu, krefs = cpu_baseline(args.seed, ksys)
        log("cpu baseline: %s" % cpu)

    kappa = None
    if ksys is not None:
        log("kappa leg")
        kappa = kappa_leg(torch, lupp, ksys, xk_true, krefs)
        ksys = None

    mixed = None
    if not args.no_mixed and args.dtype == "f64":
        A = None
        torch.cuda.empty_cache()
        log("mixed-precision leg")
        runs = [("fp16", "gmres"), ("bf16", "gmres"), ("fp8", "gmres"), ("fp16", "classical"), ("bf16", "classical")]
        mixed = {"n%d" % n: mixed_leg(torch, lupp, A0, n, args.seed, ms_per_step, runs[:1] if args.profile_once else runs)}
        if not args.profile_once:
            A0 = None
            torch.cuda.empty_cache()
            mixed["n16384"] = mixed16_leg(torch, lupp, args.seed)

    qrres = None
    if not args.no_qr and not args.profile_once:
        A = None
        torch.cuda.empty_cache()
        log("qr leg")
        qrres = qr_leg(torch, lupp, args.seed)

    utvres = None
    if not args.no_utv and not args.profile_once:
        A = None
        torch.cuda.empty_cache()
        log("randutv leg")
        utvres = utv_leg(torch, lupp, args.seed)

    batched = None
    if not args.no_batched:
        log("batched leg")
        if args.profile_once:  # counter runs: eager calls, no graph replays
            batched = {"f64": batched_leg(torch, lupp, args.seed, replays=1, graph=False)}
        else:
            batched = {"f64": batched_leg(torch, lupp, args.seed),
                       "f32": batched_leg(torch, lupp, args.seed, dtype="f32")}

    large = None
    if not args.no_large and not args.profile_once and args.dtype == "f64":
        A = A0 = None  # release the headline size's matrices
        torch.cuda.empty_cache()
        log("large mixed-precision leg (n=%d)" % args.large_n)
        large = large_leg(torch, lupp, args.large_n, args.seed)

    out = {
        "metric": "LU TFLOP/s @n=32768: FP64 vs mixed+IR at FP64 backward err; batched LUs/s",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.dtype == "f64" else "f32",
        "data": "synthetic: A iid U(-1,1) from seed %d (Philox-4x64-10)" % args.seed,
        "config": {"workload": "plain blocked LUPP FP64 n=%d" % n if args.dtype == "f64"
                   else "plain blocked LUPP FP32 n=%d" % n,
                   "n": n, "nb": args.nb or 512, "lookahead": 0 if args.no_lookahead else 1,
                   "flops_per_step": flops, "parallelism": "single GPU"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "phases": phases,
        "check": check,
        "c2": c2,
        "kappa": kappa,
        "mixed": mixed,
        "batched": batched,
        "large": large,
        "dataflow": dataflow,
        "qr": qrres,
        "randutv": utvres,
    }
    print(json.dumps(out), flush=True)
    h.close()


if __name__ == "__main__":
    main()
