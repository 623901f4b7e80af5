"""Throughput of the factored FIO inverse solve on one MI355X.

A step is one pass of the whole hot path over one batch of right-hand sides:
layout in, Kd^* (butterfly adjoint, complex64), Gd (skeletonization sweeps and
the FP64 top-level block), one FP64 refinement step r = u - Kd x (complex128
factors) followed by the complex64 correction Gd Kd^* r, and layout out.

The default workload is the largest one-GPU configuration: the 2D generalized
Radon FIO (section 6, Example 3) at n = 256 (N = 65536) with 256 right-hand
sides, eps = 1e-4.  Every run also solves, untimed, a batch whose known-truth
columns come from the oracle's direct summation (u = K fhat), and prints no
value if their error exceeds 10 eps.

Prints one JSON line (see the keys below).  Inputs are synthetic (seeded
Gaussian right-hand sides) and resident in HBM before timing starts.
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

from fio_synth import WORKLOADS, gaussian_complex, uniform_indices  # noqa: E402

PEAK_TFLOPS = {"c64": 157.3, "c128": 78.6}   # MI355X dense MFMA FP32 / FP64
PEAK_HBM_GBS = 8000.0

# HBM bytes per launch of a stage-kernel instance on the measured workload, from
# rocprofv3 FETCH_SIZE (x2) and WRITE_SIZE (x1) scaled by a 1 GiB copy kernel
# (summaries under profiles/), valid only for the kernel source and the factor set
# (its nonzero count) they were measured on.
TRAFFIC = {
    # 2D Example 3, n=256, 256 RHS (profiles/k_stage_mfma_f32_3m_2d_n256_traffic.md)
    "k_stage_mfma<float, 2, 2, 3M>": {
        "bytes": 4.1708e9,
        "kernels_sha256": "0dbfb62eb9d369702b13a55035612be69e056af0e78babd229ec27fcf0557140",
        "bf_nnz": 1138753536,
    },
}


# Matrix-core counters per launch (rocprofv3 SQ_INSTS_VALU_MFMA_MOPS_F32 x 512 and
# SQ_VALU_MFMA_BUSY_CYCLES; summary under profiles/), under the same validity rule.
MFMA_COUNTERS = {
    "k_stage_mfma<float, 2, 2, 3M>": {
        "executed_flop": 3.4403e11,
        "busy": 0.6285,
        "kernels_sha256": "0dbfb62eb9d369702b13a55035612be69e056af0e78babd229ec27fcf0557140",
        "bf_nnz": 1138753536,
    },
}


# HBM bytes per plain FP64 single-RHS solve (every launch), the same counters and
# calibration, default kernel choices (profiles/plain_fp64_2d_n256_traffic.md).
PLAIN_TRAFFIC = {
    "plain_fp64": {
        "bytes": 2.1873e10,
        "kernels_sha256": "0dbfb62eb9d369702b13a55035612be69e056af0e78babd229ec27fcf0557140",
        "bf_nnz": 1138753536,
    },
}


def counted(table, name, bf_nnz):
    """The entry of a counter table for this kernel, or None if the kernel source or
    the factors (their nonzero count) differ from the ones profiled."""
    import hashlib
    t = table.get(name.split(" (")[0])
    if not t or t.get("bf_nnz") != bf_nnz:
        return None
    src = os.path.join(ROOT, "paper_2105_02995_amd", "csrc", "kernels.hip")
    with open(src, "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != t["kernels_sha256"]:
            return None
    return t


def mfma_counters_for(name, bf_nnz, avg_launch_ms, peak):
    t = counted(MFMA_COUNTERS, name, bf_nnz)
    if t is None:
        return None
    ex = t["executed_flop"] / (avg_launch_ms * 1e-3) / 1e12
    return {"executed_flop_per_launch": t["executed_flop"], "executed_tflops": round(ex, 3),
            "executed_frac": round(ex / peak, 4), "mfma_busy": t["busy"]}


def traffic_for(name, bf_nnz):
    """HBM bytes per launch from the committed counter runs, or None if the kernel
    source or the factors (their nonzero count) differ from the ones profiled."""
    t = counted(TRAFFIC, name, bf_nnz)
    return None if t is None else t["bytes"]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="2d_n256", choices=sorted(WORKLOADS))
    ap.add_argument("--refine", type=int, default=1, help="FP64 refinement steps per solve")
    ap.add_argument("--mode", choices=("refine", "pcg"), default="refine",
                    help="refine: complex64 applies + FP64 refinement; pcg: CG on Kd^*Kd preconditioned "
                         "by Gd (complex128 applies) to a relative residual of 1e-8, the 2D n=64 configuration")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-calibration", action="store_true",
                    help="skip the measured device ceilings (streaming read, matrix-core loop)")
    ap.add_argument("--no-plain", action="store_true", help="skip the FP64 single-RHS comparator")
    ap.add_argument("--no-serve", action="store_true", help="skip the small serving leg")
    ap.add_argument("--plan-file", default=None,
                    help="load the factors from this plan file if it exists, else build them and save them there")
    ap.add_argument("--plain-only", action="store_true",
                    help="run only the FP64 single-RHS comparator (for profiling its kernels)")
    ap.add_argument("--plain-untuned", action="store_true",
                    help="FP64 single-RHS comparator on the default kernel choices (no autotuning: "
                         "profiled runs then launch the same kernels, whatever the profiler does to timings)")
    ap.add_argument("--trace", action="store_true",
                    help="named library ranges (fio_set_trace) during the timed steps, for a marker trace")
    ap.add_argument("--no-tune", action="store_true", help="use the built-in kernel heuristics")
    ap.add_argument("--serve", action="store_true",
                    help="run the serving mix (Poisson arrivals over many keys) instead of the solve bench")
    ap.add_argument("--serve-requests", type=int, default=200)
    ap.add_argument("--no-multi", action="store_true",
                    help="serving: run every batch on its own (no multi-instance solves)")
    return ap.parse_args()


SERVE_KEYS_FULL = ([(1, n, "1d_ex1", e) for n in (1024, 2048, 4096, 8192, 16384, 32768, 65536)
                    for e in (1e-4, 1e-6)] + [(2, n, "2d_radon", 1e-4) for n in (32, 64, 128, 256)])
SERVE_KEYS_SMALL = [(1, 4096, "1d_ex1", 1e-6), (1, 65536, "1d_ex1", 1e-6), (2, 64, "2d_radon", 1e-4)]


def serving_run(F, plans, keys, nreq, fracs, seed, max_batch=256, graphs=True, multi=True, trim=False):
    """Poisson arrivals (seeded) of solves over the given resident keys, 1..32
    right-hand sides each; the rate is a fraction of the measured saturation rate
    (all requests at t=0).  Batches of different keys admitted together run as one
    multi-instance solve (multi).  Returns p50/p99 latency and RHS*N/s per rate."""
    from paper_2105_02995_amd.serve import (GpuExecutor, Scheduler, ServeRequest, latency_stats,
                                            throughput)
    rng = np.random.default_rng(seed)
    pools = {k: gaussian_complex((k[1] ** k[0], 32), 7000 + i) for i, k in enumerate(keys)}
    kidx = rng.integers(len(keys), size=nreq)
    nrhs = rng.integers(1, 33, size=nreq)
    ex = GpuExecutor({k: plans[k] for k in keys}, max_batch_rhs=max_batch, refine=1, use_graphs=graphs,
                     use_multi=multi, trim=trim)

    def make(times):
        return [ServeRequest(j, keys[kidx[j]], float(times[j]), pools[keys[kidx[j]]][:, :nrhs[j]])
                for j in range(nreq)]

    sch = Scheduler(ex, hbm_budget=200 << 30, max_batch_rhs=max_batch)
    for k in keys:
        if not sch.register(k):
            raise RuntimeError("key %s does not fit the HBM budget" % (k,))
    log("serving: saturation burst of %d requests" % nreq)
    t0 = time.perf_counter()
    sch.run(make(np.zeros(nreq)))
    sat = nreq / (time.perf_counter() - t0)
    out = {"saturation_req_per_s": sat, "keys": len(keys), "requests": nreq, "graphs": graphs, "multi": multi,
           "rates": []}
    for frac in fracs:
        sch.finished = []
        sch.batches_started = sch.groups_started = 0
        times = np.cumsum(rng.exponential(1.0 / (frac * sat), nreq))
        done = sch.run(make(times))
        st = latency_stats(done)
        rec = {"rate_frac": frac, "req_per_s": frac * sat, "p50_ms": st["p50_ms"],
               "p99_ms": st["p99_ms"], "rhs_n_per_s": throughput(done),
               "batches": sch.batches_started, "multi_groups": sch.groups_started, "per_key": {}}
        for k in keys:  # the tail by key: large keys' batches run longest
            dk = [r for r in done if r.key == k]
            if dk:
                sk = latency_stats(dk)
                rec["per_key"]["%dd_n%d_eps%g" % (k[0], k[1], k[3])] = {
                    "requests": len(dk), "p50_ms": round(sk["p50_ms"], 3), "p99_ms": round(sk["p99_ms"], 3)}
        log("serving at %.2f x saturation: p50 %.2f ms, p99 %.2f ms, %.3e RHS*N/s" % (
            frac, st["p50_ms"], st["p99_ms"], rec["rhs_n_per_s"]))
        out["rates"].append(rec)
    return out


def build_plans(F, keys, have=None):
    plans = dict(have or {})
    for k in keys:
        if k in plans:
            continue
        t0 = time.perf_counter()
        plans[k] = F.fio_build(F.make_problem(k[0], k[1], k[2], eps=k[3], device=0))
        log("built %s in %.1f s" % (k, time.perf_counter() - t0))
    return plans


def serve_main(args):
    import torch  # noqa: F401
    from paper_2105_02995_amd import fio as F
    plans = build_plans(F, SERVE_KEYS_FULL)
    res = serving_run(F, plans, SERVE_KEYS_FULL, args.serve_requests, (0.5, 0.8, 0.95), 2000,
                      multi=not args.no_multi, trim=True)
    head = res["rates"][1]
    out = {"metric": "serving mix: p50/p99 latency and RHS*N/s of factored FIO solves",
           "value": head["rhs_n_per_s"], "unit": "RHS*N/s", "n_gpus": 1,
           "higher_is_better": True, "data": "synthetic",
           "config": {"workload": "Poisson arrivals over %d resident keys (1D N=1024..65536 at eps 1e-4/1e-6, "
                                  "2D n=32,64,128,256 at eps 1e-4), 1-32 RHS per request, complex64 + 1 FP64 "
                                  "refinement step, HIP-graph replay, plans trimmed to the images the solve "
                                  "uses" % len(SERVE_KEYS_FULL)},
           "serving": res}
    print(json.dumps(out), flush=True)


VNAME = {1: (1, 4), 2: (2, 4), 3: (1, 2), 4: (2, 2), 5: (1, 1), 6: (2, 1), 8: (4, 4), 9: (4, 2)}
PAIR_NT = {1: 1, 2: 2, 3: 4}
PAIR_STACKED = 4  # fused pair with sibling blocks stacked into one operand


def chain_timing(F, plan, torch, dtype, op, nrhs, reps=5):
    """Every launch of one chain apply (op = K or KH) as the library schedules it
    (single stages and fused stage pairs), timed with HIP events on the launch
    stream.  Returns one dict per launch: kernel instance name, average ms,
    algorithmic flops (8 per complex multiply-add of the block products) and
    algorithmic HBM bytes: the factor entries of the launch's stages read once,
    plus the chain's input vector (first launch) and output vector (last launch);
    the coefficient vectors passed between launches are an implementation cost,
    not algorithmic work."""
    st = F.fio_plan_stats(plan)
    S = st["n_stages"]
    N = st["n"] ** st["d"]
    fwd_info = [F.fio_stage_info(plan, s) for s in range(S)]

    def io(k):
        """stage k of the chain of op: its factor info, input and output entry counts"""
        f = k if op == F.FIO_OP_K else S - 1 - k
        i = fwd_info[f]
        rows_o = i["n_out"] * i["r_out"]
        rows_i = N if f == 0 else fwd_info[f - 1]["n_out"] * fwd_info[f - 1]["r_out"]
        return (i, rows_i, rows_o) if op == F.FIO_OP_K else (i, rows_o, rows_i)
    csize = 8 if dtype == F.FIO_C64 else 16
    r = "float" if dtype == F.FIO_C64 else "double"
    sched = F.fio_chain_schedule(plan, op, dtype, nrhs)
    maxlen = max(max(max(io(k)[1], io(k)[2]) for k in range(S)), N)
    ctype = torch.complex64 if dtype == F.FIO_C64 else torch.complex128
    a = torch.randn(maxlen * nrhs, dtype=ctype, device="cuda")
    b = torch.zeros_like(a)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in sched]
    tot = np.zeros(len(sched))
    for rep in range(reps):
        for j, (first, count, v) in enumerate(sched):
            ev[j][0].record(stream)
            if count == 3:
                F.fio_stage_triple_apply(plan, op, first, dtype, a, b, nrhs, stream)
            elif count == 2:
                F.fio_stage_pair_apply(plan, op, first, dtype, a, b, nrhs, stream)
            else:
                F.fio_stage_apply(plan, op, first, dtype, a, b, nrhs, stream)
            ev[j][1].record(stream)
            a, b = b, a
        torch.cuda.synchronize()
        if rep > 0:
            tot += np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    tot /= max(reps - 1, 1)
    out = []
    for j, (first, count, v) in enumerate(sched):
        ks = list(range(first, first + count))
        flops = sum(8.0 * io(k)[0]["nnz"] * nrhs for k in ks)
        byts = sum(io(k)[0]["nnz"] * csize for k in ks)
        if j == 0:
            byts += N * nrhs * csize
        if j == len(sched) - 1:
            byts += N * nrhs * csize
        moved = sum(io(k)[0]["nnz"] * csize + 4 * io(k)[0]["n_out"] * io(k)[0]["fan"] for k in ks)
        moved += (io(ks[0])[1] + io(ks[-1])[2]) * nrhs * csize
        if count == 3:
            name = "k_stage3s_mfma<%s, %d, %d>" % (r, 2 if dtype == F.FIO_C64 else 1,
                                                   3 if max(io(k)[0]["r_out"] if op == F.FIO_OP_K else io(k)[0]["r_in"]
                                                            for k in ks) <= 24 else 4)
        elif count == 2 and v == PAIR_STACKED:
            rmax = max(io(k)[0]["r_out"] if op == F.FIO_OP_K else io(k)[0]["r_in"] for k in ks)
            name = "k_stage2s_mfma<%s, %d, %d>" % (r, 2 if dtype == F.FIO_C64 else 1, 3 if rmax <= 24 else 4)
        elif count == 2:
            mt = 2 if max(io(k)[0]["r_out"] if op == F.FIO_OP_K else io(k)[0]["r_in"] for k in ks) > 16 else 1
            name = "k_stage2_mfma<%s, %d, %d>" % (r, mt, PAIR_NT[v])
        elif v == 0:
            name = "k_stage<%s2>" % r
        elif v == 7:
            name = "k_stage_nb<%s2>" % r
        elif v in (12, 13, 14):
            name = "k_stage_mfma<%s, %d, %d, 3M>" % ((r,) + {12: (2, 4), 13: (4, 2), 14: (2, 2)}[v])
        elif v in (10, 11):
            ro = io(ks[0])[0]["r_out"] if op == F.FIO_OP_K else io(ks[0])[0]["r_in"]
            name = "k_stage_lds<%s, %d, %d>" % (r, 1 if ro <= 64 else (2 if ro <= 128 else 3), 4 if v == 10 else 2)
        else:
            name = "k_stage_mfma<%s, %d, %d>" % ((r,) + VNAME[v])
        out.append({"name": name, "ms": float(tot[j]), "flops": flops, "bytes": float(byts),
                    "launch_io_bytes": float(moved), "stages": ks})
    return out


def calibration():
    """Measured ceilings of the device (paper_2105_02995_amd/fio_calibrate, a child
    process): streaming read rate and register-only FP32/FP64 matrix-core loop rates,
    beside the published peaks the roofline fractions use."""
    import subprocess
    exe = os.path.join(ROOT, "paper_2105_02995_amd", "fio_calibrate")
    out = {}
    for mode in ("read", "mfma"):
        try:
            r = subprocess.run([exe, mode], capture_output=True, text=True, timeout=120)
        except (OSError, subprocess.TimeoutExpired) as exc:
            log("calibration %s: %s" % (mode, exc))
            return None
        if r.returncode != 0:
            log("calibration %s failed: %s" % (mode, r.stderr.strip()))
            return None
        parse_calibration(r.stdout.splitlines(), out)
    log("calibration: %s" % out)
    return out


def parse_calibration(lines, out=None):
    """The figures of fio_calibrate's output lines: the best streaming-read rate over
    its launch shapes (TB/s) and the matrix-core loop rates (TFLOP/s)."""
    import re
    out = {} if out is None else out
    for line in lines:
        m = re.match(r"read: .* (\d+) workgroups, ([0-9.]+) TB/s", line)
        if m:
            out["read_tbs"] = max(out.get("read_tbs", 0.0), float(m.group(2)))
        m = re.match(r"mfma (f32|f64) 16x16x4: ([0-9.]+) TFLOP/s", line)
        if m:
            out["mfma_loop_%s_tflops" % m.group(1)] = float(m.group(2))
    return out


def oracle_leg(F, torch, plan, wl, stream, refine, ncol=4, mode="refine"):
    """The FP64 oracle on a bounded sample of the workload (CPU, all cores).

    1. Known truth: fhat for `ncol` columns (seeded Gaussian) and u = K fhat by the
       oracle's direct summation (section 1, eq6) at full N; this product is timed.
    2. The GPU solves (untimed) a full batch whose columns spread over it carry
       these u; the max relative error against fhat is rel_err_vs_oracle.
    3. CPU baseline: the oracle's solve at this N is CG on K^*K with
       direct-summation products (section 6, eq_NR_1), 2 products per iteration
       plus K^* u.  Its rate is extrapolated from the timed product and the
       oracle's own CG count at the small size of the same example (dense K).
       A dense LU solve of the small size (K formation, LU, all right-hand
       sides) is timed as a measured point.
    """
    import oracle as O
    N, B = wl.N, wl.nrhs
    ncol = min(ncol, B)
    p = O.OracleProblem(wl.d, wl.n, wl.phase, wl.c_div)
    fh = gaussian_complex((N, ncol), wl.seed + 100)
    log("oracle: direct summation u = K fhat, N=%d, %d columns ..." % (N, ncol))
    t0 = time.perf_counter()
    u_true = O.apply_direct(p, fh)
    t_prod = time.perf_counter() - t0
    log("oracle: %.1f s" % t_prod)
    u = gaussian_complex((N, B), wl.seed + 101)
    cols = np.unique(np.linspace(0, B - 1, ncol).round().astype(np.int64))
    u[:, cols] = u_true
    U = torch.from_numpy(np.ascontiguousarray(u.T)).cuda()
    X = torch.zeros_like(U)
    if mode == "pcg":
        F.fio_solve(plan, F.FIO_SOLVE_PCG, F.FIO_C128, U, X, B, N, tol=1e-8, maxit=200, precondition=1,
                    stream=stream)
    else:
        F.fio_solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, U, X, B, N, tol=0.0, maxit=refine, stream=stream,
                    want_info=False)
    torch.cuda.synchronize()
    x = X.cpu().numpy().T
    finite = bool(np.isfinite(x).all())
    err = O.rel_err(x[:, cols], fh) if finite else np.full(len(cols), np.inf)
    # the oracle's CG count and a measured dense solve at the small size: K formation,
    # LU and the solves, median of 3 with the BLAS on all its threads, and once with
    # one thread
    small_n = min(wl.n, 4096 if wl.d == 1 else 64)
    ps = O.OracleProblem(wl.d, small_n, wl.phase, wl.c_div)
    Ns = ps.N
    us = gaussian_complex((Ns, B), wl.seed + 102)

    def dense_solve():
        t0 = time.perf_counter()
        Kd = O.dense_K(ps)
        O.solve_dense(ps, us, Kd)
        return time.perf_counter() - t0, Kd

    from threadpoolctl import threadpool_info, threadpool_limits
    blas_threads = max([i.get("num_threads", 0) for i in threadpool_info()] or [0])
    runs = [dense_solve() for _ in range(3)]
    t_lu = float(np.median([r[0] for r in runs]))
    K = runs[0][1]
    del runs
    with threadpool_limits(limits=1):
        t_lu1, _ = dense_solve()
    _, iters = O.cg_normal(lambda v: K @ v, lambda v: K.conj().T @ v, gaussian_complex(Ns, 99), tol=1e-8)
    del K
    per_solve = (2 * iters + 1) * t_prod          # ncol right-hand sides
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    base = {"value": ncol * N / per_solve, "unit": "RHS*N/s", "cores": cores, "kind": "oracle, extrapolated",
            "sample": "one direct-summation product K fhat on %d RHS at N=%d (%.1f s, timed), times %d products "
                      "of the oracle's CG on K^*K (%d iterations: the oracle's CG count at %s, same phase, "
                      "to 1e-8)" % (ncol, N, t_prod, 2 * iters + 1, iters,
                                    "N=%d" % small_n if wl.d == 1 else "n=%d" % small_n),
            "measured_small": {"value": B * Ns / t_lu, "unit": "RHS*N/s", "seconds": t_lu,
                               "blas_threads": blas_threads, "os_cpu_count": os.cpu_count(),
                               "sample": "dense LU oracle solve at %s (N=%d): K formation, LU, %d RHS; "
                                         "median of 3" % ("N=%d" % small_n if wl.d == 1 else "2D n=%d" % small_n,
                                                          Ns, B)},
            "measured_small_1thread": {"value": B * Ns / t_lu1, "unit": "RHS*N/s", "seconds": t_lu1,
                                       "blas_threads": 1, "sample": "the same solve, BLAS limited to one thread"}}
    check = {"rel_err_vs_oracle": float(err.max()), "rel_err_median": float(np.median(err)),
             "columns": [int(c) for c in cols], "bound": 10 * wl.eps, "finite": finite}
    return base, check


def measure_serving(F, wl, plan, args):
    """Small serving leg: Poisson arrivals over a few resident keys including the
    workload's own plan, at 0.8 of the measured saturation rate."""
    key = (wl.d, wl.n, wl.phase, wl.eps)
    keys = list(SERVE_KEYS_SMALL)
    if key not in keys:
        keys.append(key)
    plans = build_plans(F, keys, {key: plan})
    try:
        return serving_run(F, plans, keys, 400, (0.8,), 2000, multi=not args.no_multi)
    finally:
        for k, pl in plans.items():
            if pl is not plan:
                pl.close()


def roofline_of(F, torch, plan, stats, B, refine, mode="refine"):
    """Dominant butterfly kernel instance of the step and its roofline figures.
    The complex64 adjoint chain runs twice per step, the complex128 forward chain
    once per refinement step.  The bound is the roof the instance reaches first:
    HBM if its algorithmic bytes take longer at 8 TB/s than its flops at the
    matrix-core peak of its precision."""
    if mode == "pcg":  # every iteration applies Kd and Kd^* in complex128
        legs = ((chain_timing(F, plan, torch, F.FIO_C128, F.FIO_OP_KH, B), 1, PEAK_TFLOPS["c128"]),
                (chain_timing(F, plan, torch, F.FIO_C128, F.FIO_OP_K, B), 1, PEAK_TFLOPS["c128"]))
    else:
        legs = ((chain_timing(F, plan, torch, F.FIO_C64, F.FIO_OP_KH, B), 2, PEAK_TFLOPS["c64"]),
                (chain_timing(F, plan, torch, F.FIO_C128, F.FIO_OP_K, B), refine, PEAK_TFLOPS["c128"]))
    l64, l128 = legs[0][0], legs[1][0]
    n64, n128 = ("c128_KH", "c128_K") if mode == "pcg" else ("c64_KH", "c128_K")
    inst = {}
    for launches, weight, pk in legs:
        for ln in launches:
            e = inst.setdefault(ln["name"], {"l": [], "w": weight, "pk": pk})
            e["l"].append(ln)
    best = max(inst, key=lambda n: inst[n]["w"] * sum(x["ms"] for x in inst[n]["l"]))
    e = inst[best]
    tms = np.array([x["ms"] for x in e["l"]])
    fl = np.array([x["flops"] for x in e["l"]])
    by = np.array([x["bytes"] for x in e["l"]])
    pk = e["pk"]
    tf = fl.sum() / (tms.sum() * 1e-3) / 1e12
    gbs = by.sum() / (tms.sum() * 1e-3) / 1e9
    hbm_bound = by.sum() / (PEAK_HBM_GBS * 1e9) >= fl.sum() / (pk * 1e12)
    traffic = traffic_for(best, stats["bf_nnz"])
    roof = {"bound": "hbm" if hbm_bound else "mfma",
            "achieved": round(gbs if hbm_bound else tf, 3),
            "peak": PEAK_HBM_GBS if hbm_bound else pk,
            "unit": "GB/s" if hbm_bound else "TFLOP/s",
            "frac": round((gbs / PEAK_HBM_GBS) if hbm_bound else (tf / pk), 4),
            "traffic": traffic, "kernel": best,
            "traffic_over_algorithmic": round(traffic / float(by.mean()), 3) if traffic else None,
            "mfma_counters": mfma_counters_for(best, stats["bf_nnz"], float(tms.mean()), pk),
            "launches_per_chain": len(e["l"]),
            "avg_launch_ms": round(float(tms.mean()), 5),
            "flops_per_launch": float(fl.mean()), "bytes_per_launch": float(by.mean()),
            "intensity_flop_per_byte": round(float(fl.sum() / by.sum()), 2),
            "other_roof": {"mfma_tflops": round(tf, 3), "mfma_frac": round(tf / pk, 4),
                           "hbm_gbs": round(gbs, 1), "hbm_frac": round(gbs / PEAK_HBM_GBS, 4)},
            "chain_ms": {n64: round(sum(x["ms"] for x in l64), 4),
                         n128: round(sum(x["ms"] for x in l128), 4)},
            "chain_tflops": {n64: round(sum(x["flops"] for x in l64) / (sum(x["ms"] for x in l64) * 1e9), 2),
                             n128: round(sum(x["flops"] for x in l128) / (sum(x["ms"] for x in l128) * 1e9), 2)},
            "chain_bytes": {n64: {"algorithmic": sum(x["bytes"] for x in l64),
                                  "launch_io": sum(x["launch_io_bytes"] for x in l64)},
                            n128: {"algorithmic": sum(x["bytes"] for x in l128),
                                   "launch_io": sum(x["launch_io_bytes"] for x in l128)}},
            "instances": {n: {"launches": len(v["l"]), "ms_per_chain": round(sum(x["ms"] for x in v["l"]), 4)}
                          for n, v in inst.items()}}
    log("roofline: %s avg %.4f ms/launch over %d launches: %.2f TFLOP/s (%.1f%% of %.1f), "
        "%.0f GB/s (%.1f%% of HBM), bound %s" % (best, tms.mean(), len(e["l"]), tf, 100 * tf / pk, pk,
                                                 gbs, 100 * gbs / PEAK_HBM_GBS, roof["bound"]))
    log("chains: %s %.4f ms (%.1f TFLOP/s), %s %.4f ms (%.1f TFLOP/s)" % (
        n64, roof["chain_ms"][n64], roof["chain_tflops"][n64], n128, roof["chain_ms"][n128],
        roof["chain_tflops"][n128]))
    return roof


def plain_fp64(F, torch, plan, U, N, stream, ncols=16, tune=True):
    """Plain FP64 path: complex128 factors, one right-hand side per call, direct
    solve (Gd Kd^* u), with the kernels autotuned for that width as the batched
    path is for its own (tune=False: the library's default choices)."""
    if tune:
        t0 = time.perf_counter()
        F.fio_autotune(plan, F.FIO_C128, 1, 3, stream)
        log("autotuned the single-RHS FP64 path in %.1f s" % (time.perf_counter() - t0))
    Uc = [U[j % U.shape[0]:j % U.shape[0] + 1].contiguous() for j in range(ncols)]  # workloads of < ncols RHS cycle
    Xc = [torch.zeros_like(Uc[0]) for _ in range(ncols)]
    for j in range(2):
        F.fio_solve(plan, F.FIO_SOLVE_DIRECT, F.FIO_C128, Uc[j], Xc[j], 1, N, stream=stream, want_info=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j in range(ncols):
        F.fio_solve(plan, F.FIO_SOLVE_DIRECT, F.FIO_C128, Uc[j], Xc[j], 1, N, stream=stream, want_info=False)
    torch.cuda.synchronize()
    tp = time.perf_counter() - t0
    st = F.fio_plan_stats(plan)
    # algorithmic bytes of one complex128 direct solve: the Kd^* factors, the Gd
    # factors twice (the up sweep reads T^*, L^-1, M and the down sweep M^*, L^-*, T;
    # the triangle of L^-1 only), the root block, and u in / fhat out
    byts = (st["bf_nnz"] + 2 * st["hif_sweep_nnz"] + st["root_size"] ** 2 + 2 * N) * 16
    tp_entry = counted(PLAIN_TRAFFIC, "plain_fp64", st["bf_nnz"])
    traffic_plain = None if tp_entry is None else tp_entry["bytes"]
    gbs = byts / (tp / ncols) / 1e9
    out = {"value": ncols * N / tp, "ms_per_rhs": 1000 * tp / ncols, "dtype": "c128", "nrhs_per_call": 1,
           "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                        "frac": round(gbs / PEAK_HBM_GBS, 4), "bytes_per_rhs": byts,
                        "traffic": traffic_plain, "traffic_over_algorithmic":
                            None if traffic_plain is None else round(traffic_plain / byts, 3),
                        "what": "whole direct solve (every launch of Kd^*, Gd and layout)"}}
    log("plain FP64 single-RHS: %.3f ms/RHS, %.3e RHS*N/s, %.0f GB/s of factor bytes" % (
        1000 * tp / ncols, out["value"], gbs))
    return out


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the factored solve is measured on a single "
              "MI355X (sharding over several GPUs is described, not implemented)", file=sys.stderr)
        sys.exit(2)
    if args.serve:
        return serve_main(args)
    import torch
    from paper_2105_02995_amd import fio as F

    wl = WORKLOADS[args.workload]
    N, B = wl.N, wl.nrhs
    log("workload %s: d=%d n=%d N=%d nrhs=%d eps=%g" % (wl.name, wl.d, wl.n, N, B, wl.eps))
    t0 = time.perf_counter()
    if args.plan_file and os.path.exists(args.plan_file):
        plan = F.fio_load(args.plan_file, 0)
        log("loaded %s in %.1f s" % (args.plan_file, time.perf_counter() - t0))
    else:
        # large 2D builds take a while: print their progress
        plan = F.fio_build(F.make_problem(wl.d, wl.n, wl.phase, eps=wl.eps, c_div=wl.c_div, device=0,
                                          verbose=1 if wl.N * wl.d >= 2 * 65536 else 0))
        if args.plan_file:
            F.fio_save(plan, args.plan_file)
            log("saved the factors to %s" % args.plan_file)
    build_s = time.perf_counter() - t0
    stats = F.fio_plan_stats(plan)
    log("built in %.1f s: bf_nnz=%d hif_nnz=%d root=%d device_bytes=%.2f GB" % (
        build_s, stats["bf_nnz"], stats["hif_nnz"], stats["root_size"], stats["device_bytes"] / 1e9))

    u = gaussian_complex((N, B), wl.seed)
    U = torch.from_numpy(np.ascontiguousarray(u.T)).cuda()
    X = torch.zeros_like(U)
    stream = torch.cuda.current_stream()
    if args.plain_only:
        print(json.dumps({"workload": wl.name, "plain_fp64_single_rhs": plain_fp64(F, torch, plan, U, N, stream,
                                                                                tune=not args.plain_untuned)}),
              flush=True)
        plan.close()
        return

    if not args.no_tune:
        t0 = time.perf_counter()
        F.fio_autotune(plan, F.FIO_C64, B, 3, stream)
        F.fio_autotune(plan, F.FIO_C128, B, 3, stream)
        log("autotuned stage kernels for %d RHS in %.1f s" % (B, time.perf_counter() - t0))

    def solve(Uin, Xout):
        if args.mode == "pcg":
            return F.fio_solve(plan, F.FIO_SOLVE_PCG, F.FIO_C128, Uin, Xout, B, N, tol=1e-8, maxit=200,
                               precondition=1, stream=stream)
        return F.fio_solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, Uin, Xout, B, N, tol=0.0, maxit=args.refine,
                           stream=stream, want_info=False)

    def step():
        solve(U, X)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    if args.trace:
        F.fio_set_trace(True)
    t0 = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record(stream)
        step()
        evs[k][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    if args.trace:
        F.fio_set_trace(False)
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    ms = 1000.0 * elapsed / args.steps
    value = B * N / (elapsed / args.steps)
    log("timed %d steps: %.3f ms/step, %.3e RHS*N/s" % (args.steps, ms, value))
    its, corr = F.fio_solve(plan, F.FIO_SOLVE_REFINE, F.FIO_C64, U, X, B, N, tol=0.0,
                            maxit=args.refine, stream=stream)
    pcg = None
    if args.mode == "pcg":
        # iterations with Gd, and the same solve with Kd^* alone (no preconditioner)
        its_g, res_g = F.fio_solve(plan, F.FIO_SOLVE_PCG, F.FIO_C128, U, X, B, N, tol=1e-8, maxit=200,
                                   precondition=1, stream=stream)
        X0 = torch.zeros_like(U)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        its_0, res_0 = F.fio_solve(plan, F.FIO_SOLVE_PCG, F.FIO_C128, U, X0, B, N, tol=1e-8, maxit=200,
                                   precondition=0, stream=stream)
        torch.cuda.synchronize()
        t_0 = time.perf_counter() - t1
        pcg = {"tol": 1e-8, "iters_with_gd": its_g, "rel_resid_with_gd": res_g, "iters_kd_only": its_0,
               "rel_resid_kd_only": res_0, "ms_kd_only": 1000 * t_0}
        log("pcg: %d iterations with Gd (rel resid %.2e), %d with Kd^* alone (%.1f ms)"
            % (its_g, res_g, its_0, 1000 * t_0))
        del X0

    # optional spatial output f = n^d F* fhat of the batch (not part of the step)
    Fs = torch.empty_like(X)
    F.fio_inverse_dft(plan, X, Fs, B, N, stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(5):
        F.fio_inverse_dft(plan, X, Fs, B, N, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    spatial_ms = e0.elapsed_time(e1) / 5
    del Fs
    log("spatial output (inverse DFT of the batch): %.4f ms" % spatial_ms)

    roof = roofline_of(F, torch, plan, stats, B, args.refine, args.mode)
    plain = None if args.no_plain else plain_fp64(F, torch, plan, U, N, stream, tune=not args.plain_untuned)
    del X
    serving = None if args.no_serve else measure_serving(F, wl, plan, args)

    calib = None if args.no_calibration else calibration()
    cpu, check = None, None
    if not args.no_cpu_baseline:
        cpu, check = oracle_leg(F, torch, plan, wl, stream, args.refine, mode=args.mode)
        log("oracle check: max rel err %.3e over columns %s (bound %.1e); cpu baseline %.3e RHS*N/s on %d cores"
            % (check["rel_err_vs_oracle"], check["columns"], check["bound"], cpu["value"], cpu["cores"]))

    ok = check is None or (check["finite"] and check["rel_err_vs_oracle"] <= check["bound"])
    out = {
        "metric": "RHS*N/s of factored FIO inverse solve at rel err <= 10 eps; p50/p99 latency",
        "value": value if ok else None, "unit": "RHS*N/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128" if args.mode == "pcg" else "c64+f64", "data": "synthetic",
        "config": {"workload": "%s: %s, N=%d, %d RHS, eps=%g, %s"
                               % (wl.name, "1D FIO Example 1 phase c(x)=(2+sin 2pi x)/16" if wl.d == 1 else
                                  "2D FIO Example 3 (generalized Radon phase), n=%d" % wl.n,
                                  N, B, wl.eps,
                                  "CG on Kd^*Kd preconditioned by Gd to 1e-8, complex128 applies"
                                  if args.mode == "pcg" else
                                  "complex64 applies + %d FP64 refinement step(s)" % args.refine),
                   "N": N, "nrhs": B, "eps": wl.eps, "mode": args.mode},
        "rel_err_vs_oracle": check,
        "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99)),
                       "what": "per-step (%d-RHS batch) latency, HIP events" % B},
        "serving": serving,
        "last_correction_rel": corr,
        "pcg": pcg,
        "spatial_output_ms": spatial_ms,
        "roofline": roof,
        "cpu_baseline": cpu,
        "plain_fp64_single_rhs": plain,
        "speedup_vs_plain": (value / plain["value"]) if plain else None,
        "calibration": calib,
        "build_seconds": build_s,
        "plan": {k: stats[k] for k in ("bf_nnz", "hif_nnz", "root_size", "max_rank_bf",
                                       "max_rank_h", "device_bytes", "L")},
    }
    print(json.dumps(out), flush=True)
    plan.close()
    if not ok:
        log("rel_err_vs_oracle %.3e exceeds 10 eps = %.1e: no value reported"
            % (check["rel_err_vs_oracle"], check["bound"]))
        sys.exit(1)


if __name__ == "__main__":
    main()
