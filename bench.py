"""Benchmark of the low-rank IgA optimal-control hot path on one MI355X.

One step = the whole path on the perturbed-cube workload, in FP64: TT assembly of the
Kronecker factors of M and K (assemble_factors), the KKT operator (kkt_create) and the
block-AMEn solve (amen_solve) to tolerance 1e-6. Workload: unit cube whose 8x8x8 cubic
control net carries a seeded smooth perturbation of amplitude 0.1, degree 3, n = 128 free
dofs per direction (2,097,152 dofs per field, 6,291,456 KKT unknowns), beta = 1e-6, Fourier
desired state, weight TT tolerance 1e-6. Inputs (control points, desired-state TT cores)
are seeded and synthetic and are uploaded before the timed region. Every solve's status
and FP64 KKT residual is checked: a step whose solve did not converge, or whose residual is
above 1e-6, marks the line invalid ("valid": false) and names the step.

Printed JSON line:
  value      local TT-matvec GFLOP/s inside the timed solves: algorithmic flops of every
             projected local matvec (banded middle stage counted over the band and the
             nonzero rank blocks) / their GPU time (HIP events on the library stream);
  solve_time_s, assembly_time_s, kkt_residual, statuses, per-part solve times, ranks;
  mixed_vs_fp64  the same solve in the mixed forms (FP32 local contractions, or BF16
             products with FP32 accumulation, inside FP64 iterative refinement) and in
             FP64, from one assembly: solve times, statuses, residuals, state differences
             against the FP64 form, speedups (null for a form whose solve is invalid);
  annulus_n64  the twisted-annulus workload at n = 64 (FP64, tol 1e-7): one step's times;
  annulus_n256  the twisted annulus at n = 256 (16.7 M dofs per field, tol 1e-6): the solve
             with ranks capped at 40 (stops above tolerance with IGA_ERANK), the uncapped
             solve, and the times of the reduced cost, its desired-state gradient and its
             control-point gradient at the uncapped solution (differentiation form);
  batching   64 uneven local TT-matvecs, one call per problem versus one batched call;
  time_dependent  the time-dependent KKT system on the annulus geometry and desired state
             with 10 implicit Euler steps (3 x 10 x 64^3 = 7.9 M unknowns), AMEn to 1e-6:
             FP64 solve time, residual, ranks, time parts; the FP32 and BF16 forms' solve
             times, residuals and state differences against FP64;
  in_solve_band_stage  the banded middle stage of the local matvecs inside the timed solves
             (HIP events recorded by the library on its stream around every such stage);
  roofline   the dominant kernel of the local TT-matvec at the workload's microbenchmark
             shape (r, R_M, R_K, n, p) = (40, 15, 80, 128, 3): the banded middle stage of
             the K operator, timed by the library with HIP events on its stream; traffic
             from the committed rocprofv3 counter summary when it was taken from the current
             kernel source, else null; beside it the whole local matvec's fraction of peak;
  cpu_baseline  the oracle's local TT-matvec (numpy FP64) at the same shape, timed on the
             host cores of this machine on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (matrix cores)
PEAK_FP32_TFLOPS = 157.3  # MI355X dense FP32 (matrix cores)
PEAK_BF16_TFLOPS = 2500.0  # MI355X dense BF16 (matrix cores)
MICRO = dict(r=40, RM=15, RK=80, n=128, p=3)
WORKLOAD = "perturbed_cube_n128"
SECONDARY = "annulus_n64"
RES_BAR = 1e-6  # KKT relative residual every timed solve must reach
COPY_BYTES = 256 << 20
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "band_stage_K_n128shape_traffic.txt")
KERNEL_SOURCES = ["paper_1811_06797_amd/csrc/k_gemm.hip", "paper_1811_06797_amd/csrc/localop.cpp"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--micro-iters", type=int, default=20)
    ap.add_argument("--solve-only", action="store_true",
                    help="one step (assembly and solve) of the workload and its statistics, for tracing")
    ap.add_argument("--workload", default=WORKLOAD,
                    help="workload of --solve-only (perturbed_cube_n128, annulus_n64, annulus_n256, cube_n16)")
    ap.add_argument("--precision", default="FP64", choices=["FP64", "FP32", "BF16"],
                    help="precision form of --solve-only")
    ap.add_argument("--micro-only", action="store_true",
                    help="only the local TT-matvec microbenchmark and the reference copy (for counter runs)")
    return ap.parse_args()


# the dominant kernel of the local matvec at the microbenchmark shape: the banded stage of the
# K operator (R = 80: an 80-row register-staged tile, one tile per 80 operator ranks)
ROOFLINE_KERNEL = "gemm2_kernel"


def solve_ok(rc, st):
    """A timed solve counts only if it converged and its FP64 KKT residual meets the bar."""
    return rc == 0 and st.get("converged", 0) == 1 and st["residual"] <= RES_BAR


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per launch of the dominant kernel from the committed counter summary, if it
    was taken from the current kernel sources (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m_hash = re.search(r"^source_hash:\s*(\S+)", txt, re.M)
    m_bytes = re.search(r"^traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt, re.M)
    if not (m_hash and m_bytes) or m_hash.group(1) != kernel_source_hash():
        return None
    return float(m_bytes.group(1))


def mixed_compare(iga, ctx, torch, geo, c, Y, steps):
    """The workload's solve in the mixed forms (FP32 local contractions or BF16 products, FP64
    refinement) and in FP64 from the same assembled operators: solve times, residuals, state
    differences."""
    n, p, beta = c["n"], c["degree"], c["beta"]
    M, K, _ = iga.assemble_factors(ctx, geo, p, n, weight_tol=c["weight_tol"])
    kk = iga.kkt_create(ctx, M, K, beta)
    out = {}
    fulls = {}
    for name, prec in (("fp64", iga.FP64), ("mixed", iga.FP32), ("mixed_bf16", iga.BF16)):
        times, sts, rcs = [], [], []
        for i in range(steps + 1):  # the first solve is a warm-up
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol, st, rc = iga.amen_solve(ctx, kk, Y, c["tol"], precision=prec)
            t1 = time.perf_counter()
            if i > 0:
                times.append(t1 - t0)
                sts.append(st)
                rcs.append(rc)
            if i == steps:
                fulls[name] = iga.btt_to_full(ctx, sol)[0].cpu().numpy()
            iga.btt_destroy(sol)
        last = sts[-1]
        d = {"solve_time_s": sum(times) / len(times), "kkt_residual": max(x["residual"] for x in sts),
             "status": rcs, "converged": [x["converged"] for x in sts],
             "valid": all(solve_ok(r_, x) for r_, x in zip(rcs, sts)),
             "half_sweeps": last["half_sweeps"], "ranks": last["ranks"], "local_iterations": last["local_iterations"]}
        for part in ("t_local_matvec", "t_local_matvec_fp32", "t_interfaces", "t_svd", "t_precond", "t_krylov_other",
                     "t_residual"):
            d[part] = sum(x[part] for x in sts) / len(sts)
        if prec != iga.FP64:
            d["refinements"] = last["refinements"]
            d["local_matvecs_fp32"] = last["local_matvecs_fp32"]
            d["local_matvec_gflops_fp32"] = (sum(x["local_matvec_flops_fp32"] for x in sts)
                                             / sum(x["t_local_matvec_fp32"] for x in sts) / 1e9)
        d["local_matvec_gflops_fp64"] = (sum(x["local_matvec_flops"] for x in sts)
                                         / sum(x["t_local_matvec"] for x in sts) / 1e9)
        out[name] = d
    import numpy as np
    y64 = fulls["fp64"]
    for name in ("mixed", "mixed_bf16"):
        yl = fulls[name]
        out[name]["state_rel_diff_vs_fp64"] = float(np.linalg.norm(yl - y64) / np.linalg.norm(y64))
        both = out[name]["valid"] and out["fp64"]["valid"]
        out[name]["speedup_vs_fp64"] = out["fp64"]["solve_time_s"] / out[name]["solve_time_s"] if both else None
    iga.kkt_destroy(kk)
    iga.ttop_destroy(M)
    iga.ttop_destroy(K)
    return out


def n256_leg(iga, ctx, torch):
    """The differentiation form's workload: twisted annulus, degree 3, n = 256 (16.7 M dofs per
    field), beta = 1e-6, tol 1e-6. With the ranks capped at 40 the solve stops above tolerance
    (IGA_ERANK; residual reached and ranks reported); uncapped it converges, and on that solution
    the reduced cost, its desired-state gradient and its control-point gradient are timed."""
    import numpy as np
    import synth
    geo, yc, c = synth.config("annulus_n256")
    n, p, beta = c["n"], c["degree"], c["beta"]
    Y = iga.tt_create(ctx, yc)
    M, K, _ = iga.assemble_factors(ctx, geo, p, n, weight_tol=c["weight_tol"])
    kk = iga.kkt_create(ctx, M, K, beta)
    out = {"config": c["name"] + ", beta %g, weight tol %g, tol %g" % (beta, c["weight_tol"], c["tol"])}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol, st, rc = iga.amen_solve(ctx, kk, Y, c["tol"], r_max=c["r_max"])
    out["capped"] = {"r_max": c["r_max"], "status": rc, "solve_time_s": time.perf_counter() - t0,
                     "kkt_residual": st["residual"], "max_local_residual": st["max_local_residual"],
                     "ranks": st["ranks"], "half_sweeps": st["half_sweeps"]}
    iga.btt_destroy(sol)
    sol, st, rc = iga.amen_solve(ctx, kk, Y, c["tol"])  # warm-up
    iga.btt_destroy(sol)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sol, st, rc = iga.amen_solve(ctx, kk, Y, c["tol"])
    out["uncapped"] = {"status": rc, "valid": solve_ok(rc, st), "solve_time_s": time.perf_counter() - t0,
                       "kkt_residual": st["residual"], "ranks": st["ranks"], "half_sweeps": st["half_sweeps"],
                       "t_local_matvec": st["t_local_matvec"], "t_svd": st["t_svd"], "t_precond": st["t_precond"],
                       "t_interfaces": st["t_interfaces"], "t_residual": st["t_residual"]}
    grads = {}
    for name, fn in (("objective", lambda: iga.objective(ctx, kk, Y, sol)),
                     ("grad_yhat", lambda: iga.grad_yhat(ctx, kk, Y, sol, (n, n, n))),
                     ("grad_geometry", lambda: iga.grad_geometry(ctx, geo, p, n, beta, Y, sol))):
        fn()  # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        val = fn()
        torch.cuda.synchronize()
        grads[name + "_s"] = time.perf_counter() - t0
        if name == "objective":
            grads["objective"] = val
        if name == "grad_geometry":
            grads["grad_geometry_norm"] = float(np.linalg.norm(val))
    out["differentiation"] = grads
    iga.btt_destroy(sol)
    iga.kkt_destroy(kk)
    iga.ttop_destroy(M)
    iga.ttop_destroy(K)
    iga.tt_destroy(Y)
    return out


def batching_bench(iga, ctx, torch, nprob=64, seed=100, iters=3):
    """Batching form: the local TT-matvecs of nprob problems with uneven shapes drawn like the
    batched workload (n in {32,48,64,96,128}, degree in {2,3}, ranks r ~ U{8..32}, R_M ~ U{1..6},
    R_K ~ U{3..24}, beta log-uniform in [1e-8, 1e-2]) on seeded N(0,1) operands: one problem per
    call versus one batched call (grouped launches, autotuned tiles), FP64 and FP32."""
    import numpy as np
    import synth
    rng = np.random.default_rng(seed)
    probs, flops = [], 0.0
    for i in range(nprob):
        n = int(rng.choice([32, 48, 64, 96, 128]))
        p = int(rng.choice([2, 3]))
        r = int(rng.integers(8, 33))
        RM = int(rng.integers(1, 7))
        RK = int(rng.integers(3, 25))
        beta = float(10.0 ** rng.uniform(-8, -2))
        prob = synth.random_local_problem(r, RM, RK, n, p, seed=seed + i)
        dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in prob.items()}
        probs.append(dict(r0=r, n=n, r1=r, degree=p, RM0=RM, RM1=RM, RK0=RK, RK1=RK, beta=beta, PhiL_M=dev["PhiL_M"],
                          PhiR_M=dev["PhiR_M"], PhiL_K=dev["PhiL_K"], PhiR_K=dev["PhiR_K"], Mcore=dev["M"],
                          Kcore=dev["K"], x=dev["x"], y=torch.empty_like(dev["x"])))
        flops += iga.local_matvec_flops(r, n, r, p, RM, RM, RK, RK)
    out = {"problems": nprob, "flops_per_pass": flops}
    for name, prec in (("fp64", iga.FP64), ("fp32", iga.FP32)):
        def seq():
            for q in probs:
                iga.local_matvec(ctx, q["r0"], q["n"], q["r1"], q["degree"], q["RM0"], q["RM1"], q["RK0"], q["RK1"],
                                 q["PhiL_M"], q["PhiR_M"], q["PhiL_K"], q["PhiR_K"], q["Mcore"], q["Kcore"],
                                 q["beta"], q["x"], q["y"], prec)
        seq()
        iga.local_matvec_batched(ctx, probs, prec, autotune=True)  # tunes the buckets once
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(iters):
            seq()
        torch.cuda.synchronize()
        ts = (time.perf_counter() - t0) / iters
        t0 = time.perf_counter()
        for _ in range(iters):
            iga.local_matvec_batched(ctx, probs, prec, autotune=True)
        torch.cuda.synchronize()
        tb = (time.perf_counter() - t0) / iters
        out[name] = {"one_call_per_problem_s": ts, "batched_s": tb, "speedup": ts / tb,
                     "batched_gflops": flops / tb / 1e9, "one_call_per_problem_gflops": flops / ts / 1e9}
    return out


def time_dependent_bench(iga, ctx, torch, geo, c, Y, nt=10):
    """The time-dependent system (implicit Euler, nt steps, tau = 1 / nt) on the workload's
    geometry and desired state, AMEn tolerance 1e-6: FP64 (one warm-up solve, one timed), then
    the FP32 and BF16 forms (one timed solve each) with their state's distance to FP64's."""
    n, p, beta = c["n"], c["degree"], c["beta"]
    M, K, _ = iga.assemble_factors(ctx, geo, p, n, weight_tol=c["weight_tol"])
    kk = iga.kkt_create_parabolic(ctx, M, K, beta, nt, 1.0 / nt)
    out = {"time_steps": nt, "unknowns": 3 * nt * n ** 3}
    ref = None
    for name, prec, runs in (("fp64", iga.FP64, 2), ("fp32", iga.FP32, 1), ("bf16", iga.BF16, 1)):
        for i in range(runs):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            sol, st, rc = iga.amen_solve(ctx, kk, Y, 1e-6, precision=prec)
            t1 = time.perf_counter()
            if i + 1 < runs:
                iga.btt_destroy(sol)
        full = iga.btt_to_full(ctx, sol)
        iga.btt_destroy(sol)
        rec = {"solve_time_s": t1 - t0, "status": rc, "valid": solve_ok(rc, st), "kkt_residual": st["residual"],
               "half_sweeps": st["half_sweeps"], "ranks": st["ranks"], "t_svd": st["t_svd"]}
        if name == "fp64":
            ref = full
            rec.update({"local_iterations": st["local_iterations"], "t_local_matvec": st["t_local_matvec"],
                        "t_precond": st["t_precond"],
                        "local_matvec_gflops": st["local_matvec_flops"] / st["t_local_matvec"] / 1e9
                        if st["t_local_matvec"] else None})
            out.update(rec)
        else:
            rec["state_rel_diff_vs_fp64"] = float((full - ref).norm() / ref.norm())
            rec["speedup_vs_fp64"] = out["solve_time_s"] / rec["solve_time_s"]
            out[name] = rec
        del full
    del ref
    iga.kkt_destroy(kk)
    iga.ttop_destroy(M)
    iga.ttop_destroy(K)
    return out


def micro_bench(iga, ctx, torch, iters):
    """Local TT-matvec at the microbenchmark shape on seeded N(0,1) inputs; the library times
    the banded stage of each operator with HIP events on its stream."""
    import numpy as np
    import synth
    s = MICRO
    prob = synth.random_local_problem(s["r"], s["RM"], s["RK"], s["n"], s["p"], seed=1)
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in prob.items()}
    y = torch.empty_like(dev["x"])
    args = (ctx, s["r"], s["n"], s["r"], s["p"], s["RM"], s["RM"], s["RK"], s["RK"], dev["PhiL_M"],
            dev["PhiR_M"], dev["PhiL_K"], dev["PhiR_K"], dev["M"], dev["K"], 1e-6, dev["x"], y)
    for _ in range(3):
        iga.local_matvec(*args)
    # a plain device copy of known size (256 MiB read, 256 MiB written): the reference that
    # scales the HBM counters (FETCH_SIZE, WRITE_SIZE) in a counter run of this program
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    iga.profile_start(ctx)
    e0.record(stream)
    for _ in range(iters):
        iga.local_matvec(*args)
    e1.record(stream)
    prof = iga.profile_stop(ctx)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    flops = iga.local_matvec_flops(s["r"], s["n"], s["r"], s["p"], s["RM"], s["RM"], s["RK"], s["RK"])
    out = {"shape": dict(s), "ms": ms, "gflops": flops / ms / 1e6, "flops": flops, "profile": prof,
           "stages": stage_rates(prof, (0, 1))}
    # the same product in the mixed forms (operands converted to FP32 inside each call; BF16
    # rounds them once more as the products stage them)
    for name, prec, slot, peak in (("fp32", iga.FP32, 3, PEAK_FP32_TFLOPS), ("bf16", iga.BF16, 5, PEAK_BF16_TFLOPS)):
        for _ in range(3):
            iga.local_matvec(*args, prec)
        torch.cuda.synchronize()
        iga.profile_start(ctx)
        e0.record(stream)
        for _ in range(iters):
            iga.local_matvec(*args, prec)
        e1.record(stream)
        pr = iga.profile_stop(ctx)
        torch.cuda.synchronize()
        msl = e0.elapsed_time(e1) / iters
        band = pr["flops"][slot] / (pr["ms"][slot] * 1e-3) / 1e12 if pr["ms"][slot] else None
        out[name] = {"ms": msl, "gflops": flops / msl / 1e6, "band_K_tflops": band,
                     "band_K_frac_of_%s_peak" % name: band / peak if band else None}
    return out, prob


# microbenchmark shapes (r, R_M, R_K, n, p): the three workload shapes, then a sweep over r at
# the first one's operator ranks
SHAPES = [(32, 10, 60, 64, 3), (40, 15, 80, 128, 3), (40, 10, 60, 256, 3)] + \
         [(r, 10, 60, 64, 3) for r in (16, 24, 40, 64)]


def shapes_bench(iga, ctx, torch, warmup=10, calls=50):
    """FP64 local TT-matvec on seeded N(0,1) operands at each shape: median of per-call HIP
    event times after warm-up, algorithmic GFLOP/s, and the banded K stage's TF/s from the
    library's event profile of the same calls."""
    import numpy as np
    import synth
    out = []
    stream = torch.cuda.current_stream()
    for (r, RM, RK, n, p) in SHAPES:
        prob = synth.random_local_problem(r, RM, RK, n, p, seed=1)
        dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in prob.items()}
        y = torch.empty_like(dev["x"])
        args = (ctx, r, n, r, p, RM, RM, RK, RK, dev["PhiL_M"], dev["PhiR_M"], dev["PhiL_K"], dev["PhiR_K"],
                dev["M"], dev["K"], 1e-6, dev["x"], y)
        for _ in range(warmup):
            iga.local_matvec(*args)
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(calls)]
        torch.cuda.synchronize()
        iga.profile_start(ctx)
        for e0, e1 in ev:
            e0.record(stream)
            iga.local_matvec(*args)
            e1.record(stream)
        pr = iga.profile_stop(ctx)
        torch.cuda.synchronize()
        ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ev]))
        flops = iga.local_matvec_flops(r, n, r, p, RM, RM, RK, RK)
        out.append({"shape": {"r": r, "RM": RM, "RK": RK, "n": n, "p": p}, "median_ms": ms,
                    "gflops": flops / ms / 1e6,
                    "band_K_tflops": pr["flops"][1] / (pr["ms"][1] * 1e-3) / 1e12 if pr["ms"][1] else None})
        del dev, y
    return out


def cpu_baseline(prob, budget_s=15.0, max_calls=400):
    """The oracle's local projected matvec (numpy FP64 einsum stages) at the microbenchmark
    shape, timed on the host cores."""
    from oracle import tt
    from paper_1811_06797_amd import iga
    s = MICRO
    Md = tt.banded_to_dense(prob["M"], s["p"])
    Kd = tt.banded_to_dense(prob["K"], s["p"])
    x = prob["x"]
    flops = iga.local_matvec_flops(s["r"], s["n"], s["r"], s["p"], s["RM"], s["RM"], s["RK"], s["RK"])
    calls = 0
    t0 = time.perf_counter()
    while True:
        for l in range(3):
            tt.local_apply(prob["PhiL_M"], Md, prob["PhiR_M"], x[l])
        for l in (0, 2):
            tt.local_apply(prob["PhiL_K"], Kd, prob["PhiR_K"], x[l])
        calls += 1
        if time.perf_counter() - t0 > budget_s or calls >= max_calls:
            break
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    return {"value": flops * calls / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "%d local projected matvecs (3 M + 2 K operator applications each) of the oracle's "
                      "numpy einsum contraction at (r, R_M, R_K, n, p) = (%d, %d, %d, %d, %d), %.1f s, "
                      "os.cpu_count() = %s" % (calls, s["r"], s["RM"], s["RK"], s["n"], s["p"], dt, os.cpu_count())}


def oracle_legs():
    """The oracle timed on the host cores on two more bounded samples: the identity-cube
    workload (n = 16, degree 2) end to end, full 3-D assembly plus its reduced PCG solve (its
    sparse-LU KKT solve takes about a minute and is not timed), and the matrix-free KKT
    residual at n = 128 on the perturbed cube, one 3 x 3 x 3 box of rows (the element-by-element
    product the tests sample) after the weight interpolation it needs."""
    import numpy as np
    import synth
    from oracle import assembly, kkt, tt
    out = {}
    geo, yc, c = synth.config("cube_n16")
    yh = tt.tt_full(yc).ravel()
    t0 = time.perf_counter()
    Mo, Ko = assembly.assemble(geo, c["n"], c["degree"], mode="exact")
    t1 = time.perf_counter()
    y, u, lam, its = kkt.solve_reduced(Mo, Ko, c["beta"], yh)
    t2 = time.perf_counter()
    out["identity_cube_n16"] = {"assembly_s": t1 - t0, "reduced_solve_s": t2 - t1, "pcg_iterations": int(its),
                                "residual": float(kkt.residual(Mo, Ko, c["beta"], yh, np.concatenate([y, u, lam])))}
    geo, yc, c = synth.config("perturbed_cube_n128")
    n, p = c["n"], c["degree"]
    t0 = time.perf_counter()
    W = assembly.interpolate_weights(geo, assembly.Space(n, p))
    t1 = time.perf_counter()
    rng = np.random.default_rng(0)
    fields = [rng.standard_normal((n,) * 3) for _ in range(4)]
    box = ((62, 65), (30, 33), (90, 93))
    assembly.apply_box(geo, n, p, fields, box, mode="interp", Wint=W)
    t2 = time.perf_counter()
    out["perturbed_cube_n128_box_residual"] = {
        "weights_s": t1 - t0, "box_s": t2 - t1, "rows_per_box": 27,
        "full_residual_s_extrapolated": (t2 - t1) * n ** 3 / 27}
    return out


def stage_rates(prof, ops):
    """TF/s and summed ms of the three local-matvec stages (left interface, banded operator core,
    right interface) over the given operator indices of a library event profile."""
    out = {}
    for name, ms_key, fl_key in (("left_interface", "s1_ms", "s1_flops"), ("band", "ms", "flops"),
                                 ("right_interface", "s3_ms", "s3_flops")):
        ms = sum(prof[ms_key][i] for i in ops)
        fl = sum(prof[fl_key][i] for i in ops)
        out[name] = {"ms": ms, "tflops": fl / (ms * 1e-3) / 1e12 if ms else None}
    return out


def run_step(iga, ctx, torch, geo, c, Y, precision=None):
    """One step: assembly, KKT operator and block-AMEn solve of one workload; statistics of the
    solve with the wall times of both parts and the solve's status."""
    n, p, beta = c["n"], c["degree"], c["beta"]
    t0 = time.perf_counter()
    M, K, ranks = iga.assemble_factors(ctx, geo, p, n, weight_tol=c["weight_tol"])
    kk = iga.kkt_create(ctx, M, K, beta)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    opts = {"precision": precision if precision is not None else iga.FP64}
    if "r_max" in c:
        opts["r_max"] = c["r_max"]
    sol, st, rc = iga.amen_solve(ctx, kk, Y, c["tol"], **opts)
    t2 = time.perf_counter()
    st["assembly_s"] = t1 - t0
    st["solve_wall_s"] = t2 - t1
    st["rc"] = rc
    st["valid"] = solve_ok(rc, st)
    st["op_ranks"] = [iga.ttop_info(M)[1], iga.ttop_info(K)[1]]
    st["weight_ranks"] = [[int(v) for v in row] for row in ranks]
    iga.btt_destroy(sol)
    iga.kkt_destroy(kk)
    iga.ttop_destroy(M)
    iga.ttop_destroy(K)
    return st


STAT_KEYS = ("half_sweeps", "converged", "ranks", "local_solves", "local_iterations", "local_matvecs",
             "local_matvec_flops", "t_local_matvec", "t_precond", "t_svd", "t_interfaces", "t_krylov_other",
             "t_residual", "op_ranks")


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this implementation runs on one GPU; multi-GPU runs are not supported "
              "(use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_1811_06797_amd import iga

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = iga.ctx_create(0, stream.cuda_stream)

    if a.micro_only:
        micro, _ = micro_bench(iga, ctx, torch, a.micro_iters)
        prof = micro["profile"]
        print(json.dumps({"shape": micro["shape"], "ms": micro["ms"], "gflops": micro["gflops"],
                          "band_K_ms_per_launch": prof["ms"][1] / max(prof["launches"][1], 1),
                          "band_K_flops_per_launch": prof["flops"][1] / max(prof["launches"][1], 1)}), flush=True)
        iga.ctx_destroy(ctx)
        return

    if a.solve_only:
        geo, yc, c = synth.config(a.workload)
        Y = iga.tt_create(ctx, yc)
        torch.cuda.synchronize()
        st = run_step(iga, ctx, torch, geo, c, Y, getattr(iga, a.precision))
        print(json.dumps({k: st[k] for k in ("assembly_s", "solve_wall_s", "rc", "valid", "residual", "ranks",
                                             "half_sweeps", "local_iterations", "local_matvecs", "t_local_matvec",
                                             "t_svd", "t_precond", "t_interfaces", "op_ranks")}), flush=True)
        iga.tt_destroy(Y)
        iga.ctx_destroy(ctx)
        return

    geo, yc, c = synth.config(WORKLOAD)
    Y = iga.tt_create(ctx, yc)
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        run_step(iga, ctx, torch, geo, c, Y)
    torch.cuda.synchronize()
    iga.profile_start(ctx)
    t0 = time.perf_counter()
    stats = [run_step(iga, ctx, torch, geo, c, Y) for _ in range(a.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    band = iga.profile_stop(ctx)
    ms_per_step = (t1 - t0) * 1e3 / a.steps
    print("bench: %d timed steps done, %.1f ms per step" % (a.steps, ms_per_step), file=sys.stderr, flush=True)

    flops = sum(s["local_matvec_flops"] for s in stats)
    t_mv = sum(s["t_local_matvec"] for s in stats)
    gflops = flops / t_mv / 1e9
    valid = all(s["valid"] for s in stats)
    invalid_steps = [i for i, s in enumerate(stats) if not s["valid"]]
    mixed = mixed_compare(iga, ctx, torch, geo, c, Y, 2)
    print("bench: mixed-precision comparison done", file=sys.stderr, flush=True)
    geo2, yc2, c2 = synth.config(SECONDARY)
    Y2 = iga.tt_create(ctx, yc2)
    run_step(iga, ctx, torch, geo2, c2, Y2)
    s2 = run_step(iga, ctx, torch, geo2, c2, Y2)
    secondary = {"config": c2["name"] + ", tol %g, FP64" % c2["tol"], "assembly_time_s": s2["assembly_s"],
                 "solve_time_s": s2["solve_wall_s"], "status": s2["rc"], "valid": s2["valid"],
                 "kkt_residual": s2["residual"], "ranks": s2["ranks"], "half_sweeps": s2["half_sweeps"],
                 "local_matvec_gflops": s2["local_matvec_flops"] / s2["t_local_matvec"] / 1e9}
    geo1, yc1, c1 = synth.config("cube_n16")
    Y1 = iga.tt_create(ctx, yc1)
    run_step(iga, ctx, torch, geo1, c1, Y1)
    s1 = run_step(iga, ctx, torch, geo1, c1, Y1)
    iga.tt_destroy(Y1)
    cube16 = {"config": c1["name"] + ", beta %g, tol %g, FP64" % (c1["beta"], c1["tol"]),
              "assembly_time_s": s1["assembly_s"], "solve_time_s": s1["solve_wall_s"], "status": s1["rc"],
              "kkt_residual": s1["residual"], "ranks": s1["ranks"]}
    n256 = n256_leg(iga, ctx, torch)
    batching = batching_bench(iga, ctx, torch)
    timedep = time_dependent_bench(iga, ctx, torch, geo2, c2, Y2)
    iga.tt_destroy(Y2)
    print("bench: secondary workloads done", file=sys.stderr, flush=True)
    micro, prob = micro_bench(iga, ctx, torch, a.micro_iters)
    shapes = shapes_bench(iga, ctx, torch)
    peaks = iga.measure_peaks(ctx)
    prof = micro["profile"]
    k_ms = prof["ms"][1] / max(prof["launches"][1], 1)
    k_flops = prof["flops"][1] / max(prof["launches"][1], 1)
    achieved = k_flops / (k_ms * 1e-3) / 1e12
    traffic = traffic_from_profile()
    last = stats[-1]
    band_ms = band["ms"][0] + band["ms"][1]
    band_flops = band["flops"][0] + band["flops"][1]

    line = {
        "metric": "local TT-matvec GFLOP/s + KKT solve time to 1e-6 residual, mixed vs FP64",
        "value": gflops,
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded perturbed-cube geometry and Fourier desired state)",
        "config": {"workload": "perturbed unit cube (8x8x8 cubic control net, seeded smooth perturbation of "
                               "amplitude 0.1), degree 3, n = 128 free dofs per direction (2,097,152 per field, "
                               "6,291,456 KKT unknowns), beta = 1e-6, Fourier desired state, weight TT tol %g, "
                               "block-AMEn tol %g, FP64; one step = assembly + KKT operator + solve"
                               % (c["weight_tol"], c["tol"])},
        "valid": valid,
        "invalid_steps": invalid_steps,
        "status": [s["rc"] for s in stats],
        "solve_time_s": sum(s["solve_wall_s"] for s in stats) / len(stats),
        "assembly_time_s": sum(s["assembly_s"] for s in stats) / len(stats),
        "kkt_residual": max(s["residual"] for s in stats),
        "solve": {k: last[k] for k in STAT_KEYS},
        "weight_ranks": last["weight_ranks"],
        "in_solve_stages": stage_rates(band, (0, 1)),
        "in_solve_band_stage": {"stages": band["stages"][0] + band["stages"][1],
                                "launches": band["launches"][0] + band["launches"][1],
                                "ms": band_ms, "flops": band_flops,
                                "tflops": band_flops / (band_ms * 1e-3) / 1e12 if band_ms else None,
                                "frac_of_fp64_peak": band_flops / (band_ms * 1e-3) / 1e12 / PEAK_FP64_TFLOPS
                                if band_ms else None},
        "mixed_vs_fp64": mixed,
        "annulus_n256": n256,
        "annulus_n64": secondary,
        "identity_cube_n16": cube16,
        "batching": batching,
        "time_dependent": timedep,
        "microbench_local_matvec": {k: micro[k] for k in ("shape", "ms", "gflops", "flops", "stages", "fp32", "bf16")},
        "microbench_shapes": shapes,
        "measured_peaks": peaks,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP64_TFLOPS, "traffic": traffic,
                     "peak_measured": peaks["mfma_f64_4x4x4_tflops"],
                     "frac_of_measured": achieved / peaks["mfma_f64_4x4x4_tflops"],
                     "kernel": ROOFLINE_KERNEL + ": banded middle stage of the K operator in the "
                               "local TT-matvec at (r, R_M, R_K, n, p) = (%d, %d, %d, %d, %d)"
                               % (MICRO["r"], MICRO["RM"], MICRO["RK"], MICRO["n"], MICRO["p"]),
                     "flops_per_launch": k_flops, "ms_per_launch": k_ms, "launches": prof["launches"][1],
                     "whole_local_matvec_tflops": micro["gflops"] / 1e3,
                     "whole_local_matvec_frac": micro["gflops"] / 1e3 / PEAK_FP64_TFLOPS,
                     "in_solve_local_matvec_frac": gflops / 1e3 / PEAK_FP64_TFLOPS},
    }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob)
        line["cpu_baseline"]["oracle_legs"] = oracle_legs()
    iga.tt_destroy(Y)
    iga.ctx_destroy(ctx)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
