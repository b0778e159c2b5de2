"""Benchmark of the low-rank IgA optimal-control hot path on one MI355X.

One step = the whole path on one synthetic workload: TT assembly of M and K
(assemble_factors), the KKT operator (kkt_create) and the block-AMEn solve to
a KKT relative residual below 1e-6 (amen_solve), in FP64. The workload is the
twisted quarter annulus (radii 1, 2, seeded twist), degree 3, n = 64 free
dofs per direction (262,144 dofs per field), beta = 1e-6, Fourier desired
state, weight TT tolerance 1e-10. Inputs (control points, desired-state TT)
are synthetic and seeded.

Printed JSON line: metric value = local TT-matvec GFLOP/s inside the timed
solves (algorithmic flops of every projected local matvec / their GPU time,
HIP events on the library's stream), plus the solve time, the residual, a
roofline object for the dominant kernel and the CPU oracle baseline.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64_TFLOPS = 78.6  # MI355X dense FP64 (vector and matrix)
PEAK_HBM_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--micro-iters", type=int, default=20)
    return ap.parse_args()


def local_shapes_micro():
    # projected local TT-matvec at the n = 64 benchmark shape (r, R_M, R_K, n, p)
    return dict(r=32, RM=10, RK=60, n=64, p=3)


def micro_bench(iga, ctx, torch, iters):
    """Time iga_local_matvec on seeded random inputs at the benchmark shape with HIP events."""
    import numpy as np
    import synth
    s = local_shapes_micro()
    prob = synth.random_local_problem(s["r"], s["RM"], s["RK"], s["n"], s["p"], seed=1)
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in prob.items()}
    y = torch.empty_like(dev["x"])
    args = (ctx, s["r"], s["n"], s["r"], s["p"], s["RM"], s["RM"], s["RK"], s["RK"], dev["PhiL_M"],
            dev["PhiR_M"], dev["PhiL_K"], dev["PhiR_K"], dev["M"], dev["K"], 1e-6, dev["x"], y)
    for _ in range(3):
        iga.local_matvec(*args)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(iters):
        iga.local_matvec(*args)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / iters
    flops = iga.local_matvec_flops(s["r"], s["n"], s["r"], s["p"], s["RM"], s["RM"], s["RK"], s["RK"])
    return {"shape": s, "ms": ms, "gflops": flops / ms / 1e6, "flops": flops}, prob


def cpu_baseline(prob, budget_s=15.0):
    """The oracle's local projected matvec (numpy FP64) at the same shape, timed on the host."""
    import numpy as np
    from oracle import tt
    from paper_1811_06797_amd import iga
    s = local_shapes_micro()
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
        if time.perf_counter() - t0 > budget_s or calls >= 50:
            break
    dt = time.perf_counter() - t0
    try:
        from threadpoolctl import threadpool_info
        threads = max([int(i.get("num_threads", 1)) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    return {"value": flops * calls / dt / 1e9, "unit": "GFLOP/s", "cores": threads, "kind": "oracle",
            "sample": "%d calls of the oracle's einsum local projected matvec (3 M + 2 K applications) "
                      "at (r, R_M, R_K, n, p) = (32, 10, 60, 64, 3), %.1f s" % (calls, dt)}


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_1811_06797_amd import iga

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    ctx = iga.ctx_create(0, stream.cuda_stream)
    geo, yc, c = synth.config("c2")
    n, p, beta = c["n"], c["degree"], c["beta"]
    Y = iga.tt_create(ctx, yc)
    torch.cuda.synchronize()

    def step():
        M, K, ranks = iga.assemble_factors(ctx, geo, p, n, weight_tol=c["weight_tol"])
        kk = iga.kkt_create(ctx, M, K, beta)
        t = time.perf_counter()
        sol, st, rc = iga.amen_solve(ctx, kk, Y, c["tol"])
        st["solve_wall_s"] = time.perf_counter() - t
        st["rc"] = rc
        st["op_ranks"] = [iga.ttop_info(M)[1], iga.ttop_info(K)[1]]
        iga.btt_destroy(sol)
        iga.kkt_destroy(kk)
        iga.ttop_destroy(M)
        iga.ttop_destroy(K)
        return st

    for _ in range(a.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = [step() for _ in range(a.steps)]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / a.steps

    flops = sum(s["local_matvec_flops"] for s in stats)
    t_mv = sum(s["t_local_matvec"] for s in stats)
    gflops = flops / t_mv / 1e9
    solve_s = sum(s["solve_wall_s"] for s in stats) / len(stats)
    micro, prob = micro_bench(iga, ctx, torch, a.micro_iters)

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
        "data": "synthetic",
        "config": {"workload": "twisted quarter annulus, p=3, n=64 per direction (262,144 dofs), "
                               "beta=1e-6, Fourier desired state, weight TT tol 1e-10, AMEn tol %g" % c["tol"],
                   "global_batch": 1, "parallelism": "single GPU"},
        "solve_time_s": solve_s,
        "kkt_residual": max(s["residual"] for s in stats),
        "solve": {k: stats[-1][k] for k in ("half_sweeps", "ranks", "local_solves", "local_iterations",
                                            "local_matvecs", "t_local_matvec", "t_precond", "t_svd",
                                            "t_interfaces", "t_krylov_other", "op_ranks")},
        "microbench_local_matvec": micro,
        "roofline": {"bound": "mfma", "achieved": micro["gflops"] / 1e3, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": micro["gflops"] / 1e3 / PEAK_FP64_TFLOPS, "traffic": None,
                     "kernel": "projected local TT-matvec at (r, R_M, R_K, n, p) = (32, 10, 60, 64, 3)"},
    }
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(prob)
    iga.tt_destroy(Y)
    iga.ctx_destroy(ctx)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
