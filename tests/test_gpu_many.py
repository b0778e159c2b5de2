"""GPU batching form for whole solves (iga_amen_solve_many): independent block-AMEn solves run
concurrently by worker threads with their own streams. Each solve runs the kernels of a lone
iga_amen_solve in the same order, so the results must equal the sequential ones exactly; one
problem is also checked against the oracle's direct solve."""
import numpy as np
import pytest

import synth
from oracle import assembly, kkt as okkt, tt
from tests.gpu_util import rel_err

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="iga_amen_solve_many is switched off: a run of 64 problems of the batching "
                            "workload through it faulted the GPU and the cause has not been found"),
]


def _systems(gpu_ctx, problems):
    from paper_1811_06797_amd import iga
    ops, kkts, ys = [], [], []
    for geo, yc, c in problems:
        M, K, _ = iga.assemble_factors(gpu_ctx, geo, c["degree"], c["n"], weight_tol=0.0)
        ops += [M, K]
        kkts.append(iga.kkt_create(gpu_ctx, M, K, c["beta"]))
        ys.append(iga.tt_create(gpu_ctx, yc))
    return ops, kkts, ys


def _release(ops, kkts, ys):
    from paper_1811_06797_amd import iga
    for y in ys:
        iga.tt_destroy(y)
    for k in kkts:
        iga.kkt_destroy(k)
    for o in ops:
        iga.ttop_destroy(o)


def test_concurrent_solves_equal_sequential(gpu_ctx):
    from paper_1811_06797_amd import iga
    problems = synth.batch_problems(6, seed0=200, n_choices=(6, 8, 10))
    ops, kkts, ys = _systems(gpu_ctx, problems)
    try:
        seq = []
        for k, y in zip(kkts, ys):
            sol, st, rc = iga.amen_solve(gpu_ctx, k, y, 1e-8)
            seq.append((iga.btt_to_full(gpu_ctx, sol).cpu().numpy(), rc, st["half_sweeps"]))
            iga.btt_destroy(sol)
        sols, stats, status = iga.amen_solve_many(gpu_ctx, kkts, ys, 1e-8, workers=3)
        try:
            for i, s in enumerate(sols):
                assert s is not None and status[i] == seq[i][1]
                f = iga.btt_to_full(gpu_ctx, s).cpu().numpy()
                assert np.array_equal(f, seq[i][0]), i
                assert stats[i]["half_sweeps"] == seq[i][2]
        finally:
            for s in sols:
                if s is not None:
                    iga.btt_destroy(s)
    finally:
        _release(ops, kkts, ys)
    # one of them against the oracle's direct solve of the same system
    geo, yc, c = problems[0]
    M, K = assembly.assemble(geo, c["n"], c["degree"], mode="interp")
    y, u, lam = okkt.solve_direct(M, K, c["beta"], tt.tt_full(yc).ravel())
    assert rel_err(seq[0][0][0].ravel(), y) < 1e-6


def test_statuses_and_refusals(gpu_ctx):
    from paper_1811_06797_amd import iga
    problems = synth.batch_problems(3, seed0=300, n_choices=(6,))
    ops, kkts, ys = _systems(gpu_ctx, problems)
    try:
        # one half-sweep cannot converge: every solve reports that and still returns a solution
        sols, stats, status = iga.amen_solve_many(gpu_ctx, kkts, ys, 1e-12, workers=2, nswp=1)
        try:
            assert all(s is not None for s in sols)
            assert all(rc in (iga.ENOCONV, iga.ERANK) for rc in status)
        finally:
            for s in sols:
                iga.btt_destroy(s)
        with pytest.raises(iga.IgaError):
            iga.amen_solve_many(gpu_ctx, kkts, ys, 1e-8, workers=0)
        with pytest.raises(iga.IgaError):
            iga.amen_solve_many(gpu_ctx, kkts, ys, [1e-8, 2.0, 1e-8], workers=2)
    finally:
        _release(ops, kkts, ys)
