"""Batching form: local TT-matvecs of many problems of uneven n, degree and ranks through one
grouped launch per stage, against the oracle and against the one-problem entry point."""
import numpy as np
import pytest

import synth
from tests.gpu_util import elem_err, rel_err
from tests.test_gpu_localmatvec import FP32_TOL, _reference

pytestmark = pytest.mark.gpu

SHAPES = [  # r0, RM, RK, n, p, r1
    (3, 1, 2, 5, 1, 3), (5, 2, 3, 9, 2, 4), (7, 3, 5, 13, 3, 7), (1, 1, 3, 6, 2, 4), (17, 2, 9, 23, 3, 17),
    (12, 4, 12, 32, 2, 9), (20, 3, 15, 48, 3, 24), (9, 1, 7, 64, 3, 9)]


def _problems(torch, seed0=0):
    out, refs = [], []
    for j, (r, RM, RK, n, p, rr) in enumerate(SHAPES):
        prob = synth.random_local_problem(r, RM, RK, n, p, seed=seed0 + 31 * j, r_right=rr)
        beta = 10.0 ** (-1 - j % 5)
        dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in prob.items()}
        q = dict(r0=r, n=n, r1=rr, degree=p, RM0=RM, RM1=RM, RK0=RK, RK1=RK, beta=beta, PhiL_M=dev["PhiL_M"],
                 PhiR_M=dev["PhiR_M"], PhiL_K=dev["PhiL_K"], PhiR_K=dev["PhiR_K"], Mcore=dev["M"], Kcore=dev["K"],
                 x=dev["x"], y=torch.zeros_like(dev["x"]))
        out.append(q)
        refs.append(_reference(prob, p, beta))
    return out, refs


def test_batched_fp64_matches_oracle_and_single_calls(gpu_ctx):
    import torch
    from paper_1811_06797_amd import iga
    probs, refs = _problems(torch)
    iga.local_matvec_batched(gpu_ctx, probs, iga.FP64, autotune=False)
    torch.cuda.synchronize()
    ys = [q["y"].cpu().numpy() for q in probs]
    for q, y, ref in zip(probs, ys, refs):
        assert rel_err(y, ref) < 1e-13
        assert elem_err(y, ref) < 1e-13
        single = torch.zeros_like(q["y"])
        iga.local_matvec(gpu_ctx, q["r0"], q["n"], q["r1"], q["degree"], q["RM0"], q["RM1"], q["RK0"], q["RK1"],
                         q["PhiL_M"], q["PhiR_M"], q["PhiL_K"], q["PhiR_K"], q["Mcore"], q["Kcore"], q["beta"],
                         q["x"], single)
        torch.cuda.synchronize()
        assert rel_err(y, single.cpu().numpy()) < 1e-14
    # tile shapes picked by timing give the same bits (every shape accumulates K in one order)
    for q in probs:
        q["y"].zero_()
    iga.local_matvec_batched(gpu_ctx, probs, iga.FP64, autotune=True)
    iga.local_matvec_batched(gpu_ctx, probs, iga.FP64, autotune=True)
    torch.cuda.synchronize()
    for q, y in zip(probs, ys):
        assert np.array_equal(q["y"].cpu().numpy(), y)


def test_batched_fp32_matches_oracle(gpu_ctx):
    import torch
    from paper_1811_06797_amd import iga
    probs, refs = _problems(torch, seed0=5)
    iga.local_matvec_batched(gpu_ctx, probs, iga.FP32, autotune=True)
    torch.cuda.synchronize()
    for q, ref in zip(probs, refs):
        assert rel_err(q["y"].cpu().numpy(), ref) < FP32_TOL


def test_batched_edge_cases(gpu_ctx):
    import torch
    from paper_1811_06797_amd import iga
    iga.local_matvec_batched(gpu_ctx, [], iga.FP64)
    probs, _ = _problems(torch)
    bad = dict(probs[0])
    bad["degree"] = 0
    with pytest.raises(iga.IgaError):
        iga.local_matvec_batched(gpu_ctx, [bad], iga.FP64)
