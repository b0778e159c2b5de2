"""The allocation-free local TT-matvec (iga_local_matvec_noalloc) against the allocating entry
point iga_local_matvec (FP64) on the same inputs, through the C ABI: two calls in a row, the
second on a smaller problem, so the second runs on a scratch array that still holds the
first call's intermediates; and a shape whose workspace exceeds the fixed array is refused."""
import numpy as np
import pytest

import synth
from tests.gpu_util import rel_err

pytestmark = pytest.mark.gpu

SHAPES = [(24, 4, 12, 40, 3), (16, 3, 9, 24, 2)]  # (r, R_M, R_K, n, p): second smaller than first


def _dev(prob, torch):
    return {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in prob.items()}


def test_noalloc_matches_allocating_entry_point(gpu_ctx):
    import torch
    from paper_1811_06797_amd import iga
    for seed, (r, RM, RK, n, p) in enumerate(SHAPES):
        print("noalloc case", (r, RM, RK, n, p), flush=True)
        prob = synth.random_local_problem(r, RM, RK, n, p, seed=40 + seed)
        d = _dev(prob, torch)
        args = (gpu_ctx, r, n, r, p, RM, RM, RK, RK, d["PhiL_M"], d["PhiR_M"], d["PhiL_K"], d["PhiR_K"], d["M"],
                d["K"], 1e-3, d["x"])
        y_ref = torch.empty_like(d["x"])
        y_na = torch.full_like(d["x"], float("nan"))
        iga.local_matvec(*args, y_ref, iga.FP64)
        iga.local_matvec_noalloc(*args, y_na)
        torch.cuda.synchronize()
        a, b = y_na.cpu().numpy(), y_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        err = rel_err(a, b)
        print("noalloc vs allocating entry point: rel err %.3e, max abs diff %.3e" % (err, np.abs(a - b).max()),
              flush=True)
        # the same kernels in the same order on the same inputs
        assert err <= 1e-14


def test_noalloc_refuses_shapes_beyond_the_scratch(gpu_ctx):
    import torch
    from paper_1811_06797_amd import iga
    # (r, R_M, R_K, n, p) = (64, 10, 60, 64, 3) needs several hundred MB of intermediates
    r, RM, RK, n, p = 64, 10, 60, 64, 3
    x = torch.zeros(3 * r * n * r, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    small = torch.zeros(RK * r * r, dtype=torch.float64, device="cuda")
    core = torch.zeros(RK * n * (2 * p + 1) * RK, dtype=torch.float64, device="cuda")
    with pytest.raises(iga.IgaError) as ei:
        iga.local_matvec_noalloc(gpu_ctx, r, n, r, p, RM, RM, RK, RK, small, small, small, small, core, core, 1e-3,
                                 x, y)
    assert ei.value.code == iga.EINVAL and "exceeds" in str(ei.value)
