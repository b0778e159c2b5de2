"""GPU parity of the projected local TT-matvec (eq. KKT_red) against the oracle's einsum
definition, which is itself pinned to F^T A F x on tiny cases (tests/test_oracle_tt.py)."""
import numpy as np
import pytest

import synth
from oracle import tt
from tests.gpu_util import elem_err, kkt_rows, rel_err

pytestmark = pytest.mark.gpu


def _reference(prob, p, beta):
    Md = tt.banded_to_dense(prob["M"], p)
    Kd = tt.banded_to_dense(prob["K"], p)
    x = prob["x"]
    Mf = [tt.local_apply(prob["PhiL_M"], Md, prob["PhiR_M"], x[l]) for l in range(3)]
    Kf = [tt.local_apply(prob["PhiL_K"], Kd, prob["PhiR_K"], x[l]) for l in range(3)]
    return np.stack(kkt_rows(Mf, Kf, beta))


def _run(gpu_ctx, prob, r, n, p, RM, RK, beta, precision, rr=None):
    import torch
    from paper_1811_06797_amd import iga
    rr = r if rr is None else rr
    dev = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in prob.items()}
    y = torch.empty_like(dev["x"])
    iga.local_matvec(gpu_ctx, r, n, rr, p, RM, RM, RK, RK, dev["PhiL_M"], dev["PhiR_M"], dev["PhiL_K"],
                     dev["PhiR_K"], dev["M"], dev["K"], beta, dev["x"], y, precision)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.mark.parametrize("r,RM,RK,n,p,rr", [(3, 1, 2, 5, 1, None), (5, 2, 3, 9, 2, None), (7, 3, 5, 13, 3, 4),
                                             (1, 1, 3, 6, 2, 4), (17, 2, 9, 23, 3, None),
                                             (24, 1, 1, 40, 3, 30),
                                             # banded K stage on the LDS-direct wide tile: N = 2 r^2 = 2178
                                             # is 17 column tiles and a ragged one, M = 50 a partial tile,
                                             # K = 350 a partial K tile; odd R_K = 51 takes the
                                             # register-staged kernel instead
                                             (33, 4, 50, 32, 3, None), (33, 4, 51, 32, 3, None),
                                             # 64 x 128 tiles on tall products with more than 64
                                             # columns: the right-interface stage (M = r n = 320
                                             # and 720, N = r' = 72 and 90), and the left one
                                             # (M = R_K r = 360, N = n r' = 2160)
                                             (20, 2, 5, 16, 3, 72), (30, 3, 12, 24, 2, 90),
                                             # banded stages with 17..32 output ranks (the
                                             # re-laid core's product on 24-row tiles up to 24
                                             # ranks, 32-row ones above): p = 3, a ragged p = 2
                                             # case, p = 1 with both operators there (R_M = 17,
                                             # R_K = 30), and 21 and 23 ranks with n = 29
                                             (20, 3, 24, 18, 3, None), (12, 2, 19, 37, 2, 13),
                                             (9, 17, 30, 20, 1, 7), (11, 21, 23, 29, 3, 5)])
def test_local_matvec_matches_oracle(gpu_ctx, r, RM, RK, n, p, rr):
    from paper_1811_06797_amd import iga
    prob = synth.random_local_problem(r, RM, RK, n, p, seed=r + n, r_right=rr)
    beta = 1e-3
    y = _run(gpu_ctx, prob, r, n, p, RM, RK, beta, iga.FP64, rr)
    ref = _reference(prob, p, beta)
    assert rel_err(y, ref) < 1e-13
    assert elem_err(y, ref) < 1e-13


# FP32 form: inputs rounded to FP32 (relative 6e-8) and FP32 accumulation over the three
# stages' contraction lengths (at most a few thousand terms of N(0,1) data) give a relative
# Frobenius error of order 6e-8 * sqrt(K) <= 1e-5; the bar leaves a factor 5.
FP32_TOL = 5e-5


@pytest.mark.parametrize("r,RM,RK,n,p,rr", [(3, 1, 2, 5, 1, None), (5, 2, 3, 9, 2, None), (7, 3, 5, 13, 3, 4),
                                             (1, 1, 3, 6, 2, 4), (17, 2, 9, 23, 3, None),
                                             # banded K stage on the FP32 LDS-direct wide tile (N = 2312:
                                             # a ragged column tile, M = 52 and K = 364 partial tiles);
                                             # R_K = 50 is not a multiple of 4 and takes the
                                             # register-staged kernel
                                             (34, 4, 52, 32, 3, None), (34, 4, 50, 32, 3, None)])
def test_local_matvec_fp32_matches_oracle(gpu_ctx, r, RM, RK, n, p, rr):
    from paper_1811_06797_amd import iga
    prob = synth.random_local_problem(r, RM, RK, n, p, seed=r + n, r_right=rr)
    beta = 1e-3
    y = _run(gpu_ctx, prob, r, n, p, RM, RK, beta, iga.FP32, rr)
    assert rel_err(y, _reference(prob, p, beta)) < FP32_TOL


def test_local_matvec_benchmark_shape(gpu_ctx):
    """The n = 64 benchmark shape (r, R_M, R_K, n, b) = (32, 10, 60, 64, 7)."""
    from paper_1811_06797_amd import iga
    r, RM, RK, n, p = 32, 10, 60, 64, 3
    prob = synth.random_local_problem(r, RM, RK, n, p, seed=1)
    y = _run(gpu_ctx, prob, r, n, p, RM, RK, 1e-6, iga.FP64)
    ref = _reference(prob, p, 1e-6)
    assert rel_err(y, ref) < 1e-13
    assert elem_err(y, ref) < 1e-13
    yf = _run(gpu_ctx, prob, r, n, p, RM, RK, 1e-6, iga.FP32)
    assert rel_err(yf, ref) < FP32_TOL


# BF16 form: every contraction operand is rounded to bfloat16 (relative 2^-9 = 2e-3) and
# products accumulate in FP32. Against the exact FP64 product the three stages compound to a
# relative error of about sqrt(3) * sqrt(2) * 2e-3 = 5e-3; the bar leaves a factor 6.
BF16_TOL = 3e-2


def _bf16(a):
    """Nearest bfloat16 (ties to even) of the FP32 rounding of a, returned in FP64."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _reference_bf16(prob, p, beta):
    """The BF16 form's arithmetic written out: each stage's operands rounded to bfloat16,
    exact products, intermediates stored in FP32."""
    f32 = lambda a: np.asarray(a, dtype=np.float32).astype(np.float64)

    def apply(PhiL, A, PhiR, x):
        t1 = f32(np.einsum("pxa,ajb->pxjb", _bf16(PhiL), _bf16(x), optimize=True))
        t2 = f32(np.einsum("pijq,pxjb->qxib", _bf16(A), _bf16(t1), optimize=True))
        return f32(np.einsum("qxib,qyb->xiy", _bf16(t2), _bf16(PhiR), optimize=True))

    Md = tt.banded_to_dense(prob["M"], p)
    Kd = tt.banded_to_dense(prob["K"], p)
    x = prob["x"]
    Mf = [apply(prob["PhiL_M"], Md, prob["PhiR_M"], x[l]) for l in range(3)]
    Kf = [apply(prob["PhiL_K"], Kd, prob["PhiR_K"], x[l]) for l in range(3)]
    return np.stack(kkt_rows(Mf, Kf, beta))


def test_bf16_rounding_helper():
    """The test's rounding: exact values stay, halfway cases go to the even neighbour."""
    one_ulp = 2.0 ** -7  # bfloat16 spacing in [1, 2)
    v = np.array([1.0, 1.0 + one_ulp, 1.0 + one_ulp / 2, 1.0 + 1.5 * one_ulp, -3.0, 0.0])
    assert np.array_equal(_bf16(v), [1.0, 1.0 + one_ulp, 1.0, 1.0 + 2 * one_ulp, -3.0, 0.0])


@pytest.mark.parametrize("r,RM,RK,n,p,rr", [(3, 1, 2, 5, 1, None), (5, 2, 3, 9, 2, None), (7, 3, 5, 13, 3, 4),
                                             (1, 1, 3, 6, 2, 4), (17, 2, 9, 23, 3, None), (40, 3, 20, 37, 3, 24)])
def test_local_matvec_bf16_matches_oracle(gpu_ctx, r, RM, RK, n, p, rr):
    """Against the exact product (rounding bound) and against the written-out BF16 arithmetic:
    the kernel's FP32 intermediates differ from the FP64-accumulated ones by ~1e-7, which moves
    a bfloat16 rounding only for values within that of a midpoint, so 1e-3 is ample there."""
    from paper_1811_06797_amd import iga
    prob = synth.random_local_problem(r, RM, RK, n, p, seed=r + n, r_right=rr)
    beta = 1e-3
    y = _run(gpu_ctx, prob, r, n, p, RM, RK, beta, iga.BF16, rr)
    exact = rel_err(y, _reference(prob, p, beta))
    assert exact < BF16_TOL
    assert exact > 1e-5  # the products really are in reduced precision
    assert rel_err(y, _reference_bf16(prob, p, beta)) < 1e-3


def test_local_matvec_bf16_benchmark_shape(gpu_ctx):
    """At (32, 10, 60, 64, 3), with millions of intermediates, the midpoint moves average
    out: the product matches the written-out BF16 arithmetic to 2e-4 (an unrounded operand
    would leave ~1e-3)."""
    from paper_1811_06797_amd import iga
    r, RM, RK, n, p = 32, 10, 60, 64, 3
    prob = synth.random_local_problem(r, RM, RK, n, p, seed=1)
    y = _run(gpu_ctx, prob, r, n, p, RM, RK, 1e-6, iga.BF16)
    assert rel_err(y, _reference(prob, p, 1e-6)) < BF16_TOL
    assert rel_err(y, _reference_bf16(prob, p, 1e-6)) < 2e-4


def _sampled_reference(prob, p, beta, samples):
    """Outputs y[l][a', i, b'] of the local matvec written out one by one from the definition
    sum PhiL[al][a'][a] A[al][i][j][be] x[a][j][b] PhiR[be][b'][b] over the band j = i + o - p
    (the full product is out of reach of the oracle at these sizes)."""
    x = prob["x"]

    def one(PhiL, core, PhiR, xl, a1, i, b1):
        n = xl.shape[1]
        js = [i + o - p for o in range(2 * p + 1) if 0 <= i + o - p < n]
        os_ = [j - i + p for j in js]
        t1 = np.einsum("pa,ajb->pjb", PhiL[:, a1, :], xl[:, js, :])
        t2 = np.einsum("pjq,pjb->qb", core[:, i, os_, :], t1)
        return np.einsum("qb,qb->", t2, PhiR[:, b1, :])

    out = []
    for (a1, i, b1) in samples:
        Mf = [one(prob["PhiL_M"], prob["M"], prob["PhiR_M"], x[l], a1, i, b1) for l in range(3)]
        Kf = [one(prob["PhiL_K"], prob["K"], prob["PhiR_K"], x[l], a1, i, b1) for l in range(3)]
        out.append(kkt_rows(Mf, Kf, beta))
    return np.array(out)  # [sample][row]


@pytest.mark.parametrize("shape", [(40, 15, 80, 128, 3), (40, 10, 60, 256, 3)])
def test_local_matvec_full_size_sampled(gpu_ctx, shape):
    """The n = 128 and n = 256 benchmark shapes (r, R_M, R_K, n, p): 24 sampled outputs of each
    of the three rows against the definition, including the first and last rows of the band."""
    from paper_1811_06797_amd import iga
    r, RM, RK, n, p = shape
    prob = synth.random_local_problem(r, RM, RK, n, p, seed=7)
    rng = np.random.default_rng(11)
    samples = [(int(rng.integers(r)), int(i), int(rng.integers(r)))
               for i in [0, 1, 2, n // 2, n - 3, n - 2, n - 1] + list(rng.integers(0, n, 17))]
    ref = _sampled_reference(prob, p, 1e-6, samples)
    y = _run(gpu_ctx, prob, r, n, p, RM, RK, 1e-6, iga.FP64)
    got = np.array([[y[l, a1, i, b1] for l in range(3)] for (a1, i, b1) in samples])
    assert rel_err(got, ref) < 1e-12
    y32 = _run(gpu_ctx, prob, r, n, p, RM, RK, 1e-6, iga.FP32)
    got32 = np.array([[y32[l, a1, i, b1] for l in range(3)] for (a1, i, b1) in samples])
    assert rel_err(got32, ref) < FP32_TOL


def test_local_matvec_flops_formula():
    from paper_1811_06797_amd import iga
    r, RM, RK, n, p = 32, 10, 60, 64, 3
    nnz = sum(min(n - 1, i + p) - max(0, i - p) + 1 for i in range(n))
    per = lambda R: 2 * r * r * R * n * r + 2 * r * r * R * R * nnz + 2 * r * n * R * r * r
    assert abs(iga.local_matvec_flops(r, n, r, p, RM, RM, RK, RK) - (3 * per(RM) + 2 * per(RK))) < 1.0
