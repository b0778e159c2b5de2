"""GPU parity of TT rounding (iga_tt_round) against the oracle's TT-SVD of the expanded tensor.

Rounding a TT x to rel_tol runs the library's truncation SVDs (pivoted Householder QR of each
unfolding, then the Jacobi iteration on the small factor) after a right-to-left
orthogonalisation; the oracle expands x and runs LAPACK's TT-SVD with the same per-unfolding
tolerance rel_tol / sqrt(2) ||x||. In exact arithmetic both give the same truncation, so where
the singular values have a clear gap at the cut the two results agree elementwise to rounding;
in general each is within rel_tol ||x|| of x and their ranks agree up to one.
"""
import numpy as np
import pytest

from oracle import tt

pytestmark = pytest.mark.gpu


def _random_cores(n, r, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [scale * rng.standard_normal((r[d], n[d], r[d + 1])) for d in range(3)]


def _tt_sum(a, b):
    """Cores of the TT of full(a) + full(b) (ranks add)."""
    a0, a1, a2 = a
    b0, b1, b2 = b
    c0 = np.concatenate([a0, b0], axis=2)
    c1 = np.zeros((a1.shape[0] + b1.shape[0], a1.shape[1], a1.shape[2] + b1.shape[2]))
    c1[:a1.shape[0], :, :a1.shape[2]] = a1
    c1[a1.shape[0]:, :, a1.shape[2]:] = b1
    c2 = np.concatenate([a2, b2], axis=0)
    return [c0, c1, c2]


def _round(gpu_ctx, cores, rel_tol):
    from paper_1811_06797_amd import iga
    h = iga.tt_create(gpu_ctx, cores)
    try:
        o = iga.tt_round(gpu_ctx, h, rel_tol)
        try:
            n, r = iga.tt_info(o)
            out = iga.tt_get_cores(gpu_ctx, o)
        finally:
            iga.tt_destroy(o)
    finally:
        iga.tt_destroy(h)
    return r, out


@pytest.mark.parametrize("n, rb", [((20, 24, 18), (6, 6)), ((60, 64, 50), (40, 40))])
def test_round_low_rank_plus_small_matches_oracle(gpu_ctx, n, rb):
    """x = a + 1e-9 b, a of ranks (3, 4), b of ranks rb: rounding to 1e-6 recovers ranks (3, 4),
    and with singular-value gaps of about 1e9 at both cuts the library's result equals the
    oracle's TT-SVD of full(x) elementwise. With rb = (40, 40) every unfolding has more than 32
    columns, so each truncation SVD runs behind the pivoted QR step."""
    a = _random_cores(n, (1, 3, 4, 1), seed=1)
    b = _random_cores(n, (1,) + rb + (1,), seed=2)
    b[0] *= 1e-9
    x = _tt_sum(a, b)
    X = tt.tt_full(x)
    r, out = _round(gpu_ctx, x, 1e-6)
    ref = tt.tt_svd(X, 1e-6)
    assert r == [1, 3, 4, 1]
    assert [c.shape[2] for c in ref[:2]] == [3, 4]
    Y, Yref = tt.tt_full(out), tt.tt_full(ref)
    scale = np.abs(X).max()
    assert np.abs(Y - Yref).max() <= 1e-12 * scale
    assert np.linalg.norm(Y - X) <= 1e-6 * np.linalg.norm(X)
    # the first core is left-orthonormal, as in the oracle's TT-SVD
    U = out[0].reshape(n[0], 3)
    assert np.abs(U.T @ U - np.eye(3)).max() < 1e-13


def test_round_zero_tolerance_keeps_the_tensor(gpu_ctx):
    """Redundant ranks (30, 25) at n = (10, 12, 9): tolerance 0 keeps every nonzero singular value,
    so the ranks fall to the unfoldings' ranks (10, 9) and the tensor is unchanged to rounding."""
    n = (10, 12, 9)
    x = _random_cores(n, (1, 30, 25, 1), seed=3)
    X = tt.tt_full(x)
    r, out = _round(gpu_ctx, x, 0.0)
    assert r == [1, 10, 9, 1]
    assert np.abs(tt.tt_full(out) - X).max() <= 1e-13 * np.abs(X).max()


@pytest.mark.parametrize("rel_tol", [1e-4, 1e-8, 1e-11])
def test_round_smooth_tensor_error_and_ranks(gpu_ctx, rel_tol):
    """A smooth tensor stored with doubled ranks (x = t + t): the rounding's error is within
    rel_tol ||x||, its ranks are within one of the oracle's TT-SVD ranks of full(x) at the same
    tolerance, and the two reconstructions differ by at most 2 rel_tol ||x|| elementwise."""
    n = (26, 31, 22)
    g = np.meshgrid(np.linspace(0, 1, n[0]), np.linspace(0, 1, n[1]), np.linspace(0, 1, n[2]), indexing="ij")
    F = 1.0 / (1.0 + g[0] + 2.0 * g[1] + 3.0 * g[2]) + 0.1 * np.sin(4.0 * g[0] * g[1] + g[2])
    t = tt.tt_svd(F, 1e-14)
    x = _tt_sum(t, t)
    X = tt.tt_full(x)
    r, out = _round(gpu_ctx, x, rel_tol)
    ref = tt.tt_svd(X, rel_tol)
    Y = tt.tt_full(out)
    nx = np.linalg.norm(X)
    assert np.linalg.norm(Y - X) <= rel_tol * nx * (1 + 1e-6) + 1e-14 * nx
    for d in (1, 2):
        assert abs(r[d] - ref[d - 1].shape[2]) <= 1, (r, [c.shape for c in ref])
    assert np.abs(Y - tt.tt_full(ref)).max() <= 2 * rel_tol * nx + 1e-13 * nx


def test_round_zero_tensor(gpu_ctx):
    """The zero tensor (ranks (2, 3)) rounds to ranks (1, 1), the smallest the format holds, with
    every entry exactly zero and no NaN from the zero singular values."""
    n = (7, 5, 6)
    x = [np.zeros((1, 7, 2)), np.zeros((2, 5, 3)), np.zeros((3, 6, 1))]
    r, out = _round(gpu_ctx, x, 1e-6)
    assert r == [1, 1, 1, 1]
    Y = tt.tt_full(out)
    assert Y.shape == n
    assert np.all(Y == 0.0)
    assert all(np.all(np.isfinite(c)) for c in out)


def test_round_refusals(gpu_ctx):
    from paper_1811_06797_amd import iga
    h = iga.tt_create(gpu_ctx, _random_cores((4, 5, 6), (1, 2, 2, 1), seed=4))
    try:
        for bad in (-1e-3, 1.0):
            with pytest.raises(iga.IgaError):
                iga.tt_round(gpu_ctx, h, bad)
    finally:
        iga.tt_destroy(h)
