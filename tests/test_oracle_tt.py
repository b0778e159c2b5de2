"""Pins of the oracle's TT layer (Sections 3 and 5): expansion, TT-SVD, frame, projections."""
import numpy as np
import pytest

import synth
from oracle import assembly, tt
from oracle.assembly import matrix_1d


def test_tt_full_rank_one_is_outer_product():
    rng = np.random.default_rng(0)
    a, b, c = rng.standard_normal(4), rng.standard_normal(5), rng.standard_normal(3)
    T = tt.tt_full([a.reshape(1, 4, 1), b.reshape(1, 5, 1), c.reshape(1, 3, 1)])
    assert np.allclose(T, np.einsum("i,j,k->ijk", a, b, c), atol=1e-15)


def test_tt_svd_accuracy_and_exact_rank():
    cores = synth.random_tt([6, 7, 5], [3, 2], seed=1)
    A = tt.tt_full(cores)
    got = tt.tt_svd(A, 1e-12)
    assert [c.shape[2] for c in got[:-1]] == [3, 2]
    assert np.linalg.norm(tt.tt_full(got) - A) < 1e-13 * np.linalg.norm(A)
    rng = np.random.default_rng(2)
    B = A + 1e-4 * rng.standard_normal(A.shape)
    for eps in (1e-2, 1e-5):
        g = tt.tt_svd(B, eps)
        assert np.linalg.norm(tt.tt_full(g) - B) <= eps * np.linalg.norm(B) * (1 + 1e-12)


def test_ttm_full_kronecker_and_laplace_form():
    n, p = 4, 2
    M1 = matrix_1d(n, p, trim=True)
    K1 = matrix_1d(n, p, 1, 1, trim=True)
    dense = [M1.reshape(1, n, n, 1)] * 3
    assert np.allclose(tt.ttm_full(dense), np.kron(np.kron(M1, M1), M1), atol=1e-16)
    # rank-(2,2) TT-matrix of K1(x)M(x)M + M(x)K1(x)M + M(x)M(x)K1
    c1 = np.stack([K1, M1], axis=-1).reshape(1, n, n, 2)
    c2 = np.zeros((2, n, n, 2))
    c2[0, :, :, 0] = M1
    c2[1, :, :, 0] = K1
    c2[1, :, :, 1] = M1
    c3 = np.stack([M1, K1], axis=0).reshape(2, n, n, 1)
    ref = sum(np.kron(np.kron(a, b), c) for a, b, c in [(K1, M1, M1), (M1, K1, M1), (M1, M1, K1)])
    assert np.allclose(tt.ttm_full([c1, c2, c3]), ref, atol=1e-15)
    # banded storage round trip
    assert np.array_equal(tt.banded_to_dense(tt.dense_to_banded(c2, p), p), c2)


def _orthonormalise(cores, d):
    """Left-orthonormal cores before d, right-orthonormal after d (by QR)."""
    cores = [c.copy() for c in cores]
    for k in range(d):
        r0, n, r1 = cores[k].shape
        Q, R = np.linalg.qr(cores[k].reshape(r0 * n, r1))
        cores[k] = Q.reshape(r0, n, -1)
        cores[k + 1] = np.einsum("ab,bjc->ajc", R, cores[k + 1])
    for k in range(len(cores) - 1, d, -1):
        r0, n, r1 = cores[k].shape
        Q, R = np.linalg.qr(cores[k].reshape(r0, n * r1).T)
        cores[k] = Q.T.reshape(-1, n, r1)
        cores[k - 1] = np.einsum("ajb,cb->ajc", cores[k - 1], R)
    return cores


@pytest.mark.parametrize("d", [0, 1, 2])
def test_frame_linearity_and_orthogonality(d):
    """f = F_{!=d} vec(F_d) (eq. ttlin); orthonormal neighbours give F^T F = I."""
    cores = _orthonormalise(synth.random_tt([4, 5, 3], [2, 3], seed=3), d)
    F = tt.frame(cores, d)
    assert np.allclose(F @ cores[d].ravel(), tt.tt_full(cores).ravel(), atol=1e-14)
    assert np.allclose(F.T @ F, np.eye(F.shape[1]), atol=1e-13)


@pytest.mark.parametrize("d", [0, 1, 2])
def test_local_apply_is_projected_operator(d):
    """Interfaces contracted core by core give F^T A F x (the reduced matrices of eq. KKT_red)."""
    rng = np.random.default_rng(4)
    ns, p = [4, 5, 4], 1
    X = synth.random_tt(ns, [2, 3], seed=5)
    Rk = [1, 2, 3, 1]
    A = [tt.banded_to_dense(rng.standard_normal((Rk[k], ns[k], 2 * p + 1, Rk[k + 1])), p) for k in range(3)]
    L, R = tt.interfaces_from_cores(X, A, X, d)
    x = rng.standard_normal(X[d].shape)
    y = tt.local_apply(L, A[d], R, x)
    F = tt.frame(X, d)
    ref = F.T @ (tt.ttm_full(A) @ (F @ x.ravel()))
    assert np.allclose(y.ravel(), ref, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("ell", [0, 1, 2])
def test_btt_full_is_the_frame_times_the_component_slice(ell):
    """Component l of a block-TT is F_{!=ell} vec(F_ell(l)) (eqs. btt and ttlin): the frame of
    the plain cores times slice l of the core that carries the component index."""
    rng = np.random.default_rng(7)
    ns, r = [4, 3, 5], [1, 2, 3, 1]
    cores = [rng.standard_normal((r[d], ns[d], r[d + 1])) for d in range(3)]
    cores[ell] = rng.standard_normal((3, r[ell], ns[ell], r[ell + 1]))
    full = tt.btt_full(cores, ell)
    assert full.shape == (3, *ns)
    for l in range(3):
        plain = [c if d != ell else c[l] for d, c in enumerate(cores)]
        F = tt.frame(plain, ell)
        assert np.allclose(full[l].ravel(), F @ cores[ell][l].ravel(), atol=1e-13)


def test_btt_full_of_rank_one_cores_is_an_outer_product_per_component():
    rng = np.random.default_rng(8)
    a = rng.standard_normal(4)
    b3 = rng.standard_normal((3, 5))
    c = rng.standard_normal(2)
    cores = [a.reshape(1, 4, 1), b3.reshape(3, 1, 5, 1), c.reshape(1, 2, 1)]
    full = tt.btt_full(cores, 1)
    for l in range(3):
        assert np.allclose(full[l], np.einsum("i,j,k->ijk", a, b3[l], c), atol=1e-15)


def test_tt_svd_with_the_ranks_it_chose_gives_the_same_tensor():
    """tt_svd_ranks at the ranks tt_svd picked for a tolerance reproduces tt_svd's tensor; at
    full ranks it reproduces the input exactly; ranks one lower give a larger error."""
    rng = np.random.default_rng(3)
    x = np.linspace(0, 1, 9)
    A = np.einsum("i,j,k->ijk", np.sin(x), np.cos(2 * x), np.exp(x)) + 1e-3 * rng.standard_normal((9, 9, 9))
    for eps in (1e-1, 1e-2):
        ref = tt.tt_svd(A, eps)
        ranks = [ref[0].shape[2], ref[1].shape[2]]
        got = tt.tt_svd_ranks(A, ranks)
        assert np.allclose(tt.tt_full(got), tt.tt_full(ref), atol=1e-13 * np.abs(A).max())
    full = tt.tt_svd_ranks(A, [9, 9])
    assert np.allclose(tt.tt_full(full), A, atol=1e-13 * np.abs(A).max())
    e_hi = np.linalg.norm(tt.tt_full(tt.tt_svd_ranks(A, [3, 3])) - A)
    e_lo = np.linalg.norm(tt.tt_full(tt.tt_svd_ranks(A, [2, 2])) - A)
    assert e_lo > e_hi
