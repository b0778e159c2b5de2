"""Pins of the oracle's KKT system and direct solve (Section 4, stationary reading)."""
import math

import numpy as np
import pytest

import synth
from oracle import assembly, bspline, kkt


def _solve(geo, n, p, beta, yhat):
    M, K = assembly.assemble(geo, n, p)
    y, u, lam = kkt.solve_direct(M, K, beta, yhat)
    return M, K, y, u, lam


def test_kkt_conditions_and_dense_crosscheck():
    geo = synth.twisted_annulus(seed=1)
    n, p, beta = 5, 2, 1e-3
    rng = np.random.default_rng(0)
    yh = rng.standard_normal(n ** 3)
    M, K, y, u, lam = _solve(geo, n, p, beta, yh)
    # grad L = 0 row by row
    assert np.linalg.norm(M @ (y - yh) + K @ lam) < 1e-10 * np.linalg.norm(M @ yh)
    assert np.linalg.norm(beta * u - lam) < 1e-12 * np.linalg.norm(lam)
    assert np.linalg.norm(K @ y - M @ u) < 1e-10 * np.linalg.norm(M @ u)
    # dense LAPACK solve of the same system
    A = kkt.kkt_matrix(M, K, beta).toarray()
    f = np.linalg.solve(A, kkt.kkt_rhs(M, yh))
    assert np.abs(f - np.concatenate([y, u, lam])).max() < 1e-9 * np.abs(f).max()


def _center_value(c, n, p):
    t = bspline.knot_vector(n, p)
    b = bspline.basis(t, p, np.array([0.5]))[0, 1:-1]
    return np.einsum("ijk,i,j,k->", c.reshape(n, n, n), b, b, b)


def test_continuum_limit_identity_cube():
    """Unit cube, yhat = prod sin(pi x_d): the continuous optimum is y = yhat/(1+beta mu^2),
    u = mu y, mu = 3 pi^2 (eigenfunction of -Laplace). The discrete solution approaches it."""
    beta = 1e-4
    mu = 3 * math.pi ** 2
    amp = 1.0 / (1.0 + beta * mu ** 2)
    assert abs(amp - 0.919398) < 1e-6
    errs = []
    for n in (6, 9, 12):
        yh = np.einsum("i,j,k->ijk", *[c[0, :, 0] for c in synth.yhat_sine(n, 2)])
        M, K, y, u, lam = _solve(synth.identity_geometry(), n, 2, beta, yh.ravel())
        yc = _center_value(y, n, 2)
        uc = _center_value(u, n, 2)
        errs.append(abs(yc - amp))
        assert abs(uc / yc - mu) < 0.05 * mu
    # second order in h (the desired state is sampled at Greville points, an O(h^2) approximation)
    assert errs[0] / errs[1] > 1.7 and errs[1] / errs[2] > 1.5
    assert errs[2] < 3e-2


def test_objective_trends_in_beta():
    """Section 6.2: the objective grows and the control norm shrinks as beta grows."""
    geo = synth.twisted_annulus(seed=1)
    n, p = 5, 2
    yh = np.einsum("i,j,k->ijk", *[c[0, :, 0] for c in synth.yhat_sine(n, p)]).ravel()
    M, K = assembly.assemble(geo, n, p)
    Js, us = [], []
    for beta in (1e-4, 1e-3, 1e-2, 1e-1, 1.0):
        y, u, lam = kkt.solve_direct(M, K, beta, yh)
        Js.append(kkt.objective(M, y, u, yh, beta))
        us.append(np.linalg.norm(u))
    assert all(a < b for a, b in zip(Js, Js[1:]))
    assert all(a > b for a, b in zip(us, us[1:]))


def test_reduced_cost_gradient_envelope():
    """The KKT solution is the constrained minimiser: d J*/d yhat = -M (y - yhat) (envelope theorem),
    checked by central differences of the oracle's own solve."""
    geo = synth.perturbed_cube(seed=3)
    n, p, beta = 4, 2, 1e-2
    M, K = assembly.assemble(geo, n, p)
    rng = np.random.default_rng(1)
    yh = rng.standard_normal(n ** 3)
    y, u, lam = kkt.solve_direct(M, K, beta, yh)
    g = -(M @ (y - yh))
    h = 1e-6
    for idx in rng.choice(n ** 3, 6, replace=False):
        e = np.zeros(n ** 3)
        e[idx] = h
        Jp = kkt.objective(M, *kkt.solve_direct(M, K, beta, yh + e)[:2], yh + e, beta)
        Jm = kkt.objective(M, *kkt.solve_direct(M, K, beta, yh - e)[:2], yh - e, beta)
        assert abs((Jp - Jm) / (2 * h) - g[idx]) < 1e-6 * max(1.0, abs(g[idx]))


def _small_system(n=5, p=2, seed=1, beta=1e-3):
    geo = synth.twisted_annulus(seed=seed)
    M, K = assembly.assemble(geo, n, p)
    return M, K, beta


def test_kkt_apply_is_the_kkt_matrix_product():
    """kkt_apply(f) equals the assembled block matrix (pinned by the optimality conditions above)
    times f, block row by block row, on random vectors (Sec. 4, eq. KKTSystem)."""
    M, K, beta = _small_system()
    A = kkt.kkt_matrix(M, K, beta)
    rng = np.random.default_rng(5)
    for _ in range(3):
        f = rng.standard_normal(A.shape[0])
        ref = A @ f
        got = kkt.kkt_apply(M, K, beta, f)
        assert np.linalg.norm(got - ref) <= 1e-14 * np.linalg.norm(ref)
    # each block row separately: a unit vector in one component excites the columns of that block
    N = M.shape[0]
    for comp in range(3):
        f = np.zeros(3 * N)
        f[comp * N: (comp + 1) * N] = rng.standard_normal(N)
        assert np.linalg.norm(kkt.kkt_apply(M, K, beta, f) - A @ f) <= 1e-14 * np.linalg.norm(A @ f)


def test_kkt_apply_maps_the_optimum_to_the_rhs_and_residual_is_its_defect():
    """At the direct solution A f = b, so the relative residual vanishes to rounding; for a
    perturbed f the residual equals ||A (f + e) - b|| / ||b|| with the assembled block matrix."""
    M, K, beta = _small_system(beta=1e-2)
    rng = np.random.default_rng(6)
    yh = rng.standard_normal(M.shape[0])
    y, u, lam = kkt.solve_direct(M, K, beta, yh)
    f = np.concatenate([y, u, lam])
    assert kkt.residual(M, K, beta, yh, f) < 1e-12
    b = kkt.kkt_rhs(M, yh)
    assert np.linalg.norm(kkt.kkt_apply(M, K, beta, f) - b) < 1e-12 * np.linalg.norm(b)
    e = 1e-3 * rng.standard_normal(f.shape)
    A = kkt.kkt_matrix(M, K, beta)
    ref = np.linalg.norm(A @ (f + e) - b) / np.linalg.norm(b)
    assert abs(kkt.residual(M, K, beta, yh, f + e) - ref) <= 1e-12 * ref


@pytest.mark.parametrize("beta", [1e-2, 1e-6])
@pytest.mark.parametrize("n,p", [(6, 2), (8, 3)])
def test_reduced_solve_matches_direct_solve(n, p, beta):
    """The reduced state equation (M + beta K M^-1 K) y = M yhat, with u = M^-1 K y and lambda =
    beta u from the second and third KKT rows, gives the (y, u, lambda) of a dense LAPACK solve of
    the whole KKT matrix. At beta = 1e-6 the KKT matrix has a condition number near 1e12, so
    forward errors of ~1e-11 separate two backward-stable solves; the bar is 1e-9, and both
    solutions must leave KKT residuals at rounding level."""
    geo = synth.twisted_annulus(seed=1)
    M, K = assembly.assemble(geo, n, p, mode="interp")
    yh = np.einsum("i,j,k->ijk", *[c[0, :, 0] for c in synth.yhat_sine(n, p)]).ravel()
    yr, ur, lr, its = kkt.solve_reduced(M, K, beta, yh)
    A = kkt.kkt_matrix(M, K, beta).toarray()
    yd, ud, ld = np.linalg.solve(A, kkt.kkt_rhs(M, yh)).reshape(3, -1)
    assert its <= 40
    for a, b in ((yr, yd), (ur, ud), (lr, ld)):
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)
    assert kkt.residual(M, K, beta, yh, np.concatenate([yr, ur, lr])) < 1e-12
    # the sparse LU of the whole system agrees to within its own conditioning
    ys, us, ls = kkt.solve_direct(M, K, beta, yh)
    assert np.linalg.norm(ys - yr) <= 1e-7 * np.linalg.norm(yr)
