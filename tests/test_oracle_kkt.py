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
