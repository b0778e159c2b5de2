"""Pins of the oracle's time-dependent KKT system (Section 4, implicit Euler, eq. KKTSystem).

Each pin reaches the solution by a route other than the block matrix: the paper's
componentwise optimality conditions, the one-step reduction to the stationary system, and
the decoupling into spatial eigenmodes of the pencil (K, M).
"""
import numpy as np
import scipy.linalg as sla
import scipy.sparse.linalg as spla

import synth
from oracle import assembly, kkt, parabolic


def _problem(n=4, p=2, seed=1):
    geo = synth.twisted_annulus(seed=seed)
    M, K = assembly.assemble(geo, n, p)
    rng = np.random.default_rng(seed)
    return M, K, rng.standard_normal(n ** 3)


def test_time_difference_matrix():
    C = parabolic.time_difference(4).toarray()
    assert np.array_equal(C, [[1, 0, 0, 0], [-1, 1, 0, 0], [0, -1, 1, 0], [0, 0, -1, 1]])


def test_componentwise_conditions():
    """grad L = 0 of the time-discrete Lagrangian, step by step (Section 4):
    tau M (y_k - yhat) - M l_{k+1} + (M + tau K) l_k = 0 (l_{Nt+1} = 0),
    tau beta M u_k - tau M l_k = 0, and the implicit Euler step
    M (y_k - y_{k-1}) + tau K y_k - tau M u_k = 0 (y_0 = 0)."""
    M, K, yh = _problem()
    beta, nt, tau = 1e-2, 5, 0.1
    y, u, lam = parabolic.solve_direct(M, K, beta, nt, tau, yh)
    scale = np.linalg.norm(tau * (M @ yh))
    for k in range(nt):
        lnext = lam[k + 1] if k + 1 < nt else np.zeros_like(yh)
        yprev = y[k - 1] if k > 0 else np.zeros_like(yh)
        r1 = tau * (M @ (y[k] - yh)) - M @ lnext + (M + tau * K) @ lam[k]
        r2 = tau * beta * (M @ u[k]) - tau * (M @ lam[k])
        r3 = M @ (y[k] - yprev) + tau * (K @ y[k]) - tau * (M @ u[k])
        assert np.linalg.norm(r1) < 1e-10 * scale
        assert np.linalg.norm(r2) < 1e-10 * scale
        assert np.linalg.norm(r3) < 1e-10 * scale


def test_state_is_the_implicit_euler_march_of_its_control():
    """Given the optimal control, marching (M + tau K) y_k = M y_{k-1} + tau M u_k from y_0 = 0
    reproduces the optimal states."""
    M, K, yh = _problem()
    beta, nt, tau = 1e-3, 6, 0.05
    y, u, lam = parabolic.solve_direct(M, K, beta, nt, tau, yh)
    lu = spla.splu((M + tau * K).tocsc())
    prev = np.zeros_like(yh)
    for k in range(nt):
        prev = lu.solve(M @ prev + tau * (M @ u[k]))
        assert np.linalg.norm(prev - y[k]) < 1e-10 * np.linalg.norm(y[k])


def test_one_step_is_the_stationary_system_with_shifted_stiffness():
    """Nt = 1: dividing every row by tau gives the stationary KKT system with K + M / tau in the
    same unknowns."""
    M, K, yh = _problem()
    beta, tau = 1e-2, 0.3
    y, u, lam = parabolic.solve_direct(M, K, beta, 1, tau, yh)
    ys, us, ls = kkt.solve_direct(M, K + M / tau, beta, yh)
    assert np.linalg.norm(y[0] - ys) < 1e-10 * np.linalg.norm(ys)
    assert np.linalg.norm(u[0] - us) < 1e-10 * np.linalg.norm(us)
    assert np.linalg.norm(lam[0] - ls) < 1e-10 * np.linalg.norm(ls)


def test_spatial_eigenmodes_decouple():
    """With K V = M V diag(mu), V^T M V = I, every mode of the pencil gives its own
    3 Nt x 3 Nt system in the time coefficients (the blocks of eq. KKTSystem with M -> 1,
    K -> mu); solving them one by one and mapping back matches the sparse LU solve."""
    M, K, yh = _problem(n=3)
    beta, nt, tau = 1e-1, 4, 0.2
    y, u, lam = parabolic.solve_direct(M, K, beta, nt, tau, yh)
    mu, V = sla.eigh(K.toarray(), M.toarray())
    g = V.T @ (M @ yh)  # desired state in the M-orthonormal mode basis
    C = parabolic.time_difference(nt).toarray()
    I = np.eye(nt)
    Z = np.zeros((nt, nt))
    coef = np.zeros((3, nt, len(mu)))
    for j, m in enumerate(mu):
        Kt = tau * m * I + C
        A = np.block([[tau * I, Z, Kt.T], [Z, tau * beta * I, -tau * I], [Kt, -tau * I, Z]])
        b = np.concatenate([tau * g[j] * np.ones(nt), np.zeros(nt), np.zeros(nt)])
        coef[:, :, j] = np.linalg.solve(A, b).reshape(3, nt)
    for c, field in enumerate((y, u, lam)):
        rec = coef[c] @ V.T
        assert np.linalg.norm(rec - field) < 1e-9 * np.linalg.norm(field)


def test_objective_and_residual():
    M, K, yh = _problem()
    beta, nt, tau = 1e-2, 3, 0.1
    y, u, lam = parabolic.solve_direct(M, K, beta, nt, tau, yh)
    f = np.stack([y, u, lam])
    assert parabolic.residual(M, K, beta, nt, tau, yh, f) < 1e-12
    J = parabolic.objective(M, y, u, yh, beta, tau)
    # the optimum beats the zero control (J(0) = sum_k tau/2 yhat^T M yhat)
    assert 0 < J < 0.5 * nt * tau * yh @ (M @ yh)
