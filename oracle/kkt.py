"""Stationary KKT system of the Poisson control problem (Section 4 with the time dimension dropped).

Test infrastructure only (see oracle/__init__.py).

Reading of the paper for the elliptic case: one time step, tau = 1, the
time-coupling matrix C -> 0, calligraphic M -> M, calligraphic K -> K. With
the Lagrangian L = 1/2 (y-yhat)^T M (y-yhat) + beta/2 u^T M u
+ lambda^T (K y - M u) the conditions grad L = 0 read

    [ M    0    K ] [y]        [M yhat]
    [ 0   bM   -M ] [u]   =    [  0   ]
    [ K   -M    0 ] [l]        [  0   ]

(eq. KKTSystem), K symmetric.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla


def kkt_matrix(M, K, beta: float):
    return sps.bmat([[M, None, K.T], [None, beta * M, -M], [K, -M, None]], format="csc")


def kkt_rhs(M, yhat):
    y = np.asarray(yhat).ravel()
    z = np.zeros_like(y)
    return np.concatenate([M @ y, z, z])


def kkt_apply(M, K, beta, f):
    """A f for f = [y; u; lambda] (stacked, each of length n^3)."""
    f = np.asarray(f).reshape(3, -1)
    y, u, lam = f
    return np.concatenate([M @ y + K.T @ lam, beta * (M @ u) - M @ lam, K @ y - M @ u])


def solve_direct(M, K, beta, yhat):
    """Direct sparse LU solve of the KKT system; returns (y, u, lambda)."""
    A = kkt_matrix(M, K, beta)
    b = kkt_rhs(M, yhat)
    f = spla.splu(A).solve(b)
    return f.reshape(3, -1)


def objective(M, y, u, yhat, beta):
    """J = 1/2 (y-yhat)^T M (y-yhat) + beta/2 u^T M u (discrete objective of Section 4)."""
    e = np.asarray(y).ravel() - np.asarray(yhat).ravel()
    u = np.asarray(u).ravel()
    return 0.5 * e @ (M @ e) + 0.5 * beta * u @ (M @ u)


def residual(M, K, beta, yhat, f):
    """||A f - b||_2 / ||b||_2 with A f from kkt_apply and b = [M yhat; 0; 0]."""
    b = kkt_rhs(M, yhat)
    return np.linalg.norm(kkt_apply(M, K, beta, f) - b) / np.linalg.norm(b)


def solve_reduced(M, K, beta, yhat, rtol: float = 1e-13, maxiter: int = 200):
    """The KKT solution through the reduced equation for the state alone.

    Rows 2 and 3 of the KKT system give lambda = beta u and u = M^-1 K y; row 1 then becomes
        (M + beta K M^-1 K) y = M yhat,
    a symmetric positive definite system (M SPD, K symmetric). It is solved by preconditioned
    conjugate gradients, M^-1 applied through a sparse LU of M. The preconditioner is
        P = (M + g K) M^-1 (M + g K),  g = sqrt(beta),
    applied as P^-1 = (M + g K)^-1 M (M + g K)^-1 through a sparse LU of M + g K (SPD once the
    boundary functions are omitted). In the basis of the generalised eigenvectors of (K, M)
    (eigenvalues mu >= 0) the reduced matrix is diag(1 + beta mu^2) and P is diag((1 + g mu)^2),
    so the preconditioned spectrum lies in [1/2, 1] and CG converges at a rate of about 0.17
    per step whatever the mesh and beta. Stops when ||r|| <= rtol ||M yhat||.
    Returns (y, u, lambda, iterations).
    """
    M = sps.csc_matrix(M)
    K = sps.csc_matrix(K)
    g = np.sqrt(beta)
    luM = spla.splu(M)
    luP = spla.splu(sps.csc_matrix(M + g * K))

    def S(v):
        return M @ v + beta * (K @ luM.solve(K @ v))

    def Pinv(v):
        return luP.solve(M @ luP.solve(v))

    b = M @ np.asarray(yhat, dtype=np.float64).ravel()
    bn = np.linalg.norm(b)
    y = np.zeros_like(b)
    r = b.copy()
    z = Pinv(r)
    d = z.copy()
    rz = r @ z
    its = 0
    while its < maxiter and np.linalg.norm(r) > rtol * bn:
        Sd = S(d)
        a = rz / (d @ Sd)
        y += a * d
        r -= a * Sd
        z = Pinv(r)
        rz_new = r @ z
        d = z + (rz_new / rz) * d
        rz = rz_new
        its += 1
    u = luM.solve(K @ y)
    lam = beta * u
    return y, u, lam, its
