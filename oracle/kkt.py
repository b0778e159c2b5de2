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
    b = kkt_rhs(M, yhat)
    return np.linalg.norm(kkt_apply(M, K, beta, f) - b) / np.linalg.norm(b)
