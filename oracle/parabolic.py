"""Time-dependent (parabolic) KKT system of the control problem (Section 4).

Test infrastructure only (see oracle/__init__.py).

Implicit Euler in time with step tau and N_t steps, rectangle rule for the
objective, y_0 = 0. With the states, controls and multipliers of all steps
stacked step-major inside each component, y = [y_1; ..; y_Nt] (likewise u,
lambda), the conditions grad L = 0 of the time-discrete Lagrangian read
(eq. KKTSystem)

    [ tau calM    0            calK^T    ] [y]     [tau calM yhat]
    [ 0           tau b calM  -tau calM  ] [u]  =  [     0       ]
    [ calK       -tau calM     0         ] [l]     [     0       ]

with calM = I_Nt (x) M and calK = I_Nt (x) tau K + C (x) M, C the Nt x Nt lower
bidiagonal matrix with 1 on the diagonal and -1 below it (the backward
difference of the implicit Euler step).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla


def time_difference(nt: int):
    """C: 1 on the diagonal, -1 on the first subdiagonal (eq. KKTSystem)."""
    return sps.diags([np.ones(nt), -np.ones(nt - 1)], [0, -1], shape=(nt, nt), format="csr")


def calM(M, nt: int):
    return sps.kron(sps.identity(nt, format="csr"), M, format="csr")


def calK(M, K, nt: int, tau: float):
    return sps.kron(sps.identity(nt, format="csr"), tau * K, format="csr") + sps.kron(time_difference(nt), M,
                                                                                        format="csr")


def kkt_matrix(M, K, beta: float, nt: int, tau: float):
    Mc = calM(M, nt)
    Kc = calK(M, K, nt, tau)
    return sps.bmat([[tau * Mc, None, Kc.T], [None, tau * beta * Mc, -tau * Mc], [Kc, -tau * Mc, None]],
                    format="csc")


def yhat_sequence(yhat, nt: int):
    """The desired state of every step: yhat given per step ([nt][N]) or one state for all."""
    y = np.asarray(yhat, dtype=np.float64)
    if y.ndim == 2 and y.shape[0] == nt:
        return y
    return np.tile(y.ravel(), (nt, 1))


def kkt_rhs(M, yhat, nt: int, tau: float):
    Y = yhat_sequence(yhat, nt)
    top = np.concatenate([tau * (M @ Y[k]) for k in range(nt)])
    z = np.zeros_like(top)
    return np.concatenate([top, z, z])


def kkt_apply(M, K, beta, nt, tau, f):
    """A f for f = [y; u; lambda], each [nt][N] stacked."""
    return kkt_matrix(M, K, beta, nt, tau) @ np.asarray(f).ravel()


def solve_direct(M, K, beta, nt, tau, yhat):
    """Direct sparse LU solve; returns (y, u, lambda), each [nt][N]."""
    A = kkt_matrix(M, K, beta, nt, tau)
    b = kkt_rhs(M, yhat, nt, tau)
    f = spla.splu(A).solve(b)
    return f.reshape(3, nt, -1)


def objective(M, y, u, yhat, beta, tau):
    """sum_k tau/2 ((y_k - yhat_k)^T M (y_k - yhat_k) + beta u_k^T M u_k) (eq. timeDiscrete, discrete)."""
    y = np.asarray(y)
    nt = y.shape[0]
    Y = yhat_sequence(yhat, nt)
    J = 0.0
    for k in range(nt):
        e = y[k] - Y[k]
        J += 0.5 * tau * (e @ (M @ e) + beta * (u[k] @ (M @ u[k])))
    return J


def residual(M, K, beta, nt, tau, yhat, f):
    b = kkt_rhs(M, yhat, nt, tau)
    return np.linalg.norm(kkt_apply(M, K, beta, nt, tau, f) - b) / np.linalg.norm(b)
