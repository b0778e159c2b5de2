"""Geometry map, Jacobian and the weight functions omega and Q (Section 2).

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np

from .bspline import basis


class GeometryError(ValueError):
    """det grad G is not positive at some evaluation point (the map folds)."""


def evaluate(geo, x1, x2, x3):
    """G and grad G on the tensor grid x1 x x2 x x3.

    G(x) = C : B(x) (eq. geometryMapping); J[..., a, b] = d G_a / d xhat_b.
    Returns G of shape (3, n1, n2, n3) and J of shape (n1, n2, n3, 3, 3).
    """
    p = geo.degree
    C = np.asarray(geo.ctrl, dtype=np.float64)
    B = [basis(geo.knots[d], p, x) for d, x in enumerate((x1, x2, x3))]
    dB = [basis(geo.knots[d], p, x, deriv=1) for d, x in enumerate((x1, x2, x3))]
    G = np.einsum("aijk,pi,qj,rk->apqr", C, B[0], B[1], B[2], optimize=True)
    J = np.empty(G.shape[1:] + (3, 3))
    for a in range(3):
        J[..., a, 0] = np.einsum("ijk,pi,qj,rk->pqr", C[a], dB[0], B[1], B[2], optimize=True)
        J[..., a, 1] = np.einsum("ijk,pi,qj,rk->pqr", C[a], B[0], dB[1], B[2], optimize=True)
        J[..., a, 2] = np.einsum("ijk,pi,qj,rk->pqr", C[a], B[0], B[1], dB[2], optimize=True)
    return G, J


def weights(J, check: bool = True):
    """omega = |det J| and Q = (J^T J)^{-1} omega at every point (Section 2).

    Raises GeometryError if det J <= 0 anywhere (omega = |det| would hide a fold).
    Returns omega (...,) and Q (..., 3, 3).
    """
    det = np.linalg.det(J)
    if check and not np.all(det > 0.0):
        raise GeometryError("det grad G <= 0 at %d points" % int(np.sum(det <= 0.0)))
    omega = np.abs(det)
    JtJ = np.einsum("...ka,...kb->...ab", J, J)
    Q = np.linalg.inv(JtJ) * omega[..., None, None]
    return omega, Q


# Order of the seven weight functions used throughout: omega, then the upper
# triangle of Q row by row.
WEIGHT_NAMES = ("omega", "q11", "q12", "q13", "q22", "q23", "q33")
Q_INDEX = {"q11": (0, 0), "q12": (0, 1), "q13": (0, 2), "q22": (1, 1), "q23": (1, 2), "q33": (2, 2)}


def weight_fields(geo, x1, x2, x3, check=True):
    """The seven weight functions on a tensor grid, stacked (7, n1, n2, n3)."""
    _, J = evaluate(geo, x1, x2, x3)
    omega, Q = weights(J, check=check)
    out = [omega]
    for nm in WEIGHT_NAMES[1:]:
        k, l = Q_INDEX[nm]
        out.append(Q[..., k, l])
    return np.stack(out, axis=0)
