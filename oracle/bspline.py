"""B-spline bases (Section 2, eq. knotVector and the Cox-de Boor recursion).

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import numpy as np


def knot_vector(n_free: int, degree: int) -> np.ndarray:
    """Open uniform knot vector of the solution space.

    Reading of the paper: ``n`` counts the free (interior) unknowns per
    direction after the Dirichlet boundary functions are omitted, so the
    space has N = n + 2 B-splines on E = N - p uniform elements. The end knots
    repeat p + 1 times (eq. knotVector).
    """
    N = n_free + 2
    E = N - degree
    if E < 1:
        raise ValueError("too few functions for this degree")
    return np.concatenate([np.zeros(degree + 1), np.arange(1, E) / E, np.ones(degree + 1)])


def uniform_knots(nbasis: int, degree: int) -> np.ndarray:
    E = nbasis - degree
    return np.concatenate([np.zeros(degree + 1), np.arange(1, E) / E, np.ones(degree + 1)])


def basis(knots: np.ndarray, degree: int, x: np.ndarray, deriv: int = 0) -> np.ndarray:
    """All B-splines beta_{i,p} (or their first derivatives) at points x.

    Cox-de Boor recursion of Section 2. Reading: the degree-0 indicator is
    half-open [t_i, t_{i+1}) except on the last non-empty span, which is
    closed so that the basis is a partition of unity at x = 1; a quotient
    with zero denominator counts as zero. The derivative is the textbook
    formula p/(t_{i+p}-t_i) beta_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) beta_{i+1,p-1}
    (the paper does not state it).

    Returns an array of shape (len(x), len(knots) - degree - 1).
    """
    t = np.asarray(knots, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    m = len(t)
    last = max(i for i in range(m - 1) if t[i] < t[i + 1])
    B = np.zeros((len(x), m - 1))
    for i in range(m - 1):
        if t[i] < t[i + 1]:
            if i == last:
                B[:, i] = (x >= t[i]) & (x <= t[i + 1])
            else:
                B[:, i] = (x >= t[i]) & (x < t[i + 1])

    def frac(num, den):
        return num / den if den != 0.0 else np.zeros_like(num) if isinstance(num, np.ndarray) else 0.0

    top = degree - 1 if deriv == 1 else degree
    for j in range(1, top + 1):
        Bn = np.zeros((len(x), m - 1 - j))
        for i in range(m - 1 - j):
            left = frac(x - t[i], t[i + j] - t[i]) * B[:, i]
            right = frac(t[i + j + 1] - x, t[i + j + 1] - t[i + 1]) * B[:, i + 1]
            Bn[:, i] = left + right
        B = Bn
    if deriv == 0:
        return B
    if deriv != 1:
        raise ValueError("only first derivatives are needed")
    p = degree
    nb = m - p - 1
    dB = np.zeros((len(x), nb))
    for i in range(nb):
        a = p / (t[i + p] - t[i]) if t[i + p] != t[i] else 0.0
        b = p / (t[i + p + 1] - t[i + 1]) if t[i + p + 1] != t[i + 1] else 0.0
        dB[:, i] = a * B[:, i] - b * B[:, i + 1]
    return dB


def greville(knots: np.ndarray, degree: int) -> np.ndarray:
    nb = len(knots) - degree - 1
    return np.array([np.mean(knots[i + 1:i + degree + 1]) for i in range(nb)])


def elements(knots: np.ndarray):
    """Non-empty knot spans as (left, right) arrays."""
    u = np.unique(knots)
    return u[:-1], u[1:]


def gauss_rule(knots: np.ndarray, nq: int = 5):
    """Gauss-Legendre points and weights on every element (5 per element in the paper's runs).

    Returns (pts, wts), each of shape (E, nq).
    """
    xg, wg = np.polynomial.legendre.leggauss(nq)
    a, b = elements(knots)
    h = b - a
    pts = a[:, None] + 0.5 * h[:, None] * (xg[None, :] + 1.0)
    wts = 0.5 * h[:, None] * wg[None, :]
    return pts, wts
