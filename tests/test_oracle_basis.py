"""Pins of the oracle's B-spline layer (Section 2) against library routines and identities."""
import numpy as np
import pytest
from scipy.interpolate import BSpline

from oracle import bspline
from oracle.assembly import matrix_1d


@pytest.mark.parametrize("p,n", [(1, 4), (2, 6), (3, 9), (7, 12)])
def test_basis_matches_scipy(p, n):
    t = bspline.knot_vector(n, p)
    x = np.linspace(0.0, 1.0, 97)[:-1] + 0.003
    x = np.concatenate([x, [0.0, 1.0]])
    B = bspline.basis(t, p, x)
    dB = bspline.basis(t, p, x, deriv=1)
    N = len(t) - p - 1
    for i in range(N):
        c = np.zeros(N)
        c[i] = 1.0
        s = BSpline(t, c, p, extrapolate=False)
        ref = np.nan_to_num(s(x))
        dref = np.nan_to_num(s.derivative()(x))
        assert np.allclose(B[:, i], ref, atol=1e-14, rtol=0)
        assert np.allclose(dB[:, i], dref, atol=1e-11, rtol=1e-12)


@pytest.mark.parametrize("p", [1, 2, 3, 5, 7])
def test_partition_of_unity_and_endpoint(p):
    t = bspline.knot_vector(10, p)
    x = np.linspace(0, 1, 201)
    B = bspline.basis(t, p, x)
    dB = bspline.basis(t, p, x, deriv=1)
    assert np.allclose(B.sum(1), 1.0, atol=1e-14)
    assert np.allclose(dB.sum(1), 0.0, atol=1e-11)
    assert B[-1, -1] == 1.0 and B[0, 0] == 1.0  # reading: last span closed at x = 1


def test_gauss_rule_exact_degree_9():
    t = bspline.knot_vector(7, 2)
    pts, wts = bspline.gauss_rule(t, 5)
    for deg in range(10):
        assert abs((wts * pts ** deg).sum() - 1.0 / (deg + 1)) < 1e-14
    p1, w1 = bspline.gauss_rule(bspline.knot_vector(1, 2), 5)  # a single element
    assert abs((w1 * p1 ** 9).sum() - 0.1) < 1e-15
    assert abs((w1 * p1 ** 10).sum() - 1.0 / 11) > 1e-6


def _golden():
    rows = {}
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "cardinal_factors.txt")
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        head, den = line.split("/")
        f = head.split()
        rows[(int(f[0]), f[1])] = np.array([float(v) for v in f[2:]]) / float(den)
    return rows


@pytest.mark.parametrize("p,n", [(2, 16), (3, 64), (3, 20)])
def test_univariate_factors_cardinal_closed_form(p, n):
    g = _golden()
    E = n + 2 - p
    h = 1.0 / E
    M = matrix_1d(n, p)
    K = matrix_1d(n, p, 1, 1)
    N = n + 2
    for i in range(2 * p, N - 2 * p):  # rows far enough from the boundary
        assert np.allclose(M[i, i - p:i + p + 1] / h, g[(p, "M")], atol=1e-14)
        assert np.allclose(K[i, i - p:i + p + 1] * h, g[(p, "K")], atol=1e-12)
    # mass sums to the length of the interval, stiffness kills constants
    assert abs(M.sum() - 1.0) < 1e-13
    assert np.abs(K @ np.ones(N)).max() < 1e-10
    assert np.abs(matrix_1d(n, p, 0, 1) @ np.ones(N)).max() < 1e-10
