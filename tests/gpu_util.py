"""Helpers shared by the GPU parity tests (expansion of library outputs for comparison)."""
import numpy as np

from oracle import tt


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (nb if nb > 0 else 1.0)


def ttop_dense(iga, ctx, op):
    """Dense matrix of a library TT-matrix (small n only)."""
    n, R, p = iga.ttop_info(op)
    cores = [tt.banded_to_dense(iga.ttop_get_core(ctx, op, d), p) for d in range(3)]
    return tt.ttm_full(cores)


def kkt_rows(Mf, Kf, beta):
    """KKT block rows from (M f_l, K f_l) lists: [M f0 + K f2, beta M f1 - M f2, K f0 - M f1]."""
    return [Mf[0] + Kf[2], beta * Mf[1] - Mf[2], Kf[0] - Mf[1]]


def elem_err(a, b):
    """Largest elementwise difference relative to the largest entry of b: max|a - b| / max|b|
    (the element-by-element counterpart of rel_err)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    mb = np.abs(b).max() if b.size else 0.0
    return (np.abs(a - b).max() if a.size else 0.0) / (mb if mb > 0 else 1.0)
