"""Tensor-train objects by their definitions (Sections 3 and 5).

Test infrastructure only (see oracle/__init__.py).

Layouts (C order, last index fastest):
  TT core             (r_{d-1}, n_d, r_d)                       eq. tt
  block-TT core       (3, r_{d-1}, n_d, r_d) at the core holding the
                      component index l, plain cores elsewhere   eq. btt
  TT-matrix core      (R_{d-1}, n_d, n_d, R_d) dense, or banded
                      (R_{d-1}, n_d, 2p+1, R_d) with column j = i + o - p
  left interface      (R, r_test, r_trial): slot alpha, test rank, trial rank
  right interface     (R, r_test, r_trial)
"""
from __future__ import annotations

import numpy as np


def tt_full(cores):
    """Full tensor of a TT: W(i1..iD) = W_1(i1) ... W_D(iD) (eq. tt)."""
    out = np.asarray(cores[0])
    for c in cores[1:]:
        out = np.tensordot(out, c, axes=(out.ndim - 1, 0))
    return out.reshape(out.shape[1:-1])


def btt_full(cores, ell_core: int):
    """The three components f_l of a block-TT (eq. btt), shape (3, n1, ..., nD)."""
    out = []
    for l in range(3):
        cs = [c if d != ell_core else c[l] for d, c in enumerate(cores)]
        out.append(tt_full(cs))
    return np.stack(out)


def banded_to_dense(core, degree: int):
    """(R0, n, 2p+1, R1) banded core -> (R0, n, n, R1) dense core."""
    R0, n, b, R1 = core.shape
    D = np.zeros((R0, n, n, R1))
    for i in range(n):
        for o in range(b):
            j = i + o - degree
            if 0 <= j < n:
                D[:, i, j, :] = core[:, i, o, :]
    return D


def dense_to_banded(core, degree: int):
    R0, n, _, R1 = core.shape
    b = 2 * degree + 1
    out = np.zeros((R0, n, b, R1))
    for i in range(n):
        for o in range(b):
            j = i + o - degree
            if 0 <= j < n:
                out[:, i, o, :] = core[:, i, j, :]
    return out


def ttm_full(dense_cores):
    """Dense matrix of a TT-matrix: sum over rank indices of Kronecker products (eq. M_kron)."""
    out = dense_cores[0]  # (1, n, n, R)
    for c in dense_cores[1:]:
        # out: (1, I, J, R), c: (R, n, n, R')
        t = np.einsum("aijr,rklb->aikjlb", out, c)
        s = t.shape
        out = t.reshape(s[0], s[1] * s[2], s[3] * s[4], s[5])
    return out[0, :, :, 0]


def tt_svd(A, eps: float):
    """TT-SVD (Oseledets 2011): sequential truncated SVDs of the unfoldings.

    Each step drops the trailing singular values whose squared sum stays
    below (eps / sqrt(D-1) * ||A||_F)^2. Returns the cores.
    """
    A = np.asarray(A, dtype=np.float64)
    shape = A.shape
    D = len(shape)
    delta = eps / np.sqrt(D - 1) * np.linalg.norm(A)
    cores = []
    r = 1
    C = A.copy()
    for d in range(D - 1):
        C = C.reshape(r * shape[d], -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        tail = np.sqrt(np.cumsum((s ** 2)[::-1]))[::-1]  # tail[k] = ||s[k:]||
        rk = len(s)
        for k in range(len(s)):
            if tail[k] <= delta:
                rk = k
                break
        rk = max(rk, 1) if np.linalg.norm(A) > 0 else 0
        if rk == 0:
            return None
        cores.append(U[:, :rk].reshape(r, shape[d], rk))
        C = s[:rk, None] * Vt[:rk]
        r = rk
    cores.append(C.reshape(r, shape[-1], 1))
    return cores


def tt_svd_ranks(A, ranks):
    """TT-SVD with prescribed ranks (r_1, .., r_{D-1}): the sequential SVDs of the unfoldings of
    tt_svd, each kept to the given rank instead of a tolerance. With the ranks tt_svd chose at a
    tolerance it returns the same tensor; used to rebuild a truncation whose ranks are known."""
    A = np.asarray(A, dtype=np.float64)
    shape = A.shape
    D = len(shape)
    if len(ranks) != D - 1:
        raise ValueError("need D - 1 ranks")
    cores = []
    r = 1
    C = A.copy()
    for d in range(D - 1):
        C = C.reshape(r * shape[d], -1)
        U, s, Vt = np.linalg.svd(C, full_matrices=False)
        rk = int(ranks[d])
        if not 1 <= rk <= len(s):
            raise ValueError("rank %d out of range at unfolding %d" % (rk, d))
        cores.append(U[:, :rk].reshape(r, shape[d], rk))
        C = s[:rk, None] * Vt[:rk]
        r = rk
    cores.append(C.reshape(r, shape[-1], 1))
    return cores


def frame(cores, d: int):
    """Frame matrix F_{!=d} (eq. frame): shape (prod n, r_{d-1} n_d r_d).

    Column (a, j, b) is X_{<d}[..., a] (x) e_j (x) X_{>d}[b, ...].
    """
    ns = [c.shape[1] for c in cores]
    left = np.ones((1, 1))
    for c in cores[:d]:
        left = np.einsum("Ia,ajb->Ijb", left, c).reshape(-1, c.shape[2])
    right = np.ones((1, 1))
    for c in reversed(cores[d + 1:]):
        right = np.einsum("ajb,bJ->ajJ", c, right).reshape(c.shape[0], -1)
    nd = ns[d]
    F = np.einsum("Ia,ij,bJ->IiJajb", left, np.eye(nd), right)
    P = left.shape[0] * nd * right.shape[1]
    return F.reshape(P, left.shape[1] * nd * right.shape[0])


def projected(Afull, F):
    """F^T A F, the projected submatrix of eq. KKT_red."""
    return F.T @ (Afull @ F)


# The three contractions below are each one einsum of their definition. The order of the
# pairwise products is given explicitly ("einsum_path" lists, operands numbered as passed,
# each product appended to the end of the list): numpy's automatic choice under its default
# memory limit can fall back to a single naive loop over all eight indices, which takes
# minutes at ranks of a few tens.


def local_apply(PhiL, A_dense, PhiR, x):
    """y[a',i,b'] = sum PhiL[al,a',a] A[al,i,j,be] x[a,j,b] PhiR[be,b',b] (the local projected matvec).

    One contraction over (al, a, j, be, b), written as the definition of eq. KKT_red's reduced
    operator applied to a core; evaluated as (PhiL x), then A, then PhiR.
    """
    return np.einsum("pxa,pijq,ajb,qyb->xiy", PhiL, A_dense, x, PhiR,
                     optimize=["einsum_path", (0, 2), (0, 2), (0, 1)])


def interface_left(PhiL, U, A_dense, V):
    """Phi'[be,b',b] = sum U[a',i,b'] PhiL[al,a',a] A[al,i,j,be] V[a,j,b] (one contraction;
    evaluated as (PhiL V), then A, then U)."""
    return np.einsum("xiy,pxa,pijq,ajb->qyb", U, PhiL, A_dense, V,
                     optimize=["einsum_path", (1, 3), (1, 2), (0, 1)])


def interface_right(PhiR, U, A_dense, V):
    """Phi'[al,a',a] = sum U[a',i,b'] PhiR[be,b',b] A[al,i,j,be] V[a,j,b] (one contraction;
    evaluated as (V PhiR), then A, then U)."""
    return np.einsum("xiy,qyb,pijq,ajb->pxa", U, PhiR, A_dense, V,
                     optimize=["einsum_path", (1, 3), (1, 2), (0, 1)])


def interfaces_from_cores(X, A_dense_cores, Y, d: int):
    """Left and right interfaces at core d by contracting cores 0..d-1 and d+1..D-1."""
    L = np.ones((1, 1, 1))
    for k in range(d):
        L = interface_left(L, X[k], A_dense_cores[k], Y[k])
    R = np.ones((1, 1, 1))
    for k in range(len(X) - 1, d, -1):
        R = interface_right(R, X[k], A_dense_cores[k], Y[k])
    return L, R
