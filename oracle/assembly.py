"""Galerkin mass and stiffness matrices by full tensor Gauss quadrature (Sections 2 and 3).

Test infrastructure only (see oracle/__init__.py).

Definitions followed:
  M_ij = int beta_i beta_j omega dxhat                 (eq. massMatrix)
  K_ij = sum_{k,l} int q_kl d_l beta_i d_k beta_j dxhat (eq. stiffnessMatrix)
with a 5-point Gauss-Legendre rule per element and direction (Section 6.1),
Dirichlet conditions imposed by omitting the boundary functions (Section 4).

Two weight modes:
  "exact"  -- omega and Q evaluated from the geometry at every quadrature point;
  "interp" -- omega and every q_kl replaced by their interpolants in the
              spline space of degree 2p+1 on the same elements, interpolated
              at its Greville points (Section 3, eq. weightEquationSystem).
              This is the integrand that the Kronecker (TT-matrix) form of
              the operators reproduces exactly when the weight tensors are
              not truncated.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sps

from .bspline import basis, gauss_rule, greville, knot_vector, uniform_knots
from .geometry import WEIGHT_NAMES, Q_INDEX, weight_fields


class Space:
    """Univariate solution space: degree p, N = n + 2 functions, E = N - p uniform elements."""

    def __init__(self, n: int, degree: int, nq: int = 5):
        self.n, self.p, self.nq = n, degree, nq
        self.N = n + 2
        self.E = self.N - degree
        self.knots = knot_vector(n, degree)
        self.pts, self.wts = gauss_rule(self.knots, nq)  # (E, nq)
        full = basis(self.knots, degree, self.pts.ravel()).reshape(self.E, nq, self.N)
        dfull = basis(self.knots, degree, self.pts.ravel(), deriv=1).reshape(self.E, nq, self.N)
        # on element e the nonzero functions are e .. e+p (open uniform knots)
        idx = np.arange(self.E)[:, None] + np.arange(degree + 1)[None, :]
        self.B = np.take_along_axis(full, idx[:, None, :].repeat(nq, axis=1), axis=2)
        self.dB = np.take_along_axis(dfull, idx[:, None, :].repeat(nq, axis=1), axis=2)
        self.first = np.arange(self.E)


class InterpSpace:
    """Weight-interpolation space of Section 3: degree pt (default 2p+1), same E elements."""

    def __init__(self, sp: Space, p_tilde: int | None = None):
        self.p = 2 * sp.p + 1 if p_tilde is None else p_tilde
        self.n = sp.E + self.p
        self.knots = uniform_knots(self.n, self.p)
        self.x = greville(self.knots, self.p)
        self.colloc = basis(self.knots, self.p, self.x)  # (n, n), B(X)


def interpolate_weights(geo, sp: Space, p_tilde: int | None = None):
    """Coefficient tensors W (omega) and V_kl (q_kl) of the interpolants, shape (7, nt, nt, nt).

    Solves vec w(X) = (B1(X1) kron B2(X2) kron B3(X3)) vec W (eq.
    weightEquationSystem) mode by mode.
    """
    it = InterpSpace(sp, p_tilde)
    F = weight_fields(geo, it.x, it.x, it.x)
    Binv = np.linalg.inv(it.colloc)
    W = np.einsum("ai,wijk->wajk", Binv, F)
    W = np.einsum("bj,wajk->wabk", Binv, W)
    W = np.einsum("ck,wabk->wabc", Binv, W)
    return W, it


def _weights_on_points(geo, sp, mode, x1, x2, x3, Wint=None):
    if mode == "exact":
        return weight_fields(geo, x1, x2, x3)
    if mode == "interp":
        W, it = Wint
        Bt = [basis(it.knots, it.p, x) for x in (x1, x2, x3)]
        out = np.einsum("wabc,pa->wpbc", W, Bt[0])
        out = np.einsum("wpbc,qb->wpqc", out, Bt[1])
        return np.einsum("wpqc,rc->wpqr", out, Bt[2])
    raise ValueError(mode)


def _block(geo, sp, mode, erange, Wint):
    """Quadrature data on the element box erange = ((a1,b1),(a2,b2),(a3,b3))."""
    pts = [sp.pts[a:b].ravel() for (a, b) in erange]
    Wq = _weights_on_points(geo, sp, mode, *pts, Wint=Wint)
    ne = [b - a for (a, b) in erange]
    nq = sp.nq
    return Wq.reshape(7, ne[0], nq, ne[1], nq, ne[2], nq)


def local_matrices(geo, sp: Space, mode="exact", erange=None, Wint=None):
    """Element matrices over an element box, one slab e1 at a time.

    Yields (e1, Mloc, Kloc) with Mloc, Kloc of shape (ne2, ne3, nl, nl), nl=(p+1)^3,
    local functions ordered (a1, a2, a3) in C order.
    """
    if erange is None:
        erange = ((0, sp.E),) * 3
    if mode == "interp" and Wint is None:
        Wint = interpolate_weights(geo, sp)
    Wq = _block(geo, sp, mode, erange, Wint)
    p1 = sp.p + 1
    (a1, b1), (a2, b2), (a3, b3) = erange
    w1, w2, w3 = sp.wts[a1:b1], sp.wts[a2:b2], sp.wts[a3:b3]
    B2, B3 = sp.B[a2:b2], sp.B[a3:b3]
    dB2, dB3 = sp.dB[a2:b2], sp.dB[a3:b3]
    for k1, e1 in enumerate(range(a1, b1)):
        B1, dB1 = sp.B[e1], sp.dB[e1]  # (nq, p1)
        # values and the three partial derivatives of the local functions at the element points:
        # shape (ne2, ne3, nq1, nq2, nq3, p1, p1, p1)
        phi = np.einsum("xa,fyb,gzc->fgxyzabc", B1, B2, B3)
        g = [np.einsum("xa,fyb,gzc->fgxyzabc", dB1, B2, B3),
             np.einsum("xa,fyb,gzc->fgxyzabc", B1, dB2, B3),
             np.einsum("xa,fyb,gzc->fgxyzabc", B1, B2, dB3)]
        ne2, ne3 = B2.shape[0], B3.shape[0]
        nq = sp.nq
        wq = np.einsum("x,fy,gz->fgxyz", w1[k1], w2, w3)  # quadrature weights
        wl = Wq[:, k1].transpose(0, 2, 4, 1, 3, 5)  # (7, ne2, ne3, nq, nq, nq)
        shp = (ne2, ne3, nq ** 3, p1 ** 3)
        phi = phi.reshape(shp)
        g = [gg.reshape(shp) for gg in g]
        wq = wq.reshape(ne2, ne3, nq ** 3)
        om = wl[0].reshape(ne2, ne3, nq ** 3)
        Mloc = np.matmul(np.swapaxes((wq * om)[..., None] * phi, -1, -2), phi)
        Q = np.empty((3, 3, ne2, ne3, nq ** 3))
        for name in WEIGHT_NAMES[1:]:
            k, l = Q_INDEX[name]
            v = wl[WEIGHT_NAMES.index(name)].reshape(ne2, ne3, nq ** 3)
            Q[k, l] = v
            Q[l, k] = v
        # K_ij = sum_{k,l} q_kl d_l beta_i d_k beta_j
        Kloc = np.zeros_like(Mloc)
        for k in range(3):
            H = sum(Q[k, l][..., None] * g[l] for l in range(3))  # sum_l q_kl d_l beta_i
            Kloc += np.matmul(np.swapaxes(wq[..., None] * H, -1, -2), g[k])
        yield e1, Mloc, Kloc


def _global_index(sp, e1, e2s, e3s):
    p1 = sp.p + 1
    a = np.arange(p1)
    i1 = e1 + a
    i2 = e2s[:, None] + a[None, :]
    i3 = e3s[:, None] + a[None, :]
    N = sp.N
    I = (i1[None, None, :, None, None] * N + i2[:, None, None, :, None]) * N + i3[None, :, None, None, :]
    return I.reshape(len(e2s), len(e3s), p1 ** 3)


def assemble(geo, n: int, degree: int, mode: str = "exact", trim: bool = True, nq: int = 5,
             Wint=None):
    """Sparse M and K over all N^3 functions, optionally restricted to the n^3 interior ones."""
    sp = Space(n, degree, nq)
    N3 = sp.N ** 3
    rows, cols, mv, kv = [], [], [], []
    e2s = np.arange(sp.E)
    e3s = np.arange(sp.E)
    for e1, Mloc, Kloc in local_matrices(geo, sp, mode, Wint=Wint):
        I = _global_index(sp, e1, e2s, e3s)
        R = np.broadcast_to(I[..., :, None], Mloc.shape)
        C = np.broadcast_to(I[..., None, :], Mloc.shape)
        rows.append(R.ravel())
        cols.append(C.ravel())
        mv.append(Mloc.ravel())
        kv.append(Kloc.ravel())
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    M = sps.csr_matrix((np.concatenate(mv), (rows, cols)), shape=(N3, N3))
    K = sps.csr_matrix((np.concatenate(kv), (rows, cols)), shape=(N3, N3))
    M.sum_duplicates()
    K.sum_duplicates()
    if trim:
        keep = interior_indices(sp.N)
        M = M[keep][:, keep]
        K = K[keep][:, keep]
    return M.tocsr(), K.tocsr()


def interior_indices(N: int) -> np.ndarray:
    """Flat C-order indices of the functions kept after omitting the boundary ones."""
    a = np.arange(1, N - 1)
    return ((a[:, None, None] * N + a[None, :, None]) * N + a[None, None, :]).ravel()


def embed(f_int: np.ndarray, N: int) -> np.ndarray:
    """Interior coefficients (n,n,n) -> full (N,N,N) with zero boundary coefficients."""
    out = np.zeros((N, N, N))
    out[1:-1, 1:-1, 1:-1] = np.asarray(f_int).reshape(N - 2, N - 2, N - 2)
    return out


def apply_box(geo, n: int, degree: int, fields, box, mode="exact", Wint=None, nq=5):
    """(M f, K f) at every interior row inside ``box`` for each field f (matrix-free).

    box = ((i1a, i1b), (i2a, i2b), (i3a, i3b)) half-open ranges of interior
    indices (0-based, 0..n-1). fields: list of interior coefficient tensors
    (n, n, n). Sums the element contributions of every element in the support
    of the box's functions -- the element-by-element definition of a
    matrix-vector product. Returns lists of arrays of the box's shape.
    """
    sp = Space(n, degree, nq)
    p = degree
    if mode == "interp" and Wint is None:
        Wint = interpolate_weights(geo, sp)
    # interior index i <-> full index i+1; function I lives on elements I-p .. I
    er = []
    for (a, b) in box:
        er.append((max(a + 1 - p, 0), min(b + 1, sp.E)))  # elements touching full indices a+1..b
    full_fields = [embed(f, sp.N) for f in fields]
    outM = [np.zeros((sp.N,) * 3) for _ in fields]
    outK = [np.zeros((sp.N,) * 3) for _ in fields]
    e2s = np.arange(*er[1])
    e3s = np.arange(*er[2])
    for e1, Mloc, Kloc in local_matrices(geo, sp, mode, erange=tuple(er), Wint=Wint):
        I = _global_index(sp, e1, e2s, e3s)
        for f, oM, oK in zip(full_fields, outM, outK):
            fe = f.ravel()[I]
            np.add.at(oM.ravel(), I.ravel(), np.einsum("fgab,fgb->fga", Mloc, fe).ravel())
            np.add.at(oK.ravel(), I.ravel(), np.einsum("fgab,fgb->fga", Kloc, fe).ravel())
    sl = tuple(slice(a + 1, b + 1) for (a, b) in box)
    return [o[sl] for o in outM], [o[sl] for o in outK]


def matrix_1d(n: int, degree: int, di: int = 0, dj: int = 0, weight=None, trim: bool = False, nq=5):
    """Univariate matrix int (d^di beta_i)(d^dj beta_j) w dx by the same Gauss rule (dense N x N)."""
    sp = Space(n, degree, nq)
    Bi = sp.dB if di else sp.B
    Bj = sp.dB if dj else sp.B
    w = sp.wts if weight is None else sp.wts * weight(sp.pts)
    A = np.zeros((sp.N, sp.N))
    for e in range(sp.E):
        loc = np.einsum("q,qa,qb->ab", w[e], Bi[e], Bj[e])
        A[e:e + degree + 1, e:e + degree + 1] += loc
    if trim:
        A = A[1:-1, 1:-1]
    return A
