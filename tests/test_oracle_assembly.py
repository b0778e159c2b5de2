"""Pins of the oracle's 3-D Galerkin assembly (Sections 2, 3, 6.1).

Each test checks the oracle against something it does not compute itself:
Kronecker closed forms on the identity and affine maps, volumes by an
independent quadrature, exact energies of the physical coordinate functions,
the rank-1 structure of the quarter annulus claimed in Section 6.1, and the
consistency of the matrix-free apply with the assembled matrices.
"""
import numpy as np
import pytest

import synth
from oracle import assembly, bspline, geometry
from oracle.assembly import matrix_1d


def kron3(a, b, c):
    return np.kron(np.kron(a, b), c)


@pytest.mark.parametrize("p,n", [(2, 5), (3, 5)])
def test_identity_is_kronecker(p, n):
    M, K = assembly.assemble(synth.identity_geometry(), n, p, trim=False)
    M1 = matrix_1d(n, p)
    K1 = matrix_1d(n, p, 1, 1)
    assert np.abs(M.toarray() - kron3(M1, M1, M1)).max() < 1e-15
    Kref = kron3(K1, M1, M1) + kron3(M1, K1, M1) + kron3(M1, M1, K1)
    assert np.abs(K.toarray() - Kref).max() < 1e-13


def test_affine_map_closed_form():
    """Constant Jacobian A: omega = |det A|, Q = (A^T A)^-1 omega, K = sum_kl q_kl (d_l on i, d_k on j)."""
    A = np.array([[1.2, 0.3, 0.1], [-0.2, 0.9, 0.25], [0.15, -0.1, 1.1]])
    geo = synth.affine_geometry(A, (0.5, -1.0, 2.0))
    n, p = 4, 2
    M, K = assembly.assemble(geo, n, p, trim=False)
    om = abs(np.linalg.det(A))
    Q = np.linalg.inv(A.T @ A) * om
    d = [[matrix_1d(n, p, di, dj) for dj in (0, 1)] for di in (0, 1)]
    Kref = 0
    for k in range(3):
        for l in range(3):
            f = [d[int(l == dd)][int(k == dd)] for dd in range(3)]
            Kref = Kref + Q[k, l] * kron3(*f)
    M1 = matrix_1d(n, p)
    assert np.abs(M.toarray() - om * kron3(M1, M1, M1)).max() < 1e-14
    assert np.abs(K.toarray() - Kref).max() < 1e-12


def _volume_and_moments(geo, nq=8):
    """int 1, int x_a over the mapped domain by Gauss on the geometry's own knot spans."""
    pts, wts = [], []
    for d in range(3):
        p_, w_ = bspline.gauss_rule(geo.knots[d], nq)
        pts.append(p_.ravel())
        wts.append(w_.ravel())
    G, J = geometry.evaluate(geo, *pts)
    om = np.abs(np.linalg.det(J))
    W = np.einsum("i,j,k->ijk", *wts) * om
    return W.sum(), np.array([(W * G[a]).sum() for a in range(3)])


def _coords_in_space(geo, n, p):
    """Coefficients of the physical coordinates x_a in the solution space (exactly representable
    when the geometry space is contained in it) by interpolation at Greville points."""
    t = bspline.knot_vector(n, p)
    g = bspline.greville(t, p)
    G, _ = geometry.evaluate(geo, g, g, g)
    Binv = np.linalg.inv(bspline.basis(t, p, g))
    c = np.einsum("ai,xijk->xajk", Binv, G)
    c = np.einsum("bj,xajk->xabk", Binv, c)
    return np.einsum("ck,xabk->xabc", Binv, c).reshape(3, -1)


@pytest.mark.parametrize("geo_name", ["twisted", "perturbed"])
def test_curved_geometry_invariants(geo_name):
    """Geometry space (p=3, 5 elements) inside the solution space (p=3, 10 elements):
    sum M = |Omega|, M 1 . x_a = int x_a, K 1 = 0, and x_a^T K x_b = delta_ab |Omega| exactly,
    because J Q J^T = omega I makes that integrand a polynomial of degree <= 8 per variable."""
    geo = synth.twisted_annulus(seed=1) if geo_name == "twisted" else synth.perturbed_cube(seed=3)
    n, p = 11, 3  # N = 13 functions on E = 10 elements
    M, K = assembly.assemble(geo, n, p, trim=False)
    vol, mom = _volume_and_moments(geo)
    one = np.ones(M.shape[0])
    assert abs(one @ (M @ one) - vol) < 1e-12 * vol
    assert np.abs(K @ one).max() < 1e-10
    X = _coords_in_space(geo, n, p)
    for a in range(3):
        assert abs(X[a] @ (M @ one) - mom[a]) < 1e-11 * max(1.0, abs(mom[a]))
        for b in range(3):
            ref = vol if a == b else 0.0
            assert abs(X[a] @ (K @ X[b]) - ref) < 1e-10 * vol
    # symmetry, and definiteness after omitting the boundary functions
    Mt, Kt = assembly.assemble(geo, 4, p, trim=True)
    assert np.abs((Mt - Mt.T).toarray()).max() < 1e-15
    assert np.abs((Kt - Kt.T).toarray()).max() < 1e-13
    assert np.linalg.eigvalsh(Mt.toarray()).min() > 0
    assert np.linalg.eigvalsh(Kt.toarray()).min() > 0


def test_box_volume_and_interp_mode_exact_for_constant_weights():
    geo = synth.box_geometry(2.0, 0.5, 1.5)
    M, K = assembly.assemble(geo, 5, 2, trim=False)
    one = np.ones(M.shape[0])
    assert abs(one @ (M @ one) - 1.5) < 1e-13
    Mi, Ki = assembly.assemble(geo, 5, 2, mode="interp", trim=False)
    # the weights are constants, which the interpolation space reproduces
    assert np.abs((Mi - M).toarray()).max() < 1e-13
    assert np.abs((Ki - K).toarray()).max() < 1e-12


def _unfolding_ranks(T, tol):
    r = []
    for k in (1, 2):
        s = np.linalg.svd(T.reshape(int(np.prod(T.shape[:k])), -1), compute_uv=False)
        r.append(int((s > tol * s[0]).sum()) if s[0] > 0 else 0)
    return r


def test_quarter_annulus_weights_have_rank_one():
    """Section 6.1: every entry of Q (and omega) of the quarter annulus has TT rank 1;
    q13 and q23 vanish."""
    geo = synth.twisted_annulus(twist_deg=0.0)
    sp = assembly.Space(12, 2)
    W, _ = assembly.interpolate_weights(geo, sp)
    scale = np.abs(W).max()
    for w, name in zip(W, geometry.WEIGHT_NAMES):
        if name in ("q13", "q23"):
            assert np.abs(w).max() < 1e-11 * scale  # zero up to the rounding of the interpolation solve
        else:
            assert _unfolding_ranks(w, 1e-12) == [1, 1], name
    # a twist about the z axis keeps omega separable but not the entries of Q
    geo_t = synth.twisted_annulus(seed=1)
    Wt, _ = assembly.interpolate_weights(geo_t, sp)
    assert _unfolding_ranks(Wt[0], 1e-10) == [1, 1]
    assert max(_unfolding_ranks(Wt[1], 1e-10)) > 1


def test_interp_mode_close_to_exact_and_converges():
    geo = synth.twisted_annulus(seed=1)
    errs = []
    for n in (4, 8):
        M, K = assembly.assemble(geo, n, 2)
        Mi, Ki = assembly.assemble(geo, n, 2, mode="interp")
        errs.append(np.linalg.norm((Ki - K).toarray()) / np.linalg.norm(K.toarray()))
        assert np.linalg.norm((Mi - M).toarray()) / np.linalg.norm(M.toarray()) < 1e-3
    assert errs[1] < errs[0] < 1e-2


@pytest.mark.parametrize("mode", ["exact", "interp"])
def test_matrix_free_box_matches_assembled_rows(mode):
    geo = synth.perturbed_cube(seed=3)
    n, p = 7, 3
    M, K = assembly.assemble(geo, n, p, mode=mode)
    rng = np.random.default_rng(0)
    f = rng.standard_normal((n, n, n))
    box = ((0, 3), (2, 7), (4, 6))
    oM, oK = assembly.apply_box(geo, n, p, [f], box, mode=mode)
    refM = (M @ f.ravel()).reshape(n, n, n)[0:3, 2:7, 4:6]
    refK = (K @ f.ravel()).reshape(n, n, n)[0:3, 2:7, 4:6]
    assert np.abs(oM[0] - refM).max() < 1e-14 * np.abs(refM).max() * 10
    assert np.abs(oK[0] - refK).max() < 1e-13 * np.abs(refK).max() * 10


def test_batch_workload_geometries_do_not_fold():
    """Every geometry of the 64-problem batching workload is one-to-one: det grad G > 0 on a
    grid that reaches within 0.005 of every face (the library refuses folded maps)."""
    from oracle import geometry
    g = np.concatenate([np.linspace(0, 1, 41), [0.005, 0.995, 0.0125, 0.9875]])
    for geo, yc, c in synth.batch_problems(64):
        G, J = geometry.evaluate(geo, g, g, g)
        d = np.linalg.det(np.moveaxis(J.reshape(3, 3, -1), -1, 0)) if J.shape[0] == 3 else np.linalg.det(J)
        assert d.min() > 0, c["name"]
