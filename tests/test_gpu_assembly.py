"""GPU parity of the TT assembly and of kkt_apply against the FP64 CPU oracle.

With weight_tol = 0 the library's Kronecker/TT operators integrate exactly the
oracle's interpolated-weight ("interp" mode) integrand, so they agree to
rounding: relative 1e-12 (Frobenius for operators, Euclidean for vectors).
"""
import numpy as np
import pytest

import synth
from oracle import assembly, geometry, kkt as okkt, tt
from tests.gpu_util import elem_err, kkt_rows, rel_err, ttop_dense

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _geo(name):
    return {
        "identity": synth.identity_geometry,
        "twisted": lambda: synth.twisted_annulus(seed=1),
        "untwisted": lambda: synth.twisted_annulus(twist_deg=0.0),
        "perturbed": lambda: synth.perturbed_cube(seed=3),
        "box": lambda: synth.box_geometry(2.0, 0.5, 1.5),
    }[name]()


@pytest.mark.parametrize("geo_name,p,n", [("identity", 2, 5), ("twisted", 3, 6), ("perturbed", 2, 5),
                                          ("untwisted", 3, 5), ("box", 1, 4), ("twisted", 2, 9)])
def test_operators_match_oracle(gpu_ctx, geo_name, p, n):
    from paper_1811_06797_amd import iga
    geo = _geo(geo_name)
    print("case", geo_name, p, n, flush=True)
    M, K, ranks = iga.assemble_factors(gpu_ctx, geo, p, n, weight_tol=0.0)
    try:
        Ml, Kl = ttop_dense(iga, gpu_ctx, M), ttop_dense(iga, gpu_ctx, K)
        Mo, Ko = assembly.assemble(geo, n, p, mode="interp")
        assert rel_err(Ml, Mo.toarray()) < TOL
        assert rel_err(Kl, Ko.toarray()) < TOL
        if geo_name in ("identity", "box"):
            Me, Ke = assembly.assemble(geo, n, p, mode="exact")
            assert rel_err(Ml, Me.toarray()) < TOL and rel_err(Kl, Ke.toarray()) < TOL
    finally:
        iga.ttop_destroy(M)
        iga.ttop_destroy(K)


def test_identity_ranks_and_kronecker_form(gpu_ctx):
    """Identity map: omega = 1 and Q = I have TT rank 1, off-diagonal q vanish,
    so M has ranks (1,1) and K = K1 M M + M K1 M + M M K1 has ranks (3,3)."""
    from paper_1811_06797_amd import iga
    M, K, ranks = iga.assemble_factors(gpu_ctx, synth.identity_geometry(), 2, 16, weight_tol=1e-10)
    try:
        assert ranks.tolist() == [[1, 1], [1, 1], [0, 0], [0, 0], [1, 1], [0, 0], [1, 1]]
        assert iga.ttop_info(M)[1] == [1, 1, 1, 1]
        assert iga.ttop_info(K)[1] == [1, 3, 3, 1]
        M1 = assembly.matrix_1d(16, 2, trim=True)
        c = [iga.ttop_get_core(gpu_ctx, M, d) for d in range(3)]
        prod = np.prod([tt.banded_to_dense(ci, 2)[0, :, :, 0] for ci in c], axis=0) ** (1.0 / 3)
        dense = [tt.banded_to_dense(ci, 2)[0, :, :, 0] for ci in c]
        full = np.kron(np.kron(dense[0], dense[1]), dense[2])
        assert rel_err(full, np.kron(np.kron(M1, M1), M1)) < TOL
        del prod
    finally:
        iga.ttop_destroy(M)
        iga.ttop_destroy(K)


def _oracle_ranks(geo, n, p, eps):
    sp = assembly.Space(n, p)
    W = geometry.weight_fields(geo, *(assembly.InterpSpace(sp).x,) * 3)
    scale = max(np.linalg.norm(w) for w in W)
    out = []
    for w in W:
        if np.linalg.norm(w) <= 1e-12 * scale:
            out.append([0, 0])
            continue
        cores = tt.tt_svd(w, eps)
        out.append([cores[0].shape[2], cores[1].shape[2]])
    return out


def test_weight_ranks_quarter_annulus_rank_one(gpu_ctx):
    """Section 6.1: TT-SVD finds rank 1 for omega and every entry of Q of the quarter annulus."""
    from paper_1811_06797_amd import iga
    geo = _geo("untwisted")
    M, K, ranks = iga.assemble_factors(gpu_ctx, geo, 3, 12, weight_tol=1e-10)
    iga.ttop_destroy(M)
    iga.ttop_destroy(K)
    assert ranks.tolist() == [[1, 1], [1, 1], [1, 1], [0, 0], [1, 1], [0, 0], [1, 1]]
    assert ranks.tolist() == _oracle_ranks(geo, 12, 3, 1e-10)


def test_weight_ranks_match_oracle_tt_svd(gpu_ctx):
    from paper_1811_06797_amd import iga
    geo = _geo("perturbed")
    M, K, ranks = iga.assemble_factors(gpu_ctx, geo, 2, 10, weight_tol=1e-6)
    iga.ttop_destroy(M)
    iga.ttop_destroy(K)
    ref = np.array(_oracle_ranks(geo, 10, 2, 1e-6))
    # rank decisions at a threshold: allow +-1 where singular values sit at the cut
    assert np.abs(ranks - ref).max() <= 1
    assert (ranks == ref).mean() > 0.8


@pytest.mark.parametrize("ell", [0, 1, 2])
def test_kkt_apply_matches_oracle(gpu_ctx, ell):
    from paper_1811_06797_amd import iga
    geo = _geo("twisted")
    p, n, beta = 2, 6, 1e-3
    M, K, _ = iga.assemble_factors(gpu_ctx, geo, p, n, weight_tol=0.0)
    kk = iga.kkt_create(gpu_ctx, M, K, beta)
    cores = synth.random_btt([n] * 3, [2, 3], ell, seed=11 + ell)
    x = iga.btt_create(gpu_ctx, cores, ell)
    y = iga.kkt_apply(gpu_ctx, kk, x)
    try:
        ny, ry, ey = iga.btt_info(y)
        nM, RM, _ = iga.ttop_info(M)
        nK, RK, _ = iga.ttop_info(K)
        assert ey == ell and ry == [1, (RM[1] + RK[1]) * 2, (RM[2] + RK[2]) * 3, 1]
        yf = iga.btt_to_full(gpu_ctx, y).cpu().numpy().reshape(3, -1)
        Mo, Ko = assembly.assemble(geo, n, p, mode="interp")
        f = tt.btt_full(cores, ell).reshape(3, -1)
        ref = okkt.kkt_apply(Mo, Ko, beta, f).reshape(3, -1)
        assert rel_err(yf, ref) < TOL
        assert elem_err(yf, ref) < TOL
        # the round trip of the input through the library is exact
        xf = iga.btt_to_full(gpu_ctx, x).cpu().numpy().reshape(3, -1)
        assert rel_err(xf, f) < 1e-15
    finally:
        for h in (y, x):
            iga.btt_destroy(h)
        iga.kkt_destroy(kk)
        iga.ttop_destroy(M)
        iga.ttop_destroy(K)


def test_kkt_apply_full_size_sampled_boxes(gpu_ctx):
    """Twisted annulus, p = 3, n = 64 (262,144 dofs per field): rows in several boxes
    (corners, faces, interior) against the oracle's element-by-element apply."""
    from paper_1811_06797_amd import iga
    geo = _geo("twisted")
    p, n, beta = 3, 64, 1e-6
    M, K, ranks = iga.assemble_factors(gpu_ctx, geo, p, n, weight_tol=0.0)
    kk = iga.kkt_create(gpu_ctx, M, K, beta)
    cores = synth.random_btt([n] * 3, [3, 4], 1, seed=5)
    x = iga.btt_create(gpu_ctx, cores, 1)
    y = iga.kkt_apply(gpu_ctx, kk, x)
    try:
        yf = iga.btt_to_full(gpu_ctx, y).cpu().numpy()
        f = tt.btt_full(cores, 1)
        Wint = assembly.interpolate_weights(geo, assembly.Space(n, p))
        for box in [((0, 4), (0, 4), (0, 4)), ((30, 34), (10, 14), (60, 64)), ((61, 64), (31, 35), (2, 6)),
                    ((20, 23), (62, 64), (40, 44))]:
            oM, oK = assembly.apply_box(geo, n, p, [f[0], f[1], f[2]], box, mode="interp", Wint=Wint)
            ref = np.stack(kkt_rows(oM, oK, beta))
            sl = (slice(None),) + tuple(slice(a, b) for a, b in box)
            assert rel_err(yf[sl], ref) < TOL, box
            assert elem_err(yf[sl], ref) < TOL, box
    finally:
        for h in (y, x):
            iga.btt_destroy(h)
        iga.kkt_destroy(kk)
        iga.ttop_destroy(M)
        iga.ttop_destroy(K)


def test_weight_truncation_error_is_bounded(gpu_ctx):
    """A truncated weight TT changes the operators by about the truncation level only."""
    from paper_1811_06797_amd import iga
    geo = _geo("twisted")
    M0, K0, _ = iga.assemble_factors(gpu_ctx, geo, 2, 6, weight_tol=0.0)
    M1, K1, r1 = iga.assemble_factors(gpu_ctx, geo, 2, 6, weight_tol=1e-6)
    try:
        e = rel_err(ttop_dense(iga, gpu_ctx, K1), ttop_dense(iga, gpu_ctx, K0))
        assert 0 < e < 1e-5
    finally:
        for h in (M0, K0, M1, K1):
            iga.ttop_destroy(h)


def test_error_paths(gpu_ctx):
    from paper_1811_06797_amd import iga
    folded = synth.identity_geometry()
    folded.ctrl = folded.ctrl.copy()
    folded.ctrl[0] = 1.0 - folded.ctrl[0]  # reflect x: det < 0 everywhere
    with pytest.raises(iga.IgaError) as e:
        iga.assemble_factors(gpu_ctx, folded, 2, 4)
    assert e.value.code == iga.EGEOM
    with pytest.raises(iga.IgaError) as e:
        iga.assemble_factors(gpu_ctx, synth.identity_geometry(), 3, [1, 4, 4])
    assert e.value.code == iga.EINVAL
    M, K, _ = iga.assemble_factors(gpu_ctx, synth.identity_geometry(), 2, 4)
    try:
        with pytest.raises(iga.IgaError) as e:
            iga.kkt_create(gpu_ctx, M, K, 0.0)
        assert e.value.code == iga.EINVAL
    finally:
        iga.ttop_destroy(M)
        iga.ttop_destroy(K)
