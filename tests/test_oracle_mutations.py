"""The pins catch plausible mistakes in the oracle. Each test plants one mistake in the oracle
(on the CPU, through monkeypatch, for the duration of the test), then runs the pins that
should catch it and requires at least one to fail. A pin that passes with the mistake in place
would be checking the oracle against itself."""
import numpy as np
import pytest
import scipy.sparse as sps

from oracle import assembly, bspline, geometry, kkt, parabolic, tt

from tests import test_oracle_assembly as t_asm
from tests import test_oracle_basis as t_basis
from tests import test_oracle_kkt as t_kkt
from tests import test_oracle_parabolic as t_par
from tests import test_oracle_tt as t_tt


def caught(*pins):
    """True if at least one pin fails (raises AssertionError)."""
    for pin in pins:
        try:
            pin()
        except AssertionError:
            return True
    return False


def test_pins_pass_without_a_planted_mistake():
    assert not caught(t_kkt.test_kkt_conditions_and_dense_crosscheck,
                      lambda: t_tt.test_local_apply_is_projected_operator(1),
                      t_basis.test_gauss_rule_exact_degree_9,
                      t_asm.test_box_volume_and_interp_mode_exact_for_constant_weights,
                      lambda: t_basis.test_basis_matches_scipy(3, 9),
                      lambda: t_basis.test_univariate_factors_cardinal_closed_form(3, 20),
                      t_asm.test_affine_map_closed_form,
                      t_par.test_state_is_the_implicit_euler_march_of_its_control,
                      t_kkt.test_kkt_apply_is_the_kkt_matrix_product,
                      t_kkt.test_kkt_apply_maps_the_optimum_to_the_rhs_and_residual_is_its_defect,
                      lambda: t_kkt.test_reduced_solve_matches_direct_solve(6, 2, 1e-2),
                      lambda: t_tt.test_btt_full_is_the_frame_times_the_component_slice(0),
                      t_tt.test_btt_full_of_rank_one_cores_is_an_outer_product_per_component)


def test_wrong_sign_of_the_control_coupling(monkeypatch):
    # +M instead of -M in the (u, lambda) block of the KKT matrix (Sec. 4, eq. KKTSystem)
    monkeypatch.setattr(kkt, "kkt_matrix", lambda M, K, beta: sps.bmat(
        [[M, None, K.T], [None, beta * M, M], [K, -M, None]], format="csc"))
    assert caught(t_kkt.test_kkt_conditions_and_dense_crosscheck)


def test_rhs_without_the_mass_matrix(monkeypatch):
    # b = [yhat; 0; 0] instead of [M yhat; 0; 0]
    def rhs(M, yhat):
        y = np.asarray(yhat).ravel()
        return np.concatenate([y, 0 * y, 0 * y])
    monkeypatch.setattr(kkt, "kkt_rhs", rhs)
    assert caught(t_kkt.test_kkt_conditions_and_dense_crosscheck)


def test_transposed_right_interface_in_the_local_matvec(monkeypatch):
    # Phi_R contracted over (beta, b', b) with its two solution-rank indices swapped (eq. KKT_red)
    def local_apply(PhiL, A_dense, PhiR, x):
        t1 = np.einsum("pxa,ajb->pxjb", PhiL, x)
        t2 = np.einsum("pijq,pxjb->qxib", A_dense, t1)
        return np.einsum("qxib,qby->xiy", t2, PhiR)
    monkeypatch.setattr(tt, "local_apply", local_apply)
    assert caught(lambda: t_tt.test_local_apply_is_projected_operator(1))


def test_gauss_weights_without_the_interval_scaling(monkeypatch):
    # element weights w_q instead of w_q h_e / 2
    true_rule = bspline.gauss_rule

    def rule(knots, nq=5):
        pts, wts = true_rule(knots, nq)
        return pts, wts * 2.0 / (knots[-1] - knots[0]) * (len(np.unique(knots)) - 1)
    monkeypatch.setattr(bspline, "gauss_rule", rule)
    monkeypatch.setattr(assembly, "gauss_rule", rule)
    assert caught(t_basis.test_gauss_rule_exact_degree_9)
    assert caught(t_asm.test_box_volume_and_interp_mode_exact_for_constant_weights)


def test_wrong_degree_factor_in_the_derivative(monkeypatch):
    # derivative recurrence with factor p - 1 instead of p
    true_basis = bspline.basis

    def basis(knots, degree, x, deriv=0):
        B = true_basis(knots, degree, x, deriv)
        return B * (degree - 1) / degree if deriv == 1 else B
    monkeypatch.setattr(bspline, "basis", basis)
    monkeypatch.setattr(assembly, "basis", basis)
    assert caught(lambda: t_basis.test_basis_matches_scipy(3, 9))
    assert caught(lambda: t_basis.test_univariate_factors_cardinal_closed_form(3, 20))


def test_transposed_jacobian_in_the_stiffness_weights(monkeypatch):
    # Q = (J J^T)^-1 omega instead of (J^T J)^-1 omega (Sec. 2)
    def weights(J, check=True):
        omega = np.abs(np.linalg.det(J))
        JJt = np.einsum("...ak,...bk->...ab", J, J)
        return omega, np.linalg.inv(JJt) * omega[..., None, None]
    monkeypatch.setattr(geometry, "weights", weights)
    assert caught(t_asm.test_affine_map_closed_form)


def test_time_difference_on_the_wrong_side_of_the_diagonal(monkeypatch):
    # -1 on the superdiagonal: a backward-in-time march
    monkeypatch.setattr(parabolic, "time_difference", lambda nt: sps.diags(
        [np.ones(nt), -np.ones(nt - 1)], [0, 1], shape=(nt, nt), format="csr"))
    assert caught(t_par.test_state_is_the_implicit_euler_march_of_its_control)


@pytest.mark.parametrize("mistake", ["dropped_band", "swapped_ranks"])
def test_interface_mistakes_in_the_left_update(monkeypatch, mistake):
    # eq. frame / ttlin: the left interface update contracts U, Phi_L, A_d and V in that order
    def interface_left(PhiL, U, A_dense, V):
        t1 = np.einsum("pxa,ajb->pxjb", PhiL, V)
        if mistake == "dropped_band":
            # only the main diagonal of each banded factor kept (the off-diagonal terms dropped)
            A_dense = np.einsum("pijq,ij->pijq", A_dense, np.eye(A_dense.shape[1]))
        t2 = np.einsum("pijq,pxjb->qxib", A_dense, t1)
        if mistake == "swapped_ranks":
            return np.einsum("xiy,qxib->qby", U, t2)
        return np.einsum("xiy,qxib->qyb", U, t2)
    monkeypatch.setattr(tt, "interface_left", interface_left)
    assert caught(lambda: t_tt.test_local_apply_is_projected_operator(1),
                  lambda: t_tt.test_local_apply_is_projected_operator(2))


def test_wrong_sign_in_the_second_row_of_the_kkt_apply(monkeypatch):
    # beta M u + M lambda instead of beta M u - M lambda in the matrix-free apply (eq. KKTSystem)
    def apply(M, K, beta, f):
        y, u, lam = np.asarray(f).reshape(3, -1)
        return np.concatenate([M @ y + K.T @ lam, beta * (M @ u) + M @ lam, K @ y - M @ u])
    monkeypatch.setattr(kkt, "kkt_apply", apply)
    assert caught(t_kkt.test_kkt_apply_is_the_kkt_matrix_product)
    assert caught(t_kkt.test_kkt_apply_maps_the_optimum_to_the_rhs_and_residual_is_its_defect)


def test_residual_against_a_rhs_without_the_mass_matrix(monkeypatch):
    def residual(M, K, beta, yhat, f):
        y = np.asarray(yhat).ravel()
        b = np.concatenate([y, 0 * y, 0 * y])
        return np.linalg.norm(kkt.kkt_apply(M, K, beta, f) - b) / np.linalg.norm(b)
    monkeypatch.setattr(kkt, "residual", residual)
    assert caught(t_kkt.test_kkt_apply_maps_the_optimum_to_the_rhs_and_residual_is_its_defect)


@pytest.mark.parametrize("mistake", ["neighbour_slice", "first_slice"])
def test_wrong_component_slice_in_the_block_tt(monkeypatch, mistake):
    # component l read from the wrong slice of the core that carries the component index (eq. btt)
    def btt_full(cores, ell_core):
        out = []
        for l in range(3):
            j = (l + 1) % 3 if mistake == "neighbour_slice" else 0
            cs = [c if d != ell_core else c[j] for d, c in enumerate(cores)]
            out.append(tt.tt_full(cs))
        return np.stack(out)
    monkeypatch.setattr(tt, "btt_full", btt_full)
    assert caught(lambda: t_tt.test_btt_full_is_the_frame_times_the_component_slice(0),
                  t_tt.test_btt_full_of_rank_one_cores_is_an_outer_product_per_component)


@pytest.mark.parametrize("mistake", ["multiplier_without_beta", "reduced_matrix_without_beta"])
def test_mistakes_in_the_reduced_solve(monkeypatch, mistake):
    # lambda = u instead of beta u, or M + K M^-1 K instead of M + beta K M^-1 K
    true_solve = kkt.solve_reduced

    def solve_reduced(M, K, beta, yhat, rtol=1e-13, maxiter=200):
        if mistake == "multiplier_without_beta":
            y, u, lam, its = true_solve(M, K, beta, yhat, rtol, maxiter)
            return y, u, u, its
        y, u, lam, its = true_solve(M, K, 1.0, yhat, rtol, maxiter)
        return y, u, beta * u, its
    monkeypatch.setattr(kkt, "solve_reduced", solve_reduced)
    assert caught(lambda: t_kkt.test_reduced_solve_matches_direct_solve(6, 2, 1e-2))
