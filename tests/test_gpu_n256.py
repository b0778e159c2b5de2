"""The differentiation form's workload at full size: twisted annulus, degree 3, n = 256 free
functions per direction (16.7 M dofs per field, 50.3 M KKT unknowns), beta = 1e-6, weight TT
tolerance 1e-10, AMEn tolerance 1e-6.

* With the solution ranks capped at 40 the solve cannot reach the tolerance (the uncapped solve
  needs ranks near (40, 160)): it must stop with IGA_ERANK, a rank at the cap and a solution.
* Uncapped it converges with FP64 KKT residual <= 1e-6.
* On the converged solution the control-point gradient of the reduced cost (Section 4, through
  the Lagrangian) matches central differences of the reduced cost: the library's assembly and
  solve repeated at control points moved by +-h along a random direction. At this size the
  oracle cannot assemble the system, so this is a property check (a gradient is the derivative
  of its function), with the oracle gradient pinned at n = 6 and 16 (tests/test_gpu_gradient.py).
  The solves use tolerance 1e-8 (rank cap 512) so that the difference quotient is not limited
  by them; the reduced cost is stationary in the control, so its solve error is second order."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _setup(gpu_ctx, geo, c):
    from paper_1811_06797_amd import iga
    M, K, _ = iga.assemble_factors(gpu_ctx, geo, c["degree"], c["n"], weight_tol=c["weight_tol"])
    kk = iga.kkt_create(gpu_ctx, M, K, c["beta"])
    return M, K, kk


def _free(iga, *hs):
    for h, f in hs:
        f(h)


def test_rank_cap_40_is_reported_and_uncapped_solve_converges(gpu_ctx):
    from paper_1811_06797_amd import iga
    geo, yc, c = synth.config("annulus_n256")
    M, K, kk = _setup(gpu_ctx, geo, c)
    Y = iga.tt_create(gpu_ctx, yc)
    try:
        sol, st, rc = iga.amen_solve(gpu_ctx, kk, Y, c["tol"], r_max=c["r_max"])
        iga.btt_destroy(sol)
        print("capped", rc, st, flush=True)
        assert rc == iga.ERANK and st["converged"] == 0 and max(st["ranks"]) >= c["r_max"]
        assert np.isfinite(st["residual"])
        sol, st, rc = iga.amen_solve(gpu_ctx, kk, Y, c["tol"])
        iga.btt_destroy(sol)
        print("uncapped", rc, st, flush=True)
        assert rc == 0 and st["converged"] == 1 and st["residual"] <= 1e-6
    finally:
        _free(iga, (Y, iga.tt_destroy), (kk, iga.kkt_destroy), (M, iga.ttop_destroy), (K, iga.ttop_destroy))


def test_geometry_gradient_matches_central_differences_n256(gpu_ctx):
    from paper_1811_06797_amd import iga
    geo, yc, c = synth.config("annulus_n256")
    Y = iga.tt_create(gpu_ctx, yc)
    tol = 1e-8

    def reduced_cost(g, grad=False):
        M, K, kk = _setup(gpu_ctx, g, c)
        sol, st, rc = iga.amen_solve(gpu_ctx, kk, Y, tol, r_max=512)
        try:
            assert rc == 0 and st["residual"] <= 1e-6, st
            J = iga.objective(gpu_ctx, kk, Y, sol)
            gC = iga.grad_geometry(gpu_ctx, g, c["degree"], c["n"], c["beta"], Y, sol) if grad else None
        finally:
            _free(iga, (sol, iga.btt_destroy), (kk, iga.kkt_destroy), (M, iga.ttop_destroy), (K, iga.ttop_destroy))
        return J, gC

    try:
        J, gC = reduced_cost(geo, grad=True)
        assert gC.shape == geo.ctrl.shape and np.all(np.isfinite(gC))
        v = np.random.default_rng(9).standard_normal(geo.ctrl.shape)
        h = 1e-5
        Jp, _ = reduced_cost(synth.Geometry(geo.degree, geo.knots, np.ascontiguousarray(geo.ctrl + h * v), geo.name))
        Jm, _ = reduced_cost(synth.Geometry(geo.degree, geo.knots, np.ascontiguousarray(geo.ctrl - h * v), geo.name))
        fd = (Jp - Jm) / (2 * h)
        g = float(np.sum(gC * v))
        print("n256 directional derivative: gradient %.10e central difference %.10e J %.6e" % (g, fd, J), flush=True)
        assert abs(g - fd) <= 1e-4 * max(abs(fd), 1e-4 * abs(J))
    finally:
        iga.tt_destroy(Y)
