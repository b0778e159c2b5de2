"""Differentiable reduced cost: torch.autograd.Function over the library's solve and adjoint.

J(yhat, C) = 1/2 (y - yhat)^T M (y - yhat) + beta/2 u^T M u, where (y, u, lambda) is the
block-AMEn solution of the KKT system (Section 4, time removed) assembled from the geometry
with control points C (Section 3). Forward: TT assembly, the KKT operator, the TT of yhat,
the solve and J, all in libiga. Backward: dJ/dyhat = -M (y - yhat) (iga_grad_yhat) and
dJ/dC (iga_grad_geometry, the derivative of the Lagrangian along the geometry). This module
only marshals arguments.
"""
from __future__ import annotations

import numpy as np
import torch

from . import iga


class _Geo:
    def __init__(self, degree, knots, ctrl):
        self.degree = int(degree)
        self.knots = [np.ascontiguousarray(np.asarray(k, dtype=np.float64)) for k in knots]
        self.ctrl = np.ascontiguousarray(np.asarray(ctrl, dtype=np.float64))


class _Handles:
    """Library handles of one forward evaluation, released when the graph lets go of them."""

    def __init__(self, ctx):
        self.ctx, self.M, self.K, self.kkt, self.Y, self.sol = ctx, None, None, None, None, None

    def __del__(self):
        if self.sol:
            iga.btt_destroy(self.sol)
        if self.Y:
            iga.tt_destroy(self.Y)
        if self.kkt:
            iga.kkt_destroy(self.kkt)
        if self.M:
            iga.ttop_destroy(self.M)
        if self.K:
            iga.ttop_destroy(self.K)


class ReducedCost(torch.autograd.Function):
    """apply(yhat, ctrl, ctx, knots, geo_degree, degree, beta, tol, opts) -> J (0-d FP64 tensor).

    yhat: (n0, n1, n2) desired-state coefficients (any device; FP64 on the GPU inside);
    ctrl: (3, ncp0, ncp1, ncp2) geometry control points; knots: three open knot vectors;
    opts: dict with optional weight_tol, yhat_tol and block-AMEn options."""

    @staticmethod
    def forward(fctx, yhat, ctrl, ctx, knots, geo_degree, degree, beta, tol, opts):
        opts = dict(opts or {})
        weight_tol = float(opts.pop("weight_tol", 0.0))
        yhat_tol = float(opts.pop("yhat_tol", 1e-14))
        geo = _Geo(geo_degree, knots, ctrl.detach().cpu().numpy())
        n = tuple(int(s) for s in yhat.shape)
        h = _Handles(ctx)
        h.M, h.K, _ = iga.assemble_factors(ctx, geo, degree, n, weight_tol=weight_tol)
        h.kkt = iga.kkt_create(ctx, h.M, h.K, beta)
        yd = yhat.detach().to(device="cuda", dtype=torch.float64).contiguous()
        h.Y = iga.tt_from_full(ctx, yd, yhat_tol)
        h.sol, stats, rc = iga.amen_solve(ctx, h.kkt, h.Y, tol, raise_on_noconv=True, **opts)
        J = iga.objective(ctx, h.kkt, h.Y, h.sol)
        fctx.h, fctx.geo, fctx.n, fctx.degree, fctx.beta = h, geo, n, degree, beta
        fctx.yhat_meta = (yhat.device, yhat.dtype)
        fctx.ctrl_meta = (ctrl.device, ctrl.dtype)
        fctx.stats = stats
        return torch.tensor(J, dtype=torch.float64, device=yhat.device)

    @staticmethod
    def backward(fctx, gJ):
        h = fctx.h
        gy = gC = None
        if fctx.needs_input_grad[0]:
            g = iga.grad_yhat(h.ctx, h.kkt, h.Y, h.sol, fctx.n)
            gy = (g.to(device=fctx.yhat_meta[0], dtype=fctx.yhat_meta[1]) * gJ.to(fctx.yhat_meta[0]))
        if fctx.needs_input_grad[1]:
            g = iga.grad_geometry(h.ctx, fctx.geo, fctx.degree, fctx.n, fctx.beta, h.Y, h.sol)
            gC = torch.from_numpy(g).to(device=fctx.ctrl_meta[0], dtype=fctx.ctrl_meta[1]) * gJ.to(fctx.ctrl_meta[0])
        return gy, gC, None, None, None, None, None, None, None


def reduced_cost(yhat, ctrl, ctx, knots, geo_degree, degree, beta, tol, **opts):
    return ReducedCost.apply(yhat, ctrl, ctx, knots, geo_degree, degree, beta, tol, opts)
