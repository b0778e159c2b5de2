// Derivatives of the reduced cost of the control problem (Section 4):
//   J = 1/2 (y - yhat)^T M (y - yhat) + beta/2 u^T M u at the solution f = (y, u, lambda).
//
// * With respect to the desired-state coefficients: at the optimum dJ/dyhat = -M (y - yhat)
//   (the Lagrangian's explicit dependence on yhat; the solution's own variation drops out).
// * With respect to the geometry control points: M and K depend on the geometry through the
//   interpolated weights omega~ = sum_m W_m beta~_m and q~_kl = sum_m V_kl,m beta~_m (Section 3,
//   eq. weightEquationSolve), W = (B~^{-1})^{(x)3} omega(Greville grid). So
//     dJ/dC = sum_g [ H_w(g) d omega(g)/dC + sum_kl H_kl(g) d q_kl(g)/dC ],
//     H = (B~^{-T})^{(x)3} G,  G_w,m = int P_w beta~_m,  G_kl,m = int P_kl beta~_m,
//   with P_w = e^2/2 + beta u^2/2 - lambda u, P_kl = (d_l lambda)(d_k y) (k_adjoint.hip). The
//   integrals use the assembly's Gauss rule on the parametric cube, with the discrete fields
//   evaluated at every quadrature point from their TT cores, slab by slab along x^_1.
//   This is the gradient of the discretisation with untruncated weight tensors.
#include <algorithm>
#include <cmath>
#include <vector>

#include "assemble.hpp"
#include "common.hpp"
#include "kernels.hpp"
#include "localop.hpp"
#include "ttops.hpp"

namespace iga {

namespace {

// Y = X x_mode A, X [n0][n1][n2], A(o, i) = A[o * sAo + i * sAi] (nout x n_mode);
// Y = alpha (product) + beta Y.
void mode_product(hipStream_t st, const double* X, const int dims[3], int mode, const double* A, long sAo,
                  long sAi, int nout, double* Y, double beta) {
  const int n0 = dims[0], n1 = dims[1], n2 = dims[2];
  k::Gemm2 g;
  g.beta = beta;
  if (mode == 0) {
    g.M = nout; g.N = n1 * n2; g.K = n0;
    g.A = A; g.sAm2 = sAo; g.sAk2 = sAi;
    g.B = X; g.sBk2 = (long)n1 * n2; g.sBn2 = 1;
    g.C = Y; g.sCm2 = (long)n1 * n2; g.sCn2 = 1;
  } else if (mode == 1) {
    g.M = nout; g.N = n2; g.K = n1;
    g.A = A; g.sAm2 = sAo; g.sAk2 = sAi;
    g.B = X; g.sBk2 = n2; g.sBn2 = 1;
    g.C = Y; g.sCm2 = n2; g.sCn2 = 1;
    g.nb1 = n0; g.sBb1 = (long)n1 * n2; g.sCb1 = (long)nout * n2;
  } else {
    g.M = n0 * n1; g.N = nout; g.K = n2;
    g.A = X; g.sAm2 = n2; g.sAk2 = 1;
    g.B = A; g.sBk2 = sAi; g.sBn2 = sAo;
    g.C = Y; g.sCm2 = nout; g.sCn2 = 1;
  }
  k::gemm2(st, g);
}

// out[s][q1][q2] = sum f(i0,i1,i2) B0[s][i0] B1[q1][i1] B2[q2][i2] for a TT f with cores
// core[d] ([r_d][n_d][r_{d+1}]); B0 holds S rows (the slab), B1 Q1 rows, B2 Q2 rows,
// B_d(q, i) = Bd[q * ldb_d + i].
void expand_at(iga_ctx* ctx, const int n[3], const int r[4], const double* const core[3], const double* B0,
               long ldb0, int S, const double* B1, long ldb1, int Q1, const double* B2, long ldb2, int Q2,
               double* out, DBuf& w1, DBuf& w2, DBuf& w3, DBuf& w4) {
  hipStream_t st = ctx->stream;
  const int r1 = r[1], r2 = r[2];
  w1.ensure(ctx, (size_t)S * r1);
  w2.ensure(ctx, (size_t)S * n[1] * r2);
  w3.ensure(ctx, (size_t)S * Q1 * r2);
  w4.ensure(ctx, (size_t)r2 * Q2);
  // w1 = B0 (S x n0) . core0 (n0 x r1)
  k::gemm_rm(st, S, r1, n[0], B0, ldb0, false, core[0], r1, false, w1.get(), r1);
  // w2 = w1 (S x r1) . core1 (r1 x n1 r2)
  k::gemm_rm(st, S, n[1] * r2, r1, w1.get(), r1, false, core[1], (long)n[1] * r2, false, w2.get(), (long)n[1] * r2);
  // w3[s][q][b] = sum_i B1[q][i] w2[s][i][b]
  const int dims[3] = {S, n[1], r2};
  mode_product(st, w2.get(), dims, 1, B1, ldb1, 1, Q1, w3.get(), 0.0);
  // w4 (r2 x Q2) = core2 (r2 x n2) . B2^T
  k::gemm_rm(st, r2, Q2, n[2], core[2], n[2], false, B2, ldb2, true, w4.get(), Q2);
  // out (S Q1 x Q2) = w3 (S Q1 x r2) . w4
  k::gemm_rm(st, S * Q1, Q2, r2, w3.get(), r2, false, w4.get(), Q2, false, out, Q2);
}

}  // namespace

int objective_impl(iga_ctx* ctx, const iga_kkt* kkt, const iga_tt* Y, const iga_btt* f, double* J, double* grad) {
  require(kkt && Y && f, IGA_EINVAL, "objective: NULL argument");
  for (int d = 0; d < 3; ++d)
    require(Y->n[d] == f->n[d] && f->n[d] == kkt->M->n[d], IGA_EINVAL, "objective: size mismatch");
  hipStream_t st = ctx->stream;
  const long N = (long)f->n[0] * f->n[1] * f->n[2];
  DBuf F(ctx, (size_t)3 * N), yh(ctx, N), Me(ctx, N), Mu(ctx, N);
  btt_expand(ctx, f, F.get());
  const double* yc[3] = {Y->core[0], Y->core[1], Y->core[2]};
  tt_expand(ctx, Y->n, Y->r, yc, yh.get());
  // e = y - yhat in place of yhat
  k::axpby(st, N, 1.0, F.get(), -1.0, yh.get());
  FullWork fw;
  full_apply_mc(ctx, kkt->M, yh.get(), Me.get(), 1.0, 0.0, fw);
  full_apply_mc(ctx, kkt->M, F.get() + N, Mu.get(), 1.0, 0.0, fw);
  if (J) *J = 0.5 * dot_host(ctx, N, yh.get(), Me.get()) + 0.5 * kkt->beta * dot_host(ctx, N, F.get() + N, Mu.get());
  if (grad) {
    IGA_HIP(hipMemcpyAsync(grad, Me.get(), N * sizeof(double), hipMemcpyDeviceToDevice, st));
    k::scale(st, N, -1.0, grad);
  }
  IGA_HIP(hipStreamSynchronize(st));
  return IGA_OK;
}

int grad_geometry_impl(iga_ctx* ctx, const iga_geometry* geo, int p, const int n[3], const iga_assembly_opts* opts,
                       double beta, const iga_tt* Y, const iga_btt* f, double* grad) {
  check_geometry(geo);
  require(Y && f && grad, IGA_EINVAL, "grad_geometry: NULL argument");
  require(p >= 1 && p <= 7, IGA_EINVAL, "grad_geometry: degree must be in 1..7");
  for (int d = 0; d < 3; ++d)
    require(n[d] >= 1 && n[d] == f->n[d] && n[d] == Y->n[d] && n[d] + 2 - p >= 1, IGA_EINVAL,
            "grad_geometry: size mismatch");
  iga_assembly_opts o = {0, 0, 0.0, 0};
  if (opts) o = *opts;
  const int pt = o.p_interp > 0 ? o.p_interp : 2 * p + 1;
  const int nq = o.nquad > 0 ? o.nquad : 5;
  require(pt <= 15 && nq <= 32, IGA_EINVAL, "interpolation degree or quadrature size too large");
  hipStream_t st = ctx->stream;
  SpaceDir dir[3];
  setup_spaces(ctx, p, n, pt, nq, dir);
  GeometryTables gt;
  geometry_tables(ctx, geo, dir, gt);
  int Q[3], nt[3];
  for (int d = 0; d < 3; ++d) {
    Q[d] = dir[d].E * nq;
    nt[d] = dir[d].nt;
  }
  // free-function tables (columns 1..N-2 of the full ones) and weighted interpolation basis
  DBuf Bq[3], Bqd[3], Tw[3];
  for (int d = 0; d < 3; ++d) {
    const int Nf = dir[d].N;
    Bq[d].reset(ctx, (size_t)Q[d] * n[d]);
    Bqd[d].reset(ctx, (size_t)Q[d] * n[d]);
    k::copy2d(st, Q[d], n[d], dir[d].Bv.get() + 1, Nf, 1, Bq[d].get(), n[d]);
    k::copy2d(st, Q[d], n[d], dir[d].Bd.get() + 1, Nf, 1, Bqd[d].get(), n[d]);
    // Tw[q][m] = qw[q] Bt[q][m]: the interpolation basis scaled by the quadrature weights
    Tw[d].reset(ctx, (size_t)Q[d] * nt[d]);
    IGA_HIP(hipMemcpyAsync(Tw[d].get(), dir[d].Bt.get(), (size_t)Q[d] * nt[d] * sizeof(double),
                           hipMemcpyDeviceToDevice, st));
    k::scale_rows(st, Q[d], nt[d], dir[d].dqw.get(), Tw[d].get(), nt[d]);
  }
  // cores of the three solution components and of yhat
  const double* comp[3][3];
  const long esz = (long)f->r[f->ell] * f->n[f->ell] * f->r[f->ell + 1];
  for (int c = 0; c < 3; ++c)
    for (int d = 0; d < 3; ++d) comp[c][d] = f->core[d].get() + (d == f->ell ? c * esz : 0);
  const double* ycores[3] = {Y->core[0], Y->core[1], Y->core[2]};

  // slab size along x^_1 so that the 19 slab arrays stay within ~2 GB
  const long plane = (long)Q[1] * Q[2];
  int S = (int)std::max<long>(1, std::min<long>(Q[0], (2L << 30) / (8L * 19 * plane)));
  const long G = (long)nt[0] * nt[1] * nt[2];
  DBuf Facc(ctx, (size_t)9 * S * plane), P(ctx, (size_t)10 * S * plane), yh(ctx, (size_t)S * plane);
  DBuf Gm(ctx, (size_t)10 * G), X1(ctx, (size_t)S * Q[1] * nt[2]), X2(ctx, (size_t)S * nt[1] * nt[2]);
  DBuf w1, w2, w3, w4;
  for (int s0 = 0; s0 < Q[0]; s0 += S) {
    const int Ss = std::min(S, Q[0] - s0);
    const long fs = (long)Ss * plane;
    // fields on the slab: e, u, lambda, d_l lambda, d_k y
    auto field = [&](const double* const* cores, int deriv_dir, double* out) {
      const double* B0 = (deriv_dir == 0 ? Bqd[0] : Bq[0]).get() + (long)s0 * n[0];
      const double* B1 = (deriv_dir == 1 ? Bqd[1] : Bq[1]).get();
      const double* B2 = (deriv_dir == 2 ? Bqd[2] : Bq[2]).get();
      expand_at(ctx, f->n, f->r, cores, B0, n[0], Ss, B1, n[1], Q[1], B2, n[2], Q[2], out, w1, w2, w3, w4);
    };
    double* Fb = Facc.get();
    field(comp[0], -1, Fb);
    expand_at(ctx, Y->n, Y->r, ycores, Bq[0].get() + (long)s0 * n[0], n[0], Ss, Bq[1].get(), n[1], Q[1],
              Bq[2].get(), n[2], Q[2], yh.get(), w1, w2, w3, w4);
    k::axpby(st, fs, -1.0, yh.get(), 1.0, Fb);  // e = y - yhat
    field(comp[1], -1, Fb + fs);
    field(comp[2], -1, Fb + 2 * fs);
    for (int l = 0; l < 3; ++l) field(comp[2], l, Fb + (3 + l) * fs);
    for (int kk = 0; kk < 3; ++kk) field(comp[0], kk, Fb + (6 + kk) * fs);
    k::adjoint_pointwise(st, fs, Fb, fs, beta, P.get(), fs);
    // G[w] += Tw0(slab)^T x_0 Tw1^T x_1 Tw2^T x_2 P[w]
    for (int w = 0; w < 10; ++w) {
      const double* Pw = P.get() + w * fs;
      // X1 (Ss Q1 x nt2) = P (Ss Q1 x Q2) . Tw2
      k::gemm_rm(st, Ss * Q[1], nt[2], Q[2], Pw, Q[2], false, Tw[2].get(), nt[2], false, X1.get(), nt[2]);
      // X2[s] (nt1 x nt2) = Tw1^T (nt1 x Q1) . X1[s]
      const int d1[3] = {Ss, Q[1], nt[2]};
      mode_product(st, X1.get(), d1, 1, Tw[1].get(), 1, nt[1], nt[1], X2.get(), 0.0);
      // G (nt0 x nt1 nt2) += Tw0[s0:s0+Ss]^T . X2
      const int d0[3] = {Ss, nt[1], nt[2]};
      mode_product(st, X2.get(), d0, 0, Tw[0].get() + (long)s0 * nt[0], 1, nt[0], nt[0], Gm.get() + w * G,
                   s0 == 0 ? 0.0 : 1.0);
    }
  }
  // H = (Binv^T)^{(x)3} G
  DBuf H(ctx, (size_t)10 * G), t1(ctx, G), t2(ctx, G);
  for (int w = 0; w < 10; ++w) {
    const int dims[3] = {nt[0], nt[1], nt[2]};
    mode_product(st, Gm.get() + w * G, dims, 0, dir[0].Binv.get(), 1, nt[0], nt[0], t1.get(), 0.0);
    mode_product(st, t1.get(), dims, 1, dir[1].Binv.get(), 1, nt[1], nt[1], t2.get(), 0.0);
    mode_product(st, t2.get(), dims, 2, dir[2].Binv.get(), 1, nt[2], nt[2], H.get() + w * G, 0.0);
  }
  // T[a][b] on the Greville grid, then the control-point contraction
  DBuf T(ctx, (size_t)9 * G);
  k::geometry_adjoint(st, nt, geo->ncp, gt.bv, gt.bd, gt.ctrl.get(), H.get(), T.get());
  const int* nc = geo->ncp;
  const long NC = (long)nc[0] * nc[1] * nc[2];
  DBuf out(ctx, (size_t)3 * NC), u1(ctx, (size_t)nc[0] * nt[1] * nt[2]), u2(ctx, (size_t)nc[0] * nc[1] * nt[2]);
  for (int a = 0; a < 3; ++a)
    for (int bdir = 0; bdir < 3; ++bdir) {
      const double* Dm[3];
      for (int d = 0; d < 3; ++d) Dm[d] = d == bdir ? gt.bd[d] : gt.bv[d];  // [nt][ncp]
      const int da[3] = {nt[0], nt[1], nt[2]};
      mode_product(st, T.get() + (3 * a + bdir) * G, da, 0, Dm[0], 1, nc[0], nc[0], u1.get(), 0.0);
      const int db[3] = {nc[0], nt[1], nt[2]};
      mode_product(st, u1.get(), db, 1, Dm[1], 1, nc[1], nc[1], u2.get(), 0.0);
      const int dc[3] = {nc[0], nc[1], nt[2]};
      mode_product(st, u2.get(), dc, 2, Dm[2], 1, nc[2], nc[2], out.get() + a * NC, bdir == 0 ? 0.0 : 1.0);
    }
  IGA_HIP(hipMemcpyAsync(grad, out.get(), (size_t)3 * NC * sizeof(double), hipMemcpyDeviceToHost, st));
  IGA_HIP(hipStreamSynchronize(st));
  return IGA_OK;
}

}  // namespace iga
