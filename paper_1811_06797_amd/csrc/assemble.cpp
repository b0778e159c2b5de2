// Low-rank TT assembly of the Galerkin mass and stiffness operators (Section 3).
//
// 1. omega = |det grad G| and Q = (grad G^T grad G)^{-1} omega on the Greville grid
//    of the weight-interpolation space (degree p~ = 2p+1 by default, same elements
//    as the solution space).
// 2. TT-SVD of each of the seven weight tensors (Oseledets' sequential truncated
//    SVDs, tolerance split as tol/sqrt(2) per unfolding).
// 3. Core-wise collocation solves B~_d(X_d)^{-1} (eq. weightEquationSolve).
// 4. For every core slice s = (r_{d-1}, r_d): the univariate weight
//    E_s(x) = sum_m W_d[r_{d-1}, m, r_d] beta~_m(x) at the Gauss points, and the
//    banded factors int (d^a beta_i)(d^b beta_j) E_s by Gauss quadrature
//    (eqs. massMatrix1D and the D^2 stiffness factors, boundary functions omitted).
// 5. M = TT-matrix of the omega factors (eq. massFinal); K = rank concatenation of
//    the nine (k,l) terms with the derivative on beta_i in direction l and on
//    beta_j in direction k (eq. stiffnessFinal).
#include <algorithm>
#include <cmath>
#include <memory>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "ttops.hpp"
#include "assemble.hpp"

namespace iga {

namespace {

std::vector<double> uniform_open_knots(int nbasis, int deg) {
  const int E = nbasis - deg;
  std::vector<double> t;
  for (int i = 0; i <= deg; ++i) t.push_back(0.0);
  for (int i = 1; i < E; ++i) t.push_back(double(i) / E);
  for (int i = 0; i <= deg; ++i) t.push_back(1.0);
  return t;
}

std::vector<double> greville(const std::vector<double>& t, int deg) {
  const int nb = (int)t.size() - deg - 1;
  std::vector<double> g(nb);
  for (int i = 0; i < nb; ++i) {
    double s = 0.0;
    for (int k = 1; k <= deg; ++k) s += t[i + k];
    g[i] = deg ? s / deg : 0.5 * (t[i] + t[i + 1]);
  }
  return g;
}

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on the three-term recurrence).
void gauss_legendre(int nq, std::vector<double>& x, std::vector<double>& w) {
  x.assign(nq, 0.0);
  w.assign(nq, 0.0);
  for (int i = 0; i < nq; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (nq + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 1; k < nq; ++k) {
        const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
        p0 = p1; p1 = p2;
      }
      const double pn = nq == 1 ? z : p1, pm = nq == 1 ? 1.0 : p0;
      dp = nq * (z * pn - pm) / (z * z - 1.0);
      const double dz = pn / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 1; k < nq; ++k) {
      const double p2 = ((2.0 * k + 1.0) * z * p1 - k * p0) / (k + 1.0);
      p0 = p1; p1 = p2;
    }
    dp = nq * (z * p1 - p0) / (z * z - 1.0);
    x[nq - 1 - i] = z;
    w[nq - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

DBuf upload(iga_ctx* ctx, const double* h, size_t n) {
  DBuf b(ctx, n);
  IGA_HIP(hipMemcpyAsync(b.get(), h, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  IGA_HIP(hipStreamSynchronize(ctx->stream));
  return b;
}

struct TT3 {
  int r[4] = {1, 0, 0, 1};
  DBuf core[3];
  bool zero = false;
};

// TT-SVD of a tensor F [nt0][nt1][nt2] with absolute tolerance delta per unfolding.
void tt_svd3(iga_ctx* ctx, const double* F, const int nt[3], double delta, int rmax, TT3& out) {
  hipStream_t st = ctx->stream;
  const int m1 = nt[1] * nt[2];
  Svd s1;
  svd_product(ctx, F, m1, nt[0], m1, /*trans=*/true, s1);
  const int R1 = trunc_rank(s1.sigma, delta, rmax);
  out.r[1] = R1;
  out.core[0].reset(ctx, (size_t)nt[0] * R1);
  k::copy2d(st, nt[0], R1, s1.V.get(), s1.p, 1, out.core[0].get(), R1);
  DBuf Y(ctx, (size_t)R1 * m1);
  k::copy2d(st, R1, m1, s1.B.get(), 1, s1.p, Y.get(), m1);
  const int m2 = R1 * nt[1], k2 = nt[2];
  Svd s2;
  std::vector<int> id;
  if (m2 >= k2) {
    svd_product(ctx, Y.get(), m2, k2, k2, false, s2);
    const int R2 = trunc_rank(s2.sigma, delta, rmax);
    out.r[2] = R2;
    std::vector<double> inv(R2), sg(R2);
    for (int j = 0; j < R2; ++j) {
      sg[j] = s2.sigma[j];
      inv[j] = s2.sigma[j] > 0 ? 1.0 / s2.sigma[j] : 0.0;
    }
    id.resize(R2);
    for (int j = 0; j < R2; ++j) id[j] = j;
    IBuf did(ctx, R2);
    DBuf dinv = upload(ctx, inv.data(), R2), dsg = upload(ctx, sg.data(), R2);
    IGA_HIP(hipMemcpyAsync(did.get(), id.data(), R2 * sizeof(int), hipMemcpyHostToDevice, st));
    out.core[1].reset(ctx, (size_t)m2 * R2);
    k::gather_cols(st, m2, k2, R2, s2.B.get(), s2.p, did.get(), dinv.get(), out.core[1].get(), R2);
    DBuf T(ctx, (size_t)k2 * R2);
    k::gather_cols(st, k2, k2, R2, s2.V.get(), s2.p, did.get(), dsg.get(), T.get(), R2);
    out.core[2].reset(ctx, (size_t)R2 * k2);
    k::copy2d(st, R2, k2, T.get(), 1, R2, out.core[2].get(), k2);
    IGA_HIP(hipStreamSynchronize(st));
  } else {
    svd_product(ctx, Y.get(), k2, m2, k2, true, s2);
    const int R2 = trunc_rank(s2.sigma, delta, rmax);
    out.r[2] = R2;
    out.core[1].reset(ctx, (size_t)m2 * R2);
    k::copy2d(st, m2, R2, s2.V.get(), s2.p, 1, out.core[1].get(), R2);
    out.core[2].reset(ctx, (size_t)R2 * k2);
    k::copy2d(st, R2, k2, s2.B.get(), 1, s2.p, out.core[2].get(), k2);
  }
}

void setup_blocks(iga_ctx* ctx, OpCore& c, const std::vector<RankBlock>& blocks) {
  (void)ctx;
  // the banded stage writes each output rank of a block once, in either orientation of the
  // core (the right interface update swaps the rank roles): the blocks must partition both the
  // left and the right ranks
  std::vector<int> cov1(c.R1, 0), cov0(c.R0, 0);
  for (const auto& b : blocks) {
    require(b.a0 >= 0 && b.na >= 1 && b.a0 + b.na <= c.R0 && b.b0 >= 0 && b.nb >= 1 && b.b0 + b.nb <= c.R1,
            IGA_EINVAL, "operator core: rank block out of range");
    for (int g = b.b0; g < b.b0 + b.nb; ++g) ++cov1[g];
    for (int g = b.a0; g < b.a0 + b.na; ++g) ++cov0[g];
  }
  for (int v : cov1) require(v == 1, IGA_EINVAL, "operator core: rank blocks must partition the right ranks");
  for (int v : cov0) require(v == 1, IGA_EINVAL, "operator core: rank blocks must partition the left ranks");
  c.blocks = blocks;
}

}  // namespace

void opcore_setup_blocks(iga_ctx* ctx, OpCore& c, const std::vector<RankBlock>& blocks) {
  setup_blocks(ctx, c, blocks);
}

int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

// TT of a full tensor [n0][n1][n2] (device) by the sequential truncated SVDs used for the
// weights, relative Frobenius tolerance rel_tol split as rel_tol / sqrt(2) per unfolding.
iga_tt* tt_from_full_impl(iga_ctx* ctx, const int n[3], const double* full, double rel_tol) {
  require(n[0] >= 1 && n[1] >= 1 && n[2] >= 1, IGA_EINVAL, "tt_from_full: bad sizes");
  require(rel_tol >= 0.0 && rel_tol < 1.0, IGA_EINVAL, "tt_from_full: tolerance must be in [0, 1)");
  const long N = (long)n[0] * n[1] * n[2];
  const double fro = std::sqrt(norm2_host(ctx, N, full));
  std::unique_ptr<iga_tt> t(new iga_tt());
  t->ctx = ctx;
  for (int d = 0; d < 3; ++d) t->n[d] = n[d];
  TT3 tt;
  tt_svd3(ctx, full, n, std::max(rel_tol, 1e-15) / std::sqrt(2.0) * fro, 0, tt);
  for (int d = 0; d < 4; ++d) t->r[d] = tt.r[d];
  for (int d = 0; d < 3; ++d) {
    t->own[d] = std::move(tt.core[d]);
    t->core[d] = t->own[d].get();
  }
  IGA_HIP(hipStreamSynchronize(ctx->stream));
  return t.release();
}

// Left factor and remainder of a truncated SVD: for the r leading singular triplets of s,
// U = B / sigma (m x r, orthonormal columns) and C = Sigma V^T (r x k), both row-major.
static void split_svd(iga_ctx* ctx, const Svd& s, int m, int k, int r, DBuf& U, DBuf& C) {
  hipStream_t st = ctx->stream;
  std::vector<int> id(r);
  std::vector<double> inv(r), sg(r);
  for (int j = 0; j < r; ++j) {
    id[j] = j;
    sg[j] = s.sigma[j];
    inv[j] = s.sigma[j] > 0 ? 1.0 / s.sigma[j] : 0.0;
  }
  IBuf did(ctx, r);
  IGA_HIP(hipMemcpyAsync(did.get(), id.data(), r * sizeof(int), hipMemcpyHostToDevice, st));
  DBuf dinv = upload(ctx, inv.data(), r), dsg = upload(ctx, sg.data(), r), CT(ctx, (size_t)k * r);
  U.reset(ctx, (size_t)m * r);
  C.reset(ctx, (size_t)r * k);
  k::gather_cols(st, m, s.p, r, s.B.get(), s.p, did.get(), dinv.get(), U.get(), r);
  k::gather_cols(st, k, s.p, r, s.V.get(), s.p, did.get(), dsg.get(), CT.get(), r);
  k::copy2d(st, r, k, CT.get(), 1, r, C.get(), k);
  IGA_HIP(hipStreamSynchronize(st));
}

// TT rounding of a three-core TT (the truncation of Sec. 5, eq. tt, applied to a TT vector):
// right-to-left orthogonalisation (cores 2 and 1 get orthonormal rows, their factors move left),
// then left-to-right truncated SVDs of the unfoldings with the absolute tolerance
// rel_tol ||x|| / sqrt(2) each, so that ||round(x) - x|| <= rel_tol ||x|| up to rounding. The
// SVDs are those of the sweep's truncations (pivoted QR, then Jacobi on the small factor).
iga_tt* tt_round_impl(iga_ctx* ctx, const iga_tt* in, double rel_tol) {
  require(rel_tol >= 0.0 && rel_tol < 1.0, IGA_EINVAL, "tt_round: tolerance must be in [0, 1)");
  hipStream_t st = ctx->stream;
  const int* n = in->n;
  int r[4] = {1, in->r[1], in->r[2], 1};
  DBuf G[3];
  for (int d = 0; d < 3; ++d) {
    const size_t len = (size_t)r[d] * n[d] * r[d + 1];
    G[d].reset(ctx, len);
    IGA_HIP(hipMemcpyAsync(G[d].get(), in->core[d], len * sizeof(double), hipMemcpyDeviceToDevice, st));
  }
  // right-to-left: G_d^T = U Sigma V^T, G_d <- U^T, G_{d-1} <- G_{d-1} V Sigma
  for (int d = 2; d >= 1; --d) {
    const int m = n[d] * r[d + 1], k = r[d];
    Svd s;
    svd(ctx, G[d].get(), m, k, m, /*trans=*/true, s);
    const int q = std::max(1, trunc_rank(s.sigma, 0.0, 0));
    DBuf U, C;
    split_svd(ctx, s, m, k, q, U, C);
    DBuf Gd(ctx, (size_t)q * m), Gp(ctx, (size_t)r[d - 1] * n[d - 1] * q);
    k::copy2d(st, q, m, U.get(), 1, q, Gd.get(), m);
    k::gemm_rm(st, r[d - 1] * n[d - 1], q, k, G[d - 1].get(), k, false, C.get(), k, true, Gp.get(), q);
    G[d] = std::move(Gd);
    G[d - 1] = std::move(Gp);
    r[d] = q;
  }
  const double fro = std::sqrt(norm2_host(ctx, (long)n[0] * r[1], G[0].get()));
  const double delta = rel_tol / std::sqrt(2.0) * fro;
  // left-to-right: G_d = U Sigma V^T, truncated; G_d <- U_r, G_{d+1} <- Sigma_r V_r^T G_{d+1}
  for (int d = 0; d <= 1; ++d) {
    const int m = r[d] * n[d], k = r[d + 1], rest = n[d + 1] * r[d + 2];
    Svd s;
    svd(ctx, G[d].get(), m, k, k, /*trans=*/false, s);
    const int rt = std::max(1, trunc_rank(s.sigma, delta, 0));
    DBuf U, C;
    split_svd(ctx, s, m, k, rt, U, C);
    DBuf Gn(ctx, (size_t)rt * rest);
    k::gemm_rm(st, rt, rest, k, C.get(), k, false, G[d + 1].get(), rest, false, Gn.get(), rest);
    G[d] = std::move(U);
    G[d + 1] = std::move(Gn);
    r[d + 1] = rt;
  }
  std::unique_ptr<iga_tt> t(new iga_tt());
  t->ctx = ctx;
  for (int d = 0; d < 3; ++d) t->n[d] = n[d];
  for (int d = 0; d < 4; ++d) t->r[d] = r[d];
  for (int d = 0; d < 3; ++d) {
    t->own[d] = std::move(G[d]);
    t->core[d] = t->own[d].get();
  }
  IGA_HIP(hipStreamSynchronize(st));
  return t.release();
}

void setup_spaces(iga_ctx* ctx, int p, const int n[3], int pt, int nq, SpaceDir dir[3]) {
  hipStream_t st = ctx->stream;
  std::vector<double> gx, gw;
  gauss_legendre(nq, gx, gw);
  for (int d = 0; d < 3; ++d) {
    SpaceDir& D = dir[d];
    D.n = n[d]; D.N = n[d] + 2; D.E = D.N - p; D.nt = D.E + pt;
    D.ksol = uniform_open_knots(D.N, p);
    D.kint = uniform_open_knots(D.nt, pt);
    D.grev = greville(D.kint, pt);
    for (int e = 0; e < D.E; ++e) {
      const double a = double(e) / D.E, h = 1.0 / D.E;
      for (int q = 0; q < nq; ++q) {
        D.qpts.push_back(a + 0.5 * h * (gx[q] + 1.0));
        D.qw.push_back(0.5 * h * gw[q]);
      }
    }
    D.dksol = upload(ctx, D.ksol.data(), D.ksol.size());
    D.dkint = upload(ctx, D.kint.data(), D.kint.size());
    D.dgrev = upload(ctx, D.grev.data(), D.grev.size());
    D.dqpts = upload(ctx, D.qpts.data(), D.qpts.size());
    D.dqw = upload(ctx, D.qw.data(), D.qw.size());
    const int Q = D.E * nq;
    D.Bv.reset(ctx, (size_t)Q * D.N);
    D.Bd.reset(ctx, (size_t)Q * D.N);
    D.Bt.reset(ctx, (size_t)Q * D.nt);
    k::bspline_tabulate(st, D.dksol.get(), (int)D.ksol.size(), p, D.dqpts.get(), Q, 0, D.Bv.get());
    k::bspline_tabulate(st, D.dksol.get(), (int)D.ksol.size(), p, D.dqpts.get(), Q, 1, D.Bd.get());
    k::bspline_tabulate(st, D.dkint.get(), (int)D.kint.size(), pt, D.dqpts.get(), Q, 0, D.Bt.get());
    // collocation matrix of the interpolation space at its Greville points, and its inverse
    DBuf Bc(ctx, (size_t)D.nt * D.nt), work(ctx, (size_t)2 * D.nt * D.nt);
    IBuf sing(ctx, 1);
    k::bspline_tabulate(st, D.dkint.get(), (int)D.kint.size(), pt, D.dgrev.get(), D.nt, 0, Bc.get());
    D.Binv.reset(ctx, (size_t)D.nt * D.nt);
    k::invert(st, D.nt, Bc.get(), D.Binv.get(), work.get(), sing.get());
    int singular = 0;
    IGA_HIP(hipMemcpyAsync(&singular, sing.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    IGA_HIP(hipStreamSynchronize(st));
    require(!singular, IGA_EINVAL, "collocation matrix of the interpolation space is singular");
  }

}

void geometry_tables(iga_ctx* ctx, const iga_geometry* geo, const SpaceDir dir[3], GeometryTables& gt) {
  hipStream_t st = ctx->stream;
  for (int d = 0; d < 3; ++d) {
    const int nk = geo->ncp[d] + geo->degree + 1;
    const int ntd = dir[d].nt;
    gt.gk[d] = upload(ctx, geo->knots[d], nk);
    gt.Bv[d].reset(ctx, (size_t)ntd * geo->ncp[d]);
    gt.Bd[d].reset(ctx, (size_t)ntd * geo->ncp[d]);
    k::bspline_tabulate(st, gt.gk[d].get(), nk, geo->degree, dir[d].dgrev.get(), ntd, 0, gt.Bv[d].get());
    k::bspline_tabulate(st, gt.gk[d].get(), nk, geo->degree, dir[d].dgrev.get(), ntd, 1, gt.Bd[d].get());
    gt.bv[d] = gt.Bv[d].get();
    gt.bd[d] = gt.Bd[d].get();
  }
  gt.ctrl = upload(ctx, geo->ctrl, (size_t)3 * geo->ncp[0] * geo->ncp[1] * geo->ncp[2]);
}

void check_geometry(const iga_geometry* geo) {
  require(geo != nullptr && geo->ctrl != nullptr, IGA_EINVAL, "geometry: NULL argument");
  require(geo->degree >= 1 && geo->degree <= 15, IGA_EINVAL, "geometry degree must be in 1..15");
  for (int d = 0; d < 3; ++d) {
    require(geo->ncp[d] > geo->degree && geo->knots[d], IGA_EINVAL, "geometry: bad control net");
    const int nk = geo->ncp[d] + geo->degree + 1;
    const double* t = geo->knots[d];
    for (int i = 0; i + 1 < nk; ++i) require(t[i] <= t[i + 1], IGA_EINVAL, "geometry knots must be non-decreasing");
    require(t[0] == 0.0 && t[nk - 1] == 1.0, IGA_EINVAL, "geometry knots must span [0, 1]");
  }
}



// Banded factor core [R0][n][2p+1][R1] of one weight TT core for one derivative type.
static void build_factor(iga_ctx* ctx, const SpaceDir& D, int p, int nq, const double* Wcore, int R0, int R1,
                         bool di, bool dj, double* out) {
  hipStream_t st = ctx->stream;
  const int Q = D.E * nq, b = 2 * p + 1;
  DBuf E(ctx, (size_t)R0 * R1 * Q), F(ctx, (size_t)R0 * R1 * D.n * b);
  k::Gemm g;
  g.M = R1; g.N = Q; g.K = D.nt;
  g.A = Wcore; g.sAm = 1; g.sAk = R1;
  g.B = D.Bt.get(); g.sBk = 1; g.sBn = D.nt;
  g.C = E.get(); g.sCm = Q; g.sCn = 1;
  g.nb1 = R0; g.sAb1 = (long)D.nt * R1; g.sCb1 = (long)R1 * Q;
  k::gemm(st, g);
  k::factor_quadrature(st, R0 * R1, D.n, p, D.E, nq, di ? D.Bd.get() : D.Bv.get(),
                       dj ? D.Bd.get() : D.Bv.get(), D.dqw.get(), E.get(), F.get());
  const int dims[4] = {R0, R1, D.n, b};
  const int perm[4] = {0, 2, 3, 1};
  k::permute4(st, F.get(), dims, perm, out);
  IGA_HIP(hipStreamSynchronize(st));  // E, F are released on return
}

int assemble_impl(iga_ctx* ctx, const iga_geometry* geo, int p, const int n[3],
                  const iga_assembly_opts* opts, iga_ttop** Mout, iga_ttop** Kout, int* ranks_out) {
  require(ctx && geo && n && Mout && Kout, IGA_EINVAL, "assemble_factors: NULL argument");
  require(p >= 1 && p <= 7, IGA_EINVAL, "assemble_factors: degree must be in 1..7");
  require(geo->degree >= 1 && geo->degree <= 15, IGA_EINVAL, "geometry degree must be in 1..15");
  for (int d = 0; d < 3; ++d) {
    require(n[d] >= 1 && n[d] <= 4096, IGA_EINVAL, "assemble_factors: n out of range");
    require(n[d] + 2 - p >= 1, IGA_EINVAL, "assemble_factors: too few functions for the degree");
    require(geo->ncp[d] > geo->degree && geo->knots[d], IGA_EINVAL, "geometry: bad control net");
  }
  require(geo->ctrl != nullptr, IGA_EINVAL, "geometry: NULL control points");
  iga_assembly_opts o = {0, 0, 0.0, 0};
  if (opts) o = *opts;
  const int pt = o.p_interp > 0 ? o.p_interp : 2 * p + 1;
  const int nq = o.nquad > 0 ? o.nquad : 5;
  require(pt <= 15 && nq <= 32, IGA_EINVAL, "interpolation degree or quadrature size too large");
  require(o.weight_tol >= 0.0 && o.weight_tol < 1.0, IGA_EINVAL, "weight_tol must be in [0, 1)");
  const double wtol = std::max(o.weight_tol, 1e-14);
  hipStream_t st = ctx->stream;
  const int b = 2 * p + 1;

  check_geometry(geo);  // geometry knots must be open on [0, 1]

  SpaceDir dir[3];
  setup_spaces(ctx, p, n, pt, nq, dir);

  // 1. weights on the Greville grid
  const int nt[3] = {dir[0].nt, dir[1].nt, dir[2].nt};
  const long G = (long)nt[0] * nt[1] * nt[2];
  DBuf fields(ctx, (size_t)7 * G);
  {
    GeometryTables gt;
    geometry_tables(ctx, geo, dir, gt);
    IBuf bad(ctx, 1);
    IGA_HIP(hipMemsetAsync(bad.get(), 0, sizeof(int), st));
    k::geometry_weights(st, nt, geo->ncp, gt.bv, gt.bd, gt.ctrl.get(), fields.get(), bad.get());
    int nbad = 0;
    IGA_HIP(hipMemcpyAsync(&nbad, bad.get(), sizeof(int), hipMemcpyDeviceToHost, st));
    IGA_HIP(hipStreamSynchronize(st));
    require(nbad == 0, IGA_EGEOM,
            "geometry map folds: det grad G <= 0 at " + std::to_string(nbad) + " interpolation points");
  }

  // 2-3. TT-SVD of each weight and core-wise collocation solves
  double fro[7], scale = 0.0;
  for (int w = 0; w < 7; ++w) {
    fro[w] = std::sqrt(norm2_host(ctx, G, fields.get() + w * G));
    scale = std::max(scale, fro[w]);
  }
  TT3 wt[7];
  for (int w = 0; w < 7; ++w) {
    if (!(fro[w] > 1e-12 * scale)) {
      wt[w].zero = true;
      wt[w].r[1] = wt[w].r[2] = 0;
      continue;
    }
    TT3 raw;
    tt_svd3(ctx, fields.get() + w * G, nt, wtol / std::sqrt(2.0) * fro[w], o.weight_rmax, raw);
    wt[w].r[1] = raw.r[1];
    wt[w].r[2] = raw.r[2];
    for (int d = 0; d < 3; ++d) {
      const int R0 = raw.r[d], R1 = raw.r[d + 1];
      wt[w].core[d].reset(ctx, (size_t)R0 * nt[d] * R1);
      k::Gemm g;
      g.M = nt[d]; g.N = R1; g.K = nt[d];
      g.A = dir[d].Binv.get(); g.sAm = nt[d]; g.sAk = 1;
      g.B = raw.core[d].get(); g.sBk = R1; g.sBn = 1;
      g.C = wt[w].core[d].get(); g.sCm = R1; g.sCn = 1;
      g.nb1 = R0; g.sBb1 = (long)nt[d] * R1; g.sCb1 = (long)nt[d] * R1;
      k::gemm(st, g);
    }
    IGA_HIP(hipStreamSynchronize(st));
  }
  require(!wt[0].zero, IGA_EGEOM, "omega vanishes identically");
  if (ranks_out)
    for (int w = 0; w < 7; ++w) {
      ranks_out[2 * w] = wt[w].r[1];
      ranks_out[2 * w + 1] = wt[w].r[2];
    }
  if (o.weight_rmax > 0)
    for (int w = 0; w < 7; ++w)
      if (!wt[w].zero && (wt[w].r[1] >= o.weight_rmax || wt[w].r[2] >= o.weight_rmax)) {
        // the cap may have cut singular values above tolerance; this is reported, not fatal
      }

  std::unique_ptr<iga_ttop> M(new iga_ttop()), K(new iga_ttop());
  for (iga_ttop* op : {M.get(), K.get()}) {
    op->ctx = ctx;
    op->p = p;
    for (int d = 0; d < 3; ++d) op->n[d] = n[d];
  }
  // 4-5. mass operator
  for (int d = 0; d < 4; ++d) M->R[d] = wt[0].r[d];
  for (int d = 0; d < 3; ++d) {
    OpCore& c = M->core[d];
    c.R0 = M->R[d]; c.R1 = M->R[d + 1]; c.n = n[d];
    c.data.reset(ctx, (size_t)c.R0 * n[d] * b * c.R1);
    build_factor(ctx, dir[d], p, nq, wt[0].core[d].get(), c.R0, c.R1, false, false, c.data.get());
    setup_blocks(ctx, c, {RankBlock{0, c.R0, 0, c.R1}});
  }
  // stiffness operator: term (k, l) uses q_kl = q_lk; derivative on beta_i in direction l,
  // on beta_j in direction k
  const int widx[3][3] = {{1, 2, 3}, {2, 4, 5}, {3, 5, 6}};
  struct Term { int k, l, w, off1, off2; };
  std::vector<Term> terms;
  int RK1 = 0, RK2 = 0;
  for (int kk = 0; kk < 3; ++kk)
    for (int ll = 0; ll < 3; ++ll) {
      const int w = widx[kk][ll];
      if (wt[w].zero) continue;
      terms.push_back({kk, ll, w, RK1, RK2});
      RK1 += wt[w].r[1];
      RK2 += wt[w].r[2];
    }
  require(!terms.empty(), IGA_EGEOM, "Q vanishes identically");
  K->R[0] = 1; K->R[1] = RK1; K->R[2] = RK2; K->R[3] = 1;
  for (int d = 0; d < 3; ++d) {
    OpCore& c = K->core[d];
    c.R0 = K->R[d]; c.R1 = K->R[d + 1]; c.n = n[d];
    const size_t sz = (size_t)c.R0 * n[d] * b * c.R1;
    c.data.reset(ctx, sz);
    k::fill(st, (long)sz, 0.0, c.data.get());
    std::vector<RankBlock> blocks;
    for (const Term& t : terms) {
      const int R0t = wt[t.w].r[d], R1t = wt[t.w].r[d + 1];
      DBuf tmp(ctx, (size_t)R0t * n[d] * b * R1t);
      build_factor(ctx, dir[d], p, nq, wt[t.w].core[d].get(), R0t, R1t, t.l == d, t.k == d, tmp.get());
      const int a0 = d == 0 ? 0 : (d == 1 ? t.off1 : t.off2);
      const int b0 = d == 0 ? t.off1 : (d == 1 ? t.off2 : 0);
      k::place_block(st, R0t, R1t, n[d] * b, tmp.get(), c.data.get(), c.R1, a0, b0);
      IGA_HIP(hipStreamSynchronize(st));
      if (d == 1) blocks.push_back(RankBlock{a0, R0t, b0, R1t});
    }
    if (d != 1) blocks = {RankBlock{0, c.R0, 0, c.R1}};
    setup_blocks(ctx, c, blocks);
  }

  // reference operators for the local preconditioner: dominant separable part of omega
  {
    TT3 r1;
    tt_svd3(ctx, fields.get(), nt, 0.0, 1, r1);
    double sw[4];
    DBuf ones(ctx, G);
    k::fill(st, G, 1.0, ones.get());
    sw[0] = dot_host(ctx, G, fields.get(), ones.get());
    const int diag_w[3] = {1, 4, 6};
    for (int d = 0; d < 3; ++d) {
      sw[d + 1] = dot_host(ctx, G, fields.get() + diag_w[d] * G, ones.get());
      M->ref_c[d] = sw[0] != 0.0 ? sw[d + 1] / sw[0] : 1.0;
    }
    DBuf wc[3];
    for (int d = 0; d < 3; ++d) {
      wc[d].reset(ctx, nt[d]);
      k::gemm_rm(st, nt[d], 1, nt[d], dir[d].Binv.get(), nt[d], false, r1.core[d].get(), 1, false,
                 wc[d].get(), 1);
    }
    // the separable factors of omega > 0 may carry pairs of sign flips: make each positive
    for (int d = 0; d < 2; ++d) {
      DBuf one(ctx, nt[d]);
      k::fill(st, nt[d], 1.0, one.get());
      if (dot_host(ctx, nt[d], wc[d].get(), one.get()) < 0.0) {
        k::scale(st, nt[d], -1.0, wc[d].get());
        k::scale(st, nt[2], -1.0, wc[2].get());
      }
    }
    for (int d = 0; d < 3; ++d) {
      M->refM[d].reset(ctx, (size_t)n[d] * b);
      M->refK[d].reset(ctx, (size_t)n[d] * b);
      build_factor(ctx, dir[d], p, nq, wc[d].get(), 1, 1, false, false, M->refM[d].get());
      build_factor(ctx, dir[d], p, nq, wc[d].get(), 1, 1, true, true, M->refK[d].get());
    }
    M->has_ref = true;
  }
  IGA_HIP(hipStreamSynchronize(st));
  *Mout = M.release();
  *Kout = K.release();
  return IGA_OK;
}

}  // namespace iga
