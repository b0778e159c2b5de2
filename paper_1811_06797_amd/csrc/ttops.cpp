// Host drivers of the TT contractions (see ttops.hpp).
#include "ttops.hpp"

#include <algorithm>
#include <cstdio>
#include <cmath>
#include <mutex>
#include <numeric>
#include <unordered_map>

#include "kernels.hpp"

namespace iga {

namespace {
std::mutex g_scratch_mu;
std::unordered_map<iga_ctx*, std::unique_ptr<Scratch>> g_scratch;
}  // namespace

Scratch& scratch_of(iga_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto& p = g_scratch[ctx];
  if (!p) p.reset(new Scratch());
  return *p;
}

void release_scratch(iga_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  g_scratch.erase(ctx);
}

OpView view_of(const iga_ttop* op, int d) {
  OpView v;
  const OpCore& c = op->core[d];
  v.R0 = c.R0; v.R1 = c.R1; v.n = c.n; v.p = op->p;
  v.A = c.data.get();
  v.lo_R1 = c.lo_of_R1.get(); v.hi_R1 = c.hi_of_R1.get();
  v.lo_R0 = c.lo_of_R0.get(); v.hi_R0 = c.hi_of_R0.get();
  long nz = 0;
  for (const auto& b : c.blocks) nz += (long)b.na * b.nb;
  v.flops_dense_factor = (c.R0 && c.R1) ? double(nz) / (double(c.R0) * c.R1) : 0.0;
  return v;
}

void local_stage12(iga_ctx* ctx, const OpView& A, const double* PhiL, int ra_out, int ra_in,
                   int rb_in, int ncol, const double* x, long xcs, double* t2) {
  Scratch& S = scratch_of(ctx);
  const int n = A.n;
  const long colsz = (long)ra_out * n * rb_in;
  S.t1.ensure(ctx, (size_t)A.R0 * ncol * colsz);
  // stage 1: t1[al][c][a'][j][b] = sum_a PhiL[al][a'][a] x[c][a][j][b]
  k::Gemm g;
  g.M = ra_out; g.N = n * rb_in; g.K = ra_in;
  g.A = PhiL; g.sAm = ra_in; g.sAk = 1;
  g.B = x; g.sBk = (long)n * rb_in; g.sBn = 1;
  g.C = S.t1.get(); g.sCm = (long)n * rb_in; g.sCn = 1;
  g.nb1 = A.R0; g.nb2 = ncol;
  g.sAb1 = (long)ra_out * ra_in; g.sAb2 = 0;
  g.sBb1 = 0; g.sBb2 = xcs;
  g.sCb1 = ncol * colsz; g.sCb2 = colsz;
  k::gemm(ctx->stream, g);
  // stage 2: t2[be][c][a'][i][b] = sum_{al, o} A[al][i][o][be] t1[al][c][a'][i+o-p][b]
  k::Band b;
  b.n = n; b.p = A.p; b.R0 = A.R0; b.R1 = A.R1; b.rev = false;
  b.m = ncol * ra_out; b.c = rb_in;
  b.A = A.A; b.lo = A.lo_R1; b.hi = A.hi_R1;
  b.in = S.t1.get(); b.out = t2;
  k::band(ctx->stream, b);
}

void local_stage3(iga_ctx* ctx, const OpView& A, const double* t2, int ncol, int c, const double* PhiR,
                  int ra_out, int rb_out, int rb_in, double* y, double alpha, double beta) {
  const int n = A.n;
  const long colsz = (long)ra_out * n * rb_in;
  // y[a'][i][b'] = sum_{be, b} t2[be][c][a'][i][b] PhiR[be][b'][b]
  k::Gemm g;
  g.M = ra_out * n; g.N = rb_out; g.K = rb_in; g.Kout = A.R1;
  g.A = t2 + c * colsz; g.sAm = rb_in; g.sAk = 1; g.sAko = ncol * colsz;
  g.B = PhiR; g.sBk = 1; g.sBn = rb_in; g.sBko = (long)rb_out * rb_in;
  g.C = y; g.sCm = rb_out; g.sCn = 1;
  g.alpha = alpha; g.beta = beta;
  k::gemm(ctx->stream, g);
}

void local_apply(iga_ctx* ctx, const OpView& A, const double* PhiL, const double* PhiR, int ra_out,
                 int ra_in, int rb_out, int rb_in, int ncol, const double* x, long xcs, double* y,
                 long ycs, double alpha, double beta) {
  Scratch& S = scratch_of(ctx);
  const long colsz = (long)ra_out * A.n * rb_in;
  S.t2.ensure(ctx, (size_t)A.R1 * ncol * colsz);
  local_stage12(ctx, A, PhiL, ra_out, ra_in, rb_in, ncol, x, xcs, S.t2.get());
  for (int c = 0; c < ncol; ++c)
    local_stage3(ctx, A, S.t2.get(), ncol, c, PhiR, ra_out, rb_out, rb_in, y + c * ycs, alpha, beta);
}

void interface_left(iga_ctx* ctx, const OpView& A, const double* Phi, const double* U,
                    const double* V, int ru0, int ru1, int rv0, int rv1, double* out) {
  Scratch& S = scratch_of(ctx);
  const int n = A.n;
  const long sz = (long)ru0 * n * rv1;
  S.t2.ensure(ctx, (size_t)A.R1 * sz);
  local_stage12(ctx, A, Phi, ru0, rv0, rv1, 1, V, 0, S.t2.get());
  // out[be][b'][b] = sum_{(a' i)} U[(a' i)][b'] t2[be][(a' i)][b]
  k::Gemm g;
  g.M = ru1; g.N = rv1; g.K = ru0 * n;
  g.A = U; g.sAm = 1; g.sAk = ru1;
  g.B = S.t2.get(); g.sBk = rv1; g.sBn = 1;
  g.C = out; g.sCm = rv1; g.sCn = 1;
  g.nb1 = A.R1; g.sBb1 = sz; g.sCb1 = (long)ru1 * rv1;
  k::gemm(ctx->stream, g);
}

void interface_right(iga_ctx* ctx, const OpView& A, const double* Phi, const double* U,
                     const double* V, int ru0, int ru1, int rv0, int rv1, double* out) {
  Scratch& S = scratch_of(ctx);
  const int n = A.n;
  const long sz = (long)rv0 * n * ru1;
  S.t1.ensure(ctx, (size_t)A.R1 * sz);
  S.t2.ensure(ctx, (size_t)A.R0 * sz);
  // s1[be][(a j)][b'] = sum_b V[(a j)][b] Phi[be][b'][b]
  k::Gemm g;
  g.M = rv0 * n; g.N = ru1; g.K = rv1;
  g.A = V; g.sAm = rv1; g.sAk = 1;
  g.B = Phi; g.sBk = 1; g.sBn = rv1;
  g.C = S.t1.get(); g.sCm = ru1; g.sCn = 1;
  g.nb1 = A.R1; g.sBb1 = (long)ru1 * rv1; g.sCb1 = sz;
  k::gemm(ctx->stream, g);
  // s2[al][a][i][b'] = sum_{be, o} A[al][i][o][be] s1[be][a][i+o-p][b']
  k::Band b;
  b.n = n; b.p = A.p; b.R0 = A.R0; b.R1 = A.R1; b.rev = true;
  b.m = rv0; b.c = ru1;
  b.A = A.A; b.lo = A.lo_R0; b.hi = A.hi_R0;
  b.in = S.t1.get(); b.out = S.t2.get();
  k::band(ctx->stream, b);
  // out[al][a'][a] = sum_{(i b')} U[a'][(i b')] s2[al][a][(i b')]
  k::Gemm h;
  h.M = ru0; h.N = rv0; h.K = n * ru1;
  h.A = U; h.sAm = (long)n * ru1; h.sAk = 1;
  h.B = S.t2.get(); h.sBk = 1; h.sBn = (long)n * ru1;
  h.C = out; h.sCm = rv0; h.sCn = 1;
  h.nb1 = A.R0; h.sBb1 = sz; h.sCb1 = (long)ru0 * rv0;
  k::gemm(ctx->stream, h);
}

void core_product(iga_ctx* ctx, const OpView& A, const double* X, int r0, int r1, double* Y,
                  double alpha, double beta) {
  k::core_product(ctx->stream, A.R0, A.R1, A.n, A.p, A.A, r0, r1, X, Y, alpha, beta);
}

void tt_expand(iga_ctx* ctx, const int n[3], const int r[4], const double* const core[3], double* out) {
  Scratch& S = scratch_of(ctx);
  g_phase = "tt_expand";
  // T (n0 n1 x r2) = core0 (n0 x r1) . core1 (r1 x n1 r2)
  S.t3.ensure(ctx, (size_t)n[0] * n[1] * r[2]);
  k::gemm_rm(ctx->stream, n[0], n[1] * r[2], r[1], core[0], r[1], false, core[1], (long)n[1] * r[2],
             false, S.t3.get(), (long)n[1] * r[2]);
  k::gemm_rm(ctx->stream, n[0] * n[1], n[2], r[2], S.t3.get(), r[2], false, core[2], n[2], false, out,
             n[2]);
}

void btt_expand(iga_ctx* ctx, const iga_btt* x, double* out) {
  const long N = (long)x->n[0] * x->n[1] * x->n[2];
  for (int l = 0; l < x->nblk; ++l) {
    const double* c[3];
    for (int d = 0; d < 3; ++d) {
      const long sz = (long)x->r[d] * x->n[d] * x->r[d + 1];
      c[d] = x->core[d].get() + (d == x->ell ? l * sz : 0);
    }
    tt_expand(ctx, x->n, x->r, c, out + l * N);
  }
}

void full_apply(iga_ctx* ctx, const iga_ttop* A, const double* x, double* y, double alpha, double beta) {
  Scratch& S = scratch_of(ctx);
  g_phase = "full_apply";
  const int n0 = A->n[0], n1 = A->n[1], n2 = A->n[2];
  const long N = (long)n0 * n1 * n2;
  S.t1.ensure(ctx, (size_t)A->R[1] * N);
  S.t2.ensure(ctx, (size_t)A->R[2] * N);
  // T1[al][i1][j2 j3] = sum_j1 A0[0][i1][j1][al] x[j1][j2 j3]
  OpView v0 = view_of(A, 0), v1 = view_of(A, 1), v2 = view_of(A, 2);
  k::Band b;
  b.n = n0; b.p = A->p; b.R0 = 1; b.R1 = A->R[1]; b.rev = false; b.m = 1; b.c = n1 * n2;
  b.A = v0.A; b.lo = v0.lo_R1; b.hi = v0.hi_R1; b.in = x; b.out = S.t1.get();
  k::band(ctx->stream, b);
  // T2[be][i1][i2][j3] = sum_{al, j2} A1[al][i2][j2][be] T1[al][i1][j2][j3]
  k::Band c;
  c.n = n1; c.p = A->p; c.R0 = A->R[1]; c.R1 = A->R[2]; c.rev = false; c.m = n0; c.c = n2;
  c.A = v1.A; c.lo = v1.lo_R1; c.hi = v1.hi_R1; c.in = S.t1.get(); c.out = S.t2.get();
  k::band(ctx->stream, c);
  // y[i1 i2][i3] = sum_{be, j3} A2[be][i3][j3][0] T2[be][i1 i2][j3]
  k::Band e;
  e.n = n2; e.p = A->p; e.R0 = A->R[2]; e.R1 = 1; e.rev = false; e.m = n0 * n1; e.c = 1;
  e.A = v2.A; e.lo = v2.lo_R1; e.hi = v2.hi_R1; e.in = S.t2.get(); e.out = y;
  e.alpha = alpha; e.beta = beta;
  k::band(ctx->stream, e);
}

iga_btt* kkt_apply_impl(iga_ctx* ctx, const iga_kkt* kkt, const iga_btt* x) {
  static thread_local char ph[160];
  std::snprintf(ph, sizeof ph, "kkt_apply ranks %d %d ell %d", x->r[1], x->r[2], x->ell);
  g_phase = ph;
  const iga_ttop* M = kkt->M;
  const iga_ttop* K = kkt->K;
  std::unique_ptr<iga_btt> y(new iga_btt());
  y->ctx = ctx;
  y->ell = x->ell;
  y->nblk = x->nblk;
  const int nbk = kkt->nblk;
  require(x->nblk == nbk, IGA_EINVAL, "kkt_apply: block count differs from the KKT system");
  int s[4];
  s[0] = 1; s[3] = 1;
  for (int d = 0; d < 3; ++d) y->n[d] = x->n[d];
  for (int d = 1; d < 3; ++d) s[d] = (M->R[d] + K->R[d]) * x->r[d];
  for (int d = 0; d < 4; ++d) y->r[d] = s[d];
  Scratch& S = scratch_of(ctx);
  for (int d = 0; d < 3; ++d) {
    const int n = x->n[d];
    const bool ellc = (d == x->ell);
    const int nl = ellc ? nbk : 1;
    const long ysz = (long)s[d] * n * s[d + 1];
    y->core[d].reset(ctx, nl * ysz);
    k::fill(ctx->stream, nl * ysz, 0.0, y->core[d].get());
    const long xsz = (long)x->r[d] * n * x->r[d + 1];
    for (int which = 0; which < 2; ++which) {
      const iga_ttop* A = which == 0 ? M : K;
      OpView v = view_of(A, d);
      const int na = A->R[d] * x->r[d], nb = A->R[d + 1] * x->r[d + 1];
      const int a0 = (which == 1 && d > 0) ? M->R[d] * x->r[d] : 0;
      const int b0 = (which == 1 && d < 2) ? M->R[d + 1] * x->r[d + 1] : 0;
      S.t3.ensure(ctx, (size_t)na * n * nb);
      for (int lo = 0; lo < nl; ++lo) {
        if (!ellc) {
          core_product(ctx, v, x->core[d].get(), x->r[d], x->r[d + 1], S.t3.get(), 1.0, 0.0);
        } else {
          // sum_l c[lo][l] A (.) x_l
          bool first = true;
          for (int l = 0; l < nbk; ++l) {
            const double c = (which == 0 ? kkt->cM : kkt->cK)[(size_t)lo * nbk + l];
            if (c == 0.0) continue;
            core_product(ctx, v, x->core[d].get() + l * xsz, x->r[d], x->r[d + 1], S.t3.get(), c,
                         first ? 0.0 : 1.0);
            first = false;
          }
          if (first) continue;  // this component receives nothing from this operator
        }
        k::place_block(ctx->stream, na, nb, n, S.t3.get(), y->core[d].get() + lo * ysz, s[d + 1], a0, b0);
      }
    }
  }
  return y.release();
}

// ---------------------------------------------------------------- SVD

void svd(iga_ctx* ctx, const double* A, int m, int k, long lda, bool trans, Svd& out) {
  require(m >= 1 && k >= 1, IGA_EINVAL, "svd: empty matrix");
  hipStream_t st = ctx->stream;
  if (m < k) {
    // work on the tall transpose: A^T = U' S V'^T  =>  A = V' S U'^T
    Svd t;
    svd(ctx, A, k, m, lda, !trans, t);
    const int p = t.p;
    std::vector<double> sg(t.sigma.begin(), t.sigma.begin() + p), inv(p);
    for (int j = 0; j < p; ++j) inv[j] = sg[j] > 0 ? 1.0 / sg[j] : 0.0;
    std::vector<int> id(p);
    std::iota(id.begin(), id.end(), 0);
    IBuf did(ctx, p);
    DBuf dsg(ctx, p), dinv(ctx, p);
    IGA_HIP(hipMemcpyAsync(did.get(), id.data(), p * sizeof(int), hipMemcpyHostToDevice, st));
    IGA_HIP(hipMemcpyAsync(dsg.get(), sg.data(), p * sizeof(double), hipMemcpyHostToDevice, st));
    IGA_HIP(hipMemcpyAsync(dinv.get(), inv.data(), p * sizeof(double), hipMemcpyHostToDevice, st));
    out.m = m; out.k = k; out.p = p;
    out.B.reset(ctx, (size_t)m * p);
    out.V.reset(ctx, (size_t)k * p);
    k::gather_cols(st, m, p, p, t.V.get(), p, did.get(), dsg.get(), out.B.get(), p);
    k::gather_cols(st, k, p, p, t.B.get(), p, did.get(), dinv.get(), out.V.get(), p);
    out.sigma = sg;
    out.passes = t.passes;
    IGA_HIP(hipStreamSynchronize(st));
    return;
  }
  // one-sided block Jacobi on the m x kp zero-padded copy
  const int bs = k::osbj_block();
  const int kp = ((k + 2 * bs - 1) / (2 * bs)) * (2 * bs);
  const int nb = kp / bs;
  DBuf B(ctx, (size_t)m * kp), V(ctx, (size_t)kp * kp);
  k::fill(st, (long)m * kp, 0.0, B.get());
  if (!trans) k::copy2d(st, m, k, A, lda, 1, B.get(), kp);
  else k::copy2d(st, m, k, A, 1, lda, B.get(), kp);
  {
    std::vector<double> eye((size_t)kp * kp, 0.0);
    for (int i = 0; i < kp; ++i) eye[(size_t)i * kp + i] = 1.0;
    IGA_HIP(hipMemcpyAsync(V.get(), eye.data(), eye.size() * sizeof(double), hipMemcpyHostToDevice, st));
    IGA_HIP(hipStreamSynchronize(st));
  }
  const double fro2 = norm2_host(ctx, (long)m * kp, B.get());
  // NaN or Inf would also break the ordering of the singular values below
  require(std::isfinite(fro2), IGA_ENUM, "svd: the matrix holds a non-finite entry");
  const double floor_col = 1e-28 * fro2;
  const double tol = 4e-16 * std::max(1.0, std::sqrt((double)m));
  const int npair = nb / 2, nround = nb - 1;
  IBuf flags(ctx, (size_t)npair * nround);
  const size_t wlen = k::osbj_work_len(m, kp, nb);
  DBuf work(ctx, wlen);
  std::vector<int> hf((size_t)npair * nround);
  int sweeps = 0;
  if (fro2 > 0) {
    for (int sweep = 0; sweep < 30; ++sweep) {
      for (int rd = 0; rd < nround; ++rd)
        k::osbj_round(st, B.get(), m, kp, V.get(), kp, kp, nb, rd, tol, floor_col, flags.get() + rd * npair,
                     work.get(), wlen);
      IGA_HIP(hipMemcpyAsync(hf.data(), flags.get(), hf.size() * sizeof(int), hipMemcpyDeviceToHost, st));
      IGA_HIP(hipStreamSynchronize(st));
      ++sweeps;
      bool any = false;
      for (int f : hf) any = any || f;
      if (!any) break;
    }
  }
  out.passes = sweeps;
  DBuf nrm(ctx, kp);
  k::colnorms(st, m, kp, B.get(), kp, nrm.get());
  std::vector<double> sig(kp);
  IGA_HIP(hipMemcpyAsync(sig.data(), nrm.get(), kp * sizeof(double), hipMemcpyDeviceToHost, st));
  IGA_HIP(hipStreamSynchronize(st));
  std::vector<int> idx(kp);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return sig[a] > sig[b]; });
  const int p = k;
  out.m = m; out.k = k; out.p = p;
  out.sigma.resize(p);
  for (int j = 0; j < p; ++j) out.sigma[j] = sig[idx[j]];
  IBuf didx(ctx, p);
  IGA_HIP(hipMemcpyAsync(didx.get(), idx.data(), p * sizeof(int), hipMemcpyHostToDevice, st));
  out.B.reset(ctx, (size_t)m * p);
  out.V.reset(ctx, (size_t)k * p);
  k::gather_cols(st, m, kp, p, B.get(), kp, didx.get(), nullptr, out.B.get(), p);
  k::gather_cols(st, k, kp, p, V.get(), kp, didx.get(), nullptr, out.V.get(), p);
  IGA_HIP(hipStreamSynchronize(st));
}

int trunc_rank(const std::vector<double>& sigma, double abs_tol, int rmax, int rmin) {
  const int k = (int)sigma.size();
  // tail[r] = ||sigma[r:]||
  std::vector<double> tail(k + 1, 0.0);
  for (int j = k - 1; j >= 0; --j) tail[j] = std::sqrt(tail[j + 1] * tail[j + 1] + sigma[j] * sigma[j]);
  int r = k;
  for (int j = 0; j <= k; ++j)
    if (tail[j] <= abs_tol) { r = j; break; }
  r = std::max(r, std::min(rmin, k));
  if (rmax > 0) r = std::min(r, rmax);
  return r;
}

// Symmetric eigen-decomposition X = Vc diag(lam) Vc^T (Vc: eigenvectors in columns, k x k).
// Small k: two-sided cyclic Jacobi in one workgroup's LDS. Larger k (X positive
// semidefinite here: mass and stiffness interfaces): the one-sided block Jacobi SVD of X,
// whose right singular vectors are the eigenvectors, with lam_j = v_j^T X v_j.
static void eig_sym(iga_ctx* ctx, int k, const double* X, double* Vc, double* lam) {
  hipStream_t st = ctx->stream;
  if (k <= k::jacobi_lds_max()) {
    DBuf H(ctx, (size_t)k * k), WT(ctx, (size_t)k * k);
    IGA_HIP(hipMemcpyAsync(H.get(), X, (size_t)k * k * sizeof(double), hipMemcpyDeviceToDevice, st));
    k::jacobi_eig(st, 1, k, H.get(), 0, WT.get(), 0, 1e-15, 60, nullptr);
    k::diag_get(st, k, H.get(), lam);
    k::transpose_square(st, 1, k, WT.get(), 0, Vc, 0);
    return;
  }
  Svd s;
  svd(ctx, X, k, k, k, false, s);
  IGA_HIP(hipMemcpyAsync(Vc, s.V.get(), (size_t)k * k * sizeof(double), hipMemcpyDeviceToDevice, st));
  k::coldots(st, k, k, s.V.get(), k, s.B.get(), k, lam);
}

void gen_eig(iga_ctx* ctx, int k, const double* A, const double* B, double* V, double* lam) {
  hipStream_t st = ctx->stream;
  DBuf U(ctx, (size_t)k * k), d(ctx, k), lb(ctx, k), Sm(ctx, (size_t)k * k), T(ctx, (size_t)k * k),
      C(ctx, (size_t)k * k), Z(ctx, (size_t)k * k);
  IBuf idx(ctx, k);
  // B = U diag(lb) U^T ; S = U diag(lb)^{-1/2} (S^T B S = I)
  eig_sym(ctx, k, B, U.get(), lb.get());
  k::vec_invsqrt(st, k, lb.get(), d.get());
  std::vector<int> id(k);
  std::iota(id.begin(), id.end(), 0);
  IGA_HIP(hipMemcpyAsync(idx.get(), id.data(), k * sizeof(int), hipMemcpyHostToDevice, st));
  k::gather_cols(st, k, k, k, U.get(), k, idx.get(), d.get(), Sm.get(), k);
  // C = S^T A S, symmetrised against rounding
  k::gemm_rm(st, k, k, k, A, k, false, Sm.get(), k, false, T.get(), k);
  k::gemm_rm(st, k, k, k, Sm.get(), k, true, T.get(), k, false, C.get(), k);
  k::symmetrize(st, 1, k, C.get(), 0);
  eig_sym(ctx, k, C.get(), Z.get(), lam);
  // V = S Z
  k::gemm_rm(st, k, k, k, Sm.get(), k, false, Z.get(), k, false, V, k);
  IGA_HIP(hipStreamSynchronize(st));
}

double dot_host(iga_ctx* ctx, long n, const double* x, const double* y) {
  Scratch& S = scratch_of(ctx);
  S.red.ensure(ctx, (size_t)k::reduce_partials() * 64 + 64);
  double* out = S.red.get() + (size_t)k::reduce_partials() * 64;
  k::dot(ctx->stream, n, x, y, S.red.get(), out);
  double h = 0.0;
  IGA_HIP(hipMemcpyAsync(&h, out, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  IGA_HIP(hipStreamSynchronize(ctx->stream));
  return h;
}

double norm2_host(iga_ctx* ctx, long n, const double* x) { return dot_host(ctx, n, x, x); }

}  // namespace iga
