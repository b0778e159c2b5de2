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
  long nz = 0;
  for (const auto& b : c.blocks) nz += (long)b.na * b.nb;
  v.flops_dense_factor = (c.R0 && c.R1) ? double(nz) / (double(c.R0) * c.R1) : 0.0;
  return v;
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
