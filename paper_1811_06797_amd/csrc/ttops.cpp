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

namespace {

// Lower Cholesky factor L (k x k, zero above the diagonal) of the symmetric G (k x k,
// row-major, destroyed), by blocks of b = chol_block_size() columns, left to right: factor
// the diagonal block (which also gives its inverse, kept in Linv[block]), solve the panel
// below it, L21 = G21 L11^-T, and update the trailing matrix, G22 -= L21 L21^T. Returns the
// number of non-positive pivots (each leaves a zero column).
int cholesky(iga_ctx* ctx, int k, double* G, double* L, double* Linv) {
  hipStream_t st = ctx->stream;
  const int cb = k::chol_block_size();
  IBuf bad(ctx, 1);
  const int zero = 0;
  IGA_HIP(hipMemcpyAsync(bad.get(), &zero, sizeof(int), hipMemcpyHostToDevice, st));
  k::fill(st, (long)k * k, 0.0, L);
  for (int j0 = 0; j0 < k; j0 += cb) {
    const int jb = std::min(cb, k - j0), nr = k - j0 - jb;
    double* Lj = Linv + (long)(j0 / cb) * cb * cb;
    k::chol_block(st, jb, G + (long)j0 * k + j0, k, L + (long)j0 * k + j0, k, Lj, bad.get());
    if (nr > 0) {
      double* L21 = L + (long)(j0 + jb) * k + j0;
      k::gemm_rm(st, nr, jb, jb, G + (long)(j0 + jb) * k + j0, k, false, Lj, cb, true, L21, k);
      k::gemm_rm(st, nr, nr, jb, L21, k, false, L21, k, true, G + (long)(j0 + jb) * k + j0 + jb, k, -1.0, 1.0);
    }
  }
  int nbad = 0;
  IGA_HIP(hipMemcpyAsync(&nbad, bad.get(), sizeof(int), hipMemcpyDeviceToHost, st));
  IGA_HIP(hipStreamSynchronize(st));
  return nbad;
}

// Q = X R^-1 for R = L^T (X, Q: m x k, row-major, distinct), block column by block column:
// Q_j = X_j Ljj^-T - Q_{<j} (L_{j,<j}^T Ljj^-T), with the diagonal-block inverses from
// cholesky(). Mj: k x chol_block_size() scratch; work: split-K partials.
void solve_right_lt(iga_ctx* ctx, int m, int k, const double* X, long ldx, const double* L, const double* Linv,
                    double* Q, long ldq, double* Mj, double* work, size_t wlen) {
  hipStream_t st = ctx->stream;
  const int cb = k::chol_block_size();
  for (int j0 = 0; j0 < k; j0 += cb) {
    const int jb = std::min(cb, k - j0);
    const double* Lj = Linv + (long)(j0 / cb) * cb * cb;
    k::gemm_rm(st, m, jb, jb, X + j0, ldx, false, Lj, cb, true, Q + j0, ldq);
    if (j0 > 0) {
      k::gemm_rm(st, j0, jb, jb, L + (long)j0 * k, k, true, Lj, cb, true, Mj, cb);
      k::gemm_rm(st, m, jb, j0, Q, ldq, false, Mj, cb, false, Q + j0, ldq, -1.0, 1.0, work, wlen);
    }
  }
}

// R^T (k x k, lower) of the triangular factor of X P, X m x k (ldx; m >= k, k <= pchol_max()),
// P the column order of column-pivoted QR, by shifted Cholesky QR in three passes (Fukaya,
// Kannan, Nakatsukasa, Yamamoto, Yanagisawa, 2020). The first pass factors the Gram matrix
// plus a shift of 11 (m k + k (k + 1)) u ||X||_F^2 with diagonal pivoting, whose pivot order
// equals column-pivoted QR's, and orthogonalises X P against that factor; the second factors
// the remainder's Gram matrix plus 11 (m k + k (k + 1)) u; the shifts keep Cholesky from
// breaking down on a rank-deficient X. The third factors the nearly orthonormal remainder
// without a shift. R = R3 R2 R1 is backward stable, ||X P - Q R|| = O(u ||X||), whatever the
// rank of X (only R is formed; Q is not needed). perm[j] (device) receives the original column
// of pivot j and XP (m x k) the permuted columns. Returns false if a shifted pass still breaks
// down.
bool cholesky_qr3_rt(iga_ctx* ctx, int m, int k, const double* X, long ldx, double fro2, double* RT, int* perm,
                     double* XP) {
  hipStream_t st = ctx->stream;
  const int cb = k::chol_block_size();
  const int nblk = (k + cb - 1) / cb;
  DBuf G(ctx, (size_t)k * k), L1(ctx, (size_t)k * k), L2(ctx, (size_t)k * k), L3(ctx, (size_t)k * k);
  DBuf Li(ctx, (size_t)nblk * cb * cb), Mj(ctx, (size_t)k * cb);
  DBuf Q1(ctx, (size_t)m * k), Q2(ctx, (size_t)m * k);
  const size_t wlen = std::max<size_t>((size_t)32 * k * k, (size_t)8 * m * cb);
  DBuf work(ctx, wlen);
  const double c = 11.0 * ((double)m * k + (double)k * (k + 1)) * std::ldexp(1.0, -53);
  // pass 1: pivoted
  {
    IBuf bad(ctx, 1);
    double shift = c * fro2;
    bool ok = false;
    for (int attempt = 0; attempt < 4 && !ok; ++attempt, shift *= 100.0) {
      const int zero = 0;
      IGA_HIP(hipMemcpyAsync(bad.get(), &zero, sizeof(int), hipMemcpyHostToDevice, st));
      k::gemm_rm(st, k, k, m, X, ldx, true, X, ldx, false, L1.get(), k, 1.0, 0.0, work.get(), wlen);
      k::add_diag(st, k, L1.get(), k, shift);
      k::pivoted_cholesky(st, k, L1.get(), perm, bad.get());
      int nbad = 0;
      IGA_HIP(hipMemcpyAsync(&nbad, bad.get(), sizeof(int), hipMemcpyDeviceToHost, st));
      IGA_HIP(hipStreamSynchronize(st));
      ok = nbad == 0;
    }
    if (!ok) return false;
  }
  k::trinv_blocks(st, k, L1.get(), k, Li.get());
  k::gather_cols(st, m, (int)ldx, k, X, ldx, perm, nullptr, XP, k);
  solve_right_lt(ctx, m, k, XP, k, L1.get(), Li.get(), Q1.get(), k, Mj.get(), work.get(), wlen);
  // passes 2 and 3: blocked Cholesky of the remainder's Gram matrix
  auto factor = [&](const double* Y, double shift, double* Lout, bool retry) {
    for (int attempt = 0; attempt < 4; ++attempt) {
      k::gemm_rm(st, k, k, m, Y, k, true, Y, k, false, G.get(), k, 1.0, 0.0, work.get(), wlen);
      if (shift > 0.0) k::add_diag(st, k, G.get(), k, shift);
      if (cholesky(ctx, k, G.get(), Lout, Li.get()) == 0 || !retry) return true;
      shift *= 100.0;
    }
    return false;
  };
  if (!factor(Q1.get(), c, L2.get(), true)) return false;
  solve_right_lt(ctx, m, k, Q1.get(), k, L2.get(), Li.get(), Q2.get(), k, Mj.get(), work.get(), wlen);
  factor(Q2.get(), 0.0, L3.get(), false);
  // R^T = R1^T R2^T R3^T = L1 (L2 L3)
  k::gemm_rm(st, k, k, k, L2.get(), k, false, L3.get(), k, false, G.get(), k);
  k::gemm_rm(st, k, k, k, L1.get(), k, false, G.get(), k, false, RT, k);
  return true;
}

}  // namespace

// How the tall problem is solved: one-sided Jacobi on A itself (PLAIN), on the pivoted
// Cholesky-QR factor with left vectors accurate only in the product U Sigma (PRODUCT, see
// svd_preconditioned), or on the factor of the rank-revealing QR step (QR, see svd_qrcp).
enum SvdMode { SVD_PLAIN, SVD_PRODUCT, SVD_QR };
// Inner Jacobi sweeps per block pair and round on a triangular factor (graded columns), and
// the size, relative to ||A||_F, below which a rotation's change of its columns is left out.
constexpr int QR_INNER_SWEEPS = 1;
constexpr double QR_ROT_FLOOR = 1e-15;
static void svd_impl(iga_ctx* ctx, const double* A, int m, int k, long lda, bool trans, Svd& out, SvdMode mode);

// Product form of the tall SVD (m >= k) of B (m x kp, zero-padded beyond column k): R of B P
// from the column-pivoted shifted Cholesky QR, then one-sided block Jacobi on R^T (k x k),
// which converges in far fewer sweeps than on B itself (Drmac and Veselic's preconditioning;
// without the pivoting it barely helps on smooth data): R^T W = U_X Sigma gives
// R = W Sigma U_X^T, so the right singular vectors of B P are U_X, the normalised columns of
// R^T W, those of B are P U_X, and B V = (B P) U_X = U Sigma. Columns with sigma = 0 get zero
// vectors. B V holds u_j only to an absolute accuracy of about u ||B|| / sigma_j: the product
// B V^T is accurate, B / sigma is not orthonormal to working accuracy for small sigma.
// Returns false (nothing written) if the Cholesky QR broke down.
static bool svd_preconditioned(iga_ctx* ctx, const double* B, int m, int k, int kp, double fro2, Svd& out) {
  hipStream_t st = ctx->stream;
  DBuf RT(ctx, (size_t)k * k), BP(ctx, (size_t)m * k);
  IBuf perm(ctx, k);
  if (!cholesky_qr3_rt(ctx, m, k, B, kp, fro2, RT.get(), perm.get(), BP.get())) return false;
  DBuf X(ctx, (size_t)k * kp);
  k::fill(st, (long)k * kp, 0.0, X.get());
  k::copy2d(st, k, k, RT.get(), k, 1, X.get(), kp);
  const int nb = kp / k::osbj_block(), npair = nb / 2, nround = nb - 1;
  const double floor_col = 1e-28 * fro2;
  const double tol = 4e-16 * std::max(1.0, std::sqrt((double)k));
  IBuf flags(ctx, (size_t)npair * nround);
  const size_t wlen = k::osbj_work_len(k, 0, nb);
  DBuf work(ctx, wlen);
  std::vector<int> hf((size_t)npair * nround);
  int sweeps = 0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    for (int rd = 0; rd < nround; ++rd)
      k::osbj_round(st, X.get(), k, kp, nullptr, 0, kp, nb, rd, tol, floor_col, flags.get() + rd * npair,
                   work.get(), wlen, QR_INNER_SWEEPS);
    IGA_HIP(hipMemcpyAsync(hf.data(), flags.get(), hf.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    IGA_HIP(hipStreamSynchronize(st));
    ++sweeps;
    bool any = false;
    for (int f : hf) any = any || f;
    if (!any) break;
  }
  DBuf nrm(ctx, kp);
  k::colnorms(st, k, kp, X.get(), kp, nrm.get());
  std::vector<double> sig(kp);
  IGA_HIP(hipMemcpyAsync(sig.data(), nrm.get(), kp * sizeof(double), hipMemcpyDeviceToHost, st));
  IGA_HIP(hipStreamSynchronize(st));
  std::vector<int> idx(kp);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return sig[a] > sig[b]; });
  const int p = k;
  std::vector<int> id(idx.begin(), idx.begin() + p);
  std::vector<double> inv(p);
  out.m = m; out.k = k; out.p = p;
  out.sigma.resize(p);
  for (int j = 0; j < p; ++j) {
    out.sigma[j] = sig[id[j]];
    inv[j] = out.sigma[j] > 0 ? 1.0 / out.sigma[j] : 0.0;
  }
  IBuf didx(ctx, p);
  DBuf dinv(ctx, p);
  IGA_HIP(hipMemcpyAsync(didx.get(), id.data(), p * sizeof(int), hipMemcpyHostToDevice, st));
  IGA_HIP(hipMemcpyAsync(dinv.get(), inv.data(), p * sizeof(double), hipMemcpyHostToDevice, st));
  out.V.reset(ctx, (size_t)k * p);
  out.B.reset(ctx, (size_t)m * p);
  k::gather_cols(st, k, kp, p, X.get(), kp, didx.get(), dinv.get(), out.V.get(), p);
  // B V in the permuted columns the factor was taken of
  k::gemm_rm(st, m, p, k, BP.get(), k, false, out.V.get(), p, false, out.B.get(), p);
  {
    // V of the permuted columns to V of A: row perm[i] of V_A is row i of V_{AP}
    std::vector<int> hp(k), inv_perm(k);
    IGA_HIP(hipMemcpyAsync(hp.data(), perm.get(), k * sizeof(int), hipMemcpyDeviceToHost, st));
    IGA_HIP(hipStreamSynchronize(st));
    for (int i = 0; i < k; ++i) inv_perm[hp[i]] = i;
    IBuf dinvp(ctx, k);
    IGA_HIP(hipMemcpyAsync(dinvp.get(), inv_perm.data(), k * sizeof(int), hipMemcpyHostToDevice, st));
    DBuf VA(ctx, (size_t)k * p);
    k::gather_rows(st, k, p, out.V.get(), p, dinvp.get(), VA.get(), p);
    out.V = std::move(VA);
  }
  out.passes = sweeps;
  IGA_HIP(hipStreamSynchronize(st));
  return true;
}

// Tall SVD (m >= k) of B (m x kp row-major, zero-padded beyond column k) through a rank-revealing
// QR step (Sec. 5, eqs. svd1-svd2: QR of the unfolding, then the SVD of the triangular factor):
// column-pivoted Householder QR, B P = Q R, stopped at the first r_c with
// ||R(r_c:, r_c:)||_F <= eta ||B||_F (eta = 1e-14, below every truncation threshold the sweep
// uses), so that B P = Q_top R_top + E with ||E||_F <= eta ||B||_F; then the one-sided Jacobi
// iteration on R_top^T (k x r_c) with the rotations accumulated: R_top^T W = Y Sigma gives
// B P ~ (Q_top W) Sigma Y^T, so U = Q_top W (orthonormal to working accuracy: the reflectors
// applied to the columns of a rotation) and V = P Y. The pivoting also preconditions the Jacobi iteration (R_top's rows are graded), and
// the iteration runs on r_c columns of length k instead of k columns of length m. Singular
// values past r_c are returned as zero.
static void svd_qrcp(iga_ctx* ctx, const double* B, int m, int k, int kp, double fro2, Svd& out) {
  hipStream_t st = ctx->stream;
  const int rmax = k;
  DBuf W(ctx, (size_t)k * m), V(ctx, (size_t)rmax * m), R(ctx, (size_t)rmax * k), beta(ctx, rmax),
      rnorm(ctx, 2 * (size_t)k);
  IBuf pivots(ctx, rmax), ctrl(ctx, 3);
  k::copy2d(st, k, m, B, 1, kp, W.get(), m);
  k::fill(st, (long)rmax * k, 0.0, R.get());
  const int zeros[3] = {0, 0, 0};
  IGA_HIP(hipMemcpyAsync(ctrl.get(), zeros, sizeof zeros, hipMemcpyHostToDevice, st));
  k::qrcp_init(st, m, k, W.get(), m, rnorm.get());
  const double eta = 1e-14;
  const double thr2 = eta * eta * fro2;
  int rc = rmax, j = 0;
  for (int chunk = 8; j < rmax;) {
    const int je = std::min(rmax, j + chunk);
    for (; j < je; ++j) {
      // step j reads the norms written by step j - 1 (the two halves of rnorm alternate)
      const double* nin = rnorm.get() + (j % 2) * (size_t)k;
      double* nout = rnorm.get() + ((j + 1) % 2) * (size_t)k;
      k::qrhh_step(st, m, k, j, W.get(), m, nin, nout, V.get(), beta.get(), R.get(), pivots.get(), ctrl.get(),
                   thr2);
    }
    int hc[3];
    IGA_HIP(hipMemcpyAsync(hc, ctrl.get(), sizeof hc, hipMemcpyDeviceToHost, st));
    IGA_HIP(hipStreamSynchronize(st));
    if (hc[0]) {
      rc = hc[2];
      break;
    }
    chunk = std::min(2 * chunk, 64);
  }
  if (rc < 1) rc = 1;  // fro2 > 0: the first step always chooses a column
  // pivot order: the chosen columns, then the others in their original order
  std::vector<int> order(k), inv_order(k), hp(rc);
  IGA_HIP(hipMemcpyAsync(hp.data(), pivots.get(), rc * sizeof(int), hipMemcpyDeviceToHost, st));
  IGA_HIP(hipStreamSynchronize(st));
  {
    std::vector<char> chosen(k, 0);
    int pos = 0;
    for (int t = 0; t < rc; ++t) {
      order[pos++] = hp[t];
      chosen[hp[t]] = 1;
    }
    for (int c = 0; c < k; ++c)
      if (!chosen[c]) order[pos++] = c;
    for (int c = 0; c < k; ++c) inv_order[order[c]] = c;
  }
  IBuf dorder(ctx, k), dinvo(ctx, k);
  IGA_HIP(hipMemcpyAsync(dorder.get(), order.data(), k * sizeof(int), hipMemcpyHostToDevice, st));
  IGA_HIP(hipMemcpyAsync(dinvo.get(), inv_order.data(), k * sizeof(int), hipMemcpyHostToDevice, st));
  // X = R_top^T in pivot order: k x rcp, zero-padded
  const int bs = k::osbj_block();
  const int rcp = ((rc + 2 * bs - 1) / (2 * bs)) * (2 * bs);
  const int nb = rcp / bs, npair = nb / 2, nround = nb - 1;
  DBuf RP(ctx, (size_t)rc * k), X(ctx, (size_t)k * rcp), Wr(ctx, (size_t)rcp * rcp);
  k::gather_cols(st, rc, k, k, R.get(), k, dorder.get(), nullptr, RP.get(), k);
  k::fill(st, (long)k * rcp, 0.0, X.get());
  k::copy2d(st, k, rc, RP.get(), 1, k, X.get(), rcp);
  {
    std::vector<double> eye((size_t)rcp * rcp, 0.0);
    for (int i = 0; i < rcp; ++i) eye[(size_t)i * rcp + i] = 1.0;
    IGA_HIP(hipMemcpyAsync(Wr.get(), eye.data(), eye.size() * sizeof(double), hipMemcpyHostToDevice, st));
    IGA_HIP(hipStreamSynchronize(st));
  }
  const double floor_col = 1e-28 * fro2;
  const double tol = 4e-16 * std::max(1.0, std::sqrt((double)k));
  IBuf flags(ctx, (size_t)npair * nround);
  const size_t wlen = k::osbj_work_len(k, rcp, nb);
  DBuf work(ctx, wlen);
  std::vector<int> hf((size_t)npair * nround);
  int sweeps = 0;
  for (int sweep = 0; sweep < 30; ++sweep) {
    for (int rd = 0; rd < nround; ++rd)
      k::osbj_round(st, X.get(), k, rcp, Wr.get(), rcp, rcp, nb, rd, tol, floor_col, flags.get() + rd * npair,
                   work.get(), wlen, QR_INNER_SWEEPS, QR_ROT_FLOOR * QR_ROT_FLOOR * fro2);
    IGA_HIP(hipMemcpyAsync(hf.data(), flags.get(), hf.size() * sizeof(int), hipMemcpyDeviceToHost, st));
    IGA_HIP(hipStreamSynchronize(st));
    ++sweeps;
    bool any = false;
    for (int f : hf) any = any || f;
    if (!any) break;
  }
  DBuf nrm(ctx, rcp);
  k::colnorms(st, k, rcp, X.get(), rcp, nrm.get());
  std::vector<double> sig(rcp);
  IGA_HIP(hipMemcpyAsync(sig.data(), nrm.get(), rcp * sizeof(double), hipMemcpyDeviceToHost, st));
  IGA_HIP(hipStreamSynchronize(st));
  std::vector<int> idx(rcp);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return sig[a] > sig[b]; });
  const int p = k;
  out.m = m; out.k = k; out.p = p;
  out.sigma.assign(p, 0.0);
  std::vector<int> id(idx.begin(), idx.begin() + rc);
  std::vector<double> sg(rc), inv(rc);
  for (int t = 0; t < rc; ++t) {
    sg[t] = out.sigma[t] = sig[id[t]];
    inv[t] = sg[t] > 0 ? 1.0 / sg[t] : 0.0;
  }
  IBuf didx(ctx, rc);
  DBuf dsg(ctx, rc), dinv(ctx, rc);
  IGA_HIP(hipMemcpyAsync(didx.get(), id.data(), rc * sizeof(int), hipMemcpyHostToDevice, st));
  IGA_HIP(hipMemcpyAsync(dsg.get(), sg.data(), rc * sizeof(double), hipMemcpyHostToDevice, st));
  IGA_HIP(hipMemcpyAsync(dinv.get(), inv.data(), rc * sizeof(double), hipMemcpyHostToDevice, st));
  // U Sigma = Q_top (W Sigma) in the sorted order: the columns of W Sigma, padded with zero rows
  // to length m, reflected by H_{rc-1} .. H_0
  DBuf WS(ctx, (size_t)rc * rc), Yc(ctx, (size_t)rc * m), Y(ctx, (size_t)k * rc);
  k::gather_cols(st, rc, rcp, rc, Wr.get(), rcp, didx.get(), dsg.get(), WS.get(), rc);
  k::fill(st, (long)rc * m, 0.0, Yc.get());
  k::copy2d(st, rc, rc, WS.get(), 1, rc, Yc.get(), m);  // Yc[col][x] = WS[x][col]
  k::qrhh_apply(st, m, rc, V.get(), beta.get(), rc, Yc.get());
  out.B.reset(ctx, (size_t)m * p);
  out.V.reset(ctx, (size_t)k * p);
  if (rc < p) {
    k::fill(st, (long)m * p, 0.0, out.B.get());
    k::fill(st, (long)k * p, 0.0, out.V.get());
  }
  k::copy2d(st, m, rc, Yc.get(), 1, m, out.B.get(), p);  // B[x][col] = Yc[col][x]
  // V = P Y: row order[c] of V is row c of Y
  k::gather_cols(st, k, rcp, rc, X.get(), rcp, didx.get(), dinv.get(), Y.get(), rc);
  k::gather_rows(st, k, rc, Y.get(), rc, dinvo.get(), out.V.get(), p);
  out.passes = sweeps;
  IGA_HIP(hipStreamSynchronize(st));
}

void svd(iga_ctx* ctx, const double* A, int m, int k, long lda, bool trans, Svd& out) {
  svd_impl(ctx, A, m, k, lda, trans, out, SVD_QR);
}

void svd_product(iga_ctx* ctx, const double* A, int m, int k, long lda, bool trans, Svd& out) {
  svd_impl(ctx, A, m, k, lda, trans, out, SVD_PRODUCT);
}

static void svd_impl(iga_ctx* ctx, const double* A, int m, int k, long lda, bool trans, Svd& out, SvdMode mode) {
  require(m >= 1 && k >= 1, IGA_EINVAL, "svd: empty matrix");
  hipStream_t st = ctx->stream;
  if (m < k) {
    // work on the tall transpose: A^T = U' S V'^T  =>  A = V' S U'^T (A's left vectors are the
    // transpose's right vectors)
    Svd t;
    svd_impl(ctx, A, k, m, lda, !trans, t, mode);
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
  if (mode == SVD_PRODUCT && k > 2 * bs && k <= k::pchol_max() && fro2 > 0 &&
      svd_preconditioned(ctx, B.get(), m, k, kp, fro2, out))
    return;
  if (mode == SVD_QR && k > 2 * bs && fro2 > 0) {
    svd_qrcp(ctx, B.get(), m, k, kp, fro2, out);
    return;
  }
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
  // a symmetric positive definite matrix of full rank: the QR step would not shorten anything
  Svd s;
  svd_impl(ctx, X, k, k, k, false, s, SVD_PLAIN);
  IGA_HIP(hipMemcpyAsync(Vc, s.V.get(), (size_t)k * k * sizeof(double), hipMemcpyDeviceToDevice, st));
  k::coldots(st, k, k, s.V.get(), k, s.B.get(), k, lam);
}

void gen_eig(iga_ctx* ctx, int k, const double* A, const double* B, double* V, double* lam) {
  hipStream_t st = ctx->stream;
  {
    // Cholesky reduction: B = L L^T, W = L^-T (W^T B W = I), C = W^T A W = Z diag(lam) Z^T,
    // V = W Z; one symmetric eigenproblem instead of two (B's and C's). Falls through to the
    // eigen-decomposition of B if B is not numerically positive definite.
    const int cb = k::chol_block_size(), nblk = (k + cb - 1) / cb;
    const size_t wlen = (size_t)32 * k * k + (size_t)8 * k * cb;
    DBuf G(ctx, (size_t)k * k), L(ctx, (size_t)k * k), Li(ctx, (size_t)nblk * cb * cb), Mj(ctx, (size_t)k * cb),
        E(ctx, (size_t)k * k), W(ctx, (size_t)k * k), T(ctx, (size_t)k * k), C(ctx, (size_t)k * k),
        Z(ctx, (size_t)k * k), work(ctx, wlen);
    IGA_HIP(hipMemcpyAsync(G.get(), B, (size_t)k * k * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (cholesky(ctx, k, G.get(), L.get(), Li.get()) == 0) {
      k::fill(st, (long)k * k, 0.0, E.get());
      k::add_diag(st, k, E.get(), k, 1.0);
      solve_right_lt(ctx, k, k, E.get(), k, L.get(), Li.get(), W.get(), k, Mj.get(), work.get(), wlen);
      k::gemm_rm(st, k, k, k, A, k, false, W.get(), k, false, T.get(), k);
      k::gemm_rm(st, k, k, k, W.get(), k, true, T.get(), k, false, C.get(), k);
      k::symmetrize(st, 1, k, C.get(), 0);
      eig_sym(ctx, k, C.get(), Z.get(), lam);
      k::gemm_rm(st, k, k, k, W.get(), k, false, Z.get(), k, false, V, k);
      IGA_HIP(hipStreamSynchronize(st));
      return;
    }
  }
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
