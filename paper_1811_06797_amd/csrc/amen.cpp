// Block-AMEn solver of the KKT system (Section 5, eqs. btt, svd1, svd2, frame, ttlin,
// KKT_red), stationary or time-dependent (Section 4, eq. KKTSystem).
//
// The solution (y, u, lambda) -- for the time-dependent system (y_t, u_t, lambda_t) of
// every step -- is one block-TT whose component index l sits in the core being updated.
// Each local step projects the block rows onto the frame of the current solution (the
// interfaces Phi = X^T A X of M and K,
// contracted core by core) and solves the reduced KKT system. Then the core is
// split by a truncated SVD, the left (or right) factor becomes the new
// orthonormal core, and the rest -- carrying l -- is multiplied into the next core.
//
// Choices the paper leaves open (all documented with the build):
// * the sweep stores the scaled unknowns (y, sqrt(beta) u, lambda / sqrt(beta)), which
//   makes the three blocks comparable in size so that one SVD truncation serves
//   all of them; the equations stay unscaled (the local operator is A D with
//   D = diag(1, 1/sqrt(beta), sqrt(beta)), which has the same Galerkin solution
//   since D acts on the component index only), so every local residual is the
//   projected residual of the original system; the returned solution is unscaled;
// * truncation is residual-based: the smallest rank whose truncated core keeps the
//   local residual <= max(tol/2, 1.5 x that of the untruncated core), at most r_max;
// * the reduced system is solved by flexible GMRES, preconditioned by the exact
//   inverse of a reduced reference KKT operator: mass and Laplace-form stiffness
//   with the dominant separable part of omega, whose projection is a Kronecker
//   sum and is inverted by fast diagonalisation (generalised eigenvectors of the
//   left interface pair, the univariate factor pair and the right interface pair;
//   the 3x3 KKT block of every mode is solved exactly; in the time-dependent system
//   the 3 nt x 3 nt block of every spatial mode, by a tridiagonal elimination in time);
// * rank adaptivity by residual enrichment (AMEn, Dolgov & Savostyanov): a
//   rank-rho TT Z tracks the residual; its projection onto (X-left, Z-right)
//   frames (forward sweep) or (Z-left, X-right) frames (backward) supplies rho
//   new orthonormal directions appended to the truncated core;
// * stopping: every local residual of a half-sweep, measured before its solve,
//   relative to its local right-hand side, is <= tol.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <random>
#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "localop.hpp"
#include "ttops.hpp"

namespace iga {

double kkt_residual_impl(iga_ctx* ctx, const iga_kkt* kkt, const iga_tt* yhat, const iga_btt* f);

namespace {

// Accumulates GPU time of one kind of work from event pairs resolved at the end.
class EventTimer {
 public:
  explicit EventTimer(hipStream_t s) : s_(s) {}
  ~EventTimer() {
    for (auto e : pool_) (void)hipEventDestroy(e);
  }
  int begin() {
    hipEvent_t a = get(), b = get();
    IGA_HIP(hipEventRecord(a, s_));
    pairs_.push_back({a, b});
    return (int)pairs_.size() - 1;
  }
  void end(int id) { IGA_HIP(hipEventRecord(pairs_[id].second, s_)); }
  double seconds() {
    IGA_HIP(hipStreamSynchronize(s_));
    double ms = 0;
    for (auto& p : pairs_) {
      float t = 0;
      IGA_HIP(hipEventElapsedTime(&t, p.first, p.second));
      ms += t;
    }
    for (auto& p : pairs_) {
      free_.push_back(p.first);
      free_.push_back(p.second);
    }
    pairs_.clear();
    acc_ += ms * 1e-3;
    return acc_;
  }
  double total() { return seconds(); }

 private:
  hipEvent_t get() {
    if (!free_.empty()) {
      hipEvent_t e = free_.back();
      free_.pop_back();
      return e;
    }
    hipEvent_t e;
    IGA_HIP(hipEventCreate(&e));
    pool_.push_back(e);
    return e;
  }
  hipStream_t s_;
  std::vector<hipEvent_t> pool_, free_;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pairs_;
  double acc_ = 0;
};

enum Frame { FX = 0, FZ = 1 };

class Amen {
 public:
  Amen(iga_ctx* ctx, const iga_kkt* kkt, const iga_tt* Y, double tol, const iga_amen_opts& o)
      : ctx_(ctx), st_(ctx->stream), kkt_(kkt), Y_(Y), tol_(tol), o_(o),
        t_mv_(ctx->stream), t_pc_(ctx->stream), t_if_(ctx->stream), t_svd_(ctx->stream),
        t_kr_(ctx->stream), t_mv32_(ctx->stream) {
    for (int d = 0; d < 3; ++d) n_[d] = kkt->M->n[d];
    g_ = std::sqrt(kkt->beta);
    nb_ = kkt->nblk;
    ntb_ = nb_ / 3;
    if (kkt->nt > 0) block_tables();
    ops_[0] = kkt->M;
    ops_[1] = kkt->K;
    ops_[2] = kkt->Kref;
    ry_[0] = 1; ry_[3] = 1;
    ry_[1] = Y->r[1]; ry_[2] = Y->r[2];
    rng_.seed(o.seed);
    lowp_ = o.precision == IGA_FP32 || o.precision == IGA_BF16;
    bf16_ = o.precision == IGA_BF16;
    // dense cores re-laid as [n][2p+1][R0][R1] once per solve: the banded stage of the
    // local matvec then contracts over one (R0, 2p+1) index instead of two nested ones.
    // Block-structured cores with few rank pairs are re-laid too, zeros included: for them
    // one product over the whole core costs less than one small launch per block.
    // The interface updates contract the same cores, the right ones with the rank roles
    // swapped ([n][2p+1][R1][R0]); the reference operator of the preconditioner is re-laid too.
    for (int op = 0; op < 3; ++op)
      for (int d = 0; d < 3; ++d) {
        const OpCore& c = ops_[op]->core[d];
        const bool dense = c.blocks.size() == 1 && c.blocks[0].na == c.R0 && c.blocks[0].nb == c.R1;
        if (!dense && (long)c.R0 * c.R1 > kDenseRankPairs) continue;
        const int b = 2 * ops_[op]->p + 1;
        const int dims[4] = {c.R0, c.n, b, c.R1}, perm[4] = {1, 2, 0, 3}, permT[4] = {1, 2, 3, 0};
        rcore_[op][d].reset(ctx, (long)c.R0 * c.n * b * c.R1);
        k::permute4(st_, c.data.get(), dims, perm, rcore_[op][d].get());
        rcoreT_[op][d].reset(ctx, (long)c.R0 * c.n * b * c.R1);
        k::permute4(st_, c.data.get(), dims, permT, rcoreT_[op][d].get());
      }
    if (lowp_) {
      // FP32 copies of the operator cores, fixed for the whole solve
      for (int op = 0; op < 2; ++op)
        for (int d = 0; d < 3; ++d) {
          const OpCore& c = ops_[op]->core[d];
          const long sz = (long)c.R0 * c.n * (2 * ops_[op]->p + 1) * c.R1;
          fcore_[op][d].reset(ctx, sz);
          k::to_f32(st_, sz, c.data.get(), fcore_[op][d].get());
          if (rcore_[op][d].get()) {
            frcore_[op][d].reset(ctx, sz);
            k::to_f32(st_, sz, rcore_[op][d].get(), frcore_[op][d].get());
          }
        }
    }
  }

  int run(const iga_btt* x0, iga_btt** sol, iga_amen_stats* stats);

 private:
  // ---- helpers ----
  DBuf random_buf(size_t n, double scale) {
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<double> h(n);
    for (auto& v : h) v = scale * nd(rng_);
    DBuf b(ctx_, n);
    IGA_HIP(hipMemcpyAsync(b.get(), h.data(), n * sizeof(double), hipMemcpyHostToDevice, st_));
    IGA_HIP(hipStreamSynchronize(st_));
    return b;
  }
  DBuf ones1() {
    DBuf b(ctx_, 1);
    k::fill(st_, 1, 1.0, b.get());
    return b;
  }
  long core_size(int d) const { return (long)r_[d] * n_[d] * r_[d + 1]; }
  OpView view(int op, int d) const { return view_of(ops_[op], d); }
  const double* Ycore(int d) const { return Y_->core[d]; }
  int R(int op, int d) const { return ops_[op]->R[d]; }

  void right_orth_plain(DBuf* cores, int* ranks, int d, bool prev_is_ell);
  void move_ell_to_first();
  void init_interfaces();
  void update_left(int d);
  void update_right(int d);
  LocalOp make_op(int d, Frame left, Frame right) const;
  void rhs_local(int d, Frame left, Frame right, double* out);
  double solve_local(int d);
  void setup_precond(int d);
  void apply_precond(const double* v, double* z);
  void matvec(const LocalOp& L, const double* x, double* y);
  // r0 (may be null): b - A x for the x on entry, already computed by the caller
  int fgmres(const LocalOp& L, const double* b, double* x, double bnorm, double abstol,
             const double* r0 = nullptr);
  void residual_proj(int d, Frame left, Frame right, double* out);  // rhs - A x in the given frames
  void move_right(int d);
  void move_left(int d);
  void orthonormal_columns(double* A, int m, int k, int kmax, DBuf& Q, int& q, double rel_floor);
  // smallest rank whose truncated core keeps the local residual <= target (see move_right)
  template <class Recon>
  int residual_rank(int d, int kmin, int kmax, const std::vector<double>& sigma, Recon recon);
  double local_res_of(int d, const double* xk);

  iga_ctx* ctx_;
  hipStream_t st_;
  const iga_kkt* kkt_;
  const iga_tt* Y_;
  double tol_;
  iga_amen_opts o_;
  const iga_ttop* ops_[3];
  int n_[3];
  int r_[4] = {1, 1, 1, 1};
  int ry_[4];
  int rho_[4] = {1, 1, 1, 1};
  int ell_ = 0;
  int kick_ = 4;
  double g_;  // sqrt(beta): scaled unknowns are (y, g u, lambda / g)
  int nb_ = 3;   // solution blocks: 3, or 3 nt for the time-dependent system
  int ntb_ = 1;  // blocks per component (time steps)
  // time-dependent system: K column ranges and the combination tables of the local operator
  int nkr_ = 0, kb_[2] = {0, 0}, kn_[2] = {0, 0};
  IBuf toff_, tsrc_;
  DBuf tcoef_;
  void block_tables();
  DBuf X_[3], Z_[3];
  DBuf PL_[3][3], PR_[3][3];  // (X, A, X), A in {M, K, Kref}
  DBuf YL_[3], YR_[3];        // (X, M, Y)
  DBuf ZL_[2][3], ZR_[2][3];  // (Z, A, X), A in {M, K}
  DBuf ZYL_[3], ZYR_[3];      // (Z, M, Y)
  // preconditioner of the current core
  // per core: eigen-data of the left and right interface pairs, with the interface version
  // they were computed from (an interface changes only when its neighbour core is updated)
  DBuf VLc_[3], lamLc_[3], VRc_[3], lamRc_[3];
  unsigned verL_[4] = {0, 0, 0, 0}, verR_[4] = {0, 0, 0, 0};
  unsigned cverL_[3] = {~0u, ~0u, ~0u}, cverR_[3] = {~0u, ~0u, ~0u};
  int crL_[3] = {-1, -1, -1}, crR_[3] = {-1, -1, -1};
  const double *VL_ = nullptr, *lamL_ = nullptr, *VR_ = nullptr, *lamR_ = nullptr;
  int pc_r0_ = 0, pc_r1_ = 0, pc_d_ = 0;
  DBuf pt1_, pt2_, pt3_;
  // Krylov workspace
  DBuf KV_, KZ_, w_, h_, red_, bl_, tmp_;
  LocalWork lw_;
  std::mt19937_64 rng_;
  // mixed-precision form: FP32 operands of the current local operator; inside the
  // refinement's inner solve (lp_inner_) every local matvec contracts in FP32
  bool lowp_ = false, lp_inner_ = false;
  bool bf16_ = false;  // inner products on BF16 matrix cores instead of FP32
  FBuf fcore_[2][3], fPL_[2], fPR_[2], fx_, fy_;
  FBuf frcore_[2][3];  // FP32 copies of the re-laid cores
  DBuf rcore_[3][3];   // re-laid cores [n][2p+1][R0][R1] (null for block-structured ones)
  DBuf rcoreT_[3][3];  // the same with the rank roles swapped, [n][2p+1][R1][R0]
  IfaceWork iw_;       // workspace of the interface updates and the right-hand-side projections
  OpView viewr(int op, int d) const {
    OpView v = view(op, d);
    v.Ar = rcore_[op][d].get();
    return v;
  }
  const std::vector<RankBlock>& blocks_of(int op, int d) const { return ops_[op]->core[d].blocks; }
  void ileft(int op, int d, const double* Phi, const double* U, const double* V, int ru0, int ru1, int rv0, int rv1,
             double* out) {
    interface_left_mc(ctx_, viewr(op, d), blocks_of(op, d), Phi, U, V, ru0, ru1, rv0, rv1, out, iw_);
  }
  void iright(int op, int d, const double* Phi, const double* U, const double* V, int ru0, int ru1, int rv0,
              int rv1, double* out) {
    interface_right_mc(ctx_, view(op, d), rcoreT_[op][d].get(), blocks_of(op, d), Phi, U, V, ru0, ru1, rv0, rv1,
                       out, iw_);
  }
  void lowp_operands(int d, LocalOp& L);
  int refine_solve(int d, const LocalOp& L, double bn, double ltol, double res0);
  // statistics
  EventTimer t_mv_, t_pc_, t_if_, t_svd_, t_kr_, t_mv32_;
  long long n_solves_ = 0, n_iters_ = 0, n_mv_ = 0, n_mv32_ = 0, n_refine_ = 0;
  double flops_ = 0, flops32_ = 0;
  double max_res_ = 0;
  // factor on the tolerance part of the truncation target: 1 while the half-sweeps make
  // progress, cut tenfold (down to 1e-3) after each half-sweep whose largest local residual
  // did not fall below the previous one's
  double trunc_scale_ = 1.0;
  double hist_res_[IGA_MAX_HISTORY] = {};
  int hist_r_[IGA_MAX_HISTORY][2] = {};
  long long hist_st_[IGA_MAX_HISTORY] = {};
  double bnorm_ = 1.0;  // norm of the local right-hand side of the last solve
  // the FP64 local residual of X_[solved_d_] as the last local solve left it, when that solve
  // computed it (-1: not known); the truncation of that core starts from it
  double solved_res_ = -1.0;
  int solved_d_ = -1;
  DBuf xk_;
};

// Make core d right-orthonormal (rows of the (r_{d-1}) x (n r_d) unfolding), pushing
// the remaining factor into core d-1 (all three components if it holds l).
void Amen::right_orth_plain(DBuf* cores, int* ranks, int d, bool prev_is_ell) {
  const int r0 = ranks[d], r1 = ranks[d + 1], n = n_[d];
  const int m = n * r1;
  Svd s;
  svd(ctx_, cores[d].get(), m, r0, m, /*trans=*/true, s);
  int k = 0;
  for (double v : s.sigma)
    if (v > 1e-14 * s.sigma[0]) ++k;
  k = std::max(k, 1);
  std::vector<int> idx(k);
  std::vector<double> inv(k), sg(k);
  for (int j = 0; j < k; ++j) {
    idx[j] = j;
    inv[j] = s.sigma[j] > 0 ? 1.0 / s.sigma[j] : 0.0;
    sg[j] = s.sigma[j];
  }
  IBuf didx(ctx_, k);
  DBuf dinv(ctx_, k), dsg(ctx_, k), T(ctx_, (size_t)m * k), F(ctx_, (size_t)r0 * k);
  IGA_HIP(hipMemcpyAsync(didx.get(), idx.data(), k * sizeof(int), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipMemcpyAsync(dinv.get(), inv.data(), k * sizeof(double), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipMemcpyAsync(dsg.get(), sg.data(), k * sizeof(double), hipMemcpyHostToDevice, st_));
  k::gather_cols(st_, m, r0, k, s.B.get(), s.p, didx.get(), dinv.get(), T.get(), k);
  DBuf nc(ctx_, (size_t)k * m);
  k::copy2d(st_, k, m, T.get(), 1, k, nc.get(), m);
  k::gather_cols(st_, r0, r0, k, s.V.get(), s.p, didx.get(), dsg.get(), F.get(), k);
  // previous core [.][n'][r0] times F (r0 x k)
  const int rp = ranks[d - 1], np = n_[d - 1];
  const int nl = prev_is_ell ? nb_ : 1;
  DBuf pc(ctx_, (size_t)nl * rp * np * k);
  k::Gemm g;
  g.M = rp * np; g.N = k; g.K = r0;
  g.A = cores[d - 1].get(); g.sAm = r0; g.sAk = 1;
  g.B = F.get(); g.sBk = k; g.sBn = 1;
  g.C = pc.get(); g.sCm = k; g.sCn = 1;
  g.nb1 = nl; g.sAb1 = (long)rp * np * r0; g.sCb1 = (long)rp * np * k;
  k::gemm(st_, g);
  IGA_HIP(hipStreamSynchronize(st_));
  cores[d] = std::move(nc);
  cores[d - 1] = std::move(pc);
  ranks[d] = k;
}

void Amen::init_interfaces() {
  for (int d = 0; d < 4; ++d) { ++verL_[d]; ++verR_[d]; }
  for (int op = 0; op < 3; ++op) {
    PL_[op][0] = ones1();
    PR_[op][2] = ones1();
  }
  YL_[0] = ones1();
  YR_[2] = ones1();
  for (int a = 0; a < 2; ++a) {
    ZL_[a][0] = ones1();
    ZR_[a][2] = ones1();
  }
  ZYL_[0] = ones1();
  ZYR_[2] = ones1();
  for (int d = 2; d >= 1; --d) update_right(d);
}

// interfaces of core d-1 from core d (right side)
void Amen::update_right(int d) {
  g_phase = "update_right";
  const int id = t_if_.begin();
  ++verR_[d - 1];
  const int r0 = r_[d], r1 = r_[d + 1];
  for (int op = 0; op < 3; ++op) {
    PR_[op][d - 1].reset(ctx_, (size_t)R(op, d) * r0 * r0);
    iright(op, d, PR_[op][d].get(), X_[d].get(), X_[d].get(), r0, r1, r0, r1, PR_[op][d - 1].get());
  }
  YR_[d - 1].reset(ctx_, (size_t)R(0, d) * r0 * ry_[d]);
  iright(0, d, YR_[d].get(), X_[d].get(), Ycore(d), r0, r1, ry_[d], ry_[d + 1], YR_[d - 1].get());
  if (kick_ > 0) {
    const int z0 = rho_[d], z1 = rho_[d + 1];
    for (int a = 0; a < 2; ++a) {
      ZR_[a][d - 1].reset(ctx_, (size_t)R(a, d) * z0 * r0);
      iright(a, d, ZR_[a][d].get(), Z_[d].get(), X_[d].get(), z0, z1, r0, r1, ZR_[a][d - 1].get());
    }
    ZYR_[d - 1].reset(ctx_, (size_t)R(0, d) * z0 * ry_[d]);
    iright(0, d, ZYR_[d].get(), Z_[d].get(), Ycore(d), z0, z1, ry_[d], ry_[d + 1], ZYR_[d - 1].get());
  }
  t_if_.end(id);
}

// interfaces of core d+1 from core d (left side)
void Amen::update_left(int d) {
  g_phase = "update_left";
  const int id = t_if_.begin();
  ++verL_[d + 1];
  const int r0 = r_[d], r1 = r_[d + 1];
  for (int op = 0; op < 3; ++op) {
    PL_[op][d + 1].reset(ctx_, (size_t)R(op, d + 1) * r1 * r1);
    ileft(op, d, PL_[op][d].get(), X_[d].get(), X_[d].get(), r0, r1, r0, r1, PL_[op][d + 1].get());
  }
  YL_[d + 1].reset(ctx_, (size_t)R(0, d + 1) * r1 * ry_[d + 1]);
  ileft(0, d, YL_[d].get(), X_[d].get(), Ycore(d), r0, r1, ry_[d], ry_[d + 1], YL_[d + 1].get());
  if (kick_ > 0) {
    const int z0 = rho_[d], z1 = rho_[d + 1];
    for (int a = 0; a < 2; ++a) {
      ZL_[a][d + 1].reset(ctx_, (size_t)R(a, d + 1) * z1 * r1);
      ileft(a, d, ZL_[a][d].get(), Z_[d].get(), X_[d].get(), z0, z1, r0, r1, ZL_[a][d + 1].get());
    }
    ZYL_[d + 1].reset(ctx_, (size_t)R(0, d + 1) * z1 * ry_[d + 1]);
    ileft(0, d, ZYL_[d].get(), Z_[d].get(), Ycore(d), z0, z1, ry_[d], ry_[d + 1], ZYL_[d + 1].get());
  }
  t_if_.end(id);
}

// Tables of the local operator of the time-dependent system: output block o of A D x is
// sum_l cM[o][l] D_l M x_l + cK[o][l] D_l K x_l, D = (1, 1/g, g) per component (the scaled
// unknowns); K acts on the ranges of consecutive blocks where cK has entries.
void Amen::block_tables() {
  const int nb = nb_;
  const std::vector<double>& cM = kkt_->cM;
  const std::vector<double>& cK = kkt_->cK;
  std::vector<int> kcol(nb, 0), kpos(nb, -1);
  for (int o = 0; o < nb; ++o)
    for (int l = 0; l < nb; ++l)
      if (cK[(size_t)o * nb + l] != 0.0) kcol[l] = 1;
  nkr_ = 0;
  int pos = 0;
  for (int l = 0; l < nb; ++l) {
    if (!kcol[l]) continue;
    if (l == 0 || !kcol[l - 1]) {
      require(nkr_ < 2, IGA_EINVAL, "amen: more than two stiffness column ranges");
      kb_[nkr_] = l;
      kn_[nkr_] = 0;
      ++nkr_;
    }
    ++kn_[nkr_ - 1];
    kpos[l] = pos++;
  }
  auto D = [&](int l) {
    const int c = l / ntb_;
    return c == 0 ? 1.0 : (c == 1 ? 1.0 / g_ : g_);
  };
  std::vector<int> toff(nb + 1, 0), src;
  std::vector<double> coef;
  for (int o = 0; o < nb; ++o) {
    toff[o] = (int)src.size();
    for (int l = 0; l < nb; ++l) {
      const double m = cM[(size_t)o * nb + l], kk = cK[(size_t)o * nb + l];
      if (m != 0.0) { src.push_back(l); coef.push_back(m * D(l)); }
      if (kk != 0.0) { src.push_back(nb + kpos[l]); coef.push_back(kk * D(l)); }
    }
  }
  toff[nb] = (int)src.size();
  toff_.reset(ctx_, toff.size());
  tsrc_.reset(ctx_, std::max<size_t>(src.size(), 1));
  tcoef_.reset(ctx_, std::max<size_t>(coef.size(), 1));
  IGA_HIP(hipMemcpyAsync(toff_.get(), toff.data(), toff.size() * sizeof(int), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipMemcpyAsync(tsrc_.get(), src.data(), src.size() * sizeof(int), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipMemcpyAsync(tcoef_.get(), coef.data(), coef.size() * sizeof(double), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipStreamSynchronize(st_));
}

LocalOp Amen::make_op(int d, Frame left, Frame right) const {
  LocalOp L;
  L.M = view(0, d);
  L.K = view(1, d);
  L.M.Ar = rcore_[0][d].get();
  L.K.Ar = rcore_[1][d].get();
  L.Mblocks = ops_[0]->core[d].blocks;
  L.Kblocks = ops_[1]->core[d].blocks;
  L.r0 = r_[d]; L.n = n_[d]; L.r1 = r_[d + 1];
  L.nblk = nb_;
  if (toff_.get()) {
    L.nkr = nkr_;
    for (int j = 0; j < 2; ++j) { L.kb[j] = kb_[j]; L.kn[j] = kn_[j]; }
    L.toff = toff_.get(); L.src = tsrc_.get(); L.tcoef = tcoef_.get();
  }
  // A D: columns 1 and 2 carry the factors 1/g and g of the scaled unknowns
  L.coef.k02 = g_;
  L.coef.m11 = kkt_->beta / g_;
  L.coef.m12 = -g_;
  L.coef.k20 = 1.0;
  L.coef.m21 = -1.0 / g_;
  if (left == FX) {
    L.PhiL_M = PL_[0][d].get(); L.PhiL_K = PL_[1][d].get();
  } else {
    L.PhiL_M = ZL_[0][d].get(); L.PhiL_K = ZL_[1][d].get(); L.r0o = rho_[d];
  }
  if (right == FX) {
    L.PhiR_M = PR_[0][d].get(); L.PhiR_K = PR_[1][d].get();
  } else {
    L.PhiR_M = ZR_[0][d].get(); L.PhiR_K = ZR_[1][d].get(); L.r1o = rho_[d + 1];
  }
  return L;
}

// [F^T M yhat; 0; 0] projected with the given frames (block o: cb[o] F^T M yhat)
void Amen::rhs_local(int d, Frame left, Frame right, double* out) {
  const int a_out = left == FX ? r_[d] : rho_[d];
  const int b_out = right == FX ? r_[d + 1] : rho_[d + 1];
  const long e = (long)a_out * n_[d] * b_out;
  const double* PL = left == FX ? YL_[d].get() : ZYL_[d].get();
  const double* PR = right == FX ? YR_[d].get() : ZYR_[d].get();
  apply_one_mc(ctx_, viewr(0, d), blocks_of(0, d), PL, PR, a_out, ry_[d], ry_[d + 1], b_out, Ycore(d), out, iw_);
  const std::vector<double>& cb = kkt_->cb;
  for (int o = nb_ - 1; o >= 1; --o) {
    if (cb[o] == 0.0) k::fill(st_, e, 0.0, out + o * e);
    else k::axpby(st_, e, cb[o], out, 0.0, out + o * e);
  }
  if (cb[0] != 1.0) k::scale(st_, e, cb[0], out);
}

void Amen::matvec(const LocalOp& L, const double* x, double* y) {
  g_phase = "matvec";
  if (lp_inner_) {
    // FP32 (or BF16-product) contractions on FP32 copies of x; the Krylov vectors stay FP64
    const long N = L.size(), No = L.out_size();
    fx_.ensure(ctx_, N);
    fy_.ensure(ctx_, No);
    const int id = t_mv32_.begin();
    k::to_f32(st_, N, x, fx_.get());
    local_matvec_f32(ctx_, L, fx_.get(), fy_.get(), lw_, bf16_);
    k::to_f64(st_, No, fy_.get(), y);
    t_mv32_.end(id);
    ++n_mv32_;
    flops32_ += local_flops(L);
    return;
  }
  const int id = t_mv_.begin();
  local_matvec(ctx_, L, x, y, lw_);
  t_mv_.end(id);
  ++n_mv_;
  flops_ += local_flops(L);
}

// FP32 copies of the interfaces of the current local operator (the cores were converted
// once for the solve).
void Amen::lowp_operands(int d, LocalOp& L) {
  for (int op = 0; op < 2; ++op) {
    const long sl = (long)R(op, d) * r_[d] * r_[d], sr = (long)R(op, d + 1) * r_[d + 1] * r_[d + 1];
    fPL_[op].ensure(ctx_, sl);
    fPR_[op].ensure(ctx_, sr);
    k::to_f32(st_, sl, PL_[op][d].get(), fPL_[op].get());
    k::to_f32(st_, sr, PR_[op][d].get(), fPR_[op].get());
  }
  L.fPhiL_M = fPL_[0].get(); L.fPhiR_M = fPR_[0].get();
  L.fPhiL_K = fPL_[1].get(); L.fPhiR_K = fPR_[1].get();
  L.M.Af = fcore_[0][d].get();
  L.K.Af = fcore_[1][d].get();
  L.M.Arf = frcore_[0][d].get();
  L.K.Arf = frcore_[1][d].get();
}

// Mixed-precision local solve by iterative refinement: the FP64 residual r = b - A x (in
// tmp_ on entry, relative norm res0) is reduced by an inner FGMRES whose matvecs contract
// in FP32 (or on BF16 products), the correction is added in FP64, and the FP64 residual is
// recomputed, until it is <= ltol. The inner solve asks for what the low-precision operator
// can deliver (relative 2e-5 for FP32; 1e-2 for BF16, whose operands carry a relative
// rounding of 2^-9 per stage) or the remaining factor, whichever is larger. Returns the
// inner iterations.
int Amen::refine_solve(int d, const LocalOp& L, double bn, double ltol, double res0) {
  const long N = L.size();
  DBuf e(ctx_, N), r(ctx_, N);
  double res = res0;
  int its = 0;
  IGA_HIP(hipMemcpyAsync(r.get(), tmp_.get(), N * sizeof(double), hipMemcpyDeviceToDevice, st_));
  const double floor = bf16_ ? 1e-2 : 2e-5;
  for (int ref = 0; ref < 20 && res > ltol; ++ref) {
    const double rn = res * bn;
    const double inner = std::max(ltol / res, floor);
    k::fill(st_, N, 0.0, e.get());
    lp_inner_ = true;
    its += fgmres(L, r.get(), e.get(), rn, inner * rn, r.get());  // e = 0: its residual is r
    lp_inner_ = false;
    k::axpby(st_, N, 1.0, e.get(), 1.0, X_[d].get());
    matvec(L, X_[d].get(), r.get());
    k::axpby(st_, N, 1.0, bl_.get(), -1.0, r.get());
    res = std::sqrt(norm2_host(ctx_, N, r.get())) / bn;
    require(std::isfinite(res), IGA_ENUM, "amen_solve: non-finite residual in the mixed-precision refinement");
    ++n_refine_;
  }
  solved_res_ = res;
  return its;
}

void Amen::residual_proj(int d, Frame left, Frame right, double* out) {
  LocalOp L = make_op(d, left, right);
  const long e = L.out_size();
  tmp_.ensure(ctx_, e);
  rhs_local(d, left, right, out);
  local_matvec(ctx_, L, X_[d].get(), tmp_.get(), lw_);
  k::axpby(st_, e, -1.0, tmp_.get(), 1.0, out);
}

void Amen::setup_precond(int d) {
  g_phase = "setup_precond";
  const int id = t_pc_.begin();
  const int r0 = r_[d], r1 = r_[d + 1];
  pc_d_ = d; pc_r0_ = r0; pc_r1_ = r1;
  if (cverL_[d] != verL_[d] || crL_[d] != r0) {
    VLc_[d].reset(ctx_, (size_t)r0 * r0);
    lamLc_[d].reset(ctx_, r0);
    if (d == 0) {
      k::fill(st_, 1, 1.0, VLc_[d].get());
      k::fill(st_, 1, 0.0, lamLc_[d].get());
    } else {
      // Kref left interface: slot 0 = K-part, slot 1 = M-part
      DBuf H(ctx_, (size_t)2 * r0 * r0);
      IGA_HIP(hipMemcpyAsync(H.get(), PL_[2][d].get(), (size_t)2 * r0 * r0 * 8, hipMemcpyDeviceToDevice, st_));
      k::symmetrize(st_, 2, r0, H.get(), (long)r0 * r0);
      gen_eig(ctx_, r0, H.get(), H.get() + (long)r0 * r0, VLc_[d].get(), lamLc_[d].get());
    }
    cverL_[d] = verL_[d];
    crL_[d] = r0;
  }
  if (cverR_[d] != verR_[d] || crR_[d] != r1) {
    VRc_[d].reset(ctx_, (size_t)r1 * r1);
    lamRc_[d].reset(ctx_, r1);
    if (d == 2) {
      k::fill(st_, 1, 1.0, VRc_[d].get());
      k::fill(st_, 1, 0.0, lamRc_[d].get());
    } else {
      // right interface: slot 0 = M-part, slot 1 = K-part
      DBuf H(ctx_, (size_t)2 * r1 * r1);
      IGA_HIP(hipMemcpyAsync(H.get(), PR_[2][d].get(), (size_t)2 * r1 * r1 * 8, hipMemcpyDeviceToDevice, st_));
      k::symmetrize(st_, 2, r1, H.get(), (long)r1 * r1);
      gen_eig(ctx_, r1, H.get() + (long)r1 * r1, H.get(), VRc_[d].get(), lamRc_[d].get());
    }
    cverR_[d] = verR_[d];
    crR_[d] = r1;
  }
  VL_ = VLc_[d].get(); lamL_ = lamLc_[d].get();
  VR_ = VRc_[d].get(); lamR_ = lamRc_[d].get();
  t_pc_.end(id);
}

// z = (V_L (x) V_n (x) V_R) D^{-1} (V_L (x) V_n (x) V_R)^T v, D the per-mode KKT blocks
void Amen::apply_precond(const double* v, double* z) {
  g_phase = "apply_precond";
  const int id = t_pc_.begin();
  const int r0 = pc_r0_, r1 = pc_r1_, n = n_[pc_d_];
  const long e = (long)r0 * n * r1;
  pt1_.ensure(ctx_, nb_ * e);
  pt2_.ensure(ctx_, nb_ * e);
  pt3_.ensure(ctx_, nb_ * e);
  const double* Vn = kkt_->Vn[pc_d_].get();
  // pass 0: pt1 <- W^T v (modes a, j, b), solve the mode blocks in place;
  // pass 1: z <- W pt1
  for (int pass = 0; pass < 2; ++pass) {
    const bool tr = pass == 0;
    const double* src = tr ? v : pt1_.get();
    // mode a: out[l][a'][(j b)] = sum_a VL(a, a') in[l][a][(j b)]
    k::Gemm ga;
    ga.M = r0; ga.N = n * r1; ga.K = r0;
    ga.A = VL_; ga.sAm = tr ? 1 : r0; ga.sAk = tr ? r0 : 1;
    ga.B = src; ga.sBk = (long)n * r1; ga.sBn = 1;
    ga.C = pt2_.get(); ga.sCm = (long)n * r1; ga.sCn = 1;
    ga.nb1 = nb_; ga.sBb1 = e; ga.sCb1 = e;
    k::gemm(st_, ga);
    // mode j: out[(l a')][i'][b] = sum_j Vn(j, i') in[(l a')][j][b]
    double* jout = tr ? pt1_.get() : pt3_.get();
    k::Gemm gj;
    gj.M = n; gj.N = r1; gj.K = n;
    gj.A = Vn; gj.sAm = tr ? 1 : n; gj.sAk = tr ? n : 1;
    gj.B = pt2_.get(); gj.sBk = r1; gj.sBn = 1;
    gj.C = jout; gj.sCm = r1; gj.sCn = 1;
    gj.nb1 = nb_ * r0; gj.sBb1 = (long)n * r1; gj.sCb1 = (long)n * r1;
    k::gemm(st_, gj);
    // mode b: out[(l a' i')][b'] = sum_b in[..][b] VR(b, b')
    double* bout = tr ? pt2_.get() : z;
    k::Gemm gb;
    gb.M = nb_ * r0 * n; gb.N = r1; gb.K = r1;
    gb.A = jout; gb.sAm = r1; gb.sAk = 1;
    gb.B = VR_; gb.sBk = tr ? r1 : 1; gb.sBn = tr ? 1 : r1;
    gb.C = bout; gb.sCm = r1; gb.sCn = 1;
    k::gemm(st_, gb);
    if (!tr) k::scale3(st_, ntb_ * e, 1.0, g_, 1.0 / g_, z);  // D^{-1}: to the scaled unknowns
    if (tr) {
      if (kkt_->nt > 0)
        k::fd_solve_time(st_, r0, n, r1, kkt_->nt, lamL_, kkt_->lamn[pc_d_].get(), lamR_, kkt_->beta, kkt_->tau,
                         pt2_.get(), pt3_.get());
      else
        k::fd_solve(st_, r0, n, r1, lamL_, kkt_->lamn[pc_d_].get(), lamR_, kkt_->beta, 1.0, pt2_.get());
      std::swap(pt1_, pt2_);
    }
  }
  t_pc_.end(id);
}

// Right-preconditioned restarted flexible GMRES with classical Gram-Schmidt applied twice.
// Returns the number of iterations; x is updated in place.
int Amen::fgmres(const LocalOp& L, const double* b, double* x, double bnorm, double abstol, const double* r0) {
  g_phase = "fgmres";
  const long N = L.size();
  const int m = std::max(2, std::min(o_.local_restart, 63));
  const int maxit = o_.local_maxit;
  static thread_local char phase[160];
  std::snprintf(phase, sizeof(phase), "fgmres basis N=%ld m=%d r=%d,%d,%d n=%d", N, m, L.r0, L.r1, L.out1(), L.n);
  g_phase = phase;
  KV_.ensure(ctx_, (size_t)(m + 1) * N);
  KZ_.ensure(ctx_, (size_t)m * N);
  g_phase = "fgmres";
  w_.ensure(ctx_, N);
  h_.ensure(ctx_, 130);
  red_.ensure(ctx_, (size_t)k::reduce_partials() * 64);
  double* V = KV_.get();
  double* Zb = KZ_.get();
  double* w = w_.get();
  double* h = h_.get();
  int it = 0;
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), hh(m + 2), y(m);
  bool first = true;
  while (it < maxit) {
    // r = b - A x (given for the first cycle)
    if (first && r0) {
      IGA_HIP(hipMemcpyAsync(V, r0, N * sizeof(double), hipMemcpyDeviceToDevice, st_));
    } else {
      matvec(L, x, V);
      k::axpby(st_, N, 1.0, b, -1.0, V);
    }
    first = false;
    const double beta0 = std::sqrt(norm2_host(ctx_, N, V));
    require(std::isfinite(beta0), IGA_ENUM, "amen_solve: non-finite residual norm in the local Krylov solve");
    if (beta0 <= abstol || !(beta0 > 0)) break;
    k::scale(st_, N, 1.0 / beta0, V);
    std::fill(gv.begin(), gv.end(), 0.0);
    gv[0] = beta0;
    int j = 0;
    bool done = false;
    for (; j < m && it < maxit; ++j, ++it) {
      apply_precond(V + j * N, Zb + j * N);
      matvec(L, Zb + j * N, w);
      const int id = t_kr_.begin();
      // CGS2
      k::multidot(st_, N, j + 1, V, N, w, red_.get(), h);
      k::multiaxpy(st_, N, j + 1, V, N, h, -1.0, w);
      k::multidot(st_, N, j + 1, V, N, w, red_.get(), h + 64);
      k::multiaxpy(st_, N, j + 1, V, N, h + 64, -1.0, w);
      k::dot(st_, N, w, w, red_.get(), h + 128);
      IGA_HIP(hipMemcpyAsync(hh.data(), h, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, st_));
      std::vector<double> h2(j + 1);
      IGA_HIP(hipMemcpyAsync(h2.data(), h + 64, (j + 1) * sizeof(double), hipMemcpyDeviceToHost, st_));
      double wn2 = 0;
      IGA_HIP(hipMemcpyAsync(&wn2, h + 128, sizeof(double), hipMemcpyDeviceToHost, st_));
      IGA_HIP(hipStreamSynchronize(st_));
      t_kr_.end(id);
      for (int i = 0; i <= j; ++i) hh[i] += h2[i];
      const double hn = std::sqrt(std::max(wn2, 0.0));
      hh[j + 1] = hn;
      if (hn > 0) k::axpby(st_, N, 1.0 / hn, w, 0.0, V + (j + 1) * N);
      // Givens
      for (int i = 0; i < j; ++i) {
        const double t = cs[i] * hh[i] + sn[i] * hh[i + 1];
        hh[i + 1] = -sn[i] * hh[i] + cs[i] * hh[i + 1];
        hh[i] = t;
      }
      const double den = std::hypot(hh[j], hh[j + 1]);
      cs[j] = den > 0 ? hh[j] / den : 1.0;
      sn[j] = den > 0 ? hh[j + 1] / den : 0.0;
      hh[j] = den;
      hh[j + 1] = 0.0;
      gv[j + 1] = -sn[j] * gv[j];
      gv[j] = cs[j] * gv[j];
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hh[i];
      if (std::fabs(gv[j + 1]) <= abstol || hn == 0.0) {
        ++j;
        ++it;
        done = true;
        break;
      }
    }
    // x += Z y,  H y = g
    const int kdim = j;
    for (int i = kdim - 1; i >= 0; --i) {
      double s = gv[i];
      for (int l = i + 1; l < kdim; ++l) s -= H[(size_t)i * m + l] * y[l];
      y[i] = H[(size_t)i * m + i] != 0.0 ? s / H[(size_t)i * m + i] : 0.0;
    }
    if (kdim > 0) {
      IGA_HIP(hipMemcpyAsync(h, y.data(), kdim * sizeof(double), hipMemcpyHostToDevice, st_));
      k::multiaxpy(st_, N, kdim, Zb, N, h, 1.0, x);
      IGA_HIP(hipStreamSynchronize(st_));
    }
    if (done) break;
  }
  (void)bnorm;
  return it;
}

double Amen::solve_local(int d) {
  g_phase = "solve_local";
  LocalOp L = make_op(d, FX, FX);
  const long N = L.size();
  bl_.ensure(ctx_, N);
  tmp_.ensure(ctx_, N);
  rhs_local(d, FX, FX, bl_.get());
  double bn = std::sqrt(norm2_host(ctx_, N, bl_.get()));
  require(std::isfinite(bn), IGA_ENUM, "amen_solve: non-finite local right-hand side");
  if (!(bn > 0)) bn = 1.0;
  bnorm_ = bn;
  matvec(L, X_[d].get(), tmp_.get());
  k::axpby(st_, N, 1.0, bl_.get(), -1.0, tmp_.get());
  const double res = std::sqrt(norm2_host(ctx_, N, tmp_.get())) / bn;
  // a NaN compares false with every tolerance, so it would pass for convergence
  require(std::isfinite(res), IGA_ENUM, "amen_solve: non-finite local residual (the iterate holds NaN or Inf)");
  ++n_solves_;
  const double ltol = o_.local_tol;
  solved_d_ = d;
  solved_res_ = res;  // kept if no solve is needed
  if (res > ltol) {
    setup_precond(d);
    if (lowp_) {
      lowp_operands(d, L);
      n_iters_ += refine_solve(d, L, bn, ltol, res);  // leaves solved_res_ at its final residual
    } else {
      solved_res_ = -1.0;
      n_iters_ += fgmres(L, bl_.get(), X_[d].get(), bn, ltol * bn, tmp_.get());
    }
  }
  return res;
}

// Orthonormal basis of the column space of the m x k matrix A (row-major, destroyed),
// at most kmax columns, dropping directions below rel_floor of the largest.
void Amen::orthonormal_columns(double* A, int m, int k, int kmax, DBuf& Q, int& q, double rel_floor) {
  Svd s;
  svd(ctx_, A, m, k, k, false, s);
  q = 0;
  if (s.sigma.empty() || !(s.sigma[0] > 1e-300)) return;
  for (int j = 0; j < k && q < kmax; ++j)
    if (s.sigma[j] > rel_floor * s.sigma[0]) ++q;
  if (q == 0) return;
  std::vector<int> idx(q);
  std::vector<double> inv(q);
  for (int j = 0; j < q; ++j) {
    idx[j] = j;
    inv[j] = 1.0 / s.sigma[j];
  }
  IBuf didx(ctx_, q);
  DBuf dinv(ctx_, q);
  IGA_HIP(hipMemcpyAsync(didx.get(), idx.data(), q * sizeof(int), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipMemcpyAsync(dinv.get(), inv.data(), q * sizeof(double), hipMemcpyHostToDevice, st_));
  Q.reset(ctx_, (size_t)m * q);
  k::gather_cols(st_, m, k, q, s.B.get(), s.p, didx.get(), dinv.get(), Q.get(), q);
  IGA_HIP(hipStreamSynchronize(st_));
}

// Local relative residual ||b_loc - A_loc x|| / ||b_loc|| of a candidate core in the
// current (X, X) frames of core d.
double Amen::local_res_of(int d, const double* xk) {
  LocalOp L = make_op(d, FX, FX);
  const long N = L.size();
  tmp_.ensure(ctx_, N);
  matvec(L, xk, tmp_.get());
  k::axpby(st_, N, 1.0, bl_.get(), -1.0, tmp_.get());
  return std::sqrt(norm2_host(ctx_, N, tmp_.get())) / bnorm_;
}

// Residual-based truncation: the smallest k in [kmin, kmax] such that the rank-k
// approximation of the solved core has local residual <= max(s tol / 2, 1.5 min(r_full, tol)),
// r_full the residual of the untruncated core, s = trunc_scale_ (the residual decreases with k; kmax if no
// k passes). Each test costs a local matvec, so the search starts from a prediction: one
// probe at the rank where the singular-value tail t(k) = (sum_{j >= k} s_j^2)^(1/2) drops
// below target * t(0) fits r(k)^2 = r_full^2 + (a t(k))^2, the model's smallest passing
// rank is tested, and the search gallops away from it in steps 1, 2, 4, .. until the test
// changes, then bisects the last step.
template <class Recon>
int Amen::residual_rank(int d, int kmin, int kmax, const std::vector<double>& sigma, Recon recon) {
  const long N = (long)nb_ * r_[d] * n_[d] * r_[d + 1];
  xk_.ensure(ctx_, N);
  // the solve's own final FP64 residual where it computed one (same operations, same value)
  const double full = solved_d_ == d && solved_res_ >= 0.0 ? solved_res_ : local_res_of(d, X_[d].get());
  solved_d_ = -1;
  require(std::isfinite(full), IGA_ENUM, "amen_solve: non-finite local residual in the truncation");
  // a local solve that stopped short of the tolerance (full > tol) grants no slack: the
  // truncation must then reach 1.5 tol, which keeps the rank where the solve was incomplete
  // instead of truncating to the solve's own (large) residual
  const double target = std::max(0.5 * trunc_scale_ * tol_, 1.5 * std::min(full, tol_));
  std::vector<signed char> known((size_t)kmax + 1, -1);
  double probe_res = 0.0;
  auto test = [&](int kk, double* resid) {
    if (known[kk] >= 0 && !resid) return known[kk] == 1;
    recon(kk, xk_.get());
    const double r = local_res_of(d, xk_.get());
    if (resid) *resid = r;
    known[kk] = r <= target ? 1 : 0;
    return r <= target;
  };
  auto ok = [&](int kk) { return test(kk, nullptr); };
  int lo = std::max(1, kmin), hi = kmax;  // the answer lies in [lo, hi]
  if (lo >= hi) return hi;
  // singular-value tails t(k), k = 0 .. kmax
  std::vector<double> tail((size_t)kmax + 1, 0.0);
  {
    double acc = 0.0;
    for (int j = (int)sigma.size() - 1; j >= 0; --j) {
      acc += sigma[j] * sigma[j];
      if (j <= kmax) tail[j] = std::sqrt(acc);
    }
  }
  int kp = hi;
  for (int k = lo; k <= hi; ++k)
    if (tail[k] <= target * tail[0]) { kp = k; break; }
  test(kp, &probe_res);
  int guess = kp;
  if (tail[kp] > 0.0 && probe_res > full) {
    const double a2 = (probe_res * probe_res - full * full) / (tail[kp] * tail[kp]);
    const double room = target * target - full * full;
    guess = hi;
    if (room > 0.0)
      for (int k = lo; k <= hi; ++k)
        if (a2 * tail[k] * tail[k] <= room) { guess = k; break; }
  }
  const int g = std::min(std::max(guess, lo), hi);
  if (ok(g)) {
    // passes: step down until a rank fails
    hi = g;
    int step = 1;
    while (hi > lo) {
      const int t = std::max(lo, hi - step);
      if (ok(t)) {
        hi = t;
        step *= 2;
      } else {
        lo = t;
        break;
      }
    }
    if (hi == lo) return hi;
  } else {
    // fails: step up until a rank passes
    lo = g;
    int step = 1;
    while (true) {
      const int t = std::min(hi, lo + step);
      if (t == hi) {
        if (t == g || !ok(t)) return hi;
        break;
      }
      if (ok(t)) {
        hi = t;
        break;
      }
      lo = t;
      step *= 2;
    }
  }
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (ok(mid)) hi = mid; else lo = mid;
  }
  return hi;
}

void Amen::move_right(int d) {
  g_phase = "move_right";
  const int r0 = r_[d], r1 = r_[d + 1], n = n_[d];
  const int m = r0 * n;
  const long e = (long)r0 * n * r1;
  int sid = t_svd_.begin();
  // residual projections with the solved core
  DBuf zc, rz;
  if (kick_ > 0) {
    zc.reset(ctx_, (long)nb_ * rho_[d] * n * rho_[d + 1]);
    residual_proj(d, FZ, FZ, zc.get());
    rz.reset(ctx_, (long)nb_ * r0 * n * rho_[d + 1]);
    residual_proj(d, FX, FZ, rz.get());
  }
  // truncated SVD of F (r0 n) x (nb r1)
  DBuf F(ctx_, nb_ * e);
  {
    const int dims[4] = {nb_, r0, n, r1};
    const int perm[4] = {1, 2, 0, 3};
    k::permute4(st_, X_[d].get(), dims, perm, F.get());
  }
  Svd s;
  svd(ctx_, F.get(), m, nb_ * r1, nb_ * r1, false, s);
  const int K3 = nb_ * r1;
  const int rmax = std::min(o_.r_max, std::min(m, K3));
  int rt = 1;
  if (s.sigma[0] > 0) {
    int nz = 0;
    for (double v : s.sigma) nz += v > 1e-14 * s.sigma[0];
    DBuf Fk(ctx_, (size_t)m * K3);
    auto recon = [&](int kk, double* out) {
      k::gemm_rm(st_, m, K3, kk, s.B.get(), s.p, false, s.V.get(), s.p, true, Fk.get(), K3);
      const int dims[4] = {r0, n, nb_, r1};
      const int perm[4] = {2, 0, 1, 3};
      k::permute4(st_, Fk.get(), dims, perm, out);
    };
    // the search's local matvecs are timed as local matvecs, not as truncation
    t_svd_.end(sid);
    rt = residual_rank(d, 1, std::min(rmax, std::max(nz, 1)), s.sigma, recon);
    sid = t_svd_.begin();
  }
  static thread_local char ph[200];
  std::snprintf(ph, sizeof ph, "move_right d=%d r0=%d r1=%d m=%d K3=%d rt=%d rho=%d,%d r2=%d", d, r0, r1, m, K3, rt, rho_[d], rho_[d + 1], r_[d + 2]);
  g_phase = ph;
  std::vector<int> idx(rt);
  std::vector<double> inv(rt), sg(rt);
  for (int j = 0; j < rt; ++j) {
    idx[j] = j;
    inv[j] = s.sigma[j] > 0 ? 1.0 / s.sigma[j] : 0.0;
    sg[j] = s.sigma[j];
  }
  IBuf didx(ctx_, rt);
  DBuf dinv(ctx_, rt), dsg(ctx_, rt);
  IGA_HIP(hipMemcpyAsync(didx.get(), idx.data(), rt * sizeof(int), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipMemcpyAsync(dinv.get(), inv.data(), rt * sizeof(double), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipMemcpyAsync(dsg.get(), sg.data(), rt * sizeof(double), hipMemcpyHostToDevice, st_));
  DBuf U(ctx_, (size_t)m * rt);
  k::gather_cols(st_, m, K3, rt, s.B.get(), s.p, didx.get(), dinv.get(), U.get(), rt);
  // C = Sigma V^T: (rt x nb r1)
  DBuf CT(ctx_, (size_t)K3 * rt), C(ctx_, (size_t)rt * K3);
  k::gather_cols(st_, K3, K3, rt, s.V.get(), s.p, didx.get(), dsg.get(), CT.get(), rt);
  k::copy2d(st_, rt, K3, CT.get(), 1, rt, C.get(), K3);
  // enrichment directions orthogonal to U
  DBuf Qz;
  int q = 0;
  if (kick_ > 0 && rt < m) {
    const int kz = nb_ * rho_[d + 1];
    DBuf Rz(ctx_, (size_t)m * kz), T(ctx_, (size_t)rt * kz);
    const int dims[4] = {nb_, r0, n, rho_[d + 1]};
    const int perm[4] = {1, 2, 0, 3};
    k::permute4(st_, rz.get(), dims, perm, Rz.get());
    // T = U^T Rz has few output tiles and a contraction over all m rows: split it
    DBuf W(ctx_, (size_t)64 * rt * kz);
    for (int pass = 0; pass < 2; ++pass) {
      k::gemm_rm(st_, rt, kz, m, U.get(), rt, true, Rz.get(), kz, false, T.get(), kz, 1.0, 0.0, W.get(), W.size());
      k::gemm_rm(st_, m, kz, rt, U.get(), rt, false, T.get(), kz, false, Rz.get(), kz, -1.0, 1.0);
    }
    orthonormal_columns(Rz.get(), m, kz, std::min(kick_, m - rt), Qz, q, 1e-12);
  }
  const int rn = rt + q;
  DBuf Xn(ctx_, (size_t)m * rn);
  k::copy2d(st_, m, rt, U.get(), rt, 1, Xn.get(), rn);
  if (q > 0) k::copy2d(st_, m, q, Qz.get(), q, 1, Xn.get() + rt, rn);
  // next core: [rn][nb][n1][r2] = Cn (rn*nb x r1) . X_{d+1} (r1 x n1 r2), Cn = [C; 0]
  const int n1 = n_[d + 1], r2 = r_[d + 2];
  DBuf Cn(ctx_, (size_t)rn * nb_ * r1), T2(ctx_, (size_t)rn * nb_ * n1 * r2), Xd1(ctx_, (size_t)nb_ * rn * n1 * r2);
  k::fill(st_, (long)rn * nb_ * r1, 0.0, Cn.get());
  IGA_HIP(hipMemcpyAsync(Cn.get(), C.get(), (size_t)rt * nb_ * r1 * 8, hipMemcpyDeviceToDevice, st_));
  k::gemm_rm(st_, rn * nb_, n1 * r2, r1, Cn.get(), r1, false, X_[d + 1].get(), (long)n1 * r2, false, T2.get(),
             (long)n1 * r2);
  {
    const int dims[4] = {rn, nb_, n1, r2};
    const int perm[4] = {1, 0, 2, 3};
    k::permute4(st_, T2.get(), dims, perm, Xd1.get());
  }
  // residual core update
  if (kick_ > 0) {
    const int z0 = rho_[d], z1 = rho_[d + 1];
    DBuf Zm(ctx_, (long)nb_ * z0 * n * z1);
    const int dims[4] = {nb_, z0, n, z1};
    const int perm[4] = {1, 2, 0, 3};
    k::permute4(st_, zc.get(), dims, perm, Zm.get());
    DBuf Qn;
    int qz = 0;
    orthonormal_columns(Zm.get(), z0 * n, nb_ * z1, std::min(kick_, z0 * n), Qn, qz, 1e-14);
    if (qz == 0) {
      DBuf Rn = random_buf((size_t)z0 * n * kick_, 1.0);
      orthonormal_columns(Rn.get(), z0 * n, kick_, std::min(kick_, z0 * n), Qn, qz, 1e-14);
    }
    Z_[d] = std::move(Qn);
    rho_[d + 1] = qz;
  }
  IGA_HIP(hipStreamSynchronize(st_));
  t_svd_.end(sid);
  X_[d] = std::move(Xn);
  X_[d + 1] = std::move(Xd1);
  r_[d + 1] = rn;
  ell_ = d + 1;
  update_left(d);
}

void Amen::move_left(int d) {
  g_phase = "move_left";
  const int r0 = r_[d], r1 = r_[d + 1], n = n_[d];
  const int m = n * r1;
  int sid = t_svd_.begin();
  DBuf zc, rz;
  if (kick_ > 0) {
    zc.reset(ctx_, (long)nb_ * rho_[d] * n * rho_[d + 1]);
    residual_proj(d, FZ, FZ, zc.get());
    rz.reset(ctx_, (long)nb_ * rho_[d] * n * r1);
    residual_proj(d, FZ, FX, rz.get());
  }
  // SVD of F^T, F = (nb r0) x (n r1)
  Svd s;
  svd(ctx_, X_[d].get(), m, nb_ * r0, m, /*trans=*/true, s);
  const int K3 = nb_ * r0;
  const int rmax = std::min(o_.r_max, std::min(m, K3));
  int rt = 1;
  if (s.sigma[0] > 0) {
    int nz = 0;
    for (double v : s.sigma) nz += v > 1e-14 * s.sigma[0];
    auto recon = [&](int kk, double* out) {
      // F_k = V_k B_k^T: (nb r0) x (n r1) in the natural [l][a][j][b] layout
      k::gemm_rm(st_, K3, m, kk, s.V.get(), s.p, false, s.B.get(), s.p, true, out, m);
    };
    // the search's local matvecs are timed as local matvecs, not as truncation
    t_svd_.end(sid);
    rt = residual_rank(d, 1, std::min(rmax, std::max(nz, 1)), s.sigma, recon);
    sid = t_svd_.begin();
  }
  static thread_local char ph[200];
  std::snprintf(ph, sizeof ph, "move_left d=%d r0=%d r1=%d m=%d K3=%d rt=%d rho=%d,%d rp=%d", d, r0, r1, m, K3, rt, rho_[d], rho_[d + 1], r_[d - 1]);
  g_phase = ph;
  std::vector<int> idx(rt);
  std::vector<double> inv(rt), sg(rt);
  for (int j = 0; j < rt; ++j) {
    idx[j] = j;
    inv[j] = s.sigma[j] > 0 ? 1.0 / s.sigma[j] : 0.0;
    sg[j] = s.sigma[j];
  }
  IBuf didx(ctx_, rt);
  DBuf dinv(ctx_, rt), dsg(ctx_, rt);
  IGA_HIP(hipMemcpyAsync(didx.get(), idx.data(), rt * sizeof(int), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipMemcpyAsync(dinv.get(), inv.data(), rt * sizeof(double), hipMemcpyHostToDevice, st_));
  IGA_HIP(hipMemcpyAsync(dsg.get(), sg.data(), rt * sizeof(double), hipMemcpyHostToDevice, st_));
  DBuf U(ctx_, (size_t)m * rt);  // (n r1) x rt
  k::gather_cols(st_, m, K3, rt, s.B.get(), s.p, didx.get(), dinv.get(), U.get(), rt);
  DBuf C(ctx_, (size_t)K3 * rt);  // (nb r0) x rt = V Sigma
  k::gather_cols(st_, K3, K3, rt, s.V.get(), s.p, didx.get(), dsg.get(), C.get(), rt);
  DBuf Qz;
  int q = 0;
  if (kick_ > 0 && rt < m) {
    const int kz = nb_ * rho_[d];
    DBuf Rz(ctx_, (size_t)m * kz), T(ctx_, (size_t)rt * kz);
    // rz [nb][z0][n][r1] viewed as (nb z0) x (n r1); transpose to (n r1) x (nb z0)
    k::copy2d(st_, m, kz, rz.get(), 1, m, Rz.get(), kz);
    // T = U^T Rz has few output tiles and a contraction over all m rows: split it
    DBuf W(ctx_, (size_t)64 * rt * kz);
    for (int pass = 0; pass < 2; ++pass) {
      k::gemm_rm(st_, rt, kz, m, U.get(), rt, true, Rz.get(), kz, false, T.get(), kz, 1.0, 0.0, W.get(), W.size());
      k::gemm_rm(st_, m, kz, rt, U.get(), rt, false, T.get(), kz, false, Rz.get(), kz, -1.0, 1.0);
    }
    orthonormal_columns(Rz.get(), m, kz, std::min(kick_, m - rt), Qz, q, 1e-12);
  }
  const int rn = rt + q;
  DBuf Uall(ctx_, (size_t)m * rn), Xn(ctx_, (size_t)rn * m);
  k::copy2d(st_, m, rt, U.get(), rt, 1, Uall.get(), rn);
  if (q > 0) k::copy2d(st_, m, q, Qz.get(), q, 1, Uall.get() + rt, rn);
  k::copy2d(st_, rn, m, Uall.get(), 1, rn, Xn.get(), m);  // X_d = Uall^T: [rn][n][r1]
  // previous core with l: [l][(c j)][rn] = X_{d-1}[(c j)][a] Cn[l][a][rn], Cn = [C, 0]
  const int rp = r_[d - 1], np = n_[d - 1];
  DBuf Cn(ctx_, (size_t)K3 * rn), Xp(ctx_, (size_t)nb_ * rp * np * rn);
  k::fill(st_, (long)K3 * rn, 0.0, Cn.get());
  k::copy2d(st_, K3, rt, C.get(), rt, 1, Cn.get(), rn);
  k::Gemm g;
  g.M = rp * np; g.N = rn; g.K = r0;
  g.A = X_[d - 1].get(); g.sAm = r0; g.sAk = 1;
  g.B = Cn.get(); g.sBk = rn; g.sBn = 1;
  g.C = Xp.get(); g.sCm = rn; g.sCn = 1;
  g.nb1 = nb_; g.sBb1 = (long)r0 * rn; g.sCb1 = (long)rp * np * rn;
  k::gemm(st_, g);
  if (kick_ > 0) {
    const int z0 = rho_[d], z1 = rho_[d + 1];
    const int mz = n * z1;
    DBuf Zm(ctx_, (size_t)mz * nb_ * z0);
    k::copy2d(st_, mz, nb_ * z0, zc.get(), 1, mz, Zm.get(), nb_ * z0);
    DBuf Qn;
    int qz = 0;
    orthonormal_columns(Zm.get(), mz, nb_ * z0, std::min(kick_, mz), Qn, qz, 1e-14);
    if (qz == 0) {
      DBuf Rn = random_buf((size_t)mz * kick_, 1.0);
      orthonormal_columns(Rn.get(), mz, kick_, std::min(kick_, mz), Qn, qz, 1e-14);
    }
    DBuf Zt(ctx_, (size_t)qz * mz);
    k::copy2d(st_, qz, mz, Qn.get(), 1, qz, Zt.get(), mz);
    Z_[d] = std::move(Zt);
    rho_[d] = qz;
  }
  IGA_HIP(hipStreamSynchronize(st_));
  t_svd_.end(sid);
  X_[d] = std::move(Xn);
  X_[d - 1] = std::move(Xp);
  r_[d] = rn;
  ell_ = d - 1;
  update_right(d);
}

// Bring a given initial guess to the layout the sweep starts from: l in core 0,
// cores 1 and 2 right-orthonormal.
void Amen::move_ell_to_first() {
  const int saved_kick = kick_;
  kick_ = 0;
  const double saved_tol = tol_;
  tol_ = 1e-14;
  const int saved_rmax = o_.r_max;
  o_.r_max = 1 << 20;
  // plain right-orthonormalisation of cores after l, then l-moves to the left
  for (int d = 2; d > ell_; --d) right_orth_plain(X_, r_, d, d - 1 == ell_);
  while (ell_ > 0) {
    const int d = ell_;
    const int r0 = r_[d], r1 = r_[d + 1], n = n_[d];
    const int m = n * r1;
    Svd s;
    svd(ctx_, X_[d].get(), m, nb_ * r0, m, true, s);
    int rt = trunc_rank(s.sigma, 1e-14 * s.sigma[0], m);
    std::vector<int> idx(rt);
    std::vector<double> inv(rt), sg(rt);
    for (int j = 0; j < rt; ++j) {
      idx[j] = j;
      inv[j] = s.sigma[j] > 0 ? 1.0 / s.sigma[j] : 0.0;
      sg[j] = s.sigma[j];
    }
    IBuf didx(ctx_, rt);
    DBuf dinv(ctx_, rt), dsg(ctx_, rt), U(ctx_, (size_t)m * rt), C(ctx_, (size_t)nb_ * r0 * rt),
        Xn(ctx_, (size_t)rt * m);
    IGA_HIP(hipMemcpyAsync(didx.get(), idx.data(), rt * sizeof(int), hipMemcpyHostToDevice, st_));
    IGA_HIP(hipMemcpyAsync(dinv.get(), inv.data(), rt * sizeof(double), hipMemcpyHostToDevice, st_));
    IGA_HIP(hipMemcpyAsync(dsg.get(), sg.data(), rt * sizeof(double), hipMemcpyHostToDevice, st_));
    k::gather_cols(st_, m, nb_ * r0, rt, s.B.get(), s.p, didx.get(), dinv.get(), U.get(), rt);
    k::gather_cols(st_, nb_ * r0, nb_ * r0, rt, s.V.get(), s.p, didx.get(), dsg.get(), C.get(), rt);
    k::copy2d(st_, rt, m, U.get(), 1, rt, Xn.get(), m);
    const int rp = r_[d - 1], np = n_[d - 1];
    DBuf Xp(ctx_, (size_t)nb_ * rp * np * rt);
    k::Gemm g;
    g.M = rp * np; g.N = rt; g.K = r0;
    g.A = X_[d - 1].get(); g.sAm = r0; g.sAk = 1;
    g.B = C.get(); g.sBk = rt; g.sBn = 1;
    g.C = Xp.get(); g.sCm = rt; g.sCn = 1;
    g.nb1 = nb_; g.sBb1 = (long)r0 * rt; g.sCb1 = (long)rp * np * rt;
    k::gemm(st_, g);
    IGA_HIP(hipStreamSynchronize(st_));
    X_[d] = std::move(Xn);
    X_[d - 1] = std::move(Xp);
    r_[d] = rt;
    ell_ = d - 1;
  }
  kick_ = saved_kick;
  tol_ = saved_tol;
  o_.r_max = saved_rmax;
}

int Amen::run(const iga_btt* x0, iga_btt** sol, iga_amen_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  kick_ = o_.kick_rank < 0 ? 0 : o_.kick_rank;
  require(kkt_->Kref != nullptr, IGA_EINVAL,
          "amen_solve needs operators from iga_assemble_factors (preconditioner data missing)");
  // initial guess, l in core 0, cores 1, 2 right-orthonormal
  if (x0) {
    for (int d = 0; d < 4; ++d) r_[d] = x0->r[d];
    ell_ = x0->ell;
    for (int d = 0; d < 3; ++d) {
      const size_t sz = (size_t)(d == ell_ ? nb_ : 1) * core_size(d);
      X_[d].reset(ctx_, sz);
      IGA_HIP(hipMemcpyAsync(X_[d].get(), x0->core[d].get(), sz * 8, hipMemcpyDeviceToDevice, st_));
    }
    // to the scaled unknowns: u -> sqrt(beta) u, lambda -> lambda / sqrt(beta)
    const long e = ntb_ * core_size(ell_);
    k::scale(st_, e, g_, X_[ell_].get() + e);
    k::scale(st_, e, 1.0 / g_, X_[ell_].get() + 2 * e);
    move_ell_to_first();
  } else {
    const int ri = o_.init_rank;
    r_[1] = std::min(ri, n_[0]);
    r_[2] = std::min(ri, n_[2]);
    ell_ = 0;
    X_[0] = random_buf((size_t)nb_ * core_size(0), 1.0);
    X_[1] = random_buf((size_t)core_size(1), 1.0);
    X_[2] = random_buf((size_t)core_size(2), 1.0);
    right_orth_plain(X_, r_, 2, false);
    right_orth_plain(X_, r_, 1, true);
  }
  if (kick_ > 0) {
    rho_[1] = std::min(kick_, n_[0]);
    rho_[2] = std::min(kick_, n_[2]);
    for (int d = 0; d < 3; ++d) Z_[d] = random_buf((size_t)rho_[d] * n_[d] * rho_[d + 1], 1.0);
    right_orth_plain(Z_, rho_, 2, false);
    right_orth_plain(Z_, rho_, 1, false);
  }
  init_interfaces();

  bool converged = false;
  int half = 0;
  double last_max = 0;
  for (half = 0; half < o_.nswp && !converged; ++half) {
    const bool fwd = (half % 2) == 0;
    max_res_ = 0;
    for (int s = 0; s < 3; ++s) {
      const int d = fwd ? s : 2 - s;
      const double res = solve_local(d);
      max_res_ = std::isnan(res) ? res : std::max(max_res_, res);
      if (fwd && d < 2) move_right(d);
      if (!fwd && d > 0) move_left(d);
    }
    // no progress over the previous half-sweep: the truncations gave back what the solves
    // gained (a rank cut that the neighbouring core's system does not tolerate), so later
    // truncations keep more of the spectrum
    if (half > 0 && max_res_ > tol_ && !(max_res_ < last_max)) trunc_scale_ = std::max(0.1 * trunc_scale_, 1e-3);
    last_max = max_res_;
    if (half < IGA_MAX_HISTORY) {
      hist_res_[half] = max_res_;
      hist_r_[half][0] = r_[1];
      hist_r_[half][1] = r_[2];
      long long st = 0;
      for (int d = 0; d < 3; ++d) st += (long long)(d == ell_ ? nb_ : 1) * core_size(d);
      hist_st_[half] = st;
    }
    if (o_.verbose >= 2) {
      std::fprintf(stderr, "[amen] half-sweep %d ranks %d %d ell %d\n", half + 1, r_[1], r_[2], ell_);
      // exact global residual of the current iterate (diagnostics only)
      iga_btt tmpx;
      tmpx.ctx = ctx_;
      tmpx.ell = ell_;
      tmpx.nblk = nb_;
      for (int d = 0; d < 3; ++d) tmpx.n[d] = n_[d];
      for (int d = 0; d < 4; ++d) tmpx.r[d] = r_[d];
      for (int d = 0; d < 3; ++d) {
        const size_t sz = (size_t)(d == ell_ ? nb_ : 1) * core_size(d);
        tmpx.core[d].reset(ctx_, sz);
        IGA_HIP(hipMemcpyAsync(tmpx.core[d].get(), X_[d].get(), sz * 8, hipMemcpyDeviceToDevice, st_));
      }
      const long e = ntb_ * core_size(ell_);
      k::scale(st_, e, 1.0 / g_, tmpx.core[ell_].get() + e);
      k::scale(st_, e, g_, tmpx.core[ell_].get() + 2 * e);
      const double gr = kkt_residual_impl(ctx_, kkt_, Y_, &tmpx);
      std::fprintf(stderr, "[amen] half-sweep %d global residual %.3e\n", half + 1, gr);
    }
    if (o_.verbose)
      std::fprintf(stderr, "[amen] half-sweep %d max local residual %.3e ranks %d %d matvecs %lld\n", half + 1,
                   max_res_, r_[1], r_[2], n_mv_);
    converged = max_res_ <= tol_;
  }
  // back to the plain unknowns
  {
    const long e = ntb_ * core_size(ell_);
    k::scale(st_, e, 1.0 / g_, X_[ell_].get() + e);
    k::scale(st_, e, g_, X_[ell_].get() + 2 * e);
  }
  std::unique_ptr<iga_btt> out(new iga_btt());
  out->ctx = ctx_;
  out->ell = ell_;
  out->nblk = nb_;
  for (int d = 0; d < 3; ++d) out->n[d] = n_[d];
  for (int d = 0; d < 4; ++d) out->r[d] = r_[d];
  for (int d = 0; d < 3; ++d) out->core[d] = std::move(X_[d]);
  IGA_HIP(hipStreamSynchronize(st_));
  const auto t1 = std::chrono::steady_clock::now();
  if (stats) {
    std::memset(stats, 0, sizeof(*stats));
    stats->half_sweeps = half;
    stats->converged = converged ? 1 : 0;
    stats->max_local_residual = last_max;
    stats->ranks[0] = r_[1];
    stats->ranks[1] = r_[2];
    stats->local_solves = n_solves_;
    stats->local_iterations = n_iters_;
    stats->local_matvecs = n_mv_;
    stats->local_matvec_flops = flops_;
    stats->t_total = std::chrono::duration<double>(t1 - t0).count();
    stats->t_local_matvec = t_mv_.total();
    stats->t_precond = t_pc_.total();
    stats->t_krylov_other = t_kr_.total();
    stats->t_interfaces = t_if_.total();
    stats->t_svd = t_svd_.total();
    stats->local_matvecs_fp32 = n_mv32_;
    stats->local_matvec_flops_fp32 = flops32_;
    stats->t_local_matvec_fp32 = t_mv32_.total();
    stats->refinements = n_refine_;
    for (int h = 0; h < std::min(half, (int)IGA_MAX_HISTORY); ++h) {
      stats->history_max_local_residual[h] = hist_res_[h];
      stats->history_ranks[h][0] = hist_r_[h][0];
      stats->history_ranks[h][1] = hist_r_[h][1];
      stats->history_storage[h] = hist_st_[h];
    }
    const auto t2 = std::chrono::steady_clock::now();
    stats->residual = kkt_residual_impl(ctx_, kkt_, Y_, out.get());
    stats->t_residual = std::chrono::duration<double>(std::chrono::steady_clock::now() - t2).count();
  }
  *sol = out.release();
  if (converged) return IGA_OK;
  // not converged: IGA_ERANK when a solution rank sits at the cap (r_max plus the enrichment)
  bool capped = false;
  for (int d = 1; d < 3; ++d) capped = capped || r_[d] >= o_.r_max;
  return capped ? IGA_ERANK : IGA_ENOCONV;
}

}  // namespace

int amen_impl(iga_ctx* ctx, const iga_kkt* kkt, const iga_tt* yhat, double tol, const iga_amen_opts* opts,
              const iga_btt* x0, iga_btt** sol, iga_amen_stats* stats) {
  iga_amen_opts o = {};
  if (opts) o = *opts;
  if (o.nswp <= 0) o.nswp = 20;
  if (o.r_max <= 0) o.r_max = 256;
  if (o.kick_rank == 0) o.kick_rank = 4;
  if (!(o.local_tol > 0)) o.local_tol = tol / 10.0;
  if (o.local_maxit <= 0) o.local_maxit = 400;
  if (o.local_restart <= 0) o.local_restart = 40;
  if (o.init_rank <= 0) o.init_rank = 2;
  require(o.precision == IGA_FP64 || o.precision == IGA_FP32 || o.precision == IGA_BF16, IGA_EINVAL,
          "amen_solve: bad precision");
  Amen a(ctx, kkt, yhat, tol, o);
  return a.run(x0, sol, stats);
}

}  // namespace iga
