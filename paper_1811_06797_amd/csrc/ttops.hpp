// Host-side drivers of the TT contractions: projected local operator apply,
// interface updates, core-wise operator-times-TT products, expansion, SVD.
#pragma once

#include <vector>

#include "common.hpp"

namespace iga {

// Non-owning view of a banded TT-matrix core with its rank-block structure.
struct OpView {
  int R0 = 0, R1 = 0, n = 0, p = 0;
  const double* A = nullptr;
  const float* Af = nullptr;  // FP32 copy (mixed-precision form), may be null
  const double* Ar = nullptr; // the core re-laid as [n][2p+1][R0][R1] (dense cores), may be null
  const float* Arf = nullptr; // FP32 copy of Ar (mixed-precision form), may be null
  const int* lo_R1 = nullptr;  // for output right rank g: contract left ranks [lo, hi)
  const int* hi_R1 = nullptr;
  const int* lo_R0 = nullptr;  // for output left rank g: contract right ranks [lo, hi)
  const int* hi_R0 = nullptr;
  double flops_dense_factor = 1.0;  // fraction of (R0 x R1) that is nonzero
};
OpView view_of(const iga_ttop* op, int d);

// Per-context scratch buffers (all work is ordered on one stream).
struct Scratch {
  DBuf t1, t2, t3, red;
  FBuf f1, f2, f3, f4;
  IBuf ilo, ihi;
};
Scratch& scratch_of(iga_ctx* ctx);

// y[c][a'][i][b'] = alpha * sum PhiL[al][a'][a] A[al][i][j][be] x[c][a][j][b] PhiR[be][b'][b] + beta*y
// for c < ncol (x columns xcs apart, y columns ycs apart).
// PhiL [R0][ra_out][ra_in], PhiR [R1][rb_out][rb_in], x [ra_in][n][rb_in], y [ra_out][n][rb_out].
void local_apply(iga_ctx* ctx, const OpView& A, const double* PhiL, const double* PhiR, int ra_out,
                 int ra_in, int rb_out, int rb_in, int ncol, const double* x, long xcs, double* y,
                 long ycs, double alpha, double beta);

// Stages 1-2 only: t2[be][c][a'][i][b] into `t2` (size R1*ncol*ra_out*n*rb_in).
void local_stage12(iga_ctx* ctx, const OpView& A, const double* PhiL, int ra_out, int ra_in,
                   int rb_in, int ncol, const double* x, long xcs, double* t2);
// Stage 3 for one column c of a t2 from local_stage12.
void local_stage3(iga_ctx* ctx, const OpView& A, const double* t2, int ncol, int c, const double* PhiR,
                  int ra_out, int rb_out, int rb_in, double* y, double alpha, double beta);

// Phi'[be][b'][b] = sum U[a'][i][b'] Phi[al][a'][a] A[al][i][j][be] V[a][j][b]
void interface_left(iga_ctx* ctx, const OpView& A, const double* Phi, const double* U,
                    const double* V, int ru0, int ru1, int rv0, int rv1, double* out);
// Phi'[al][a'][a] = sum U[a'][i][b'] Phi[be][b'][b] A[al][i][j][be] V[a][j][b]
void interface_right(iga_ctx* ctx, const OpView& A, const double* Phi, const double* U,
                     const double* V, int ru0, int ru1, int rv0, int rv1, double* out);

// Y[(al a)][i][(be b)] = sum_j A[al][i][j][be] X[a][j][b]  (core of the product A x, eq. M_kron)
void core_product(iga_ctx* ctx, const OpView& A, const double* X, int r0, int r1, double* Y,
                  double alpha, double beta);

// Full tensor of a TT (cores given per direction, rank r[0..3]) into out [n0][n1][n2].
void tt_expand(iga_ctx* ctx, const int n[3], const int r[4], const double* const core[3], double* out);
void btt_expand(iga_ctx* ctx, const iga_btt* x, double* out);

// y = A x for a TT-matrix A and a full tensor x [n0][n1][n2], mode by mode (banded):
// y = alpha A x + beta y.
void full_apply(iga_ctx* ctx, const iga_ttop* A, const double* x, double* y, double alpha, double beta);

// y = A x for the KKT operator (exact, ranks (RM+RK) r); y allocated here.
iga_btt* kkt_apply_impl(iga_ctx* ctx, const iga_kkt* kkt, const iga_btt* x);

// Thin SVD of an m x k matrix (row-major, leading dimension lda), or of the transpose of a
// k x m row-major matrix when trans, by the one-sided block Jacobi method on the taller
// orientation: columns are rotated pairwise (in blocks) until mutually orthogonal to
// working precision; then sigma_j = ||b_j||, U = B diag(1/sigma), A = U diag(sigma) V^T.
// p = min(m, k) triplets are returned.
struct Svd {
  int m = 0, k = 0, p = 0;
  DBuf B;  // m x p, = A V = U diag(sigma), columns by decreasing sigma
  DBuf V;  // k x p, right singular vectors in columns, same order
  std::vector<double> sigma;
  int passes = 0;  // Jacobi sweeps
};
void svd(iga_ctx* ctx, const double* A, int m, int k, long lda, bool trans, Svd& out);
// Smallest r with ||sigma[r:]|| <= abs_tol, capped to [rmin, rmax] (rmax <= 0: no cap).
int trunc_rank(const std::vector<double>& sigma, double abs_tol, int rmax, int rmin = 1);

// Generalised symmetric-definite eigenproblem: V^T B V = I, V^T A V = diag(lam). V, lam on device.
void gen_eig(iga_ctx* ctx, int k, const double* A, const double* B, double* V, double* lam);

// Sum of squares of a device vector (deterministic), returned on the host (synchronises).
double norm2_host(iga_ctx* ctx, long n, const double* x);
double dot_host(iga_ctx* ctx, long n, const double* x, const double* y);

}  // namespace iga
