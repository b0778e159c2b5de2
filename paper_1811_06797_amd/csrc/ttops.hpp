// Host-side drivers of the TT operations: operator views, core-wise operator-times-TT
// products, expansion, SVD. (The projected local operator, the interface updates and the
// full-tensor operator apply are in localop.hpp.)
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

// Y[(al a)][i][(be b)] = sum_j A[al][i][j][be] X[a][j][b]  (core of the product A x, eq. M_kron)
void core_product(iga_ctx* ctx, const OpView& A, const double* X, int r0, int r1, double* Y,
                  double alpha, double beta);

// Full tensor of a TT (cores given per direction, rank r[0..3]) into out [n0][n1][n2].
void tt_expand(iga_ctx* ctx, const int n[3], const int r[4], const double* const core[3], double* out);
void btt_expand(iga_ctx* ctx, const iga_btt* x, double* out);

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
// The same outputs where only the product U Sigma V^T = B V^T matters (the TT-SVD of a tensor):
// with more than 32 columns (at most 1024) the Jacobi iteration runs on R^T of a column-pivoted
// Cholesky QR (the pivoting is what makes the iteration converge in few sweeps on smooth
// data); the columns of B = A V carry the QR's absolute error u ||A||, so B / sigma is not
// orthonormal to working accuracy for small sigma.
void svd_product(iga_ctx* ctx, const double* A, int m, int k, long lda, bool trans, Svd& out);
// Smallest r with ||sigma[r:]|| <= abs_tol, capped to [rmin, rmax] (rmax <= 0: no cap).
int trunc_rank(const std::vector<double>& sigma, double abs_tol, int rmax, int rmin = 1);

// Generalised symmetric-definite eigenproblem: V^T B V = I, V^T A V = diag(lam). V, lam on device.
void gen_eig(iga_ctx* ctx, int k, const double* A, const double* B, double* V, double* lam);

// Sum of squares of a device vector (deterministic), returned on the host (synchronises).
double norm2_host(iga_ctx* ctx, long n, const double* x);
double dot_host(iga_ctx* ctx, long n, const double* x, const double* y);

}  // namespace iga
