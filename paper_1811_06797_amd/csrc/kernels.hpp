// Launchers of the HIP kernels (gfx950). All are asynchronous on the given stream.
#pragma once

#include <hip/hip_runtime.h>

namespace iga {
namespace k {

// C[b][m][n] = alpha * sum_{ko<Kout, k<K} A[b][m][ko,k] B[b][ko,k][n] + beta * C[b][m][n]
// with arbitrary element strides; batch index b = b1 * nb2 + b2.
struct Gemm {
  int M = 0, N = 0, K = 0, Kout = 1;
  const double* A = nullptr;
  long sAm = 0, sAk = 0, sAko = 0;
  const double* B = nullptr;
  long sBk = 0, sBn = 0, sBko = 0;
  double* C = nullptr;
  long sCm = 0, sCn = 0;
  int nb1 = 1, nb2 = 1;
  long sAb1 = 0, sAb2 = 0, sBb1 = 0, sBb2 = 0, sCb1 = 0, sCb2 = 0;
  double alpha = 1.0, beta = 0.0;
  // tiles of consecutive batch entries run together (set when the batch index is the row of a
  // banded product whose B operand windows overlap from row to row)
  bool batch_inner = false;
};
// work (nullable, work_len doubles): split-K partials, so that a product with few output tiles
// and a long contraction spreads over the chip
void gemm(hipStream_t s, const Gemm& g, double* work = nullptr, size_t work_len = 0);

// FP64 MFMA GEMM with two-level index maps (k_gemm.hip): every index x of m, n, k is split
// as x = x1 * X2 + x2 (X2 = inner extent; the default 1 << 30 makes it single-level with
// stride s*2) and addressed as x1 * s*1 + x2 * s*2 per operand; batch b = b1 * nb2 + b2.
struct Gemm2 {
  int M = 0, N = 0, K = 0;
  int M2 = 1 << 30, N2 = 1 << 30, K2 = 1 << 30;
  const double* A = nullptr;
  long sAm1 = 0, sAm2 = 0, sAk1 = 0, sAk2 = 0;
  const double* B = nullptr;
  long sBk1 = 0, sBk2 = 0, sBn1 = 0, sBn2 = 0;
  double* C = nullptr;
  long sCm1 = 0, sCm2 = 0, sCn1 = 0, sCn2 = 0;
  int nb1 = 1, nb2 = 1;
  long sAb1 = 0, sAb2 = 0, sBb1 = 0, sBb2 = 0, sCb1 = 0, sCb2 = 0;
  double alpha = 1.0, beta = 0.0;
  // tiles of consecutive batch entries run together (set when the batch index is the row of a
  // banded product whose B operand windows overlap from row to row)
  bool batch_inner = false;
  // tile variant (see gemm2_pick); -1: chosen from the shape
  int variant = -1;
};
void gemm2(hipStream_t s, const Gemm2& g);
// Same, with a workspace of work_len doubles that lets short-output, long-K products be split
// along K (partials summed in a fixed order, so results are deterministic).
void gemm2(hipStream_t s, const Gemm2& g, double* work, size_t work_len);
// Grouped form: many independent products with one tile variant in one persistent launch.
// gemm2_prepare validates a product, writes its argument block (gemm2_desc_bytes() bytes)
// to host_desc and returns its tile count for the variant; gemm2_grouped runs ngemm blocks
// copied to device memory, with dev_prefix[i] = sum of the tile counts before product i
// (ngemm + 1 entries, the last = total). Every variant accumulates K in the same order, so
// the result does not depend on the variant.
int gemm2_variants();
int gemm2_pick(const Gemm2& g);  // the variant the single-product form uses
size_t gemm2_desc_bytes();
long gemm2_prepare(const Gemm2& g, int variant, void* host_desc);
void gemm2_grouped(hipStream_t s, int variant, const void* dev_desc, const int* dev_prefix, int ngemm, long total);

// The same product in FP32 on the matrix cores (FP32 inputs, FP32 accumulation), for the
// mixed-precision form (k_gemm32.hip); identical index maps.
struct Gemm2F {
  int M = 0, N = 0, K = 0;
  int M2 = 1 << 30, N2 = 1 << 30, K2 = 1 << 30;
  const float* A = nullptr;
  long sAm1 = 0, sAm2 = 0, sAk1 = 0, sAk2 = 0;
  const float* B = nullptr;
  long sBk1 = 0, sBk2 = 0, sBn1 = 0, sBn2 = 0;
  float* C = nullptr;
  long sCm1 = 0, sCm2 = 0, sCn1 = 0, sCn2 = 0;
  int nb1 = 1, nb2 = 1;
  long sAb1 = 0, sAb2 = 0, sBb1 = 0, sBb2 = 0, sCb1 = 0, sCb2 = 0;
  float alpha = 1.0f, beta = 0.0f;
  bool batch_inner = false;  // as in Gemm2
  int variant = -1;          // tile variant (see gemm2f_pick); -1: chosen from the shape
};
void gemm2_f32(hipStream_t s, const Gemm2F& g, float* work, size_t work_len);
// same products with the operands rounded to bfloat16 and BF16 matrix-core products (FP32 accumulation)
void gemm2_bf16(hipStream_t s, const Gemm2F& g, float* work, size_t work_len);
// grouped FP32 form, as gemm2_prepare / gemm2_grouped
int gemm2f_pick(const Gemm2F& g);
size_t gemm2f_desc_bytes();
long gemm2f_prepare(const Gemm2F& g, int variant, void* host_desc);
void gemm2f_grouped(hipStream_t s, int variant, const void* dev_desc, const int* dev_prefix, int ngemm, long total);

// Row-major convenience: C (MxN, ldc) = alpha op(A) op(B) + beta C, op = transpose if t*.
void gemm_rm(hipStream_t s, int M, int N, int K, const double* A, long lda, bool tA,
             const double* B, long ldb, bool tB, double* C, long ldc, double alpha = 1.0,
             double beta = 0.0, double* work = nullptr, size_t work_len = 0);


// y = a x + b y (n doubles)
void axpby(hipStream_t s, long n, double a, const double* x, double b, double* y);
void fill(hipStream_t s, long n, double v, double* y);
void fill_f32(hipStream_t s, long n, float v, float* y);
void scale(hipStream_t s, long n, double a, double* y);
void to_f32(hipStream_t s, long n, const double* x, float* y);
void to_f64(hipStream_t s, long n, const float* x, double* y);
// out[o0][o1][o2][o3] = in[...] with out dims = in dims permuted: out axis k is in axis perm[k]
void permute4(hipStream_t s, const double* in, const int dims[4], const int perm[4], double* out);

// Deterministic reductions into device scalars (two passes, fixed order).
// partial must hold at least reduce_partials() doubles.
int reduce_partials();
void dot(hipStream_t s, long n, const double* x, const double* y, double* partial, double* out);
// h[j] = sum_i V[j*ldv + i] w[i], j < k (k <= 64); partial holds reduce_partials()*64 doubles
void multidot(hipStream_t s, long n, int k, const double* V, long ldv, const double* w,
              double* partial, double* h);
// w[i] += sum_j coef[j] V[j*ldv + i]   (coef on device, k <= 64)
void multiaxpy(hipStream_t s, long n, int k, const double* V, long ldv, const double* coef,
               double sign, double* w);
// column norms of a row-major m x k matrix: out[j] = sqrt(sum_i A[i][j]^2)
void colnorms(hipStream_t s, int m, int k, const double* A, long lda, double* out);

// KKT block combination of the five operator applications of a local matvec
// (zM = M x0, M x1, M x2 and zK = K x0, K x2; each [e]):
//   y0 = zM0 + k02 zK(x2), y1 = m11 zM1 + m12 zM2, y2 = k20 zK(x0) + m21 zM1.
struct KktCoef {
  double k02 = 1, m11 = 0, m12 = -1, k20 = 1, m21 = -1;
};
void kkt_combine(hipStream_t s, long e, const KktCoef& c, const double* zM, const double* zK, double* y);
void kkt_combine_f32(hipStream_t s, long e, const KktCoef& c, const float* zM, const float* zK, float* y);
// Banded stage of a rank-1 operator core: y[i][c] = sum_{o < b} A[i][o] x[(i + o) ldx + c],
// i < n, c < ncols, y rows of ncols (FP64 and FP32 forms).
void band_rank1(hipStream_t s, int n, int b, long ncols, const double* A, const double* x, long ldx, double* y);
void band_rank1_f32(hipStream_t s, int n, int b, long ncols, const float* A, const float* x, long ldx, float* y);
// Banded stage of a core with R1 <= 16 right ranks: y[i][g][c] = sum_{o < b, d < R0}
// A[i][o][d][g] x[(i + o) ldx + d ldd + c], A re-laid [n][b][R0][R1], y [n][R1][ncols].
void band_small(hipStream_t s, int n, int b, int R0, int R1, long ncols, const double* A, const double* x, long ldx,
                long ldd, double* y);
void band_small_f32(hipStream_t s, int n, int b, int R0, int R1, long ncols, const float* A, const float* x, long ldx,
                    long ldd, float* y);
// General block combination: y[o][.] = sum_{t in [toff[o], toff[o+1])} coef[t] z[src[t]][.]
// for o < nblk, blocks of e elements (device tables).
void combine_blocks(hipStream_t s, long e, int nblk, const int* toff, const int* src, const double* coef,
                    const double* z, double* y);
void combine_blocks_f32(hipStream_t s, long e, int nblk, const int* toff, const int* src, const double* coef,
                        const float* z, float* y);
// Per-mode solve of the time-dependent reference KKT system (nt steps of length tau) in
// place on v [3][nt][r0 n r1]; work: nt r0 n r1 doubles.
void fd_solve_time(hipStream_t s, int r0, int n, int r1, int nt, const double* lamL, const double* lamN,
                   const double* lamR, double beta, double tau, double* v, double* work);
// Grouped helpers of the batched local operator (one launch for all items; blockIdx.y = item).
struct Segment {
  long off, len;  // base[off .. off + len) = 0
};
void fill_segments(hipStream_t s, int nseg, long maxlen, const Segment* dev_seg, double* base);
void fill_segments_f32(hipStream_t s, int nseg, long maxlen, const Segment* dev_seg, float* base);
struct CombineItem {
  long z_off;  // zM at zbase + z_off ([3][e]), zK right after it ([2][e])
  long e;
  void* y;     // [3][e] output
  KktCoef coef;
};
void combine_grouped(hipStream_t s, int nitem, long maxe, const CombineItem* dev_items, const double* zbase);
void combine_grouped_f32(hipStream_t s, int nitem, long maxe, const CombineItem* dev_items, const float* zbase);
struct ConvSegment {
  const void* src;
  void* dst;
  long len;
};
// dst = (float) src (to_f32) or (double) src for every segment
void convert_segments(hipStream_t s, int nseg, long maxlen, const ConvSegment* dev_seg, bool to_f32);

// y[l][.] *= scale[l] for the three components of a [3][e] vector
void scale3(hipStream_t s, long e, double s0, double s1, double s2, double* y);
// Fast-diagonalisation solve of the per-mode 3x3 KKT blocks [[1,0,k],[0,c,-1],[k,-1,0]],
// k = g (lamL[a] + lamN[i] + lamR[b]), in place on v [3][r0][n][r1].
void fd_solve(hipStream_t s, int r0, int n, int r1, const double* lamL, const double* lamN,
              const double* lamR, double c, double g, double* v);
// H <- (H + H^T) / 2 for nmat k x k matrices stored stride apart
void symmetrize(hipStream_t s, int nmat, int k, double* H, long stride);
// Y[(al a)][i][(be b)] = alpha sum_o A[al][i][o][be] X[a][i+o-p][b] + beta Y (banded A [R0][n][2p+1][R1])
void core_product(hipStream_t s, int R0, int R1, int n, int p, const double* A, int r0, int r1,
                  const double* X, double* Y, double alpha, double beta);
// out[i][j] = in[i*si + j*sj], i < m, j < k (out row-major, ldo)
void copy2d(hipStream_t s, int m, int k, const double* in, long si, long sj, double* out, long ldo);
// out[j] = 1/sqrt(H[j][j]) (0 if H[j][j] <= 0)
void diag_invsqrt(hipStream_t s, int k, const double* H, double* out);
// out[j] = H[j][j]
void diag_get(hipStream_t s, int k, const double* H, double* out);
// out[j] = 1/sqrt(v[j]) (0 if v[j] <= 0)
void vec_invsqrt(hipStream_t s, int k, const double* v, double* out);
// A[i][j] *= sc[i] (m x k, row-major, leading dimension lda)
void scale_rows(hipStream_t s, int m, int k, const double* sc, double* A, long lda);
// out[j] = sum_i A[i][j] B[i][j], j < k (row-major, leading dimensions lda, ldb)
void coldots(hipStream_t s, int m, int k, const double* A, long lda, const double* B, long ldb, double* out);

// Reduced-cost gradient kernels (k_adjoint.hip). f: 9 fields at npts points, fstride apart
// (e = y - yhat, u, lambda, d_0..2 lambda, d_0..2 y); P: 10 outputs, pstride apart:
// P_w = e^2/2 + beta u^2/2 - lambda u, then P_kl = (d_l lambda)(d_k y) at 1 + 3k + l.
void adjoint_pointwise(hipStream_t s, long npts, const double* f, long fstride, double beta, double* P,
                       long pstride);
// T[3a+b][g] = H_w(g) d omega/d J_ab + sum_kl H_kl(g) d q_kl/d J_ab on the grid np (tables as
// for geometry_weights); H: [10][G] in the order of P.
void geometry_adjoint(hipStream_t s, const int np[3], const int ncp[3], const double* const Bv[3],
                      const double* const Bd[3], const double* ctrl, const double* H, double* T);

// Symmetric Jacobi eigen-decomposition, one workgroup per matrix, nmat matrices of size k
// (k <= 512): H (in: symmetric, out: diagonal holds the eigenvalues), WT (out: row i is
// the i-th eigenvector, H_in = WT^T diag WT). Rotations are skipped when
// |h_pq| <= max(tol * sqrt(|h_pp h_qq|), 1e-30 trace). sweeps_out[mat] (nullable) counts
// the sweeps that rotated anything (0: H was already diagonal to that tolerance).
void jacobi_eig(hipStream_t s, int nmat, int k, double* H, long strideH, double* WT, long strideW,
                double tol, int max_sweeps, int* sweeps_out);
// One round of the one-sided block Jacobi SVD on B (m x kp, kp = nb * osbj_block(), nb even)
// with V (kv x kp) accumulated; flags[nb/2] receive 1 for pairs that rotated.
// work holds osbj_work_len(m, kv, nb) doubles (partial Gram matrices and pair rotations);
// inner: cyclic sweeps on each pair's Gram matrix per round (ended early once converged);
// abs2 > 0: rotations that would move the larger column by at most sqrt(abs2) are skipped.
void osbj_round(hipStream_t s, double* B, int m, long ldb, double* V, int kv, long ldv, int nb, int round,
                double tol, double floor_col, int* flags, double* work, size_t work_len, int inner = 1,
                double abs2 = 0.0);
size_t osbj_work_len(int m, int kv, int nb);
int osbj_block();
// largest k for which jacobi_eig keeps the matrix in LDS
int jacobi_lds_max();
void transpose_square(hipStream_t s, int nmat, int k, const double* in, long sin, double* out,
                      long sout);
// Cholesky of one diagonal block (jb <= chol_block_size()) of a symmetric matrix whose earlier
// columns are eliminated: lower factor into L (ldl), its inverse into Linv (chol_block_size()^2,
// row-major); a non-positive pivot gives a zero column and adds one to *bad (device int).
int chol_block_size();
void chol_block(hipStream_t s, int jb, const double* G, long ldg, double* L, long ldl, double* Linv, int* bad);
// Cholesky with diagonal pivoting of a symmetric PSD k x k G (k <= pchol_max(), row-major, full
// storage, destroyed; one workgroup): lower L in G with P^T G P = L L^T, perm[j] = original
// index of pivot j (device), a non-positive pivot gives a zero column and adds one to *bad.
int pchol_max();
void pivoted_cholesky(hipStream_t s, int k, double* G, int* perm, int* bad);
// Column-pivoted Householder QR (k_qrcp.hip). W: column c at W + c * ldw (m entries, reflected
// in place); qrcp_init sets nrm2[k] to the squared column norms. Step j (launched for
// j = 0, 1, ... < rmax in order) reads the squared remaining norms from nin and writes them to
// nout (swap the two arrays between steps; -1 marks a chosen column), writes reflector j into
// row j of V (rmax x m) and beta[j], row j of R (rmax x k, original column indices, zero on
// entry) and pivots[j]; when the remaining squared Frobenius norm is <= thr2 it stops the
// factorisation instead (ctrl[0] = 1, ctrl[2] = j; ctrl: 3 ints, zero on entry) and later
// steps do nothing. qrhh_apply: Y <- H_0 ... H_{rc-1} Y for ncol columns (column c at
// Y + c * m).
void qrcp_init(hipStream_t s, int m, int k, const double* W, long ldw, double* nrm2);
void qrhh_step(hipStream_t s, int m, int k, int j, double* W, long ldw, const double* nin, double* nout,
               double* V, double* beta, double* R, int* pivots, int* ctrl, double thr2);
void qrhh_apply(hipStream_t s, int m, int rc, const double* V, const double* beta, int ncol, double* Y);
// Inverses of the chol_block_size() diagonal blocks of a lower-triangular k x k L, into Linv.
void trinv_blocks(hipStream_t s, int k, const double* L, long ldl, double* Linv);
// out[i][:] = in[idx[i]][:], i < m, k columns
void gather_rows(hipStream_t s, int m, int k, const double* in, long ldi, const int* idx, double* out, long ldo);
// A[i][i] += v, i < k
void add_diag(hipStream_t s, int k, double* A, long lda, double v);
// out[i][j] = in[i][idx[j]] * (scale ? scale[j] : 1), i < m, j < kout
void gather_cols(hipStream_t s, int m, int kin, int kout, const double* in, long ldi, const int* idx,
                 const double* scale, double* out, long ldo);
// src [na][inner][nb] -> dst [R0dst][inner][R1dst] at rank offsets (a0, b0)
void place_block(hipStream_t s, int na, int nb, int inner, const double* src, double* dst, int R1dst,
                 int a0, int b0);

// Inverse of a dense k x k matrix (row-major) by Gauss-Jordan with partial pivoting,
// one workgroup; work holds 2*k*k doubles. Sets *singular if a pivot is exactly zero.
void invert(hipStream_t s, int k, const double* A, double* Ainv, double* work, int* singular);

// ---- assembly ----
// Values (deriv=0) or first derivatives (deriv=1) of all B-splines of an open knot
// vector at the given points: out[np][nknots-deg-1].
void bspline_tabulate(hipStream_t s, const double* knots, int nknots, int deg, const double* pts,
                      int np, int deriv, double* out);
// omega, q11, q12, q13, q22, q23, q33 on a tensor grid from the geometry:
// Bv_d/Bd_d: basis values/derivatives [np_d][ncp_d]; ctrl [3][ncp0][ncp1][ncp2];
// out [7][np0][np1][np2]; *bad counts points with det <= 0.
void geometry_weights(hipStream_t s, const int np[3], const int ncp[3], const double* const Bv[3],
                      const double* const Bd[3], const double* ctrl, double* out, int* bad);
// Univariate factor quadrature (eqs. massMatrix1D and the D^2 stiffness factors):
//   out[s][i][o] = sum_q w[q] Bi(q, i+1) Bj(q, j+1) E[s][q], j = i + o - p, interior i, j only,
// Bi/Bj: dense tables [Q][N] of values or derivatives, Q = nel*nq points (element-major).
void factor_quadrature(hipStream_t s, int S, int n, int p, int nel, int nq, const double* Bi,
                       const double* Bj, const double* w, const double* E, double* out);

}  // namespace k
}  // namespace iga

struct iga_ctx;
namespace iga {
namespace k {
// Measured device ceilings (k_probe.hip): out[0..3] TFLOP/s of the FP64 4x4x4, FP64 16x16x4,
// FP32 16x16x4 and BF16 16x16x32 MFMA instructions; out[4], out[5] GB/s of a copy and a read.
void measure_peaks(iga_ctx* ctx, double* out);
}  // namespace k
}  // namespace iga
