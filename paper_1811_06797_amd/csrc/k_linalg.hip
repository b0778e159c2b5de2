// Small dense linear algebra in one workgroup: cyclic Jacobi eigen-decomposition
// of symmetric matrices, Gauss-Jordan inverse, column gathers and block copies.
#include <algorithm>

#include <mutex>

#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

constexpr int JT = 512;        // threads per Jacobi workgroup
constexpr int LDS_MAX_K = 120;      // H kept in LDS up to this size ((k+1)*k*8 bytes)
constexpr int LDS_BOTH_MAX_K = 96;  // H and the eigenvector rows both in LDS up to this size

// Parallel cyclic Jacobi with round-robin pairing (circle method): in every round the k/2
// disjoint pairs (p, q) are rotated at once, H <- J^T H J, and the eigenvectors are
// accumulated as rows of WT (WT <- J^T WT, i.e. W <- W J). After the rotation parameters of
// the round are known, one pass updates H by 2 x 2 blocks {p_t1, q_t1} x {p_t2, q_t2} (rows
// by rotation t1 and columns by rotation t2 together; the blocks are disjoint and cover H)
// and rows p, q of WT. A rotation is skipped when |h_pq| <= max(tol * sqrt(|h_pp h_qq|),
// 1e-30 trace), or when both h_pp and h_qq are below 1e-28 trace (directions at the
// rounding level of the largest one). A rotated diagonal block is stored exactly (zero
// off-diagonal, closed-form diagonal), so rounding noise in h_pq cannot keep sweeps going.
// MODE 0: H and WT in global memory; 1: H in LDS; 2: H and WT in LDS.
template <int MODE>
__global__ __launch_bounds__(JT) void jacobi_kernel(int k, double* Hs, long sH, double* WTs,
                                                    long sW, double tol, int max_sweeps,
                                                    int* sweeps_out) {
  extern __shared__ double lds[];
  double* Hg = Hs + blockIdx.x * sH;
  double* WTg = WTs + blockIdx.x * sW;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int ld = MODE >= 1 ? k + 1 : k;
  double* H = MODE >= 1 ? lds : Hg;
  double* WT = MODE == 2 ? lds + (size_t)(k + 1) * k : WTg;
  if (MODE >= 1)
    for (int e = tid; e < k * k; e += nt) H[(e / k) * ld + e % k] = Hg[e];
  for (int e = tid; e < k * k; e += nt) WT[e] = (e / k == e % k) ? 1.0 : 0.0;
  __shared__ double cs[JT / 2], sn[JT / 2], dp[JT / 2], dq[JT / 2];
  __shared__ int pp[JT / 2], qq[JT / 2];  // this round's pairs, found once by their rotation's thread
  __shared__ int rotated;
  __shared__ double trace;
  __syncthreads();
  if (tid == 0) {
    double t = 0.0;
    for (int i = 0; i < k; ++i) t += fabs(H[i * ld + i]);
    trace = t;
  }
  __syncthreads();
  const double floor_abs = 1e-30 * trace;
  const double floor_col = 1e-28 * trace;
  const int kk = k + (k & 1);
  const int npair = kk / 2;
  // circle method: position 0 fixed, positions 1..kk-1 rotate
  auto pair_of = [&](int t, int round, int& p, int& q) {
    auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (kk - 1); };
    p = player(t);
    q = player(kk - 1 - t);
    if (p > q) { const int x = p; p = q; q = x; }
  };
  int sweeps = 0;
  for (int sweep = 0; sweep < max_sweeps; ++sweep) {
    if (tid == 0) rotated = 0;
    __syncthreads();
    for (int round = 0; round < kk - 1; ++round) {
      for (int t = tid; t < npair; t += nt) {
        int p, q;
        pair_of(t, round, p, q);
        double c = 1.0, s = 0.0, np = 0.0, nq = 0.0;
        if (q < k) {
          const double app = H[p * ld + p], aqq = H[q * ld + q], apq = H[p * ld + q];
          const double thr = fmax(tol * sqrt(fabs(app * aqq)), floor_abs);
          const bool negligible = fabs(app) <= floor_col && fabs(aqq) <= floor_col;
          if (!negligible && fabs(apq) > thr) {
            const double tau = (aqq - app) / (2.0 * apq);
            const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + tt * tt);
            s = tt * c;
            np = app - tt * apq;
            nq = aqq + tt * apq;
            rotated = 1;
          }
        }
        cs[t] = c; sn[t] = s; dp[t] = np; dq[t] = nq;
        pp[t] = p; qq[t] = q;
      }
      __syncthreads();
      // H by 2 x 2 blocks
      for (int blk = tid; blk < npair * npair; blk += nt) {
        const int t1 = blk / npair, t2 = blk - t1 * npair;
        const double s1 = sn[t1], s2 = sn[t2];
        if (s1 == 0.0 && s2 == 0.0) continue;
        const int p1 = pp[t1], q1 = qq[t1], p2 = pp[t2], q2 = qq[t2];
        if (t1 == t2) {
          H[p1 * ld + p1] = dp[t1];
          H[q1 * ld + q1] = dq[t1];
          H[p1 * ld + q1] = 0.0;
          H[q1 * ld + p1] = 0.0;
          continue;
        }
        const double c1 = cs[t1], c2 = cs[t2];
        const bool hq1 = q1 < k, hq2 = q2 < k;  // q = k is the padding index of odd k (never rotated)
        const double a = H[p1 * ld + p2];
        const double bq = hq2 ? H[p1 * ld + q2] : 0.0;
        const double cp = hq1 ? H[q1 * ld + p2] : 0.0;
        const double d = (hq1 && hq2) ? H[q1 * ld + q2] : 0.0;
        const double a1 = c1 * a - s1 * cp, c1p = s1 * a + c1 * cp;
        const double b1 = c1 * bq - s1 * d, d1 = s1 * bq + c1 * d;
        H[p1 * ld + p2] = c2 * a1 - s2 * b1;
        if (hq2) H[p1 * ld + q2] = s2 * a1 + c2 * b1;
        if (hq1) H[q1 * ld + p2] = c2 * c1p - s2 * d1;
        if (hq1 && hq2) H[q1 * ld + q2] = s2 * c1p + c2 * d1;
      }
      // rows p, q of WT
      for (int e = tid; e < npair * k; e += nt) {
        const int t = e / k, j = e - t * k;
        const double s = sn[t];
        if (s == 0.0) continue;
        const double c = cs[t];
        const int p = pp[t], q = qq[t];
        const double wp = WT[p * k + j], wq = WT[q * k + j];
        WT[p * k + j] = c * wp - s * wq;
        WT[q * k + j] = s * wp + c * wq;
      }
      __syncthreads();
    }
    if (!rotated) break;
    ++sweeps;
    __syncthreads();
  }
  if (MODE >= 1)
    for (int e = tid; e < k * k; e += nt) Hg[e] = H[(e / k) * ld + e % k];
  if (MODE == 2)
    for (int e = tid; e < k * k; e += nt) WTg[e] = WT[e];
  if (tid == 0 && sweeps_out) sweeps_out[blockIdx.x] = sweeps;
}

__global__ void transpose_sq(int k, const double* in, long sin, double* out, long sout) {
  const double* a = in + blockIdx.y * sin;
  double* b = out + blockIdx.y * sout;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)k * k;
       e += (long)gridDim.x * blockDim.x) {
    const int i = e / k, j = e % k;
    b[(long)j * k + i] = a[e];
  }
}

__global__ __launch_bounds__(1024) void gauss_jordan(int k, const double* A, double* Ainv,
                                                     double* work, int* singular) {
  // work: [k][2k] augmented matrix
  const int tid = threadIdx.x, nt = blockDim.x;
  const int w = 2 * k;
  for (int e = tid; e < k * w; e += nt) {
    const int i = e / w, j = e % w;
    work[e] = (j < k) ? A[i * k + j] : ((j - k == i) ? 1.0 : 0.0);
  }
  __shared__ double best[1024];
  __shared__ int besti[1024];
  __shared__ int piv;
  if (tid == 0) *singular = 0;
  __syncthreads();
  for (int c = 0; c < k; ++c) {
    double bv = -1.0;
    int bi = c;
    for (int r = c + tid; r < k; r += nt) {
      const double v = fabs(work[r * w + c]);
      if (v > bv) { bv = v; bi = r; }
    }
    best[tid] = bv; besti[tid] = bi;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s && (best[tid + s] > best[tid] ||
                      (best[tid + s] == best[tid] && besti[tid + s] < besti[tid]))) {
        best[tid] = best[tid + s]; besti[tid] = besti[tid + s];
      }
      __syncthreads();
    }
    if (tid == 0) {
      piv = besti[0];
      if (best[0] == 0.0) *singular = 1;
    }
    __syncthreads();
    const int pr = piv;
    if (pr != c)
      for (int j = tid; j < w; j += nt) {
        const double t = work[c * w + j];
        work[c * w + j] = work[pr * w + j];
        work[pr * w + j] = t;
      }
    __syncthreads();
    const double d = work[c * w + c];
    const double inv = d != 0.0 ? 1.0 / d : 0.0;
    __syncthreads();
    for (int j = tid; j < w; j += nt) work[c * w + j] *= inv;
    __syncthreads();
    for (int e = tid; e < k * w; e += nt) {
      const int i = e / w, j = e % w;
      if (i == c || j == c) continue;
      work[e] -= work[i * w + c] * work[c * w + j];
    }
    __syncthreads();
    for (int i = tid; i < k; i += nt)
      if (i != c) work[i * w + c] = 0.0;
    __syncthreads();
  }
  for (int e = tid; e < k * k; e += nt) Ainv[e] = work[(e / k) * w + k + e % k];
}

__global__ void gather_cols_kernel(int m, int kin, int kout, const double* in, long ldi,
                                   const int* idx, const double* scale, double* out, long ldo) {
  const long total = (long)m * kout;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int i = e / kout, j = e % kout;
    double v = in[(long)i * ldi + idx[j]];
    if (scale) v *= scale[j];
    out[(long)i * ldo + j] = v;
  }
}

__global__ void place_block_kernel(int na, int nb, int inner, const double* src, double* dst,
                                   int R1dst, int a0, int b0) {
  // src [na][inner][nb] -> dst [..][inner][R1dst] at (a0 + a, ., b0 + b)
  const long total = (long)na * inner * nb;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total;
       e += (long)gridDim.x * blockDim.x) {
    const int b = e % nb;
    const long t = e / nb;
    const int x = t % inner;
    const int a = t / inner;
    dst[((long)(a0 + a) * inner + x) * R1dst + b0 + b] = src[e];
  }
}

// ---- one-sided block Jacobi SVD ----

constexpr int OSB = 16;        // columns per block
constexpr int OSP = 2 * OSB;   // columns per block pair
constexpr int OST = 256;       // threads per pair workgroup
constexpr int OSR = 64;        // rows per LDS tile
constexpr int OSL = OSP + 4;   // LDS row pitch: the 16 (k, column) fragment addresses of one
                               // FP64 MFMA step fall in distinct banks

__device__ inline void circle_pair(int t, int round, int nplayers, int& a, int& b) {
  auto player = [&](int pos) { return pos == 0 ? 0 : 1 + (pos - 1 + round) % (nplayers - 1); };
  a = player(t);
  b = player(nplayers - 1 - t);
  if (a > b) { const int x = a; a = b; b = x; }
}

// One round of the one-sided block Jacobi method, in four launches so that the work over
// the m rows spreads across the chip. The round-robin schedule pairs block I with block J;
// for each pair:
//   osbj_gram:  partial 32 x 32 Gram matrices of the pair's columns, one per chunk of rows;
//   osbj_sum:   their sum (fixed order);
//   osbj_rot:   cyclic Jacobi on the summed Gram matrix in LDS, giving the rotation W
//               (32 x 32); flags[pair] = 1 if anything rotated;
//   osbj_apply: [B_I B_J] <- [B_I B_J] W and [V_I V_J] <- [V_I V_J] W, chunk by chunk.
// The Gram and apply products run on the FP64 matrix cores (v_mfma_f64_4x4x4_4b, lane
// l = 16 lx + 4 lb + ly: A operand at (row 4 r + ly, k lx), B operand at (k lx, column
// 16 c + 4 lb + ly), result at (row 4 r + lx, column 16 c + 4 lb + ly)).
__global__ __launch_bounds__(OST) void osbj_gram_kernel(const double* B, int m, long ldb, int nb, int round,
                                                        int chunk, double* P) {
  __shared__ double T[OSR][OSL];
  const int tid = threadIdx.x, pair = blockIdx.x, c = blockIdx.y;
  int I, J;
  circle_pair(pair, round, nb, I, J);
  auto col = [&](int q) { return q < OSB ? I * OSB + q : J * OSB + (q - OSB); };
  const int rb = c * chunk, re = min(m, rb + chunk);
  // wave w owns Gram rows 8 w .. 8 w + 7 and all 32 columns: G[i][j] = sum_row T[row][i] T[row][j]
  const int wave = tid / 64, lane = tid % 64;
  const int lx = lane / 16, lb = (lane / 4) % 4, ly = lane % 4;
  const int wm0 = 8 * wave;
  double acc[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  for (int r0 = rb; r0 < re; r0 += OSR) {
    for (int e = tid; e < OSR * OSP; e += OST) {
      const int rr = e / OSP, q = e % OSP, row = r0 + rr;
      T[rr][q] = row < re ? B[(long)row * ldb + col(q)] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int ks = 0; ks < OSR; ks += 4) {
      double fa[2], fb[2];
#pragma unroll
      for (int r = 0; r < 2; ++r) fa[r] = T[ks + lx][wm0 + 4 * r + ly];
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) fb[cc] = T[ks + lx][16 * cc + 4 * lb + ly];
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
          acc[r][cc] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[r], fb[cc], acc[r][cc], 0, 0, 0);
    }
    __syncthreads();
  }
  double* out = P + ((long)pair * gridDim.y + c) * (OSP * OSP);
#pragma unroll
  for (int r = 0; r < 2; ++r)
#pragma unroll
    for (int cc = 0; cc < 2; ++cc) out[(wm0 + 4 * r + lx) * OSP + 16 * cc + 4 * lb + ly] = acc[r][cc];
}

constexpr int ORT = 256;  // threads per pair in osbj_rot: one per 2 x 2 block of the 32 x 32 Gram matrix
static_assert(ORT == (OSP / 2) * (OSP / 2), "one thread per 2 x 2 block");
// Inner Jacobi sweeps per pair and round (at most `inner`; a sweep that rotates nothing ends
// them). The pair's rotation need not diagonalise its Gram matrix fully: the outer iteration
// revisits every pair each sweep and stops only when no pair needs a rotation at the outer
// threshold. On the triangular factor of a pivoted QR, whose columns are graded, solving the
// pair's problem to convergence about halves the outer sweeps; the inner sweeps run in LDS,
// so they cost little beside the Gram and update passes over the rows.

// Gsum[pair] = sum over chunks of P[pair][chunk] (chunk order), 256 elements per workgroup,
// eight chunks of loads in flight per thread.
__global__ __launch_bounds__(256) void osbj_sum_kernel(const double* P, int nchunk, double* Gsum) {
  const int pair = blockIdx.x, e = blockIdx.y * 256 + threadIdx.x;
  const double* in = P + (long)pair * nchunk * (OSP * OSP) + e;
  constexpr int CB = 8;
  double a = 0.0;
  for (int c0 = 0; c0 < nchunk; c0 += CB) {
    double v[CB];
#pragma unroll
    for (int u = 0; u < CB; ++u) v[u] = c0 + u < nchunk ? in[(long)(c0 + u) * (OSP * OSP)] : 0.0;
#pragma unroll
    for (int u = 0; u < CB; ++u) a += v[u];
  }
  Gsum[(long)pair * (OSP * OSP) + e] = a;
}

// Round-robin partner of the 32-player schedule (as circle_pair with nplayers = 32), with the
// modulo 31 done by one conditional subtraction (pos - 1 + round <= 60).
__device__ __forceinline__ void circle_pair32(int t, int round, int& a, int& b) {
  auto player = [&](int pos) {
    int x = pos - 1 + round;
    x = x >= OSP - 1 ? x - (OSP - 1) : x;
    return pos == 0 ? 0 : 1 + x;
  };
  a = player(t);
  b = player(OSP - 1 - t);
  if (a > b) { const int x = a; a = b; b = x; }
}

// Rotation of pair (p, q) of the cyclic Jacobi method on a symmetric matrix:
// |apq| > tol sqrt(|app aqq|) (squared: no square root on the path of every rotation) unless
// both columns are negligible; then t = tan(theta) = sign(tau) / (|tau| + sqrt(1 + tau^2)) with
// tau = dd / ee, written as sign(tau) |ee| / (|dd| + sqrt(dd^2 + ee^2)) (one division and one
// root fewer), c = 1 / sqrt(1 + t^2), s = t c, and the new diagonal app - t apq, aqq + t apq.
// abs2 > 0 also skips a rotation that would move the larger column by at most sqrt(abs2) in
// norm (t^2 max(app, aqq) <= abs2): on graded columns the block updates leave the small ones
// with rounding noise of the size of u times the large ones, which the relative test alone
// keeps chasing.
struct Rot {
  double c, s, np, nq;
  bool on;
};
__device__ __forceinline__ Rot jacobi_rot(double app, double aqq, double apq, double tol, double floor_col,
                                          double abs2) {
  Rot r{1.0, 0.0, app, aqq, false};
  const bool negligible = app <= floor_col && aqq <= floor_col;
  if (!negligible && apq * apq > tol * tol * fabs(app * aqq)) {
    const double dd = aqq - app, ee = 2.0 * apq;
    const double sg = (dd == 0.0 || (dd > 0.0) == (ee > 0.0)) ? 1.0 : -1.0;
    const double t = sg * fabs(ee) / (fabs(dd) + sqrt(dd * dd + ee * ee));
    if (t * t * fmax(app, aqq) <= abs2) return r;
    r.c = 1.0 / sqrt(1.0 + t * t);
    r.s = t * r.c;
    r.np = app - t * apq;
    r.nq = aqq + t * apq;
    r.on = true;
  }
  return r;
}

__global__ __launch_bounds__(ORT) void osbj_rot_kernel(const double* Gsum, double tol, double floor_col,
                                                       double abs2, int inner, double* Wout, int* flags) {
  __shared__ double G[OSP][OSP + 1];
  __shared__ double W[OSP][OSP + 1];
  __shared__ double cs[OSP / 2], sn[OSP / 2], dp[OSP / 2], dq[OSP / 2];
  __shared__ int rot_any, rot_sweep;
  const int tid = threadIdx.x, pair = blockIdx.x;
  const double* in = Gsum + (long)pair * (OSP * OSP);
  for (int e = tid; e < OSP * OSP; e += ORT) {
    const int i = e / OSP, j = e % OSP;
    G[i][j] = in[e];
    W[i][j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid == 0) rot_any = 0;
  __syncthreads();
  {
    // a pair with nothing above the threshold exits before the sweep
    int need = 0;
    for (int e = tid; e < OSP * OSP; e += ORT) {
      const int i = e / OSP, jj = e % OSP;
      if (i < jj) need |= jacobi_rot(G[i][i], G[jj][jj], G[i][jj], tol, floor_col, abs2).on ? 1 : 0;
    }
    if (!__syncthreads_or(need)) {
      if (tid == 0) flags[pair] = 0;
      return;
    }
  }
  // Each round: the 16 disjoint rotations (p_t, q_t) of the round-robin schedule are found by
  // threads 0..15; then thread (t1, t2) applies rows of rotation t1 and columns of rotation t2
  // to the 2 x 2 block {p_t1, q_t1} x {p_t2, q_t2} of G at once (the blocks are disjoint and
  // cover G), and rows i = tid / 16, tid / 16 + 16 of W take rotation tid % 16. Diagonal blocks
  // of rotated pairs are stored exactly (zero off-diagonal, closed-form diagonal), so rounding
  // noise in g_pq cannot trigger further rotations.
  const int t1 = tid / (OSP / 2), t2 = tid % (OSP / 2);
  for (int sweep = 0; sweep < inner; ++sweep) {
    if (tid == 0) rot_sweep = 0;
    __syncthreads();
    for (int r2 = 0; r2 < OSP - 1; ++r2) {
      if (tid < OSP / 2) {
        int p, q;
        circle_pair32(tid, r2, p, q);
        const Rot R = jacobi_rot(G[p][p], G[q][q], G[p][q], tol, floor_col, abs2);
        if (R.on) rot_sweep = 1;
        cs[tid] = R.c; sn[tid] = R.s; dp[tid] = R.np; dq[tid] = R.nq;
      }
      __syncthreads();
      {
        int p1, q1, p2, q2;
        circle_pair32(t1, r2, p1, q1);
        circle_pair32(t2, r2, p2, q2);
        const double c1 = cs[t1], s1 = sn[t1], c2 = cs[t2], s2 = sn[t2];
        if (s1 != 0.0 || s2 != 0.0) {
          if (t1 == t2) {
            G[p1][p1] = dp[t1];
            G[q1][q1] = dq[t1];
            G[p1][q1] = 0.0;
            G[q1][p1] = 0.0;
          } else {
            const double a = G[p1][p2], bq = G[p1][q2], cp = G[q1][p2], d = G[q1][q2];
            // rows (rotation t1), then columns (rotation t2)
            const double a1 = c1 * a - s1 * cp, c1p = s1 * a + c1 * cp;
            const double b1 = c1 * bq - s1 * d, d1 = s1 * bq + c1 * d;
            G[p1][p2] = c2 * a1 - s2 * b1;
            G[p1][q2] = s2 * a1 + c2 * b1;
            G[q1][p2] = c2 * c1p - s2 * d1;
            G[q1][q2] = s2 * c1p + c2 * d1;
          }
        }
        // W <- W J: rows tid / 16 and tid / 16 + 16, rotation tid % 16
        if (s2 != 0.0) {
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int i = t1 + h * (OSP / 2);
            const double wp = W[i][p2], wq = W[i][q2];
            W[i][p2] = c2 * wp - s2 * wq;
            W[i][q2] = s2 * wp + c2 * wq;
          }
        }
      }
      __syncthreads();
    }
    const int any = rot_sweep;
    if (sweep == 0 && tid == 0) rot_any = any;
    __syncthreads();
    if (!any) break;
  }
  double* out = Wout + (long)pair * (OSP * OSP);
  for (int e = tid; e < OSP * OSP; e += ORT) out[e] = W[e / OSP][e % OSP];
  if (tid == 0) flags[pair] = rot_any;
}

__global__ __launch_bounds__(OST) void osbj_apply_kernel(double* B, int m, long ldb, double* V, int kv, long ldv,
                                                         int nb, int round, int chunk, int nchunkB,
                                                         const double* Wg, const int* flags) {
  __shared__ double W[OSP][OSL];
  __shared__ double T[OSR][OSL];
  const int tid = threadIdx.x, pair = blockIdx.x, c = blockIdx.y;
  if (!flags[pair]) return;
  int I, J;
  circle_pair(pair, round, nb, I, J);
  auto col = [&](int q) { return q < OSB ? I * OSB + q : J * OSB + (q - OSB); };
  for (int e = tid; e < OSP * OSP; e += OST) W[e / OSP][e % OSP] = Wg[(long)pair * (OSP * OSP) + e];
  const bool onB = c < nchunkB;
  double* X = onB ? B : V;
  const int rows = onB ? m : kv;
  const long ld = onB ? ldb : ldv;
  const int rb = (onB ? c : c - nchunkB) * chunk, re = min(rows, rb + chunk);
  // wave w owns tile rows 16 w .. 16 w + 15 and all 32 columns: X[row][q] = sum_t T[row][t] W[t][q]
  const int wave = tid / 64, lane = tid % 64;
  const int lx = lane / 16, lb = (lane / 4) % 4, ly = lane % 4;
  const int wm0 = 16 * wave;
  __syncthreads();
  for (int r0 = rb; r0 < re; r0 += OSR) {
    for (int e = tid; e < OSR * OSP; e += OST) {
      const int rr = e / OSP, q = e % OSP, row = r0 + rr;
      T[rr][q] = row < re ? X[(long)row * ld + col(q)] : 0.0;
    }
    __syncthreads();
    double acc[4][2] = {{0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
    for (int ks = 0; ks < OSP; ks += 4) {
      double fa[4], fb[2];
#pragma unroll
      for (int r = 0; r < 4; ++r) fa[r] = T[wm0 + 4 * r + ly][ks + lx];
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) fb[cc] = W[ks + lx][16 * cc + 4 * lb + ly];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int cc = 0; cc < 2; ++cc)
          acc[r][cc] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[r], fb[cc], acc[r][cc], 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = r0 + wm0 + 4 * r + lx;
      if (row >= re) continue;
#pragma unroll
      for (int cc = 0; cc < 2; ++cc) X[(long)row * ld + col(16 * cc + 4 * lb + ly)] = acc[r][cc];
    }
    __syncthreads();
  }
}

// Cholesky factor of a jb x jb diagonal block (jb <= CHB) of a symmetric matrix whose earlier
// columns have already been eliminated: reads the lower triangle of G, writes the lower factor
// to L and its inverse to Linv (CHB x CHB, row-major, zero above the diagonal). Columns are
// eliminated in order; a pivot that is not positive (a semidefinite or indefinite block, or a
// NaN) gives a zero column of L and of Linv and adds one to *bad.
constexpr int CHB = 32;
__global__ __launch_bounds__(256) void chol_block_kernel(const double* G, long ldg, int jb, double* L, long ldl,
                                                         double* Linv, int* bad) {
  __shared__ double S[CHB][CHB + 1];
  __shared__ double X[CHB][CHB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < CHB * CHB; e += 256) {
    const int i = e / CHB, j = e % CHB;
    S[i][j] = (i < jb && j <= i) ? G[(long)i * ldg + j] : 0.0;
    X[i][j] = 0.0;
  }
  __syncthreads();
  for (int c = 0; c < jb; ++c) {
    if (tid == 0) {
      const double d = S[c][c];
      const bool ok = d > 0.0;
      S[c][c] = ok ? sqrt(d) : 0.0;
      if (!ok) atomicAdd(bad, 1);
    }
    __syncthreads();
    const double piv = S[c][c];
    for (int r = c + 1 + tid; r < jb; r += 256) S[r][c] = piv > 0.0 ? S[r][c] / piv : 0.0;
    __syncthreads();
    const int w = jb - c - 1;
    for (int e = tid; e < w * w; e += 256) {
      const int r = c + 1 + e / w, q = c + 1 + e % w;
      if (q <= r) S[r][q] -= S[r][c] * S[q][c];
    }
    __syncthreads();
  }
  // Linv: forward substitution L x = e_j, one column per thread
  if (tid < jb) {
    const int j = tid;
    const double djj = S[j][j];
    X[j][j] = djj > 0.0 ? 1.0 / djj : 0.0;
    for (int r = j + 1; r < jb; ++r) {
      double a = 0.0;
      for (int t = j; t < r; ++t) a += S[r][t] * X[t][j];
      X[r][j] = S[r][r] > 0.0 ? -a / S[r][r] : 0.0;
    }
  }
  __syncthreads();
  for (int e = tid; e < CHB * CHB; e += 256) {
    const int i = e / CHB, j = e % CHB;
    if (i < jb && j <= i) L[(long)i * ldl + j] = S[i][j];
    Linv[e] = X[i][j];
  }
}

// Cholesky factorisation with diagonal pivoting of a symmetric positive semidefinite k x k
// matrix G (row-major, full storage, destroyed), by one workgroup: at step j the largest
// remaining diagonal entry of the Schur complement (the first one on ties) is swapped to
// position j, rows and columns alike, the column of the factor is formed and the whole
// trailing block is updated. The pivot order is the greedy order of column-pivoted QR of any
// A with A^T A = G. On return the lower triangle of G holds L with P^T G P = L L^T (zeros
// above the diagonal), perm[j] the original index of pivot j; a pivot that is not positive
// gives a zero column and adds one to *bad. The trailing updates read and write G in global
// memory (L2-resident at the sizes this serves, k <= PCHOL_MAX).
constexpr int PCHOL_MAX = 1024;
constexpr int PCHOL_LDS_MAX = 140;  // G itself in LDS (k^2 doubles) up to this size
template <bool InLds>
__global__ __launch_bounds__(256) void pchol_kernel(double* Gg, int k, int* perm, int* bad) {
  constexpr int KM = InLds ? PCHOL_LDS_MAX : PCHOL_MAX;
  extern __shared__ double Gl[];
  __shared__ double dg[KM];
  __shared__ int pm[KM];
  __shared__ double rv[256];
  __shared__ int ri[256];
  const int tid = threadIdx.x;
  double* G = InLds ? Gl : Gg;
  if (InLds) {
    for (int e = tid; e < k * k; e += 256) Gl[e] = Gg[e];
    __syncthreads();
  }
  for (int i = tid; i < k; i += 256) {
    dg[i] = G[(long)i * k + i];
    pm[i] = i;
  }
  __syncthreads();
  for (int j = 0; j < k; ++j) {
    // argmax of dg[j..k), the smallest index among equal values
    double bv = -1.0;
    int bi = j;
    for (int i = j + tid; i < k; i += 256)
      if (dg[i] > bv) { bv = dg[i]; bi = i; }
    rv[tid] = bv;
    ri[tid] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) {
        const double ov = rv[tid + w];
        const int oi = ri[tid + w];
        if (ov > rv[tid] || (ov == rv[tid] && oi < ri[tid])) { rv[tid] = ov; ri[tid] = oi; }
      }
      __syncthreads();
    }
    const int p = ri[0];
    if (p != j) {
      // swap rows j and p, then columns j and p
      for (int t = tid; t < k; t += 256) {
        const double a = G[(long)j * k + t], b = G[(long)p * k + t];
        G[(long)j * k + t] = b;
        G[(long)p * k + t] = a;
      }
      __syncthreads();
      for (int t = tid; t < k; t += 256) {
        const double a = G[(long)t * k + j], b = G[(long)t * k + p];
        G[(long)t * k + j] = b;
        G[(long)t * k + p] = a;
      }
      if (tid == 0) {
        const double dv = dg[j]; dg[j] = dg[p]; dg[p] = dv;
        const int pv = pm[j]; pm[j] = pm[p]; pm[p] = pv;
      }
      __syncthreads();
    }
    const double d = G[(long)j * k + j];
    const bool ok = d > 0.0;
    const double ljj = ok ? sqrt(d) : 0.0;
    __syncthreads();
    if (tid == 0) {
      G[(long)j * k + j] = ljj;
      if (!ok) atomicAdd(bad, 1);
    }
    for (int i = j + 1 + tid; i < k; i += 256) G[(long)i * k + j] = ok ? G[(long)i * k + j] / ljj : 0.0;
    __syncthreads();
    // trailing update of the full block (both triangles stay symmetric for later swaps)
    const int w = k - j - 1;
    for (long e = tid; e < (long)w * w; e += 256) {
      const int i = j + 1 + (int)(e / w), t = j + 1 + (int)(e % w);
      G[(long)i * k + t] -= G[(long)i * k + j] * G[(long)t * k + j];
    }
    __syncthreads();
    for (int i = j + 1 + tid; i < k; i += 256) dg[i] = G[(long)i * k + i];
    __syncthreads();
  }
  // the lower triangle, zeros above
  for (long e = tid; e < (long)k * k; e += 256) {
    const int i = (int)(e / k), t = (int)(e % k);
    Gg[e] = t > i ? 0.0 : G[e];
  }
  for (int i = tid; i < k; i += 256) perm[i] = pm[i];
}

// Inverses of the CHB x CHB diagonal blocks of a lower-triangular L (k x k, ldl): block b into
// Linv[b] (CHB x CHB, row-major, zero above the diagonal), by forward substitution, one
// column per thread; a zero diagonal entry gives a zero row and column.
__global__ __launch_bounds__(64) void trinv_blocks_kernel(const double* L, long ldl, int k, double* Linv) {
  __shared__ double S[CHB][CHB + 1];
  __shared__ double X[CHB][CHB + 1];
  const int b = blockIdx.x, j0 = b * CHB, jb = min(CHB, k - j0), tid = threadIdx.x;
  for (int e = tid; e < CHB * CHB; e += 64) {
    const int i = e / CHB, j = e % CHB;
    S[i][j] = (i < jb && j <= i) ? L[(long)(j0 + i) * ldl + j0 + j] : 0.0;
    X[i][j] = 0.0;
  }
  __syncthreads();
  if (tid < jb) {
    const int j = tid;
    X[j][j] = S[j][j] > 0.0 ? 1.0 / S[j][j] : 0.0;
    for (int r = j + 1; r < jb; ++r) {
      double a = 0.0;
      for (int t = j; t < r; ++t) a += S[r][t] * X[t][j];
      X[r][j] = S[r][r] > 0.0 ? -a / S[r][r] : 0.0;
    }
  }
  __syncthreads();
  double* out = Linv + (long)b * CHB * CHB;
  for (int e = tid; e < CHB * CHB; e += 64) out[e] = X[e / CHB][e % CHB];
}

// out[i][:] = in[idx[i]][:], i < m, k columns
__global__ void gather_rows_kernel(int m, int k, const double* in, long ldi, const int* idx, double* out, long ldo) {
  const long total = (long)m * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int i = (int)(e / k), j = (int)(e % k);
    out[(long)i * ldo + j] = in[(long)idx[i] * ldi + j];
  }
}

__global__ void add_diag_kernel(int k, double* A, long lda, double v) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < k; i += gridDim.x * blockDim.x) A[(long)i * lda + i] += v;
}

}  // namespace

static int osbj_chunk(int m, int nb) {
  // rows per chunk: enough chunks that the gram and apply launches hold ~512 workgroups
  const int npair = nb / 2;
  const int want = std::max(1, 512 / npair);
  int chunk = (m + want - 1) / want;
  chunk = ((chunk + OSR - 1) / OSR) * OSR;
  return std::max(chunk, OSR);
}

size_t osbj_work_len(int m, int kv, int nb) {
  const int chunk = osbj_chunk(m, nb);
  const long nchunk = (m + chunk - 1) / chunk;
  (void)kv;
  return (size_t)(nb / 2) * (nchunk + 2) * (OSP * OSP);
}

void osbj_round(hipStream_t s, double* B, int m, long ldb, double* V, int kv, long ldv, int nb, int round,
                double tol, double floor_col, int* flags, double* work, size_t work_len, int inner,
                double abs2) {
  require(nb >= 2 && nb % 2 == 0, IGA_EINVAL, "osbj_round: block count must be even");
  require(m >= 1 && kv >= 0, IGA_EINVAL, "osbj_round: bad sizes");
  require(work_len >= osbj_work_len(m, kv, nb), IGA_EINVAL, "osbj_round: workspace too small");
  const int npair = nb / 2, chunk = osbj_chunk(m, nb);
  const int nchunkB = (m + chunk - 1) / chunk, nchunkV = (kv + chunk - 1) / chunk;
  double* P = work;
  double* Gs = work + (size_t)npair * nchunkB * (OSP * OSP);
  double* Wg = Gs + (size_t)npair * (OSP * OSP);
  osbj_gram_kernel<<<dim3(npair, nchunkB), OST, 0, s>>>(B, m, ldb, nb, round, chunk, P);
  IGA_HIP(hipGetLastError());
  osbj_sum_kernel<<<dim3(npair, OSP * OSP / 256), 256, 0, s>>>(P, nchunkB, Gs);
  IGA_HIP(hipGetLastError());
  osbj_rot_kernel<<<npair, ORT, 0, s>>>(Gs, tol, floor_col, abs2, std::max(1, inner), Wg, flags);
  IGA_HIP(hipGetLastError());
  osbj_apply_kernel<<<dim3(npair, nchunkB + nchunkV), OST, 0, s>>>(B, m, ldb, V, kv, ldv, nb, round, chunk,
                                                                   nchunkB, Wg, flags);
  IGA_HIP(hipGetLastError());
}

int osbj_block() { return OSB; }
int jacobi_lds_max() { return LDS_MAX_K; }

void jacobi_eig(hipStream_t s, int nmat, int k, double* H, long strideH, double* W, long strideW,
                double tol, int max_sweeps, int* sweeps_out) {
  // one rotation per thread pair slot: the per-round tables hold JT / 2 pairs
  require(k >= 1 && k <= JT, IGA_EINVAL, "jacobi_eig: k out of range");
  // once per process (solves may run in several host threads)
  static std::once_flag attr_once;
  std::call_once(attr_once, [] {
    IGA_HIP(hipFuncSetAttribute((const void*)jacobi_kernel<1>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (LDS_MAX_K + 1) * LDS_MAX_K * (int)sizeof(double)));
    IGA_HIP(hipFuncSetAttribute((const void*)jacobi_kernel<2>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                ((LDS_BOTH_MAX_K + 1) * LDS_BOTH_MAX_K + LDS_BOTH_MAX_K * LDS_BOTH_MAX_K) *
                                    (int)sizeof(double)));
  });
  if (k <= LDS_BOTH_MAX_K) {
    const size_t lds = ((size_t)(k + 1) * k + (size_t)k * k) * sizeof(double);
    jacobi_kernel<2><<<nmat, JT, lds, s>>>(k, H, strideH, W, strideW, tol, max_sweeps, sweeps_out);
  } else if (k <= LDS_MAX_K) {
    const size_t lds = (size_t)(k + 1) * k * sizeof(double);
    jacobi_kernel<1><<<nmat, JT, lds, s>>>(k, H, strideH, W, strideW, tol, max_sweeps, sweeps_out);
  } else {
    jacobi_kernel<0><<<nmat, JT, 0, s>>>(k, H, strideH, W, strideW, tol, max_sweeps, sweeps_out);
  }
  IGA_HIP(hipGetLastError());
}

void transpose_square(hipStream_t s, int nmat, int k, const double* in, long sin, double* out,
                      long sout) {
  dim3 grid((unsigned)std::max<long>(1, std::min<long>(((long)k * k + 255) / 256, 1024)), nmat);
  transpose_sq<<<grid, 256, 0, s>>>(k, in, sin, out, sout);
  IGA_HIP(hipGetLastError());
}

void invert(hipStream_t s, int k, const double* A, double* Ainv, double* work, int* singular) {
  gauss_jordan<<<1, 1024, 0, s>>>(k, A, Ainv, work, singular);
  IGA_HIP(hipGetLastError());
}

int chol_block_size() { return CHB; }

void chol_block(hipStream_t s, int jb, const double* G, long ldg, double* L, long ldl, double* Linv, int* bad) {
  require(jb >= 1 && jb <= CHB, IGA_EINVAL, "chol_block: block size out of range");
  chol_block_kernel<<<1, 256, 0, s>>>(G, ldg, jb, L, ldl, Linv, bad);
  IGA_HIP(hipGetLastError());
}

int pchol_max() { return PCHOL_MAX; }

void pivoted_cholesky(hipStream_t s, int k, double* G, int* perm, int* bad) {
  require(k >= 1 && k <= PCHOL_MAX, IGA_EINVAL, "pivoted_cholesky: size out of range");
  if (k <= PCHOL_LDS_MAX) {
    static std::once_flag attr_once;
    std::call_once(attr_once, [] {
      IGA_HIP(hipFuncSetAttribute((const void*)pchol_kernel<true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                  PCHOL_LDS_MAX * PCHOL_LDS_MAX * (int)sizeof(double)));
    });
    pchol_kernel<true><<<1, 256, (size_t)k * k * sizeof(double), s>>>(G, k, perm, bad);
  } else {
    pchol_kernel<false><<<1, 256, 0, s>>>(G, k, perm, bad);
  }
  IGA_HIP(hipGetLastError());
}

void trinv_blocks(hipStream_t s, int k, const double* L, long ldl, double* Linv) {
  if (k <= 0) return;
  trinv_blocks_kernel<<<(k + CHB - 1) / CHB, 64, 0, s>>>(L, ldl, k, Linv);
  IGA_HIP(hipGetLastError());
}

void gather_rows(hipStream_t s, int m, int k, const double* in, long ldi, const int* idx, double* out, long ldo) {
  const long total = (long)m * k;
  if (total <= 0) return;
  gather_rows_kernel<<<(unsigned)std::min<long>((total + 255) / 256, 4096), 256, 0, s>>>(m, k, in, ldi, idx, out, ldo);
  IGA_HIP(hipGetLastError());
}

void add_diag(hipStream_t s, int k, double* A, long lda, double v) {
  if (k <= 0) return;
  add_diag_kernel<<<(unsigned)std::min(1024, (k + 255) / 256), 256, 0, s>>>(k, A, lda, v);
  IGA_HIP(hipGetLastError());
}

void gather_cols(hipStream_t s, int m, int kin, int kout, const double* in, long ldi, const int* idx,
                 const double* scale, double* out, long ldo) {
  const long total = (long)m * kout;
  if (total <= 0) return;
  gather_cols_kernel<<<(unsigned)std::min<long>((total + 255) / 256, 4096), 256, 0, s>>>(
      m, kin, kout, in, ldi, idx, scale, out, ldo);
  IGA_HIP(hipGetLastError());
}

void place_block(hipStream_t s, int na, int nb, int inner, const double* src, double* dst, int R1dst,
                 int a0, int b0) {
  const long total = (long)na * inner * nb;
  if (total <= 0) return;
  place_block_kernel<<<(unsigned)std::min<long>((total + 255) / 256, 4096), 256, 0, s>>>(
      na, nb, inner, src, dst, R1dst, a0, b0);
  IGA_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace iga
