// Generic kernels: strided batched GEMM, banded rank contraction, elementwise
// updates, permutations and deterministic reductions (FP64; GEMM/band also FP32).
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

constexpr int TM = 64, TN = 64, TK = 16, NT = 256;

template <typename T>
struct GemmArgs {
  int M, N, K, Kout;
  const T* A;
  long sAm, sAk, sAko;
  const T* B;
  long sBk, sBn, sBko;
  T* C;
  long sCm, sCn;
  int nb2;
  long sAb1, sAb2, sBb1, sBb2, sCb1, sCb2;
  T alpha, beta;
};

// 64x64 output tile per 256-thread workgroup, 4x4 outputs per thread, K staged
// through LDS in slabs of 16. Loads are coalesced along whichever of the two
// tile axes has unit stride.
template <typename T>
__global__ __launch_bounds__(NT) void gemm_kernel(GemmArgs<T> g) {
  __shared__ T As[TK][TM + 1];
  __shared__ T Bs[TK][TN + 1];
  const int b = blockIdx.z;
  const int b1 = b / g.nb2, b2 = b % g.nb2;
  const T* A = g.A + b1 * g.sAb1 + b2 * g.sAb2;
  const T* B = g.B + b1 * g.sBb1 + b2 * g.sBb2;
  T* C = g.C + b1 * g.sCb1 + b2 * g.sCb2;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  T acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = T(0);
  const long Ktot = (long)g.K * g.Kout;
  const bool a_kfast = (g.sAk == 1);
  const bool b_nfast = (g.sBn == 1);
  for (long k0 = 0; k0 < Ktot; k0 += TK) {
    for (int e = threadIdx.x; e < TM * TK; e += NT) {
      int mm, kk;
      if (a_kfast) { kk = e % TK; mm = e / TK; } else { mm = e % TM; kk = e / TM; }
      const long k = k0 + kk;
      const int m = m0 + mm;
      T v = T(0);
      if (m < g.M && k < Ktot) {
        const long ko = k / g.K, ki = k - ko * g.K;
        v = A[m * g.sAm + ki * g.sAk + ko * g.sAko];
      }
      As[kk][mm] = v;
    }
    for (int e = threadIdx.x; e < TN * TK; e += NT) {
      int nn, kk;
      if (b_nfast) { nn = e % TN; kk = e / TN; } else { kk = e % TK; nn = e / TK; }
      const long k = k0 + kk;
      const int nidx = n0 + nn;
      T v = T(0);
      if (nidx < g.N && k < Ktot) {
        const long ko = k / g.K, ki = k - ko * g.K;
        v = B[ki * g.sBk + nidx * g.sBn + ko * g.sBko];
      }
      Bs[kk][nn] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TK; ++kk) {
      T a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + ty + 16 * i;
    if (m >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int nidx = n0 + tx + 16 * j;
      if (nidx >= g.N) continue;
      T* c = C + m * g.sCm + nidx * g.sCn;
      T v = g.alpha * acc[i][j];
      if (g.beta != T(0)) v += g.beta * *c;
      *c = v;
    }
  }
}

template <typename T, typename G>
void launch_gemm(hipStream_t s, const G& d) {
  if (d.M <= 0 || d.N <= 0 || d.nb1 <= 0 || d.nb2 <= 0) return;
  GemmArgs<T> a{d.M, d.N, d.K, d.Kout, d.A, d.sAm, d.sAk, d.sAko, d.B, d.sBk, d.sBn, d.sBko,
                d.C, d.sCm, d.sCn, d.nb2, d.sAb1, d.sAb2, d.sBb1, d.sBb2, d.sCb1, d.sCb2,
                d.alpha, d.beta};
  if (d.K <= 0 || d.Kout <= 0) {
    // empty contraction: C = beta * C
    a.K = 0;
  }
  long nb = (long)d.nb1 * d.nb2;
  require(nb <= 65535, IGA_EINVAL, "gemm: batch too large");
  dim3 grid((d.N + TN - 1) / TN, (d.M + TM - 1) / TM, (unsigned)nb);
  gemm_kernel<T><<<grid, NT, 0, s>>>(a);
  IGA_HIP(hipGetLastError());
}

__global__ void axpby_kernel(long n, double a, const double* x, double b, double* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (b == 0.0) ? a * x[i] : a * x[i] + b * y[i];
}
template <class T>
__global__ void fill_kernel(long n, T v, T* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = v;
}
__global__ void scale_kernel(long n, double a, double* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] *= a;
}
__global__ void to_f32_kernel(long n, const double* x, float* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}
__global__ void to_f64_kernel(long n, const float* x, double* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    y[i] = (double)x[i];
}

unsigned grid_for(long n) { return (unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 4096)); }

struct Perm4 {
  int od[4];   // output dims
  long is[4];  // input stride of output axis k
};
__global__ void permute4_kernel(const double* in, double* out, Perm4 P, long total) {
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    long t = idx;
    long off = 0;
#pragma unroll
    for (int k = 3; k >= 0; --k) {
      const int ik = t % P.od[k];
      t /= P.od[k];
      off += ik * P.is[k];
    }
    out[idx] = in[off];
  }
}

constexpr int RED_BLOCKS = 512;

__device__ double block_sum(double v) {
  __shared__ double sh[256];
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void dot_partial(long n, const double* x, const double* y,
                                                   double* partial) {
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc = fma(x[i], y[i], acc);
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
__global__ __launch_bounds__(256) void sum_partials(int np, int nrow, const double* partial,
                                                    double* out) {
  // one block per output row, fixed order
  const int row = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) acc += partial[(long)row * np + i];
  const double s = block_sum(acc);
  if (threadIdx.x == 0 && row < nrow) out[row] = s;
}

constexpr int MD_CHUNKS = 128;
__global__ __launch_bounds__(256) void multidot_partial(long n, const double* V, long ldv,
                                                        const double* w, double* partial) {
  const int j = blockIdx.y;
  const double* v = V + j * ldv;
  double acc = 0.0;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    acc = fma(v[i], w[i], acc);
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partial[(long)j * gridDim.x + blockIdx.x] = s;
}
__global__ __launch_bounds__(256) void multiaxpy_kernel(long n, int k, const double* V, long ldv,
                                                        const double* coef, double sign, double* w) {
  __shared__ double c[64];
  if ((int)threadIdx.x < k) c[threadIdx.x] = sign * coef[threadIdx.x];
  __syncthreads();
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    double acc = w[i];
    for (int j = 0; j < k; ++j) acc = fma(c[j], V[j * ldv + i], acc);
    w[i] = acc;
  }
}
__global__ __launch_bounds__(256) void colnorm_kernel(int m, int k, const double* A, long lda,
                                                      double* out) {
  const int j = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double v = A[(long)i * lda + j];
    acc = fma(v, v, acc);
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) out[j] = sqrt(s);
}

template <typename T>
__global__ void kkt_combine_kernel(long e, T k02, T m11, T m12, T k20, T m21, const T* zM, const T* zK,
                                   T* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < e; i += (long)gridDim.x * blockDim.x) {
    const T a0 = zM[i], a1 = zM[e + i], a2 = zM[2 * e + i];
    const T b0 = zK[i], b2 = zK[e + i];
    y[i] = a0 + k02 * b2;
    y[e + i] = m11 * a1 + m12 * a2;
    y[2 * e + i] = k20 * b0 + m21 * a1;
  }
}

// Banded stage of a rank-1 operator core (one left and one right rank): row i of y is the
// band combination y[i][c] = sum_{o < b} A[i][o] x[i + o][c] of the b rows of x around it,
// o in increasing order (blockIdx.y = i). Memory-bound: each x row is read by b output rows.
template <typename T>
__global__ __launch_bounds__(256) void band_rank1_kernel(int b, long ncols, const T* A, const T* x, long ldx, T* y) {
  const int i = blockIdx.y;
  const long c = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ncols) return;
  const T* a = A + (long)i * b;
  const T* xc = x + (long)i * ldx + c;
  T acc = a[0] * xc[0];
  for (int o = 1; o < b; ++o) acc += a[o] * xc[(long)o * ldx];
  y[(long)i * ncols + c] = acc;
}

// Banded stage of an operator core with few right ranks (R1 <= 16): for row i (blockIdx.y)
// and column c, y[i][g][c] = sum_{o < b, d < R0} A[i][o][d][g] x[(i + o) ldx + d ldd + c] for
// g < R1, with A the core re-laid as [n][b][R0][R1]. A workgroup covers 64 columns; its
// BAND_WAVES waves split the rank index d (wave w takes d = w, w + BAND_WAVES, ...), so the
// chain of dependent loads per thread is b * R0 / BAND_WAVES long, and the partial sums are
// added in LDS in the fixed wave order. The coefficients are the same for a whole wave and are
// read as scalars.
constexpr int BAND_WAVES = 4;

template <typename T, int R1>
__global__ __launch_bounds__(64 * BAND_WAVES) void band_small_kernel(int b, int R0, long ncols, const T* A,
                                                                     const T* x, long ldx, long ldd, T* y) {
  __shared__ T red[(BAND_WAVES - 1) * R1 * 64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int i = blockIdx.y;
  const long c = (long)blockIdx.x * 64 + lane;
  const bool live = c < ncols;
  T acc[R1];
#pragma unroll
  for (int g = 0; g < R1; ++g) acc[g] = T(0);
  if (live) {
    const T* ai = A + (long)i * b * R0 * R1;
    for (int o = 0; o < b; ++o) {
      const T* xo = x + (long)(i + o) * ldx + c;
      const T* ao = ai + (long)o * R0 * R1;
#pragma unroll 4
      for (int d = w; d < R0; d += BAND_WAVES) {
        const T v = xo[(long)d * ldd];
#pragma unroll
        for (int g = 0; g < R1; ++g) acc[g] += ao[d * R1 + g] * v;
      }
    }
  }
  if (w > 0) {
#pragma unroll
    for (int g = 0; g < R1; ++g) red[((w - 1) * R1 + g) * 64 + lane] = acc[g];
  }
  __syncthreads();
  if (w == 0 && live) {
#pragma unroll
    for (int g = 0; g < R1; ++g) {
      T s = acc[g];
#pragma unroll
      for (int v = 0; v < BAND_WAVES - 1; ++v) s += red[(v * R1 + g) * 64 + lane];
      y[((long)i * R1 + g) * ncols + c] = s;
    }
  }
}

// y[o] = sum of coef[t] z[src[t]] over the terms t of output block o (blockIdx.y = o).
template <typename T>
__global__ void combine_blocks_kernel(long e, const int* toff, const int* src, const double* coef, const T* z, T* y) {
  const int o = blockIdx.y;
  const int t0 = toff[o], t1 = toff[o + 1];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < e; i += (long)gridDim.x * blockDim.x) {
    T a = T(0);
    for (int t = t0; t < t1; ++t) a += T(coef[t]) * z[(long)src[t] * e + i];
    y[(long)o * e + i] = a;
  }
}

// Per spatial mode (a, i, b) of the reference operator (mass -> 1, stiffness -> mu =
// lamL[a] + lamN[i] + lamR[b]) the time-dependent KKT system couples the nt steps:
//   tau y + A^T l = f1,  tau beta u - tau l = f2,  A y - tau u = f3,  A = tau mu I + C
// (C lower bidiagonal 1, -1). Eliminating u and y leaves the SPD tridiagonal system
//   (A A^T / tau + tau / beta I) l = A f1 / tau - f3 - f2 / beta,
// solved by forward elimination and back substitution (Thomas); then
// y = (f1 - A^T l) / tau and u = (f2 + tau l) / (tau beta). v: [3][nt][e] in place; work:
// [nt][e] elimination factors.
__global__ void fd_solve_time_kernel(int r0, int n, int r1, int nt, const double* lamL, const double* lamN,
                                     const double* lamR, double beta, double tau, double* v, double* work) {
  const long e = (long)r0 * n * r1;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < e;
       idx += (long)gridDim.x * blockDim.x) {
    const int b = idx % r1;
    const int i = (idx / r1) % n;
    const int a = idx / ((long)r1 * n);
    const double aa = tau * (lamL[a] + lamN[i] + lamR[b]) + 1.0;  // diagonal of A
    const double off = -aa / tau;                                   // off-diagonal of the system
    double* f1 = v + idx;
    double* f2 = v + (long)nt * e + idx;
    double* f3 = v + 2L * nt * e + idx;
    double cprev = 0.0, dprev = 0.0, f1prev = 0.0;
    for (int t = 0; t < nt; ++t) {
      const double x1 = f1[t * e], x2 = f2[t * e], x3 = f3[t * e];
      const double rhs = (aa * x1 - f1prev) / tau - x3 - x2 / beta;
      const double diag = (aa * aa + (t > 0 ? 1.0 : 0.0)) / tau + tau / beta;
      const double den = diag - off * cprev;
      const double cp = off / den, dp = (rhs - off * dprev) / den;
      work[t * e + idx] = cp;
      f3[t * e] = dp;
      cprev = cp;
      dprev = dp;
      f1prev = x1;
    }
    double lnext = 0.0;
    for (int t = nt - 1; t >= 0; --t) {
      const double l = f3[t * e] - work[t * e + idx] * lnext;
      const double y = (f1[t * e] - (aa * l - lnext)) / tau;
      const double u = (f2[t * e] + tau * l) / (tau * beta);
      f1[t * e] = y;
      f2[t * e] = u;
      f3[t * e] = l;
      lnext = l;
    }
  }
}

// Grouped forms for the batched local operator: blockIdx.y selects the item.
template <typename T>
__global__ void fill_segments_kernel(const Segment* seg, T* base) {
  const Segment sg = seg[blockIdx.y];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < sg.len; i += (long)gridDim.x * blockDim.x)
    base[sg.off + i] = T(0);
}

template <typename T>
__global__ void combine_grouped_kernel(const CombineItem* items, const T* zbase) {
  const CombineItem it = items[blockIdx.y];
  const T* zM = zbase + it.z_off;
  const T* zK = zM + 3 * it.e;
  T* y = static_cast<T*>(it.y);
  const T k02 = T(it.coef.k02), m11 = T(it.coef.m11), m12 = T(it.coef.m12), k20 = T(it.coef.k20),
          m21 = T(it.coef.m21);
  const long e = it.e;
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < e; i += (long)gridDim.x * blockDim.x) {
    const T a0 = zM[i], a1 = zM[e + i], a2 = zM[2 * e + i];
    const T b0 = zK[i], b2 = zK[e + i];
    y[i] = a0 + k02 * b2;
    y[e + i] = m11 * a1 + m12 * a2;
    y[2 * e + i] = k20 * b0 + m21 * a1;
  }
}

__global__ void convert_segments_kernel(const ConvSegment* seg, int to_f32) {
  const ConvSegment sg = seg[blockIdx.y];
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < sg.len; i += (long)gridDim.x * blockDim.x) {
    if (to_f32) static_cast<float*>(sg.dst)[i] = (float)static_cast<const double*>(sg.src)[i];
    else static_cast<double*>(sg.dst)[i] = (double)static_cast<const float*>(sg.src)[i];
  }
}

__global__ void scale3_kernel(long e, double s0, double s1, double s2, double* y) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < 3 * e; i += (long)gridDim.x * blockDim.x) {
    const int c = i / e;
    y[i] *= (c == 0 ? s0 : (c == 1 ? s1 : s2));
  }
}

__global__ void fd_solve_kernel(int r0, int n, int r1, const double* lamL, const double* lamN,
                                const double* lamR, double c, double g, double* v) {
  const long e = (long)r0 * n * r1;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < e;
       idx += (long)gridDim.x * blockDim.x) {
    const int b = idx % r1;
    const int i = (idx / r1) % n;
    const int a = idx / ((long)r1 * n);
    const double k = g * (lamL[a] + lamN[i] + lamR[b]);
    const double f1 = v[idx], f2 = v[e + idx], f3 = v[2 * e + idx];
    // [[1,0,k],[0,c,-1],[k,-1,0]] [y;u;l] = [f1;f2;f3]:  u = k y - f3, l = c u - f2
    const double y = (f1 + k * f2 + c * k * f3) / (1.0 + c * k * k);
    const double u = k * y - f3;
    v[idx] = y;
    v[e + idx] = u;
    v[2 * e + idx] = c * u - f2;
  }
}

__global__ void symmetrize_kernel(int k, double* Hs, long stride) {
  double* H = Hs + blockIdx.y * stride;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < (long)k * k;
       e += (long)gridDim.x * blockDim.x) {
    const int i = e / k, j = e % k;
    if (j <= i) continue;
    const double m = 0.5 * (H[(long)i * k + j] + H[(long)j * k + i]);
    H[(long)i * k + j] = m;
    H[(long)j * k + i] = m;
  }
}

__global__ void core_product_kernel(int R0, int R1, int n, int p, const double* A, int r0, int r1,
                                    const double* X, double* Y, double alpha, double beta) {
  const int b = 2 * p + 1;
  const long total = (long)R0 * r0 * n * R1 * r1;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    long t = idx;
    const int bb = t % r1; t /= r1;
    const int be = t % R1; t /= R1;
    const int i = t % n; t /= n;
    const int a = t % r0;
    const int al = t / r0;
    double acc = 0.0;
    const int olo = max(0, p - i), ohi = min(b, n - i + p);
    for (int o = olo; o < ohi; ++o) {
      const int j = i + o - p;
      acc = fma(A[(((long)al * n + i) * b + o) * R1 + be], X[((long)a * n + j) * r1 + bb], acc);
    }
    double v = alpha * acc;
    if (beta != 0.0) v += beta * Y[idx];
    Y[idx] = v;
  }
}

__global__ void copy2d_kernel(int m, int k, const double* in, long si, long sj, double* out, long ldo) {
  const long total = (long)m * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int i = e / k, j = e % k;
    out[(long)i * ldo + j] = in[(long)i * si + (long)j * sj];
  }
}

__global__ void diag_kernel(int k, const double* H, long step, double* out, int mode) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x) {
    const double v = H[(long)j * step];
    out[j] = mode ? (v > 0.0 ? 1.0 / sqrt(v) : 0.0) : v;
  }
}

__global__ void scale_rows_kernel(int m, int k, const double* sc, double* A, long lda) {
  const long total = (long)m * k;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int i = e / k, j = e - (long)i * k;
    A[(long)i * lda + j] *= sc[i];
  }
}

// out[j] = sum_i A[i][j] B[i][j] (one thread per column, fixed order)
__global__ void coldot_kernel(int m, int k, const double* A, long lda, const double* B, long ldb, double* out) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < k; j += gridDim.x * blockDim.x) {
    double a = 0.0;
    for (int i = 0; i < m; ++i) a = fma(A[(long)i * lda + j], B[(long)i * ldb + j], a);
    out[j] = a;
  }
}

}  // namespace

void kkt_combine(hipStream_t s, long e, const KktCoef& c, const double* zM, const double* zK, double* y) {
  if (e <= 0) return;
  kkt_combine_kernel<double><<<grid_for(e), 256, 0, s>>>(e, c.k02, c.m11, c.m12, c.k20, c.m21, zM, zK, y);
  IGA_HIP(hipGetLastError());
}

template <typename T>
static void combine_blocks_launch(hipStream_t s, long e, int nblk, const int* toff, const int* src,
                                  const double* coef, const T* z, T* y) {
  if (e <= 0 || nblk <= 0) return;
  require(nblk <= 65535, IGA_EINVAL, "combine_blocks: too many blocks");
  dim3 g((unsigned)std::min<long>((e + 255) / 256, 1024), nblk);
  combine_blocks_kernel<T><<<g, 256, 0, s>>>(e, toff, src, coef, z, y);
  IGA_HIP(hipGetLastError());
}

void combine_blocks(hipStream_t s, long e, int nblk, const int* toff, const int* src, const double* coef,
                    const double* z, double* y) {
  combine_blocks_launch<double>(s, e, nblk, toff, src, coef, z, y);
}

void combine_blocks_f32(hipStream_t s, long e, int nblk, const int* toff, const int* src, const double* coef,
                        const float* z, float* y) {
  combine_blocks_launch<float>(s, e, nblk, toff, src, coef, z, y);
}

void fd_solve_time(hipStream_t s, int r0, int n, int r1, int nt, const double* lamL, const double* lamN,
                   const double* lamR, double beta, double tau, double* v, double* work) {
  const long e = (long)r0 * n * r1;
  if (e <= 0 || nt <= 0) return;
  fd_solve_time_kernel<<<grid_for(e), 256, 0, s>>>(r0, n, r1, nt, lamL, lamN, lamR, beta, tau, v, work);
  IGA_HIP(hipGetLastError());
}

void fill_segments(hipStream_t s, int nseg, long maxlen, const Segment* dev_seg, double* base) {
  if (nseg <= 0 || maxlen <= 0) return;
  require(nseg <= 65535, IGA_EINVAL, "fill_segments: too many segments");
  dim3 g((unsigned)std::min<long>((maxlen + 255) / 256, 1024), nseg);
  fill_segments_kernel<double><<<g, 256, 0, s>>>(dev_seg, base);
  IGA_HIP(hipGetLastError());
}
void fill_segments_f32(hipStream_t s, int nseg, long maxlen, const Segment* dev_seg, float* base) {
  if (nseg <= 0 || maxlen <= 0) return;
  require(nseg <= 65535, IGA_EINVAL, "fill_segments: too many segments");
  dim3 g((unsigned)std::min<long>((maxlen + 255) / 256, 1024), nseg);
  fill_segments_kernel<float><<<g, 256, 0, s>>>(dev_seg, base);
  IGA_HIP(hipGetLastError());
}
void combine_grouped(hipStream_t s, int nitem, long maxe, const CombineItem* dev_items, const double* zbase) {
  if (nitem <= 0 || maxe <= 0) return;
  require(nitem <= 65535, IGA_EINVAL, "combine_grouped: too many items");
  dim3 g((unsigned)std::min<long>((maxe + 255) / 256, 1024), nitem);
  combine_grouped_kernel<double><<<g, 256, 0, s>>>(dev_items, zbase);
  IGA_HIP(hipGetLastError());
}
void combine_grouped_f32(hipStream_t s, int nitem, long maxe, const CombineItem* dev_items, const float* zbase) {
  if (nitem <= 0 || maxe <= 0) return;
  require(nitem <= 65535, IGA_EINVAL, "combine_grouped: too many items");
  dim3 g((unsigned)std::min<long>((maxe + 255) / 256, 1024), nitem);
  combine_grouped_kernel<float><<<g, 256, 0, s>>>(dev_items, zbase);
  IGA_HIP(hipGetLastError());
}
void convert_segments(hipStream_t s, int nseg, long maxlen, const ConvSegment* dev_seg, bool to_f32) {
  if (nseg <= 0 || maxlen <= 0) return;
  require(nseg <= 65535, IGA_EINVAL, "convert_segments: too many segments");
  dim3 g((unsigned)std::min<long>((maxlen + 255) / 256, 1024), nseg);
  convert_segments_kernel<<<g, 256, 0, s>>>(dev_seg, to_f32 ? 1 : 0);
  IGA_HIP(hipGetLastError());
}

void scale3(hipStream_t s, long e, double s0, double s1, double s2, double* y) {
  if (e <= 0) return;
  scale3_kernel<<<grid_for(3 * e), 256, 0, s>>>(e, s0, s1, s2, y);
  IGA_HIP(hipGetLastError());
}

void fd_solve(hipStream_t s, int r0, int n, int r1, const double* lamL, const double* lamN,
              const double* lamR, double c, double g, double* v) {
  const long e = (long)r0 * n * r1;
  if (e <= 0) return;
  fd_solve_kernel<<<grid_for(e), 256, 0, s>>>(r0, n, r1, lamL, lamN, lamR, c, g, v);
  IGA_HIP(hipGetLastError());
}

void symmetrize(hipStream_t s, int nmat, int k, double* H, long stride) {
  if (k <= 1 || nmat <= 0) return;
  dim3 grid((unsigned)std::max<long>(1, std::min<long>(((long)k * k + 255) / 256, 1024)), nmat);
  symmetrize_kernel<<<grid, 256, 0, s>>>(k, H, stride);
  IGA_HIP(hipGetLastError());
}

template <typename T>
static void band_rank1_launch(hipStream_t s, int n, int b, long ncols, const T* A, const T* x, long ldx, T* y) {
  if (n <= 0 || ncols <= 0) return;
  require(n <= 65535 && b >= 1, IGA_EINVAL, "band_rank1: bad sizes");
  dim3 grid((unsigned)((ncols + 255) / 256), (unsigned)n);
  band_rank1_kernel<T><<<grid, 256, 0, s>>>(b, ncols, A, x, ldx, y);
  IGA_HIP(hipGetLastError());
}

template <typename T>
static void band_small_launch(hipStream_t s, int n, int b, int R0, int R1, long ncols, const T* A, const T* x,
                              long ldx, long ldd, T* y) {
  if (n <= 0 || ncols <= 0) return;
  require(n <= 65535 && b >= 1 && R0 >= 1 && R1 >= 1 && R1 <= 16, IGA_EINVAL, "band_small: bad sizes");
  require((ncols + 63) / 64 <= 0x7fffffffL, IGA_EINVAL, "band_small: too many columns");
  dim3 grid((unsigned)((ncols + 63) / 64), (unsigned)n);
  switch (R1) {
#define IGA_BAND_SMALL(r) \
  case r: band_small_kernel<T, r><<<grid, 64 * BAND_WAVES, 0, s>>>(b, R0, ncols, A, x, ldx, ldd, y); break;
    IGA_BAND_SMALL(1) IGA_BAND_SMALL(2) IGA_BAND_SMALL(3) IGA_BAND_SMALL(4) IGA_BAND_SMALL(5) IGA_BAND_SMALL(6)
    IGA_BAND_SMALL(7) IGA_BAND_SMALL(8) IGA_BAND_SMALL(9) IGA_BAND_SMALL(10) IGA_BAND_SMALL(11) IGA_BAND_SMALL(12)
    IGA_BAND_SMALL(13) IGA_BAND_SMALL(14) IGA_BAND_SMALL(15) IGA_BAND_SMALL(16)
#undef IGA_BAND_SMALL
  }
  IGA_HIP(hipGetLastError());
}

void band_small(hipStream_t s, int n, int b, int R0, int R1, long ncols, const double* A, const double* x, long ldx,
                long ldd, double* y) {
  band_small_launch<double>(s, n, b, R0, R1, ncols, A, x, ldx, ldd, y);
}

void band_small_f32(hipStream_t s, int n, int b, int R0, int R1, long ncols, const float* A, const float* x, long ldx,
                    long ldd, float* y) {
  band_small_launch<float>(s, n, b, R0, R1, ncols, A, x, ldx, ldd, y);
}

void band_rank1(hipStream_t s, int n, int b, long ncols, const double* A, const double* x, long ldx, double* y) {
  band_rank1_launch<double>(s, n, b, ncols, A, x, ldx, y);
}

void band_rank1_f32(hipStream_t s, int n, int b, long ncols, const float* A, const float* x, long ldx, float* y) {
  band_rank1_launch<float>(s, n, b, ncols, A, x, ldx, y);
}

void kkt_combine_f32(hipStream_t s, long e, const KktCoef& c, const float* zM, const float* zK, float* y) {
  if (e <= 0) return;
  kkt_combine_kernel<float><<<grid_for(e), 256, 0, s>>>(e, (float)c.k02, (float)c.m11, (float)c.m12,
                                                        (float)c.k20, (float)c.m21, zM, zK, y);
  IGA_HIP(hipGetLastError());
}

void core_product(hipStream_t s, int R0, int R1, int n, int p, const double* A, int r0, int r1,
                  const double* X, double* Y, double alpha, double beta) {
  const long total = (long)R0 * r0 * n * R1 * r1;
  if (total <= 0) return;
  core_product_kernel<<<grid_for(total), 256, 0, s>>>(R0, R1, n, p, A, r0, r1, X, Y, alpha, beta);
  IGA_HIP(hipGetLastError());
}

void copy2d(hipStream_t s, int m, int k, const double* in, long si, long sj, double* out, long ldo) {
  const long total = (long)m * k;
  if (total <= 0) return;
  copy2d_kernel<<<grid_for(total), 256, 0, s>>>(m, k, in, si, sj, out, ldo);
  IGA_HIP(hipGetLastError());
}

void diag_invsqrt(hipStream_t s, int k, const double* H, double* out) {
  diag_kernel<<<(k + 255) / 256, 256, 0, s>>>(k, H, k + 1, out, 1);
  IGA_HIP(hipGetLastError());
}
void diag_get(hipStream_t s, int k, const double* H, double* out) {
  diag_kernel<<<(k + 255) / 256, 256, 0, s>>>(k, H, k + 1, out, 0);
  IGA_HIP(hipGetLastError());
}
void vec_invsqrt(hipStream_t s, int k, const double* v, double* out) {
  diag_kernel<<<(k + 255) / 256, 256, 0, s>>>(k, v, 1, out, 1);
  IGA_HIP(hipGetLastError());
}
void scale_rows(hipStream_t s, int m, int k, const double* sc, double* A, long lda) {
  const long total = (long)m * k;
  if (total <= 0) return;
  scale_rows_kernel<<<(unsigned)std::min<long>((total + 255) / 256, 4096), 256, 0, s>>>(m, k, sc, A, lda);
  IGA_HIP(hipGetLastError());
}
void coldots(hipStream_t s, int m, int k, const double* A, long lda, const double* B, long ldb, double* out) {
  coldot_kernel<<<(k + 255) / 256, 256, 0, s>>>(m, k, A, lda, B, ldb, out);
  IGA_HIP(hipGetLastError());
}

// FP64 products run on the matrix cores: the (ko, k) contraction index is the two-level K
// of gemm2 (outer stride s*ko, inner stride s*k).
void gemm(hipStream_t s, const Gemm& g, double* work, size_t work_len) {
  if (g.M <= 0 || g.N <= 0) return;
  Gemm2 d;
  d.M = g.M; d.N = g.N; d.K = g.K * g.Kout; d.K2 = std::max(g.K, 1);
  d.A = g.A; d.sAm2 = g.sAm; d.sAk1 = g.sAko; d.sAk2 = g.sAk;
  d.B = g.B; d.sBk1 = g.sBko; d.sBk2 = g.sBk; d.sBn2 = g.sBn;
  d.C = g.C; d.sCm2 = g.sCm; d.sCn2 = g.sCn;
  d.nb1 = g.nb1; d.nb2 = g.nb2;
  d.sAb1 = g.sAb1; d.sAb2 = g.sAb2; d.sBb1 = g.sBb1; d.sBb2 = g.sBb2; d.sCb1 = g.sCb1; d.sCb2 = g.sCb2;
  d.alpha = g.alpha; d.beta = g.beta;
  if (d.K == 0) {
    // empty contraction: C = beta C
    require(g.nb1 == 1 && g.nb2 == 1, IGA_EINVAL, "gemm: empty batched contraction");
    launch_gemm<double>(s, g);
    return;
  }
  gemm2(s, d, work, work_len);
}

void gemm_rm(hipStream_t s, int M, int N, int K, const double* A, long lda, bool tA,
             const double* B, long ldb, bool tB, double* C, long ldc, double alpha, double beta,
             double* work, size_t work_len) {
  Gemm g;
  g.M = M; g.N = N; g.K = K;
  g.A = A; g.sAm = tA ? 1 : lda; g.sAk = tA ? lda : 1;
  g.B = B; g.sBk = tB ? 1 : ldb; g.sBn = tB ? ldb : 1;
  g.C = C; g.sCm = ldc; g.sCn = 1;
  g.alpha = alpha; g.beta = beta;
  gemm(s, g, work, work_len);
}

void axpby(hipStream_t s, long n, double a, const double* x, double b, double* y) {
  if (n <= 0) return;
  axpby_kernel<<<grid_for(n), 256, 0, s>>>(n, a, x, b, y);
  IGA_HIP(hipGetLastError());
}
void fill(hipStream_t s, long n, double v, double* y) {
  if (n <= 0) return;
  fill_kernel<double><<<grid_for(n), 256, 0, s>>>(n, v, y);
  IGA_HIP(hipGetLastError());
}
void fill_f32(hipStream_t s, long n, float v, float* y) {
  if (n <= 0) return;
  fill_kernel<float><<<grid_for(n), 256, 0, s>>>(n, v, y);
  IGA_HIP(hipGetLastError());
}
void scale(hipStream_t s, long n, double a, double* y) {
  if (n <= 0) return;
  scale_kernel<<<grid_for(n), 256, 0, s>>>(n, a, y);
  IGA_HIP(hipGetLastError());
}
void to_f32(hipStream_t s, long n, const double* x, float* y) {
  if (n <= 0) return;
  to_f32_kernel<<<grid_for(n), 256, 0, s>>>(n, x, y);
  IGA_HIP(hipGetLastError());
}
void to_f64(hipStream_t s, long n, const float* x, double* y) {
  if (n <= 0) return;
  to_f64_kernel<<<grid_for(n), 256, 0, s>>>(n, x, y);
  IGA_HIP(hipGetLastError());
}

void permute4(hipStream_t s, const double* in, const int dims[4], const int perm[4], double* out) {
  Perm4 P;
  long stride[4];
  stride[3] = 1;
  for (int k = 2; k >= 0; --k) stride[k] = stride[k + 1] * dims[k + 1];
  long total = 1;
  for (int k = 0; k < 4; ++k) {
    P.od[k] = dims[perm[k]];
    P.is[k] = stride[perm[k]];
    total *= dims[k];
  }
  if (total <= 0) return;
  permute4_kernel<<<grid_for(total), 256, 0, s>>>(in, out, P, total);
  IGA_HIP(hipGetLastError());
}

int reduce_partials() { return RED_BLOCKS; }

void dot(hipStream_t s, long n, const double* x, const double* y, double* partial, double* out) {
  dot_partial<<<RED_BLOCKS, 256, 0, s>>>(n, x, y, partial);
  sum_partials<<<1, 256, 0, s>>>(RED_BLOCKS, 1, partial, out);
  IGA_HIP(hipGetLastError());
}

void multidot(hipStream_t s, long n, int k, const double* V, long ldv, const double* w,
              double* partial, double* h) {
  if (k <= 0) return;
  require(k <= 64, IGA_EINVAL, "multidot: k > 64");
  multidot_partial<<<dim3(MD_CHUNKS, k), 256, 0, s>>>(n, V, ldv, w, partial);
  sum_partials<<<k, 256, 0, s>>>(MD_CHUNKS, k, partial, h);
  IGA_HIP(hipGetLastError());
}

void multiaxpy(hipStream_t s, long n, int k, const double* V, long ldv, const double* coef,
               double sign, double* w) {
  if (k <= 0) return;
  require(k <= 64, IGA_EINVAL, "multiaxpy: k > 64");
  multiaxpy_kernel<<<grid_for(n), 256, 0, s>>>(n, k, V, ldv, coef, sign, w);
  IGA_HIP(hipGetLastError());
}

void colnorms(hipStream_t s, int m, int k, const double* A, long lda, double* out) {
  if (k <= 0) return;
  colnorm_kernel<<<k, 256, 0, s>>>(m, k, A, lda, out);
  IGA_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace iga
