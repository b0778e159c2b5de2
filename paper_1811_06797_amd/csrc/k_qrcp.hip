// Column-pivoted Householder QR of a tall m x k matrix, stopped once the columns not yet chosen
// have a Frobenius norm (of their rows below the factored ones) at or below a threshold: the
// QR step in front of the truncation SVD (the unfolding is factored, then only the small
// triangular factor goes to the SVD; Sec. 5, eqs. svd1-svd2). Greedy pivoting (the column with
// the largest remaining norm) makes the factor rank revealing: the part left out is exactly
// the remaining block.
//
// Layout: the working copy W holds column c contiguously at W + c * ldw (m entries, reflected in
// place); V holds reflector t in row t (entries t..m-1); R is rmax x k row-major over the
// original column indices, zero on entry; the squared remaining norms are recomputed exactly at
// every step, -1 once a column is chosen.
//
// One step is one launch with one workgroup per column: every workgroup finds the same argmax
// and the same remaining norm (fixed reduction order), builds the reflector from the pivot
// column, which no workgroup writes in that step, and reflects its own column. The norms are
// double-buffered (read one array, write the other), so no workgroup reads a value another one
// writes in the same launch. (Modified Gram-Schmidt with reorthogonalisation needs three
// dependent launches per step, and a chunk of steps in one cooperative launch with grid-wide
// barriers measured five times slower per step than those launches.)
#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

constexpr int QT = 256;       // threads per workgroup of the pivot and update kernels
constexpr int QWAVES = QT / 64;

__device__ inline double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// sum over the workgroup (QT threads), the same value in every thread
__device__ double block_total(double v) {
  __shared__ double sh[QWAVES];
  v = wave_sum(v);
  if (threadIdx.x % 64 == 0) sh[threadIdx.x / 64] = v;
  __syncthreads();
  double r = 0.0;
  for (int w = 0; w < QWAVES; ++w) r += sh[w];
  __syncthreads();
  return r;
}

// argmax of nrm2 over the columns not yet chosen (the smallest index on ties) and the sum of
// their squared norms, identical in every workgroup
__device__ void pivot_of(int k, const double* nrm2, int& p, double& tail) {
  __shared__ double bv[QT], sv[QT];
  __shared__ int bi[QT];
  const int tid = threadIdx.x;
  double best = -1.0, sum = 0.0;
  int bidx = -1;
  for (int c = tid; c < k; c += QT) {
    const double v = nrm2[c];
    if (v >= 0.0) {
      sum += v;
      if (v > best) { best = v; bidx = c; }
    }
  }
  bv[tid] = best; bi[tid] = bidx; sv[tid] = sum;
  __syncthreads();
  for (int w = QT / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const double ov = bv[tid + w];
      const int oi = bi[tid + w];
      if (ov > bv[tid] || (ov == bv[tid] && oi >= 0 && (bi[tid] < 0 || oi < bi[tid]))) { bv[tid] = ov; bi[tid] = oi; }
      sv[tid] += sv[tid + w];
    }
    __syncthreads();
  }
  p = bi[0];
  tail = sv[0];
  __syncthreads();
}

// squared column norms, one workgroup per column
__global__ __launch_bounds__(QT) void qrcp_init_kernel(int m, const double* W, long ldw, double* nrm2) {
  const double* w = W + (long)blockIdx.x * ldw;
  double acc = 0.0;
  for (int x = threadIdx.x; x < m; x += QT) acc = fma(w[x], w[x], acc);
  acc = block_total(acc);
  if (threadIdx.x == 0) nrm2[blockIdx.x] = acc;
}

// Step j: one workgroup per column c. ctrl[0]: done flag, ctrl[2]: number of columns chosen.
// nin[c] = ||W[c][j:m)||^2 (-1 once chosen) is only read and nout only written, so the argmax
// that every workgroup takes first sees the same values in all of them. The reflector
// H = I - beta v v^T maps the pivot column's rows j..m-1 to alpha e_j, alpha = -sign(x_j) ||x||;
// v = x - alpha e_j is built by every workgroup from the pivot column, which nobody writes in
// this step. Column c's rows j..m-1 are reflected in place; row j becomes R[j][c] and the new
// squared norm of rows j+1..m-1 goes to nout[c]. With RC > 0 (m <= QT RC) the column stays in
// registers between the dot product and the update.
template <int RC>
__global__ __launch_bounds__(QT) void qrhh_step_kernel(int m, int k, int j, double* W, long ldw, const double* nin,
                                                       double* nout, double* V, double* beta, double* R,
                                                       int* pivots, int* ctrl, double thr2) {
  if (ctrl[0]) return;
  int p;
  double tail;
  pivot_of(k, nin, p, tail);
  if (p < 0 || !(tail > thr2)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctrl[0] = 1;
      ctrl[2] = j;
    }
    return;
  }
  const double* a = W + (long)p * ldw;
  const double x0 = a[j], xn = sqrt(nin[p]);
  const double alpha = x0 >= 0.0 ? -xn : xn;
  const double v0 = x0 - alpha;
  const double vn2 = 2.0 * xn * (xn + fabs(x0));  // ||v||^2 without cancellation
  const double bt = vn2 > 0.0 ? 2.0 / vn2 : 0.0;
  const int c = blockIdx.x;
  if (c == p) {
    for (int x = j + threadIdx.x; x < m; x += QT) V[(long)j * m + x] = x == j ? v0 : a[x];
    if (threadIdx.x == 0) {
      R[(long)j * k + p] = alpha;
      beta[j] = bt;
      pivots[j] = p;
      nout[p] = -1.0;
    }
    return;
  }
  if (nin[c] < 0.0) {
    if (threadIdx.x == 0) nout[c] = -1.0;
    return;
  }
  double* w = W + (long)c * ldw;
  auto vat = [&](int x) { return x == j ? v0 : a[x]; };
  double acc = 0.0, n2 = 0.0;
  if constexpr (RC > 0) {
    double wr[RC];
#pragma unroll
    for (int u = 0; u < RC; ++u) {
      const int x = threadIdx.x + u * QT;
      const bool in = x >= j && x < m;
      wr[u] = in ? w[x] : 0.0;
      acc = fma(in ? vat(x) : 0.0, wr[u], acc);
    }
    const double g = bt * block_total(acc);
#pragma unroll
    for (int u = 0; u < RC; ++u) {
      const int x = threadIdx.x + u * QT;
      if (x >= j && x < m) {
        const double v = fma(-g, vat(x), wr[u]);
        w[x] = v;
        if (x == j)
          R[(long)j * k + c] = v;
        else
          n2 = fma(v, v, n2);
      }
    }
  } else {
    for (int x = j + threadIdx.x; x < m; x += QT) acc = fma(vat(x), w[x], acc);
    const double g = bt * block_total(acc);
    for (int x = j + threadIdx.x; x < m; x += QT) {
      const double v = fma(-g, vat(x), w[x]);
      w[x] = v;
      if (x == j)
        R[(long)j * k + c] = v;
      else
        n2 = fma(v, v, n2);
    }
  }
  n2 = block_total(n2);
  if (threadIdx.x == 0) nout[c] = n2;
}

// Y <- H_0 H_1 ... H_{rc-1} Y for the columns of Y (column col at Y + col * m, m entries), one
// workgroup per column: the reflectors applied from the last to the first.
template <int RC>
__global__ __launch_bounds__(QT) void qrhh_apply_kernel(int m, int rc, const double* V, const double* beta,
                                                        double* Y) {
  double* y = Y + (long)blockIdx.x * m;
  if constexpr (RC > 0) {
    double yr[RC];
#pragma unroll
    for (int u = 0; u < RC; ++u) {
      const int x = threadIdx.x + u * QT;
      yr[u] = x < m ? y[x] : 0.0;
    }
    for (int t = rc - 1; t >= 0; --t) {
      const double* v = V + (long)t * m;
      double acc = 0.0;
#pragma unroll
      for (int u = 0; u < RC; ++u) {
        const int x = threadIdx.x + u * QT;
        if (x >= t && x < m) acc = fma(v[x], yr[u], acc);
      }
      const double g = beta[t] * block_total(acc);
#pragma unroll
      for (int u = 0; u < RC; ++u) {
        const int x = threadIdx.x + u * QT;
        if (x >= t && x < m) yr[u] = fma(-g, v[x], yr[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < RC; ++u) {
      const int x = threadIdx.x + u * QT;
      if (x < m) y[x] = yr[u];
    }
  } else {
    for (int t = rc - 1; t >= 0; --t) {
      const double* v = V + (long)t * m;
      double acc = 0.0;
      for (int x = t + threadIdx.x; x < m; x += QT) acc = fma(v[x], y[x], acc);
      const double g = beta[t] * block_total(acc);
      for (int x = t + threadIdx.x; x < m; x += QT) y[x] = fma(-g, v[x], y[x]);
      __syncthreads();
    }
  }
}

}  // namespace

void qrcp_init(hipStream_t st, int m, int k, const double* W, long ldw, double* nrm2) {
  qrcp_init_kernel<<<k, QT, 0, st>>>(m, W, ldw, nrm2);
  IGA_HIP(hipGetLastError());
}

void qrhh_step(hipStream_t st, int m, int k, int j, double* W, long ldw, const double* nin, double* nout,
               double* V, double* beta, double* R, int* pivots, int* ctrl, double thr2) {
  if (m <= 8 * QT)
    qrhh_step_kernel<8><<<k, QT, 0, st>>>(m, k, j, W, ldw, nin, nout, V, beta, R, pivots, ctrl, thr2);
  else if (m <= 16 * QT)
    qrhh_step_kernel<16><<<k, QT, 0, st>>>(m, k, j, W, ldw, nin, nout, V, beta, R, pivots, ctrl, thr2);
  else if (m <= 48 * QT)
    qrhh_step_kernel<48><<<k, QT, 0, st>>>(m, k, j, W, ldw, nin, nout, V, beta, R, pivots, ctrl, thr2);
  else
    qrhh_step_kernel<0><<<k, QT, 0, st>>>(m, k, j, W, ldw, nin, nout, V, beta, R, pivots, ctrl, thr2);
  IGA_HIP(hipGetLastError());
}

void qrhh_apply(hipStream_t st, int m, int rc, const double* V, const double* beta, int ncol, double* Y) {
  if (ncol <= 0 || rc <= 0) return;
  if (m <= 8 * QT)
    qrhh_apply_kernel<8><<<ncol, QT, 0, st>>>(m, rc, V, beta, Y);
  else if (m <= 16 * QT)
    qrhh_apply_kernel<16><<<ncol, QT, 0, st>>>(m, rc, V, beta, Y);
  else if (m <= 48 * QT)
    qrhh_apply_kernel<48><<<ncol, QT, 0, st>>>(m, rc, V, beta, Y);
  else
    qrhh_apply_kernel<0><<<ncol, QT, 0, st>>>(m, rc, V, beta, Y);
  IGA_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace iga
