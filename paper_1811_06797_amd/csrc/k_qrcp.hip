// Column-pivoted QR of a tall m x k matrix by modified Gram-Schmidt with one
// reorthogonalisation of each new direction, stopped once the columns not yet chosen have a
// Frobenius norm at or below a threshold: the QR step in front of the truncation SVD (the
// unfolding is factored, then only the small triangular factor goes to the SVD; Sec. 5,
// eqs. svd1-svd2). Greedy pivoting (the column with the largest remaining norm) makes the
// factor rank revealing: the part left out is exactly the remaining columns.
//
// Layout: the working copy W holds column c contiguously at W + c * ldw (m entries); Q holds
// direction t as row t (m entries); R is rmax x k row-major over the original column indices;
// nrm2[c] is the squared norm of column c's remaining part, -1 once c is chosen.
//
// One step j is three launches: pivot (every workgroup finds the same argmax and the same
// remaining norm, in a fixed reduction order; the dots of the chosen column with the earlier
// directions), form (the column minus its components along the earlier directions, with
// per-workgroup partial norms) and update (normalise, project every remaining column, store
// its coefficient in R and recompute its remaining norm). The step index is a launch argument,
// so no workgroup ever reads a counter that another one writes in the same launch. (A chunk of
// steps in one cooperative launch, the phases separated by grid-wide barriers, measured five
// times slower per step than the three launches.)
#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

constexpr int QT = 256;       // threads per workgroup of the pivot and update kernels
constexpr int QWAVES = QT / 64;
constexpr int FT = 64;        // threads per workgroup of the form kernel (one element each)

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

// ctrl[0]: done flag, ctrl[1]: pivot of the current step, ctrl[2]: number of columns chosen.
// Workgroup t (t < j) forms s_t = q_t . a_p; launched with max(j, 1) workgroups.
__global__ __launch_bounds__(QT) void qrcp_pivot_kernel(int m, int k, int j, const double* W, long ldw,
                                                        const double* nrm2, const double* Q, double* s,
                                                        int* ctrl, double thr2) {
  if (ctrl[0]) return;
  int p;
  double tail;
  pivot_of(k, nrm2, p, tail);
  if (p < 0 || !(tail > thr2)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      ctrl[0] = 1;
      ctrl[2] = j;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) ctrl[1] = p;
  const int t = blockIdx.x;
  if (t >= j) return;
  const double* a = W + (long)p * ldw;
  const double* q = Q + (long)t * m;
  double acc = 0.0;
  for (int x = threadIdx.x; x < m; x += QT) acc = fma(q[x], a[x], acc);
  acc = block_total(acc);
  if (threadIdx.x == 0) s[t] = acc;
}

// qraw = a_p - sum_{t<j} s_t q_t; part[block] = its partial squared norm
__global__ __launch_bounds__(FT) void qrcp_form_kernel(int m, int j, const double* W, long ldw, const double* Q,
                                                       const double* s, const int* ctrl, double* qraw,
                                                       double* part) {
  if (ctrl[0]) return;
  const int p = ctrl[1];
  const int x = blockIdx.x * FT + threadIdx.x;
  double v = 0.0;
  if (x < m) {
    // four independent partial sums keep several loads in flight
    double a0 = W[(long)p * ldw + x], a1 = 0.0, a2 = 0.0, a3 = 0.0;
    int t = 0;
    for (; t + 4 <= j; t += 4) {
      a0 = fma(-s[t], Q[(long)t * m + x], a0);
      a1 = fma(-s[t + 1], Q[(long)(t + 1) * m + x], a1);
      a2 = fma(-s[t + 2], Q[(long)(t + 2) * m + x], a2);
      a3 = fma(-s[t + 3], Q[(long)(t + 3) * m + x], a3);
    }
    for (; t < j; ++t) a0 = fma(-s[t], Q[(long)t * m + x], a0);
    v = (a0 + a1) + (a2 + a3);
    qraw[x] = v;
  }
  const double tot = wave_sum(v * v);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// one workgroup per column: normalise the new direction (every workgroup its slice of rows),
// project the column, store its coefficient and its new remaining norm
__global__ __launch_bounds__(QT) void qrcp_update_kernel(int m, int k, int j, double* W, long ldw, double* Q,
                                                         const double* s, const double* qraw,
                                                         const double* part, int nparts, double* R,
                                                         double* nrm2, int* pivots, const int* ctrl) {
  if (ctrl[0]) return;
  const int p = ctrl[1];
  // every workgroup sums the partial norms in the same order
  double a = 0.0;
  for (int b = threadIdx.x; b < nparts; b += QT) a += part[b];
  // block_total's order is fixed, so all workgroups get the same rjj
  const double rjj = sqrt(block_total(a));
  const double inv = rjj > 0.0 ? 1.0 / rjj : 0.0;
  {
    const int per = (m + gridDim.x - 1) / gridDim.x;
    const int x0 = blockIdx.x * per, x1 = min(m, x0 + per);
    for (int x = x0 + threadIdx.x; x < x1; x += QT) Q[(long)j * m + x] = qraw[x] * inv;
  }
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < j; t += QT) R[(long)t * k + p] += s[t];
    if (threadIdx.x == 0) {
      R[(long)j * k + p] = rjj;
      nrm2[p] = -1.0;
      pivots[j] = p;
    }
  }
  const int c = blockIdx.x;
  if (c == p || nrm2[c] < 0.0) return;
  double* w = W + (long)c * ldw;
  double acc = 0.0;
  for (int x = threadIdx.x; x < m; x += QT) acc = fma(qraw[x], w[x], acc);
  const double r = block_total(acc) * inv;
  const double g = r * inv;
  double n2 = 0.0;
  for (int x = threadIdx.x; x < m; x += QT) {
    const double v = fma(-g, qraw[x], w[x]);
    w[x] = v;
    n2 = fma(v, v, n2);
  }
  n2 = block_total(n2);
  if (threadIdx.x == 0) {
    R[(long)j * k + c] = r;
    nrm2[c] = n2;
  }
}

}  // namespace

int qrcp_form_blocks(int m) { return (m + FT - 1) / FT; }

void qrcp_init(hipStream_t st, int m, int k, const double* W, long ldw, double* nrm2) {
  qrcp_init_kernel<<<k, QT, 0, st>>>(m, W, ldw, nrm2);
  IGA_HIP(hipGetLastError());
}

void qrcp_step(hipStream_t st, int m, int k, int j, double* W, long ldw, double* nrm2, double* Q, double* R,
               double* s, double* qraw, double* part, int* pivots, int* ctrl, double thr2) {
  const int nparts = qrcp_form_blocks(m);
  qrcp_pivot_kernel<<<std::max(j, 1), QT, 0, st>>>(m, k, j, W, ldw, nrm2, Q, s, ctrl, thr2);
  IGA_HIP(hipGetLastError());
  qrcp_form_kernel<<<nparts, FT, 0, st>>>(m, j, W, ldw, Q, s, ctrl, qraw, part);
  IGA_HIP(hipGetLastError());
  qrcp_update_kernel<<<k, QT, 0, st>>>(m, k, j, W, ldw, Q, s, qraw, part, nparts, R, nrm2, pivots, ctrl);
  IGA_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace iga
