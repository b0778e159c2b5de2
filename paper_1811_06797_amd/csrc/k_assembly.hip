// Kernels of the low-rank assembly (Sections 2 and 3): B-spline tabulation by
// the Cox-de Boor recursion, the geometry weights omega and Q on a tensor grid,
// and the Gauss quadrature of the banded univariate factors.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

constexpr int MAXDEG = 15;

// Span s with t[s] <= x < t[s+1]; the last non-empty span is closed at its right end.
__device__ int find_span(const double* t, int nk, int deg, double x) {
  const int nb = nk - deg - 1;
  int lo = deg, hi = nb;  // valid spans for an open knot vector: deg .. nb-1
  if (x >= t[nb]) {
    int s = nb - 1;
    while (s > deg && !(t[s] < t[s + 1])) --s;
    return s;
  }
  if (x <= t[deg]) return deg;
  while (hi - lo > 1) {
    const int mid = (lo + hi) / 2;
    if (x < t[mid]) hi = mid; else lo = mid;
  }
  return lo;
}

__global__ void tabulate_kernel(const double* t, int nk, int deg, const double* pts, int np,
                                int deriv, double* out) {
  const int nb = nk - deg - 1;
  for (int ip = blockIdx.x * blockDim.x + threadIdx.x; ip < np; ip += gridDim.x * blockDim.x) {
    const double x = pts[ip];
    const int s = find_span(t, nk, deg, x);
    // val[j] holds beta_{s-k+j, k}(x), j = 0..k, built up degree by degree
    double val[MAXDEG + 1], nv[MAXDEG + 1];
    val[0] = 1.0;
    const int top = deriv ? deg - 1 : deg;
    for (int k = 1; k <= top; ++k) {
      for (int j = 0; j <= k; ++j) {
        const int i = s - k + j;
        const double left = (j >= 1) ? val[j - 1] : 0.0;   // beta_{i, k-1}
        const double right = (j <= k - 1) ? val[j] : 0.0;  // beta_{i+1, k-1}
        const double d1 = t[i + k] - t[i];
        const double d2 = t[i + k + 1] - t[i + 1];
        double v = 0.0;
        if (d1 != 0.0) v += (x - t[i]) / d1 * left;
        if (d2 != 0.0) v += (t[i + k + 1] - x) / d2 * right;
        nv[j] = v;
      }
      for (int j = 0; j <= k; ++j) val[j] = nv[j];
    }
    double* row = out + (long)ip * nb;
    for (int i = 0; i < nb; ++i) row[i] = 0.0;
    if (!deriv) {
      for (int j = 0; j <= deg; ++j) row[s - deg + j] = val[j];
    } else {
      // beta'_{i,p} = p/(t_{i+p}-t_i) beta_{i,p-1} - p/(t_{i+p+1}-t_{i+1}) beta_{i+1,p-1}
      for (int j = 0; j <= deg; ++j) {
        const int i = s - deg + j;
        const double bl = (j >= 1) ? val[j - 1] : 0.0;
        const double br = (j <= deg - 1) ? val[j] : 0.0;
        const double d1 = t[i + deg] - t[i];
        const double d2 = t[i + deg + 1] - t[i + 1];
        double v = 0.0;
        if (d1 != 0.0) v += deg / d1 * bl;
        if (d2 != 0.0) v -= deg / d2 * br;
        row[i] = v;
      }
    }
  }
}

struct GeoArgs {
  int np[3], ncp[3];
  const double* Bv[3];
  const double* Bd[3];
  const double* ctrl;
  double* out;
  int* bad;
};

// One thread per grid point: grad G from the control net, then
// omega = |det J|, Q = (J^T J)^{-1} omega = adj(J^T J) / |det J|.
__global__ __launch_bounds__(256) void geometry_kernel(GeoArgs a) {
  const long total = (long)a.np[0] * a.np[1] * a.np[2];
  const long stride_w = total;
  const int n0 = a.ncp[0], n1 = a.ncp[1], n2 = a.ncp[2];
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int x3 = idx % a.np[2];
    const int x2 = (idx / a.np[2]) % a.np[1];
    const int x1 = idx / ((long)a.np[2] * a.np[1]);
    const double* bv0 = a.Bv[0] + (long)x1 * n0;
    const double* bd0 = a.Bd[0] + (long)x1 * n0;
    const double* bv1 = a.Bv[1] + (long)x2 * n1;
    const double* bd1 = a.Bd[1] + (long)x2 * n1;
    const double* bv2 = a.Bv[2] + (long)x3 * n2;
    const double* bd2 = a.Bd[2] + (long)x3 * n2;
    double J[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
    for (int i = 0; i < n0; ++i) {
      const double v0 = bv0[i], d0 = bd0[i];
      if (v0 == 0.0 && d0 == 0.0) continue;
      for (int j = 0; j < n1; ++j) {
        const double v1 = bv1[j], d1 = bd1[j];
        if (v1 == 0.0 && d1 == 0.0) continue;
        for (int k = 0; k < n2; ++k) {
          const double v2 = bv2[k], d2 = bd2[k];
          if (v2 == 0.0 && d2 == 0.0) continue;
          const double w0 = d0 * v1 * v2, w1 = v0 * d1 * v2, w2 = v0 * v1 * d2;
          const long c = ((long)i * n1 + j) * n2 + k;
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            const double C = a.ctrl[ax * (long)n0 * n1 * n2 + c];
            J[ax][0] = fma(C, w0, J[ax][0]);
            J[ax][1] = fma(C, w1, J[ax][1]);
            J[ax][2] = fma(C, w2, J[ax][2]);
          }
        }
      }
    }
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                       J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                       J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    if (!(det > 0.0)) atomicAdd(a.bad, 1);
    double S[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) S[p][q] = J[0][p] * J[0][q] + J[1][p] * J[1][q] + J[2][p] * J[2][q];
    const double om = fabs(det);
    const double inv = om > 0.0 ? 1.0 / om : 0.0;
    const double a00 = S[1][1] * S[2][2] - S[1][2] * S[2][1];
    const double a01 = S[0][2] * S[2][1] - S[0][1] * S[2][2];
    const double a02 = S[0][1] * S[1][2] - S[0][2] * S[1][1];
    const double a11 = S[0][0] * S[2][2] - S[0][2] * S[2][0];
    const double a12 = S[0][2] * S[1][0] - S[0][0] * S[1][2];
    const double a22 = S[0][0] * S[1][1] - S[0][1] * S[1][0];
    double* o = a.out + idx;
    o[0] = om;
    o[1 * stride_w] = a00 * inv;
    o[2 * stride_w] = a01 * inv;
    o[3 * stride_w] = a02 * inv;
    o[4 * stride_w] = a11 * inv;
    o[5 * stride_w] = a12 * inv;
    o[6 * stride_w] = a22 * inv;
  }
}

__global__ __launch_bounds__(256) void factor_kernel(int S, int n, int p, int nel, int nq,
                                                     const double* Bi, const double* Bj,
                                                     const double* w, const double* E,
                                                     double* out) {
  const int b = 2 * p + 1;
  const int N = n + 2;
  const int Q = nel * nq;
  const long total = (long)S * n * b;
  for (long idx = blockIdx.x * (long)blockDim.x + threadIdx.x; idx < total;
       idx += (long)gridDim.x * blockDim.x) {
    const int o = idx % b;
    const int i = (idx / b) % n;
    const int s = idx / ((long)b * n);
    const int I = i + 1;          // full index of the interior row
    const int Jf = I + o - p;     // full index of the column
    double acc = 0.0;
    if (Jf >= 1 && Jf <= N - 2) {
      const int e0 = max(max(I, Jf) - p, 0);
      const int e1 = min(min(I, Jf), nel - 1);
      const double* Es = E + (long)s * Q;
      for (int e = e0; e <= e1; ++e)
        for (int t = 0; t < nq; ++t) {
          const int q = e * nq + t;
          acc += w[q] * Bi[(long)q * N + I] * Bj[(long)q * N + Jf] * Es[q];
        }
    }
    out[idx] = acc;
  }
}

unsigned grid_for(long n) { return (unsigned)std::max<long>(1, std::min<long>((n + 255) / 256, 8192)); }

}  // namespace

void bspline_tabulate(hipStream_t s, const double* knots, int nknots, int deg, const double* pts,
                      int np, int deriv, double* out) {
  require(deg >= 0 && deg <= MAXDEG, IGA_EINVAL, "degree out of range (0..15)");
  require(!(deriv && deg == 0), IGA_EINVAL, "derivative of degree 0");
  if (np <= 0) return;
  tabulate_kernel<<<grid_for(np), 256, 0, s>>>(knots, nknots, deg, pts, np, deriv, out);
  IGA_HIP(hipGetLastError());
}

void geometry_weights(hipStream_t s, const int np[3], const int ncp[3], const double* const Bv[3],
                      const double* const Bd[3], const double* ctrl, double* out, int* bad) {
  GeoArgs a;
  for (int d = 0; d < 3; ++d) {
    a.np[d] = np[d]; a.ncp[d] = ncp[d]; a.Bv[d] = Bv[d]; a.Bd[d] = Bd[d];
  }
  a.ctrl = ctrl; a.out = out; a.bad = bad;
  const long total = (long)np[0] * np[1] * np[2];
  geometry_kernel<<<grid_for(total), 256, 0, s>>>(a);
  IGA_HIP(hipGetLastError());
}

void factor_quadrature(hipStream_t s, int S, int n, int p, int nel, int nq, const double* Bi,
                       const double* Bj, const double* w, const double* E, double* out) {
  const long total = (long)S * n * (2 * p + 1);
  if (total <= 0) return;
  factor_kernel<<<grid_for(total), 256, 0, s>>>(S, n, p, nel, nq, Bi, Bj, w, E, out);
  IGA_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace iga
