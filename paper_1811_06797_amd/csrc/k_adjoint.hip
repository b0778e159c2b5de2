// Kernels of the reduced-cost gradient with respect to the geometry control points.
//
// With the Lagrangian L = J + lambda^T (K y - M u) of the control problem (Section 4), the
// derivative of the reduced cost along a change of the geometry is that of L at the
// solution. M and K depend on the geometry only through the weights omega and q_kl
// interpolated in the space S~ (Section 3), so the gradient is a quadrature of
//   P_w  = e^2 / 2 + beta u^2 / 2 - lambda u           (e = y - yhat), against d omega~,
//   P_kl = (d_l lambda)(d_k y)                          against d q~_kl,
// pulled back through the interpolation to the Greville grid and then through
// omega = |det J| and Q = omega J^{-1} J^{-T} to J = grad G, and to the control points.
#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

// f: 9 fields of npts points, fstride apart: e, u, lambda, d0 lambda, d1 lambda, d2 lambda,
// d0 y, d1 y, d2 y. P: 10 outputs, pstride apart: P_w, then P_kl at 1 + 3 k + l.
__global__ __launch_bounds__(256) void pointwise_kernel(long npts, const double* f, long fstride, double beta,
                                                        double* P, long pstride) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < npts; i += (long)gridDim.x * blockDim.x) {
    const double e = f[i], u = f[fstride + i], lam = f[2 * fstride + i];
    double dl[3], dy[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dl[c] = f[(3 + c) * fstride + i];
      dy[c] = f[(6 + c) * fstride + i];
    }
    P[i] = 0.5 * e * e + 0.5 * beta * u * u - lam * u;
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int l = 0; l < 3; ++l) P[(1 + 3 * kk + l) * pstride + i] = dl[l] * dy[kk];
  }
}

struct GeoAdjArgs {
  int np[3], ncp[3];
  const double* Bv[3];
  const double* Bd[3];
  const double* ctrl;
  const double* H;  // [10][G]: adjoint weights of omega and of q_kl (k, l ordered)
  double* T;        // [9][G]: sum over weights of H * d weight / d J_ab, at 3 a + b
};

// One thread per Greville point: J from the control net (as in the assembly), S = J^{-1},
// Qh = S S^T, omega = det J (> 0 on valid maps). Then
//   d omega / d J_ab = omega S_ba,
//   d Q_kl / d J_ab  = omega (S_ba Qh_kl - S_ka Qh_bl - S_la Qh_bk).
__global__ __launch_bounds__(256) void geometry_adjoint_kernel(GeoAdjArgs a) {
  const long total = (long)a.np[0] * a.np[1] * a.np[2];
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
        for (int kq = 0; kq < n2; ++kq) {
          const double v2 = bv2[kq], d2 = bd2[kq];
          if (v2 == 0.0 && d2 == 0.0) continue;
          const double w0 = d0 * v1 * v2, w1 = v0 * d1 * v2, w2 = v0 * v1 * d2;
          const long c = ((long)i * n1 + j) * n2 + kq;
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
    // S = J^{-1} = adj(J) / det
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double id = det != 0.0 ? 1.0 / det : 0.0;
    double S[3][3];
    S[0][0] = c00 * id;
    S[1][0] = c01 * id;
    S[2][0] = c02 * id;
    S[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * id;
    S[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * id;
    S[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * id;
    S[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * id;
    S[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * id;
    S[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * id;
    double Qh[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
      for (int q = 0; q < 3; ++q) Qh[p][q] = S[p][0] * S[q][0] + S[p][1] * S[q][1] + S[p][2] * S[q][2];
    const double om = fabs(det);
    const double hw = a.H[idx];
    double Hk[3][3];
#pragma unroll
    for (int kk = 0; kk < 3; ++kk)
#pragma unroll
      for (int l = 0; l < 3; ++l) Hk[kk][l] = a.H[(1 + 3 * kk + l) * total + idx];
#pragma unroll
    for (int aa = 0; aa < 3; ++aa)
#pragma unroll
      for (int bb = 0; bb < 3; ++bb) {
        double t = hw * S[bb][aa];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
#pragma unroll
          for (int l = 0; l < 3; ++l)
            t += Hk[kk][l] * (S[bb][aa] * Qh[kk][l] - S[kk][aa] * Qh[bb][l] - S[l][aa] * Qh[bb][kk]);
        a.T[(3 * aa + bb) * total + idx] = om * t;
      }
  }
}

}  // namespace

void adjoint_pointwise(hipStream_t s, long npts, const double* f, long fstride, double beta, double* P,
                       long pstride) {
  if (npts <= 0) return;
  const unsigned g = (unsigned)std::min<long>((npts + 255) / 256, 65536);
  pointwise_kernel<<<g, 256, 0, s>>>(npts, f, fstride, beta, P, pstride);
  IGA_HIP(hipGetLastError());
}

void geometry_adjoint(hipStream_t s, const int np[3], const int ncp[3], const double* const Bv[3],
                      const double* const Bd[3], const double* ctrl, const double* H, double* T) {
  GeoAdjArgs a;
  for (int d = 0; d < 3; ++d) {
    a.np[d] = np[d];
    a.ncp[d] = ncp[d];
    a.Bv[d] = Bv[d];
    a.Bd[d] = Bd[d];
  }
  a.ctrl = ctrl;
  a.H = H;
  a.T = T;
  const long total = (long)np[0] * np[1] * np[2];
  const unsigned g = (unsigned)std::min<long>((total + 255) / 256, 65536);
  geometry_adjoint_kernel<<<g, 256, 0, s>>>(a);
  IGA_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace iga
