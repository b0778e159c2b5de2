// FP64 batched GEMM on the CDNA4 matrix cores with two-level index maps.
//
// C[b][m][n] = alpha * sum_k A[b][m][k] B[b][k][n] + beta * C[b][m][n], where each of
// m, n, k (and the batch) is split as idx = outer * inner_extent + inner with its own
// element strides per operand. This covers every contraction of the projected local
// operator (interfaces x core x interfaces) without transposes or copies.
//
// Tiling: 64 x 64 output tile per 256-thread workgroup; each of the four waves owns a
// 32 x 32 quarter and issues v_mfma_f64_4x4x4 (four independent 4x4x4 blocks per
// instruction, 512 flops). Per K-step of 4 a wave loads 8 A fragments (one per 4-row
// block, shared by the instruction's four blocks) and 2 B fragments (four 4-column
// blocks each) from LDS and issues 16 MFMAs. K is staged through LDS 16 deep, double
// buffered through registers.
//
// Operand lane layout of v_mfma_f64_4x4x4 (lane = 16x + 4b + y, b = block):
//   A_b[i][k] in lane 16k + 4b + i;  B_b[k][j] in lane 16k + 4b + j;  C_b[i][j] in lane 16i + 4b + j.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

constexpr int BM = 64, BN = 64, BK = 16, NTHR = 256;

struct G2Args {
  int M, N, K, M2, N2, K2;
  const double* A;
  long sAm1, sAm2, sAk1, sAk2;
  const double* B;
  long sBk1, sBk2, sBn1, sBn2;
  double* C;
  long sCm1, sCm2, sCn1, sCn2;
  int nb2;
  long sAb1, sAb2, sBb1, sBb2, sCb1, sCb2;
  double alpha, beta;
};

typedef double d1 __attribute__((ext_vector_type(1)));

__device__ __forceinline__ long off2(int idx, int inner, long s_outer, long s_inner) {
  const int o = idx / inner;
  return (long)o * s_outer + (long)(idx - o * inner) * s_inner;
}

__global__ __launch_bounds__(NTHR) void gemm2_kernel(G2Args g) {
  __shared__ double As[2][BK][BM + 2];
  __shared__ double Bs[2][BK][BN + 2];
  const int bz = blockIdx.z;
  const int b1 = bz / g.nb2, b2 = bz - b1 * g.nb2;
  const double* A = g.A + b1 * g.sAb1 + b2 * g.sAb2;
  const double* B = g.B + b1 * g.sBb1 + b2 * g.sBb2;
  double* C = g.C + b1 * g.sCb1 + b2 * g.sCb2;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x;

  // Each thread loads 4 A and 4 B elements per K-tile. Choose the coalesced direction:
  // consecutive threads along k if the inner k stride is 1, else along m (resp. n).
  const bool a_kfast = (g.sAk2 == 1 && g.K2 > 1) || (g.K2 == 1 && g.sAk1 == 1);
  const bool b_nfast = (g.sBn2 == 1 && g.N2 > 1) || (g.N2 == 1 && g.sBn1 == 1);
  int a_mm[4], a_kk[4], b_nn[4], b_kk[4];
  long a_row[4], b_col[4];
  bool a_ok[4], b_ok[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int e = tid + NTHR * s;
    if (a_kfast) { a_kk[s] = e % BK; a_mm[s] = e / BK; } else { a_mm[s] = e % BM; a_kk[s] = e / BM; }
    if (b_nfast) { b_nn[s] = e % BN; b_kk[s] = e / BN; } else { b_kk[s] = e % BK; b_nn[s] = e / BK; }
    const int m = m0 + a_mm[s], n = n0 + b_nn[s];
    a_ok[s] = m < g.M;
    b_ok[s] = n < g.N;
    a_row[s] = a_ok[s] ? off2(m, g.M2, g.sAm1, g.sAm2) : 0;
    b_col[s] = b_ok[s] ? off2(n, g.N2, g.sBn1, g.sBn2) : 0;
  }

  const int wave = tid / 64, lane = tid % 64;
  const int wm0 = (wave / 2) * 32, wn0 = (wave % 2) * 32;
  const int lx = lane / 16, lb = (lane / 4) % 4, ly = lane % 4;
  double acc[8][2];
#pragma unroll
  for (int i = 0; i < 8; ++i) acc[i][0] = acc[i][1] = 0.0;

  double ra[4], rb[4];
  auto load_tile = [&](int kt) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      const int ka = kt + a_kk[s];
      ra[s] = (a_ok[s] && ka < g.K) ? A[a_row[s] + off2(ka, g.K2, g.sAk1, g.sAk2)] : 0.0;
      const int kb = kt + b_kk[s];
      rb[s] = (b_ok[s] && kb < g.K) ? B[off2(kb, g.K2, g.sBk1, g.sBk2) + b_col[s]] : 0.0;
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      As[buf][a_kk[s]][a_mm[s]] = ra[s];
      Bs[buf][b_kk[s]][b_nn[s]] = rb[s];
    }
  };

  const int nkt = (g.K + BK - 1) / BK;
  if (nkt > 0) {
    load_tile(0);
    store_tile(0);
  }
  __syncthreads();
  for (int t = 0; t < nkt; ++t) {
    const int cur = t & 1;
    if (t + 1 < nkt) load_tile((t + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double fa[8], fb[2];
#pragma unroll
      for (int r = 0; r < 8; ++r) fa[r] = As[cur][ks + lx][wm0 + r * 4 + ly];
#pragma unroll
      for (int c = 0; c < 2; ++c) fb[c] = Bs[cur][ks + lx][wn0 + c * 16 + lb * 4 + ly];
#pragma unroll
      for (int r = 0; r < 8; ++r)
#pragma unroll
        for (int c = 0; c < 2; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[r], fb[c], acc[r][c], 0, 0, 0);
    }
    if (t + 1 < nkt) store_tile(cur ^ 1);
    __syncthreads();
  }
  // acc[r][c] at this lane is C[wm0 + 4r + lx][wn0 + 16c + 4lb + ly]
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    const int m = m0 + wm0 + r * 4 + lx;
    if (m >= g.M) continue;
    const long crow = off2(m, g.M2, g.sCm1, g.sCm2);
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const int n = n0 + wn0 + c * 16 + lb * 4 + ly;
      if (n >= g.N) continue;
      double* p = C + crow + off2(n, g.N2, g.sCn1, g.sCn2);
      double v = g.alpha * acc[r][c];
      if (g.beta != 0.0) v += g.beta * *p;
      *p = v;
    }
  }
}

}  // namespace

void gemm2(hipStream_t s, const Gemm2& d) {
  if (d.M <= 0 || d.N <= 0 || d.nb1 <= 0 || d.nb2 <= 0) return;
  require(d.M2 >= 1 && d.N2 >= 1 && d.K2 >= 1, IGA_EINVAL, "gemm2: inner extents must be >= 1");
  const long nb = (long)d.nb1 * d.nb2;
  require(nb <= 65535, IGA_EINVAL, "gemm2: batch too large");
  G2Args a{d.M, d.N, d.K, d.M2, d.N2, d.K2, d.A, d.sAm1, d.sAm2, d.sAk1, d.sAk2, d.B, d.sBk1, d.sBk2,
           d.sBn1, d.sBn2, d.C, d.sCm1, d.sCm2, d.sCn1, d.sCn2, d.nb2, d.sAb1, d.sAb2, d.sBb1, d.sBb2,
           d.sCb1, d.sCb2, d.alpha, d.beta};
  if (d.K < 0) a.K = 0;
  dim3 grid((d.N + BN - 1) / BN, (d.M + BM - 1) / BM, (unsigned)nb);
  gemm2_kernel<<<grid, NTHR, 0, s>>>(a);
  IGA_HIP(hipGetLastError());
}

}  // namespace k
}  // namespace iga
