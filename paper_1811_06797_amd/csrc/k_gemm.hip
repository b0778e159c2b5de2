// FP64 batched GEMM on the CDNA4 matrix cores with two-level index maps.
//
// C[b][m][n] = alpha * sum_k A[b][m][k] B[b][k][n] + beta * C[b][m][n], where each of
// m, n, k is split as idx = outer * inner_extent + inner with its own element strides per
// operand. This covers every contraction of the projected local operator (interfaces x
// banded core x interfaces) without transposes or copies.
//
// Each wave owns a (4 WM) x (16 WN) block of C and issues v_mfma_f64_4x4x4 (four
// independent 4x4x4 blocks per instruction, 512 flops): per K-step of 4 it reads WM A
// fragments (one per 4-row block, shared by the instruction's four blocks) and WN B
// fragments (four 4-column blocks each) from LDS and issues WM * WN MFMAs. Four waves
// form the workgroup tile; K is staged through LDS 16 deep with register double
// buffering. Tile variants serve tall, square and skinny outputs; when the output has too
// few tiles to fill the chip the K range is split and the partial products are summed in
// a fixed order by a second kernel (deterministic).
//
// Operand lane layout of v_mfma_f64_4x4x4 (lane = 16x + 4b + y, b = block):
//   A_b[i][k] in lane 16k + 4b + i;  B_b[k][j] in lane 16k + 4b + j;  C_b[i][j] in lane 16i + 4b + j.
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

constexpr int BK = 16, NTHR = 256;

struct G2Args {
  int M, N, K, M2, N2, K2;
  const double* A;
  long sAm1, sAm2, sAk1, sAk2;
  const double* B;
  long sBk1, sBk2, sBn1, sBn2;
  double* C;
  long sCm1, sCm2, sCn1, sCn2;
  int nb2, nbatch;
  long sAb1, sAb2, sBb1, sBb2, sCb1, sCb2;
  double alpha, beta;
  int ksplit, kchunk;   // split-K: chunk length (multiple of BK); ksplit == 1: direct store
  double* work;         // [ksplit][nbatch][M][N] partial products when ksplit > 1
};

__device__ __forceinline__ long off2(int idx, int inner, long s_outer, long s_inner) {
  const int o = idx / inner;
  return (long)o * s_outer + (long)(idx - o * inner) * s_inner;
}

// Running (outer, inner) decomposition of a k index advanced in steps of BK.
struct KIdx {
  int k1, k2;
  __device__ void init(int k, int K2) { k1 = k / K2; k2 = k - k1 * K2; }
  __device__ void step(int q, int rem, int K2) {
    k1 += q;
    k2 += rem;
    if (k2 >= K2) { k2 -= K2; ++k1; }
  }
  __device__ long off(long s1, long s2) const { return (long)k1 * s1 + (long)k2 * s2; }
};

// Row pitch of the LDS tiles: an odd multiple of 16 doubles, so that the two k rows a
// half-wave reads for one MFMA operand fall into disjoint halves of the 64 banks.
constexpr int lds_pad(int w) { return ((16 - w % 32) + 32) % 32; }

template <int WM, int WN, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(NTHR) void gemm2_kernel(G2Args g) {
  constexpr int BM = 4 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  constexpr int LA = BM * BK / NTHR, LB = BN * BK / NTHR;
  static_assert(WAVES_M * WAVES_N == 4, "four waves");
  static_assert(LA >= 1 && LB >= 1, "tile too small");
  __shared__ double As[2][BK][BM + lds_pad(BM)];
  __shared__ double Bs[2][BK][BN + lds_pad(BN)];
  const int bz = blockIdx.z;
  const int split = bz / g.nbatch, bb = bz - split * g.nbatch;
  const int b1 = bb / g.nb2, b2 = bb - b1 * g.nb2;
  const double* A = g.A + b1 * g.sAb1 + b2 * g.sAb2;
  const double* B = g.B + b1 * g.sBb1 + b2 * g.sBb2;
  const int m0 = blockIdx.y * BM, n0 = blockIdx.x * BN;
  const int tid = threadIdx.x;
  const int kbeg = split * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);

  const bool a_kfast = (g.sAk2 == 1 && g.K2 > 1) || (g.K2 == 1 && g.sAk1 == 1);
  const bool b_nfast = (g.sBn2 == 1 && g.N2 > 1) || (g.N2 == 1 && g.sBn1 == 1);
  int a_mm[LA], a_kk[LA], b_nn[LB], b_kk[LB];
  long a_row[LA], b_col[LB];
  bool a_ok[LA], b_ok[LB];
  KIdx ak[LA], bk[LB];
#pragma unroll
  for (int s = 0; s < LA; ++s) {
    const int e = tid + NTHR * s;
    if (a_kfast) { a_kk[s] = e % BK; a_mm[s] = e / BK; } else { a_mm[s] = e % BM; a_kk[s] = e / BM; }
    const int m = m0 + a_mm[s];
    a_ok[s] = m < g.M;
    a_row[s] = a_ok[s] ? off2(m, g.M2, g.sAm1, g.sAm2) : 0;
    ak[s].init(kbeg + a_kk[s], g.K2);
  }
#pragma unroll
  for (int s = 0; s < LB; ++s) {
    const int e = tid + NTHR * s;
    if (b_nfast) { b_nn[s] = e % BN; b_kk[s] = e / BN; } else { b_kk[s] = e % BK; b_nn[s] = e / BK; }
    const int n = n0 + b_nn[s];
    b_ok[s] = n < g.N;
    b_col[s] = b_ok[s] ? off2(n, g.N2, g.sBn1, g.sBn2) : 0;
    bk[s].init(kbeg + b_kk[s], g.K2);
  }
  const int kq = BK / g.K2, krem = BK - (BK / g.K2) * g.K2;

  const int wave = tid / 64, lane = tid % 64;
  const int wm0 = (wave / WAVES_N) * (4 * WM), wn0 = (wave % WAVES_N) * (16 * WN);
  const int lx = lane / 16, lb = (lane / 4) % 4, ly = lane % 4;
  double acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = 0.0;

  double ra[LA], rb[LB];
  auto load_tile = [&](int kt) {
#pragma unroll
    for (int s = 0; s < LA; ++s) {
      const int kk = kt + a_kk[s];
      ra[s] = (a_ok[s] && kk < kend) ? A[a_row[s] + ak[s].off(g.sAk1, g.sAk2)] : 0.0;
      ak[s].step(kq, krem, g.K2);
    }
#pragma unroll
    for (int s = 0; s < LB; ++s) {
      const int kk = kt + b_kk[s];
      rb[s] = (b_ok[s] && kk < kend) ? B[bk[s].off(g.sBk1, g.sBk2) + b_col[s]] : 0.0;
      bk[s].step(kq, krem, g.K2);
    }
  };
  auto store_tile = [&](int buf) {
#pragma unroll
    for (int s = 0; s < LA; ++s) As[buf][a_kk[s]][a_mm[s]] = ra[s];
#pragma unroll
    for (int s = 0; s < LB; ++s) Bs[buf][b_kk[s]][b_nn[s]] = rb[s];
  };

  const int nkt = (kend - kbeg + BK - 1) / BK;
  if (nkt > 0) {
    load_tile(kbeg);
    store_tile(0);
  }
  __syncthreads();
  for (int t = 0; t < nkt; ++t) {
    const int cur = t & 1;
    if (t + 1 < nkt) load_tile(kbeg + (t + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      double fa[WM], fb[WN];
#pragma unroll
      for (int r = 0; r < WM; ++r) fa[r] = As[cur][ks + lx][wm0 + r * 4 + ly];
#pragma unroll
      for (int c = 0; c < WN; ++c) fb[c] = Bs[cur][ks + lx][wn0 + c * 16 + lb * 4 + ly];
#pragma unroll
      for (int r = 0; r < WM; ++r)
#pragma unroll
        for (int c = 0; c < WN; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[r], fb[c], acc[r][c], 0, 0, 0);
    }
    if (t + 1 < nkt) store_tile(cur ^ 1);
    __syncthreads();
  }
  // acc[r][c] at this lane is C[wm0 + 4r + lx][wn0 + 16c + 4lb + ly]
  if (g.ksplit > 1) {
    double* W = g.work + ((long)split * g.nbatch + bb) * (long)g.M * g.N;
#pragma unroll
    for (int r = 0; r < WM; ++r) {
      const int m = m0 + wm0 + r * 4 + lx;
      if (m >= g.M) continue;
#pragma unroll
      for (int c = 0; c < WN; ++c) {
        const int n = n0 + wn0 + c * 16 + lb * 4 + ly;
        if (n < g.N) W[(long)m * g.N + n] = acc[r][c];
      }
    }
    return;
  }
  double* C = g.C + b1 * g.sCb1 + b2 * g.sCb2;
#pragma unroll
  for (int r = 0; r < WM; ++r) {
    const int m = m0 + wm0 + r * 4 + lx;
    if (m >= g.M) continue;
    const long crow = off2(m, g.M2, g.sCm1, g.sCm2);
#pragma unroll
    for (int c = 0; c < WN; ++c) {
      const int n = n0 + wn0 + c * 16 + lb * 4 + ly;
      if (n >= g.N) continue;
      double* p = C + crow + off2(n, g.N2, g.sCn1, g.sCn2);
      double v = g.alpha * acc[r][c];
      if (g.beta != 0.0) v += g.beta * *p;
      *p = v;
    }
  }
}

// C = alpha * sum_s work[s] + beta * C, splits summed in order.
__global__ __launch_bounds__(256) void splitk_reduce(G2Args g) {
  const long MN = (long)g.M * g.N;
  const long total = MN * g.nbatch;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int bb = e / MN;
    const long mn = e - bb * MN;
    const int m = mn / g.N, n = mn - (long)m * g.N;
    double s = 0.0;
    for (int sp = 0; sp < g.ksplit; ++sp) s += g.work[((long)sp * g.nbatch + bb) * MN + mn];
    const int b1 = bb / g.nb2, b2 = bb - b1 * g.nb2;
    double* p = g.C + b1 * g.sCb1 + b2 * g.sCb2 + off2(m, g.M2, g.sCm1, g.sCm2) + off2(n, g.N2, g.sCn1, g.sCn2);
    double v = g.alpha * s;
    if (g.beta != 0.0) v += g.beta * *p;
    *p = v;
  }
}

template <int WM, int WN, int WAVES_M, int WAVES_N>
void launch(hipStream_t s, G2Args a, int nbatch) {
  constexpr int BM = 4 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM, (unsigned)(nbatch * a.ksplit));
  gemm2_kernel<WM, WN, WAVES_M, WAVES_N><<<grid, NTHR, 0, s>>>(a);
}

}  // namespace

void gemm2(hipStream_t s, const Gemm2& d, double* work, size_t work_len) {
  if (d.M <= 0 || d.N <= 0 || d.nb1 <= 0 || d.nb2 <= 0) return;
  require(d.M2 >= 1 && d.N2 >= 1 && d.K2 >= 1, IGA_EINVAL, "gemm2: inner extents must be >= 1");
  const long nb = (long)d.nb1 * d.nb2;
  G2Args a{d.M, d.N, std::max(d.K, 0), d.M2, d.N2, d.K2, d.A, d.sAm1, d.sAm2, d.sAk1, d.sAk2, d.B, d.sBk1,
           d.sBk2, d.sBn1, d.sBn2, d.C, d.sCm1, d.sCm2, d.sCn1, d.sCn2, d.nb2, (int)nb, d.sAb1, d.sAb2, d.sBb1,
           d.sBb2, d.sCb1, d.sCb2, d.alpha, d.beta, 1, std::max(d.K, 0), nullptr};
  // tile shape by output shape
  int BM, BN, variant;
  if (d.M <= 16) { BM = 16; BN = 256; variant = 2; }
  else if (d.M <= 32) { BM = 32; BN = 128; variant = 1; }
  else if (d.N <= 32) { BM = 128; BN = 32; variant = 3; }
  else if (d.M <= 64 && (long)((d.N + 127) / 128) * nb >= 512) { BM = 64; BN = 128; variant = 4; }
  else { BM = 64; BN = 64; variant = 0; }
  const long tiles = (long)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN) * nb;
  // split K when the tiles cannot fill the chip and the contraction is long
  if (work && tiles < 256 && d.K >= 8 * BK) {
    int ks = (int)std::min<long>((512 + tiles - 1) / tiles, d.K / (4 * BK));
    while (ks > 1 && (size_t)ks * nb * d.M * d.N > work_len) --ks;
    if (ks > 1) {
      a.ksplit = ks;
      a.kchunk = ((d.K + ks - 1) / ks + BK - 1) / BK * BK;
      a.ksplit = (d.K + a.kchunk - 1) / a.kchunk;
      a.work = work;
    }
  }
  require((long)nb * a.ksplit <= 65535, IGA_EINVAL, "gemm2: batch too large");
  switch (variant) {
    case 2: launch<4, 4, 1, 4>(s, a, (int)nb); break;
    case 1: launch<8, 2, 1, 4>(s, a, (int)nb); break;
    case 3: launch<8, 2, 4, 1>(s, a, (int)nb); break;
    case 4: launch<8, 4, 2, 2>(s, a, (int)nb); break;
    default: launch<8, 2, 2, 2>(s, a, (int)nb); break;
  }
  IGA_HIP(hipGetLastError());
  if (a.ksplit > 1) {
    const long total = (long)d.M * d.N * nb;
    splitk_reduce<<<(unsigned)std::min<long>((total + 255) / 256, 4096), 256, 0, s>>>(a);
    IGA_HIP(hipGetLastError());
  }
}

void gemm2(hipStream_t s, const Gemm2& d) { gemm2(s, d, nullptr, 0); }

}  // namespace k
}  // namespace iga
