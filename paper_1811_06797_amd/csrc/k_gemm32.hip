// FP32-storage batched GEMMs on the CDNA4 matrix cores, with the two-level index maps of
// gemm2 (k_gemm.hip): the contractions of the mixed-precision local operator.
//
// C[b][m][n] = alpha * sum_k A[b][m][k] B[b][k][n] + beta * C[b][m][n] with FP32 operands in
// memory and FP32 accumulation, in one of two product precisions:
//  * FP32: v_mfma_f32_16x16x4f32 (one 16x16x4 product, 2048 flops). Lane layout (lane
//    l = 16 q + t, q = l / 16, t = l % 16): A[t][q] and B[q][t]; C[4 q + v][t], v = 0..3.
//  * BF16: operands are rounded to bfloat16 (nearest, ties to even) as they are staged into
//    LDS, and v_mfma_f32_16x16x32_bf16 (16x16x32, 16384 flops) multiplies them. Lane
//    layout: A[t][8 q + e] and B[8 q + e][t], e = 0..7 in one 16-byte register quadruple;
//    C as above. LDS holds the tiles in groups of 8 consecutive k per row, so that each
//    operand is one 16-byte LDS read.
// Each wave owns a (16 WM) x (16 WN) block of C; four waves form the workgroup tile; K is
// staged through LDS (16 deep in FP32, 32 in BF16), double-buffered, with the next tile's
// global loads in flight during the current tile's products. FP32 products of the wide tile
// that qualify load their operands straight into LDS instead (gemm2f_dma_kernel).
#include <algorithm>
#include <cstring>

#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

constexpr int NT = 256, BKF = 16, BKH = 32;
// FP32 wide-tile products that qualify use the LDS-direct kernel (0: never)
#ifndef IGA_DMA_F32
#define IGA_DMA_F32 1
#endif

typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

__device__ const float kZeroF[1] = {0.0f};

struct G2FArgs {
  int M, N, K, M2, N2, K2;
  const float* A;
  long sAm1, sAm2, sAk1, sAk2;
  const float* B;
  long sBk1, sBk2, sBn1, sBn2;
  float* C;
  long sCm1, sCm2, sCn1, sCn2;
  int nb2, nbatch;
  long sAb1, sAb2, sBb1, sBb2, sCb1, sCb2;
  float alpha, beta;
  int ksplit, kchunk;
  float* work;
  int batch_inner;  // tile order within an XCD's range: batch fastest (band rows; see gemm2)
};

__device__ __forceinline__ void tile_coords_f(int tile, int gx, int gy, int gz, int batch_inner, int& bx, int& by,
                                              int& bz) {
  if (batch_inner) {
    bz = tile % gz;
    const int r = tile / gz;
    bx = r % gx;
    by = r / gx;
  } else {
    bx = tile % gx;
    by = (tile / gx) % gy;
    bz = tile / (gx * gy);
  }
}

__device__ __forceinline__ long off2f(int idx, int inner, long s_outer, long s_inner) {
  const int o = idx / inner;
  return (long)o * s_outer + (long)(idx - o * inner) * s_inner;
}

// Nearest bfloat16 of a finite float, ties to even: the upper 16 bits after adding half an
// ulp of the result (less one when the result's last bit is 0).
__device__ __forceinline__ short to_bf16(float x) {
  const unsigned u = __float_as_uint(x);
  return (short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Row pitch (floats) of the LDS tiles: 16 mod 64, so the four k rows one MFMA operand read
// touches start 16 banks apart.
constexpr int lds_padf(int w) { return ((16 - w % 64) + 64) % 64; }

template <int BM, int BN, bool BF>
struct TileLdsF {
  float As[2][BKF][BM + lds_padf(BM)];
  float Bs[2][BKF][BN + lds_padf(BN)];
};
// BF16 tiles: [buffer][k / 8][row][k % 8], one spare row per k group
template <int BM, int BN>
struct TileLdsF<BM, BN, true> {
  alignas(16) short As[2][BKH / 8][BM + 1][8];
  alignas(16) short Bs[2][BKH / 8][BN + 1][8];
};

// One BM x BN output tile (column tile bx, row tile by, batch and split index bz).
template <int WM, int WN, int WAVES_M, int WAVES_N, bool BF>
__device__ __forceinline__ void gemm2f_tile(const G2FArgs& g, int bx, int by, int bz,
                                            TileLdsF<16 * WM * WAVES_M, 16 * WN * WAVES_N, BF>& L) {
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  constexpr int BK = BF ? BKH : BKF;
  constexpr int LA = BM * BK / NT, LB = BN * BK / NT;
  static_assert(WAVES_M * WAVES_N == 4, "four waves");
  static_assert(LA >= 1 && LB >= 1 && LA * NT == BM * BK && LB * NT == BN * BK, "tile does not split evenly");
  auto& As = L.As;
  auto& Bs = L.Bs;
  const int split = bz / g.nbatch, bb = bz - split * g.nbatch;
  const int b1 = bb / g.nb2, b2 = bb - b1 * g.nb2;
  const float* A = g.A + b1 * g.sAb1 + b2 * g.sAb2;
  const float* B = g.B + b1 * g.sBb1 + b2 * g.sBb2;
  const int m0 = by * BM, n0 = bx * BN;
  const int tid = threadIdx.x;
  const int kbeg = split * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);

  const bool a_kfast = (g.sAk2 == 1 && g.K2 > 1) || (g.K2 == 1 && g.sAk1 == 1);
  const bool b_nfast = (g.sBn2 == 1 && g.N2 > 1) || (g.N2 == 1 && g.sBn1 == 1);
  const int kq = BK / g.K2, krem = BK - kq * g.K2;
  const int dA = kq * (int)g.sAk1 + krem * (int)g.sAk2, dAw = dA + (int)g.sAk1 - g.K2 * (int)g.sAk2;
  const int dB = kq * (int)g.sBk1 + krem * (int)g.sBk2, dBw = dB + (int)g.sBk1 - g.K2 * (int)g.sBk2;
  int a_mm[LA], a_kk[LA], b_nn[LB], b_kk[LB], ak2[LA], bk2[LB], oa[LA], ob[LB];
  bool a_ok[LA], b_ok[LB];
#pragma unroll
  for (int s = 0; s < LA; ++s) {
    const int e = tid + NT * s;
    if (a_kfast) { a_kk[s] = e % BK; a_mm[s] = e / BK; } else { a_mm[s] = e % BM; a_kk[s] = e / BM; }
    const int m = m0 + a_mm[s];
    a_ok[s] = m < g.M;
    const int k = kbeg + a_kk[s], k1 = k / g.K2;
    ak2[s] = k - k1 * g.K2;
    oa[s] = (a_ok[s] ? (int)off2f(m, g.M2, g.sAm1, g.sAm2) : 0) + k1 * (int)g.sAk1 + ak2[s] * (int)g.sAk2;
  }
#pragma unroll
  for (int s = 0; s < LB; ++s) {
    const int e = tid + NT * s;
    if (b_nfast) { b_nn[s] = e % BN; b_kk[s] = e / BN; } else { b_kk[s] = e % BK; b_nn[s] = e / BK; }
    const int n = n0 + b_nn[s];
    b_ok[s] = n < g.N;
    const int k = kbeg + b_kk[s], k1 = k / g.K2;
    bk2[s] = k - k1 * g.K2;
    ob[s] = (b_ok[s] ? (int)off2f(n, g.N2, g.sBn1, g.sBn2) : 0) + k1 * (int)g.sBk1 + bk2[s] * (int)g.sBk2;
  }

  const int wave = tid / 64, lane = tid % 64;
  const int wm0 = (wave / WAVES_N) * (16 * WM), wn0 = (wave % WAVES_N) * (16 * WN);
  const int lq = lane / 16, lt = lane % 16;
  f4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};

  float ra[LA], rb[LB];
  auto load_tile = [&](int kt) {
    const int klim = kend - kt;
#pragma unroll
    for (int s = 0; s < LA; ++s) {
      const bool ok = a_ok[s] && a_kk[s] < klim;
      ra[s] = *(ok ? A + oa[s] : kZeroF);
      ak2[s] += krem;
      const bool w = ak2[s] >= g.K2;
      ak2[s] -= w ? g.K2 : 0;
      oa[s] += w ? dAw : dA;
    }
#pragma unroll
    for (int s = 0; s < LB; ++s) {
      const bool ok = b_ok[s] && b_kk[s] < klim;
      rb[s] = *(ok ? B + ob[s] : kZeroF);
      bk2[s] += krem;
      const bool w = bk2[s] >= g.K2;
      bk2[s] -= w ? g.K2 : 0;
      ob[s] += w ? dBw : dB;
    }
  };
  auto store_tile = [&](int buf) {
    if constexpr (BF) {
#pragma unroll
      for (int s = 0; s < LA; ++s) As[buf][a_kk[s] >> 3][a_mm[s]][a_kk[s] & 7] = to_bf16(ra[s]);
#pragma unroll
      for (int s = 0; s < LB; ++s) Bs[buf][b_kk[s] >> 3][b_nn[s]][b_kk[s] & 7] = to_bf16(rb[s]);
    } else {
#pragma unroll
      for (int s = 0; s < LA; ++s) As[buf][a_kk[s]][a_mm[s]] = ra[s];
#pragma unroll
      for (int s = 0; s < LB; ++s) Bs[buf][b_kk[s]][b_nn[s]] = rb[s];
    }
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
    if constexpr (BF) {
      // one 16x16x32 product per block: this lane's k group is lq
      s8 fa[WM], fb[WN];
#pragma unroll
      for (int r = 0; r < WM; ++r) fa[r] = *reinterpret_cast<const s8*>(&As[cur][lq][wm0 + 16 * r + lt][0]);
#pragma unroll
      for (int c = 0; c < WN; ++c) fb[c] = *reinterpret_cast<const s8*>(&Bs[cur][lq][wn0 + 16 * c + lt][0]);
#pragma unroll
      for (int r = 0; r < WM; ++r)
#pragma unroll
        for (int c = 0; c < WN; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[r], fb[c], acc[r][c], 0, 0, 0);
    } else {
#pragma unroll
      for (int ks = 0; ks < BK; ks += 4) {
        float fa[WM], fb[WN];
#pragma unroll
        for (int r = 0; r < WM; ++r) fa[r] = As[cur][ks + lq][wm0 + 16 * r + lt];
#pragma unroll
        for (int c = 0; c < WN; ++c) fb[c] = Bs[cur][ks + lq][wn0 + 16 * c + lt];
#pragma unroll
        for (int r = 0; r < WM; ++r)
#pragma unroll
          for (int c = 0; c < WN; ++c)
            acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[r], fb[c], acc[r][c], 0, 0, 0);
      }
    }
    if (t + 1 < nkt) store_tile(cur ^ 1);
    __syncthreads();
  }
  // acc[r][c][v] at this lane is C[wm0 + 16 r + 4 lq + v][wn0 + 16 c + lt]
  if (g.ksplit > 1) {
    float* W = g.work + ((long)split * g.nbatch + bb) * (long)g.M * g.N;
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm0 + 16 * r + 4 * lq + v;
        if (m >= g.M) continue;
#pragma unroll
        for (int c = 0; c < WN; ++c) {
          const int n = n0 + wn0 + 16 * c + lt;
          if (n < g.N) W[(long)m * g.N + n] = acc[r][c][v];
        }
      }
    return;
  }
  float* C = g.C + b1 * g.sCb1 + b2 * g.sCb2;
#pragma unroll
  for (int r = 0; r < WM; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wm0 + 16 * r + 4 * lq + v;
      if (m >= g.M) continue;
      const long crow = off2f(m, g.M2, g.sCm1, g.sCm2);
#pragma unroll
      for (int c = 0; c < WN; ++c) {
        const int n = n0 + wn0 + 16 * c + lt;
        if (n >= g.N) continue;
        float* p = C + crow + off2f(n, g.N2, g.sCn1, g.sCn2);
        float val = g.alpha * acc[r][c][v];
        if (g.beta != 0.0f) val += g.beta * *p;
        *p = val;
      }
    }
}

template <int WM, int WN, int WAVES_M, int WAVES_N, bool BF>
__global__ __launch_bounds__(NT) void gemm2f_kernel(G2FArgs g) {
  __shared__ TileLdsF<16 * WM * WAVES_M, 16 * WN * WAVES_N, BF> L;
  // XCD-contiguous renumbering of the workgroups (as in gemm2)
  const int gx = gridDim.x, gy = gridDim.y;
  const int total = gx * gy * gridDim.z;
  const int lin = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  const int xcd = lin % 8, q8 = lin / 8, base = total / 8, rem = total % 8;
  const int tile = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + q8;
  int bx, by, bz;
  tile_coords_f(tile, gx, gy, gridDim.z, g.batch_inner, bx, by, bz);
  gemm2f_tile<WM, WN, WAVES_M, WAVES_N, BF>(g, bx, by, bz, L);
}

// FP32 wide tile (64 x 128, four waves of 32 x 64, K tile 16) with LDS-direct operand loads:
// each global_load_lds_dwordx4 moves four floats per lane into the next 16 bytes of the wave's
// LDS window, three LDS buffers hold tiles t, t + 1 and t + 2. A windows hold four K rows of 64
// floats, B windows two K rows of 128; in K row k the 16-byte chunk c sits at position
// c ^ 4 (k % 4), so that the four rows a fragment read touches fall into disjoint banks.
// Requirements (checked on the host): single-level indices, unit strides along M in A and N in
// B, M, N and the strides multiples of 4, 16-byte aligned bases. Partial tiles read zeros.
__device__ const float kZeroF4[4] __attribute__((aligned(16))) = {0.0f, 0.0f, 0.0f, 0.0f};
constexpr int FDM = 64, FDN = 128;

__global__ __launch_bounds__(NT) void gemm2f_dma_kernel(G2FArgs g) {
  __shared__ __attribute__((aligned(16))) float A0[BKF * FDM], A1[BKF * FDM], A2[BKF * FDM];
  __shared__ __attribute__((aligned(16))) float B0[BKF * FDN], B1[BKF * FDN], B2[BKF * FDN];
  typedef __attribute__((address_space(3))) void* lds_ptr;
  typedef const __attribute__((address_space(1))) void* glb_ptr;
  const int gx = gridDim.x, gy = gridDim.y;
  const int total = gx * gy * gridDim.z;
  const int lin = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  const int xcd = lin % 8, q8 = lin / 8, base = total / 8, rem = total % 8;
  const int tile = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + q8;
  int bx, by, bz;
  tile_coords_f(tile, gx, gy, gridDim.z, g.batch_inner, bx, by, bz);
  const int split = bz / g.nbatch, bb = bz - split * g.nbatch;
  const int b1 = bb / g.nb2, b2 = bb - b1 * g.nb2;
  const float* A = g.A + b1 * g.sAb1 + b2 * g.sAb2;
  const float* B = g.B + b1 * g.sBb1 + b2 * g.sBb2;
  const int m0 = by * FDM, n0 = bx * FDN;
  const int kbeg = split * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  // this lane's chunks: A window = wave (K rows 4 wave .. 4 wave + 3), B windows 2 wave, 2 wave + 1
  int oa, ob[2], brow[2];
  bool mok, nok[2];
  const int arow = 4 * wave + (lane >> 4);
  {
    const int m = m0 + 4 * ((lane & 15) ^ (4 * (lane >> 4)));
    mok = m < g.M;
    oa = (mok ? m : 0) + (kbeg + arow) * (int)g.sAk2;
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int i = 2 * wave + u;
    brow[u] = 2 * i + (lane >> 5);
    const int n = n0 + 4 * ((lane & 31) ^ (4 * (brow[u] & 3)));
    nok[u] = n < g.N;
    ob[u] = (nok[u] ? n : 0) + (kbeg + brow[u]) * (int)g.sBk2;
  }
  const int dA = BKF * (int)g.sAk2, dB = BKF * (int)g.sBk2;
  auto issue = [&](int kt, float* As, float* Bs) {
    const int klim = kend - kt;
    {
      const float* src = (mok && arow < klim) ? A + oa : kZeroF4;
      __builtin_amdgcn_global_load_lds((glb_ptr)src, (lds_ptr)(As + wave * 256), 16, 0, 0);
      oa += dA;
    }
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const float* src = (nok[u] && brow[u] < klim) ? B + ob[u] : kZeroF4;
      __builtin_amdgcn_global_load_lds((glb_ptr)src, (lds_ptr)(Bs + (2 * wave + u) * 256), 16, 0, 0);
      ob[u] += dB;
    }
  };
  constexpr int WM = 2, WN = 4;
  const int wm0 = (wave / 2) * (16 * WM), wn0 = (wave % 2) * (16 * WN);
  const int lq = lane / 16, lt = lane % 16;
  // element (k, m) of an A buffer: (k / 4) 256 + (k % 4) 64 + 4 ((m / 4) ^ 4 (k % 4)) + m % 4;
  // element (k, n) of a B buffer: (k / 2) 256 + (k % 2) 128 + 4 ((n / 4) ^ 4 (k % 4)) + n % 4
  int offA[WM], offB[WN];
#pragma unroll
  for (int r = 0; r < WM; ++r) offA[r] = lq * 64 + 4 * (((wm0 >> 2) + 4 * r + (lt >> 2)) ^ (4 * lq)) + (lt & 3);
#pragma unroll
  for (int c = 0; c < WN; ++c)
    offB[c] = (lq >> 1) * 256 + (lq & 1) * 128 + 4 * (((wn0 >> 2) + 4 * c + (lt >> 2)) ^ (4 * lq)) + (lt & 3);
  f4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  auto compute = [&](const float* As, const float* Bs) {
#pragma unroll
    for (int ks = 0; ks < BKF; ks += 4) {
      float fa[WM], fb[WN];
#pragma unroll
      for (int r = 0; r < WM; ++r) fa[r] = As[offA[r] + ks * 64];
#pragma unroll
      for (int c = 0; c < WN; ++c) fb[c] = Bs[offB[c] + ks * 128];
#pragma unroll
      for (int r = 0; r < WM; ++r)
#pragma unroll
        for (int c = 0; c < WN; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x4f32(fa[r], fb[c], acc[r][c], 0, 0, 0);
    }
  };
  // as in gemm2_dma_kernel: wait for this wave's loads of tile t (three per wave for tile t + 1
  // may stay in flight), barrier, issue tile t + 2 into the buffer of tile t - 1, multiply tile t
  auto step = [&](int t, const float* As, const float* Bs, float* An, float* Bn) {
    __builtin_amdgcn_s_waitcnt(0x0F73);  // vmcnt(3); expcnt and lgkmcnt unconstrained
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    issue(kbeg + (t + 2) * BKF, An, Bn);
    compute(As, Bs);
  };
  const int nkt = (kend - kbeg + BKF - 1) / BKF;
  issue(kbeg, A0, B0);
  issue(kbeg + BKF, A1, B1);
  for (int t = 0; t < nkt; t += 3) {
    step(t, A0, B0, A2, B2);
    if (t + 1 >= nkt) break;
    step(t + 1, A1, B1, A0, B0);
    if (t + 2 >= nkt) break;
    step(t + 2, A2, B2, A1, B1);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0): no load may land after the workgroup ends
  // acc[r][c][v] at this lane is C[wm0 + 16 r + 4 lq + v][wn0 + 16 c + lt]
  if (g.ksplit > 1) {
    float* W = g.work + ((long)split * g.nbatch + bb) * (long)g.M * g.N;
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm0 + 16 * r + 4 * lq + v;
        if (m >= g.M) continue;
#pragma unroll
        for (int c = 0; c < WN; ++c) {
          const int n = n0 + wn0 + 16 * c + lt;
          if (n < g.N) W[(long)m * g.N + n] = acc[r][c][v];
        }
      }
    return;
  }
  float* C = g.C + b1 * g.sCb1 + b2 * g.sCb2;
#pragma unroll
  for (int r = 0; r < WM; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wm0 + 16 * r + 4 * lq + v;
      if (m >= g.M) continue;
      const long crow = off2f(m, g.M2, g.sCm1, g.sCm2);
#pragma unroll
      for (int c = 0; c < WN; ++c) {
        const int n = n0 + wn0 + 16 * c + lt;
        if (n >= g.N) continue;
        float* p = C + crow + off2f(n, g.N2, g.sCn1, g.sCn2);
        float val = g.alpha * acc[r][c][v];
        if (g.beta != 0.0f) val += g.beta * *p;
        *p = val;
      }
    }
}

// BF16-product form of the LDS-direct wide tile (64 x 128, four waves of 32 x 64, K tile 32):
// FP32 operand tiles go straight into LDS as in gemm2f_dma_kernel, and each fragment read
// rounds its eight floats to bfloat16 (nearest, ties to even: v_cvt_pk_bf16_f32) for
// v_mfma_f32_16x16x32_bf16, whose lane 16 q + t takes K rows 8 q .. 8 q + 7 of row (column)
// t. A windows hold four K rows of 64 floats, B windows two K rows of 128; in K row k the
// 16-byte chunk c sits at position c ^ 4 ((k % 4) ^ (k / 8 % 4)), so that the four lane
// groups q of one read, which share k % 4, still fall into disjoint banks.
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));

__device__ __forceinline__ unsigned cvt_bf16x2(float x, float y) {
  const b2v v = __builtin_convertvector((f2v){x, y}, b2v);
  return __builtin_bit_cast(unsigned, v);
}

__global__ __launch_bounds__(NT) void gemm2b_dma_kernel(G2FArgs g) {
  __shared__ __attribute__((aligned(16))) float A0[BKH * FDM], A1[BKH * FDM], A2[BKH * FDM];
  __shared__ __attribute__((aligned(16))) float B0[BKH * FDN], B1[BKH * FDN], B2[BKH * FDN];
  typedef __attribute__((address_space(3))) void* lds_ptr;
  typedef const __attribute__((address_space(1))) void* glb_ptr;
  const int gx = gridDim.x, gy = gridDim.y;
  const int total = gx * gy * gridDim.z;
  const int lin = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  const int xcd = lin % 8, q8 = lin / 8, base = total / 8, rem = total % 8;
  const int tile = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + q8;
  int bx, by, bz;
  tile_coords_f(tile, gx, gy, gridDim.z, g.batch_inner, bx, by, bz);
  const int split = bz / g.nbatch, bb = bz - split * g.nbatch;
  const int b1 = bb / g.nb2, b2 = bb - b1 * g.nb2;
  const float* A = g.A + b1 * g.sAb1 + b2 * g.sAb2;
  const float* B = g.B + b1 * g.sBb1 + b2 * g.sBb2;
  const int m0 = by * FDM, n0 = bx * FDN;
  const int kbeg = split * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  auto swz = [](int k) { return 4 * ((k & 3) ^ ((k >> 3) & 3)); };
  // this lane's chunks: A windows 2 wave, 2 wave + 1 (K rows 4 j .. 4 j + 3), B windows
  // 4 wave .. 4 wave + 3 (K rows 2 j, 2 j + 1)
  int oa[2], ob[4], arow[2], brow[4];
  bool mok[2], nok[4];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int j = 2 * wave + u;
    arow[u] = 4 * j + (lane >> 4);
    const int m = m0 + 4 * ((lane & 15) ^ swz(arow[u]));
    mok[u] = m < g.M;
    oa[u] = (mok[u] ? m : 0) + (kbeg + arow[u]) * (int)g.sAk2;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int j = 4 * wave + u;
    brow[u] = 2 * j + (lane >> 5);
    const int n = n0 + 4 * ((lane & 31) ^ swz(brow[u]));
    nok[u] = n < g.N;
    ob[u] = (nok[u] ? n : 0) + (kbeg + brow[u]) * (int)g.sBk2;
  }
  const int dA = BKH * (int)g.sAk2, dB = BKH * (int)g.sBk2;
  auto issue = [&](int kt, float* As, float* Bs) {
    const int klim = kend - kt;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const float* src = (mok[u] && arow[u] < klim) ? A + oa[u] : kZeroF4;
      __builtin_amdgcn_global_load_lds((glb_ptr)src, (lds_ptr)(As + (2 * wave + u) * 256), 16, 0, 0);
      oa[u] += dA;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const float* src = (nok[u] && brow[u] < klim) ? B + ob[u] : kZeroF4;
      __builtin_amdgcn_global_load_lds((glb_ptr)src, (lds_ptr)(Bs + (4 * wave + u) * 256), 16, 0, 0);
      ob[u] += dB;
    }
  };
  constexpr int WM = 2, WN = 4;
  const int wm0 = (wave / 2) * (16 * WM), wn0 = (wave % 2) * (16 * WN);
  const int q = lane / 16, t = lane % 16;
  // element (k, m) of an A buffer: (k / 4) 256 + (k % 4) 64 + 4 ((m / 4) ^ swz(k)) + m % 4;
  // element (k, n) of a B buffer: (k / 2) 256 + (k % 2) 128 + 4 ((n / 4) ^ swz(k)) + n % 4.
  // For k = 8 q + e the rows e and e + 4 lie 256 (A) or 512 (B) floats apart.
  int offA[WM][4], offB[WN][4];
#pragma unroll
  for (int r = 0; r < WM; ++r)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      offA[r][e] = 2 * q * 256 + e * 64 + 4 * (((wm0 >> 2) + 4 * r + (t >> 2)) ^ (4 * (e ^ q))) + (t & 3);
#pragma unroll
  for (int c = 0; c < WN; ++c)
#pragma unroll
    for (int e = 0; e < 4; ++e)
      offB[c][e] = (4 * q + (e >> 1)) * 256 + (e & 1) * 128 + 4 * (((wn0 >> 2) + 4 * c + (t >> 2)) ^ (4 * (e ^ q))) +
                   (t & 3);
  f4 acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = f4{0.0f, 0.0f, 0.0f, 0.0f};
  auto frag = [&](const float* X, const int (&off)[4], int step) {
    float v[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] = X[off[e]];
      v[e + 4] = X[off[e] + step];
    }
    const u4v w = {cvt_bf16x2(v[0], v[1]), cvt_bf16x2(v[2], v[3]), cvt_bf16x2(v[4], v[5]), cvt_bf16x2(v[6], v[7])};
    return __builtin_bit_cast(s8, w);
  };
  auto compute = [&](const float* As, const float* Bs) {
    s8 fa[WM], fb[WN];
#pragma unroll
    for (int r = 0; r < WM; ++r) fa[r] = frag(As, offA[r], 256);
#pragma unroll
    for (int c = 0; c < WN; ++c) fb[c] = frag(Bs, offB[c], 512);
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
      for (int c = 0; c < WN; ++c)
        acc[r][c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa[r], fb[c], acc[r][c], 0, 0, 0);
  };
  auto step = [&](int tt, const float* As, const float* Bs, float* An, float* Bn) {
    __builtin_amdgcn_s_waitcnt(0x0F76);  // vmcnt(6): this wave's loads of the next tile may stay in flight
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    issue(kbeg + (tt + 2) * BKH, An, Bn);
    compute(As, Bs);
  };
  const int nkt = (kend - kbeg + BKH - 1) / BKH;
  issue(kbeg, A0, B0);
  issue(kbeg + BKH, A1, B1);
  for (int tt = 0; tt < nkt; tt += 3) {
    step(tt, A0, B0, A2, B2);
    if (tt + 1 >= nkt) break;
    step(tt + 1, A1, B1, A0, B0);
    if (tt + 2 >= nkt) break;
    step(tt + 2, A2, B2, A1, B1);
  }
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  // acc[r][c][v] at this lane is C[wm0 + 16 r + 4 q + v][wn0 + 16 c + t]
  if (g.ksplit > 1) {
    float* W = g.work + ((long)split * g.nbatch + bb) * (long)g.M * g.N;
#pragma unroll
    for (int r = 0; r < WM; ++r)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = m0 + wm0 + 16 * r + 4 * q + v;
        if (m >= g.M) continue;
#pragma unroll
        for (int c = 0; c < WN; ++c) {
          const int n = n0 + wn0 + 16 * c + t;
          if (n < g.N) W[(long)m * g.N + n] = acc[r][c][v];
        }
      }
    return;
  }
  float* C = g.C + b1 * g.sCb1 + b2 * g.sCb2;
#pragma unroll
  for (int r = 0; r < WM; ++r)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int m = m0 + wm0 + 16 * r + 4 * q + v;
      if (m >= g.M) continue;
      const long crow = off2f(m, g.M2, g.sCm1, g.sCm2);
#pragma unroll
      for (int c = 0; c < WN; ++c) {
        const int n = n0 + wn0 + 16 * c + t;
        if (n >= g.N) continue;
        float* p = C + crow + off2f(n, g.N2, g.sCn1, g.sCn2);
        float val = g.alpha * acc[r][c][v];
        if (g.beta != 0.0f) val += g.beta * *p;
        *p = val;
      }
    }
}

// Persistent grouped form (see gemm2_grouped_kernel).
template <int WM, int WN, int WAVES_M, int WAVES_N>
__global__ __launch_bounds__(NT) void gemm2f_grouped_kernel(const G2FArgs* gs, const int* prefix, int ngemm,
                                                            int total) {
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  __shared__ TileLdsF<BM, BN, false> L;
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    int lo = 0, hi = ngemm;
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (prefix[mid] <= t) lo = mid; else hi = mid;
    }
    const G2FArgs g = gs[lo];
    const int local = t - prefix[lo];
    const int gx = (g.N + BN - 1) / BN, gy = (g.M + BM - 1) / BM;
    __syncthreads();
    gemm2f_tile<WM, WN, WAVES_M, WAVES_N, false>(g, local % gx, (local / gx) % gy, local / (gx * gy), L);
  }
}

__global__ __launch_bounds__(256) void splitk_reduce_f(G2FArgs g) {
  const long MN = (long)g.M * g.N;
  const long total = MN * g.nbatch;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    const int bb = e / MN;
    const long mn = e - bb * MN;
    const int m = mn / g.N, n = mn - (long)m * g.N;
    float s = 0.0f;
    for (int sp = 0; sp < g.ksplit; ++sp) s += g.work[((long)sp * g.nbatch + bb) * MN + mn];
    const int b1 = bb / g.nb2, b2 = bb - b1 * g.nb2;
    float* p = g.C + b1 * g.sCb1 + b2 * g.sCb2 + off2f(m, g.M2, g.sCm1, g.sCm2) + off2f(n, g.N2, g.sCn1, g.sCn2);
    float v = g.alpha * s;
    if (g.beta != 0.0f) v += g.beta * *p;
    *p = v;
  }
}

template <int WM, int WN, int WAVES_M, int WAVES_N>
void launchf(hipStream_t s, G2FArgs a, int nbatch, bool bf16) {
  constexpr int BM = 16 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM, (unsigned)(nbatch * a.ksplit));
  require((long)grid.x * grid.y * grid.z < (1L << 31), IGA_EINVAL, "gemm2_f32: grid too large");
  if (bf16)
    gemm2f_kernel<WM, WN, WAVES_M, WAVES_N, true><<<grid, NT, 0, s>>>(a);
  else
    gemm2f_kernel<WM, WN, WAVES_M, WAVES_N, false><<<grid, NT, 0, s>>>(a);
}

long spanf(int ext, int inner, long s1, long s2) {
  if (ext <= 0) return 0;
  return (long)((ext - 1) / inner) * s1 + (long)(std::min(ext, inner) - 1) * s2;
}

}  // namespace

static G2FArgs make_args_f(const Gemm2F& d) {
  require(d.M2 >= 1 && d.N2 >= 1 && d.K2 >= 1, IGA_EINVAL, "gemm2_f32: inner extents must be >= 1");
  require(d.sAm1 >= 0 && d.sAm2 >= 0 && d.sAk1 >= 0 && d.sAk2 >= 0 && d.sBk1 >= 0 && d.sBk2 >= 0 &&
              d.sBn1 >= 0 && d.sBn2 >= 0,
          IGA_EINVAL, "gemm2_f32: operand strides must be nonnegative");
  const long kA = spanf(d.K, d.K2, d.sAk1, d.sAk2) + 64L * (d.sAk1 + d.sAk2);
  const long kB = spanf(d.K, d.K2, d.sBk1, d.sBk2) + 64L * (d.sBk1 + d.sBk2);
  require(spanf(d.M, d.M2, d.sAm1, d.sAm2) + kA < (1L << 31) && spanf(d.N, d.N2, d.sBn1, d.sBn2) + kB < (1L << 31),
          IGA_EINVAL, "gemm2_f32: operand too large for 32-bit offsets");
  const long nb = (long)d.nb1 * d.nb2;
  require(nb <= 65535, IGA_EINVAL, "gemm2_f32: batch too large");
  return G2FArgs{d.M, d.N, std::max(d.K, 0), d.M2, d.N2, d.K2, d.A, d.sAm1, d.sAm2, d.sAk1, d.sAk2, d.B, d.sBk1,
                 d.sBk2, d.sBn1, d.sBn2, d.C, d.sCm1, d.sCm2, d.sCn1, d.sCn2, d.nb2, (int)nb, d.sAb1, d.sAb2,
                 d.sBb1, d.sBb2, d.sCb1, d.sCb2, d.alpha, d.beta, 1, std::max(d.K, 0), nullptr,
                 d.batch_inner ? 1 : 0};
}

static void variant_tile_f(int v, int& BM, int& BN) {
  switch (v) {
    case 1: BM = 32; BN = 128; break;
    case 2: BM = 16; BN = 256; break;
    case 3: BM = 128; BN = 32; break;
    case 4: BM = 64; BN = 128; break;
    default: BM = 64; BN = 64; break;
  }
}

int gemm2f_pick(const Gemm2F& d) {
  const long nb = (long)d.nb1 * d.nb2;
  if (d.M <= 16) return 2;
  if (d.M <= 32) return 1;
  if (d.N <= 32) return 3;
  if (d.M <= 64 && (long)((d.N + 127) / 128) * nb >= 512) return 4;
  // tall, wide products (the left-interface stage of the local matvec): 128-wide column tiles
  // halve the re-reads of the long operand (measured 1.15-1.2x on that stage)
  if (d.M > 256 && d.N > 256) return 4;
  return 0;
}

size_t gemm2f_desc_bytes() { return sizeof(G2FArgs); }

long gemm2f_prepare(const Gemm2F& d, int variant, void* host_desc) {
  G2FArgs a = make_args_f(d);
  std::memcpy(host_desc, &a, sizeof(G2FArgs));
  if (d.M <= 0 || d.N <= 0 || d.nb1 <= 0 || d.nb2 <= 0) return 0;
  int BM, BN;
  variant_tile_f(variant, BM, BN);
  return (long)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN) * a.nbatch;
}

template <int WM, int WN, int WAVES_M, int WAVES_N>
static void launch_grouped_f(hipStream_t s, const void* desc, const int* prefix, int ngemm, long total) {
  const unsigned grid = (unsigned)std::min<long>(total, 1024);
  gemm2f_grouped_kernel<WM, WN, WAVES_M, WAVES_N>
      <<<grid, NT, 0, s>>>(static_cast<const G2FArgs*>(desc), prefix, ngemm, (int)total);
}

void gemm2f_grouped(hipStream_t s, int variant, const void* dev_desc, const int* dev_prefix, int ngemm, long total) {
  if (ngemm <= 0 || total <= 0) return;
  require(total < (1L << 31), IGA_EINVAL, "gemm2f_grouped: too many tiles");
  switch (variant) {
    case 2: launch_grouped_f<1, 4, 1, 4>(s, dev_desc, dev_prefix, ngemm, total); break;
    case 1: launch_grouped_f<2, 2, 1, 4>(s, dev_desc, dev_prefix, ngemm, total); break;
    case 3: launch_grouped_f<2, 2, 4, 1>(s, dev_desc, dev_prefix, ngemm, total); break;
    case 4: launch_grouped_f<2, 4, 2, 2>(s, dev_desc, dev_prefix, ngemm, total); break;
    default: launch_grouped_f<2, 2, 2, 2>(s, dev_desc, dev_prefix, ngemm, total); break;
  }
  IGA_HIP(hipGetLastError());
}

// The FP32 LDS-direct tile moves chunks of four consecutive M (or N) elements: single-level
// indices, unit strides along M in A and N in B, extents and strides multiples of 4, 16-byte
// aligned operand bases.
static bool dma_eligible_f(const Gemm2F& d) {
  auto q4 = [](long v) { return v % 4 == 0; };
  return d.K2 >= d.K && d.M2 >= d.M && d.N2 >= d.N && d.sAm2 == 1 && d.sBn2 == 1 && q4(d.M) && q4(d.N) &&
         q4(d.sAk2) && q4(d.sBk2) && q4(d.sAb1) && q4(d.sAb2) && q4(d.sBb1) && q4(d.sBb2) &&
         reinterpret_cast<uintptr_t>(d.A) % 16 == 0 && reinterpret_cast<uintptr_t>(d.B) % 16 == 0;
}

static void gemm2_fstore(hipStream_t s, const Gemm2F& d, float* work, size_t work_len, bool bf16) {
  if (d.M <= 0 || d.N <= 0 || d.nb1 <= 0 || d.nb2 <= 0) return;
  G2FArgs a = make_args_f(d);
  const long nb = a.nbatch;
  const int variant = d.variant >= 0 ? d.variant : gemm2f_pick(d);
  int BM, BN;
  variant_tile_f(variant, BM, BN);
  const long tiles = (long)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN) * nb;
  // split K when the tiles cannot fill the chip (about four workgroups per CU), or when a long
  // contraction (K >= 4096) has fewer than ~16 workgroups per CU (about 2048 workgroups,
  // chunks of at most 8192)
  int want = 1;
  if (tiles < 512 && d.K >= 4 * 32)
    want = (int)((1024 + tiles - 1) / tiles);
  else if (tiles < 4096 && d.K >= 4096)
    want = (int)std::max<long>((2048 + tiles - 1) / tiles, (d.K + 8191) / 8192);
  if (work && want > 1) {
    int ks = (int)std::min<long>(want, d.K / 64);
    while (ks > 1 && (size_t)ks * nb * d.M * d.N > work_len) --ks;
    if (ks > 1) {
      const int bk = bf16 ? BKH : BKF;
      a.kchunk = ((d.K + ks - 1) / ks + bk - 1) / bk * bk;
      a.ksplit = (d.K + a.kchunk - 1) / a.kchunk;
      a.work = work;
    }
  }
  require((long)nb * a.ksplit <= 65535, IGA_EINVAL, "gemm2_f32: batch too large");
  if (IGA_DMA_F32 && variant == 4 && dma_eligible_f(d)) {
    dim3 grid((a.N + FDN - 1) / FDN, (a.M + FDM - 1) / FDM, (unsigned)(nb * a.ksplit));
    require((long)grid.x * grid.y * grid.z < (1L << 31), IGA_EINVAL, "gemm2_f32: grid too large");
    if (bf16)
      gemm2b_dma_kernel<<<grid, NT, 0, s>>>(a);
    else
      gemm2f_dma_kernel<<<grid, NT, 0, s>>>(a);
  } else {
  switch (variant) {
    case 2: launchf<1, 4, 1, 4>(s, a, (int)nb, bf16); break;
    case 1: launchf<2, 2, 1, 4>(s, a, (int)nb, bf16); break;
    case 3: launchf<2, 2, 4, 1>(s, a, (int)nb, bf16); break;
    case 4: launchf<2, 4, 2, 2>(s, a, (int)nb, bf16); break;
    default: launchf<2, 2, 2, 2>(s, a, (int)nb, bf16); break;
  }
  }
  IGA_HIP(hipGetLastError());
  if (a.ksplit > 1) {
    const long total = (long)d.M * d.N * nb;
    splitk_reduce_f<<<(unsigned)std::min<long>((total + 255) / 256, 4096), 256, 0, s>>>(a);
    IGA_HIP(hipGetLastError());
  }
}

void gemm2_f32(hipStream_t s, const Gemm2F& d, float* work, size_t work_len) {
  gemm2_fstore(s, d, work, work_len, false);
}

void gemm2_bf16(hipStream_t s, const Gemm2F& d, float* work, size_t work_len) {
  gemm2_fstore(s, d, work, work_len, true);
}

}  // namespace k
}  // namespace iga
