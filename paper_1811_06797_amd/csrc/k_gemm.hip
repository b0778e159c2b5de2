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
// form the workgroup tile; K is staged through LDS 16 deep (12 for the wide variant) with
// register double buffering. Tile variants serve tall, square and skinny outputs; the wide
// variant's products that qualify load their operand tiles straight into LDS instead
// (gemm2_dma_kernel). When the output has too few tiles to fill the chip the K range is
// split and the partial products are summed in a fixed order by a second kernel
// (deterministic).
//
// Operand lane layout of v_mfma_f64_4x4x4 (lane = 16x + 4b + y, b = block):
//   A_b[i][k] in lane 16k + 4b + i;  B_b[k][j] in lane 16k + 4b + j;  C_b[i][j] in lane 16i + 4b + j.
#include <algorithm>
#include <cstring>

#include "common.hpp"
#include "kernels.hpp"

namespace iga {
namespace k {
namespace {

constexpr int NTHR = 256;

// Source of the zeros that pad partial tiles.
__device__ const double kZero[1] = {0.0};

// Tile loads go through global (address space 1) pointers. Through a generic pointer the
// select against kZero compiles to flat loads, which count in the LDS counter as well, so
// every wait for an LDS fragment read would also wait for the tile loads still in flight.
__device__ __forceinline__ double gload(const double* p) {
  return *(const __attribute__((address_space(1))) double*)p;
}

// Tile of the wide variant used for M <= 64 with many column tiles (the banded stage of the
// local matvec): 64 x (32 WN) outputs, K step BK, NBUF LDS buffers.
#ifndef IGA_WIDE_WN
#define IGA_WIDE_WN 4
#endif
#ifndef IGA_WIDE_BK
#define IGA_WIDE_BK 12
#endif
#ifndef IGA_WIDE_NBUF
#define IGA_WIDE_NBUF 2
#endif
// K tiles of global loads kept in flight (1 or 2), for the wide variant and for the others
#ifndef IGA_WIDE_PREFETCH
#define IGA_WIDE_PREFETCH 2
#endif
#ifndef IGA_PREFETCH
#define IGA_PREFETCH 1
#endif
// the wide variant's products that qualify use the LDS-direct kernel (0: never)
#ifndef IGA_DMA
#define IGA_DMA 1
#endif

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
  int ksplit, kchunk;   // split-K: chunk length (multiple of the K tile); ksplit == 1: direct store
  double* work;         // [ksplit][nbatch][M][N] partial products when ksplit > 1
  int batch_inner;      // tile order within an XCD's range: batch index fastest (see tile_coords)
};

// (n-tile, m-tile, batch) of the XCD-ordered tile number: n-tile fastest by default; batch
// fastest when the batch index is the row of a banded product, so that the rows that share
// band slices of the B operand run together on one XCD while those slices are in its L2.
__device__ __forceinline__ void tile_coords(int tile, int gx, int gy, int gz, int batch_inner, int& bx, int& by,
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

__device__ __forceinline__ long off2(int idx, int inner, long s_outer, long s_inner) {
  const int o = idx / inner;
  return (long)o * s_outer + (long)(idx - o * inner) * s_inner;
}

// Row pitch of the LDS tiles: an odd multiple of 16 doubles, so that the two k rows a
// half-wave reads for one MFMA operand fall into disjoint halves of the 64 banks.
constexpr int lds_pad(int w) { return ((16 - w % 32) + 32) % 32; }

// LDS tiles of one workgroup.
template <int BM, int BN, int BK, int NBUF>
struct TileLds {
  double As[NBUF][BK][BM + lds_pad(BM)];
  double Bs[NBUF][BK][BN + lds_pad(BN)];
};

// One BM x BN output tile (column tile bx, row tile by, batch and split index bz) of the
// product g.
template <int WM, int WN, int WAVES_M, int WAVES_N, int BK, int NBUF, int PF, bool K1 = false>
__device__ __forceinline__ void gemm2_tile(const G2Args& g, int bx, int by, int bz,
                                           TileLds<4 * WM * WAVES_M, 16 * WN * WAVES_N, BK, NBUF>& L) {
  constexpr int BM = 4 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  // loads per thread and K tile; where the A tile is not a whole number of rounds of the
  // workgroup (the 24-row tile), the last round's extra threads load a duplicate of an element
  // of the tile and do not store it
  constexpr int LA = (BM * BK + NTHR - 1) / NTHR, LB = BN * BK / NTHR;
  constexpr bool PA = LA * NTHR != BM * BK;
  static_assert(WAVES_M * WAVES_N == 4, "four waves");
  static_assert(LA >= 1 && LB >= 1 && LB * NTHR == BN * BK, "tile too small");
  auto& As = L.As;
  auto& Bs = L.Bs;
  const int split = bz / g.nbatch, bb = bz - split * g.nbatch;
  const int b1 = bb / g.nb2, b2 = bb - b1 * g.nb2;
  const double* A = g.A + b1 * g.sAb1 + b2 * g.sAb2;
  const double* B = g.B + b1 * g.sBb1 + b2 * g.sBb2;
  const int m0 = by * BM, n0 = bx * BN;
  const int tid = threadIdx.x;
  const int kbeg = split * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);

  const bool a_kfast = (g.sAk2 == 1 && g.K2 > 1) || (g.K2 == 1 && g.sAk1 == 1);
  const bool b_nfast = (g.sBn2 == 1 && g.N2 > 1) || (g.N2 == 1 && g.sBn1 == 1);
  // Each thread loads LA elements of the A tile and LB of the B tile per K step, at offsets
  // advanced incrementally: k = k1 * K2 + k2 moves by BK = kq * K2 + krem, with one carry
  // into k1 when k2 wraps. Out-of-range elements are read from a zero word instead, so the
  // loads need neither branches nor a select on the loaded value (which would make each
  // load wait for its data right after issue).
  const int kq = BK / g.K2, krem = BK - kq * g.K2;
  const int dA = kq * (int)g.sAk1 + krem * (int)g.sAk2, dAw = dA + (int)g.sAk1 - g.K2 * (int)g.sAk2;
  const int dB = kq * (int)g.sBk1 + krem * (int)g.sBk2, dBw = dB + (int)g.sBk1 - g.K2 * (int)g.sBk2;
  int a_mm[LA], a_kk[LA], b_nn[LB], b_kk[LB], ak2[LA], bk2[LB];
  bool a_ok[LA], b_ok[LB], a_st[LA];
  int oa[LA], ob[LB];  // element offsets from the batch's operand base (host checks they fit)
#pragma unroll
  for (int s = 0; s < LA; ++s) {
    int e = tid + NTHR * s;
    a_st[s] = !PA || e < BM * BK;
    if (PA && !a_st[s]) e %= BM * BK;
    if (a_kfast) { a_kk[s] = e % BK; a_mm[s] = e / BK; } else { a_mm[s] = e % BM; a_kk[s] = e / BM; }
    const int m = m0 + a_mm[s];
    a_ok[s] = m < g.M;
    const int k = kbeg + a_kk[s], k1 = k / g.K2;
    ak2[s] = k - k1 * g.K2;
    oa[s] = (a_ok[s] ? (int)off2(m, g.M2, g.sAm1, g.sAm2) : 0) + k1 * (int)g.sAk1 + ak2[s] * (int)g.sAk2;
  }
#pragma unroll
  for (int s = 0; s < LB; ++s) {
    const int e = tid + NTHR * s;
    if (b_nfast) { b_nn[s] = e % BN; b_kk[s] = e / BN; } else { b_kk[s] = e % BK; b_nn[s] = e / BK; }
    const int n = n0 + b_nn[s];
    b_ok[s] = n < g.N;
    const int k = kbeg + b_kk[s], k1 = k / g.K2;
    bk2[s] = k - k1 * g.K2;
    ob[s] = (b_ok[s] ? (int)off2(n, g.N2, g.sBn1, g.sBn2) : 0) + k1 * (int)g.sBk1 + bk2[s] * (int)g.sBk2;
  }

  const int wave = tid / 64, lane = tid % 64;
  const int wm0 = (wave / WAVES_N) * (4 * WM), wn0 = (wave % WAVES_N) * (16 * WN);
  const int lx = lane / 16, lb = (lane / 4) % 4, ly = lane % 4;
  double acc[WM][WN];
#pragma unroll
  for (int i = 0; i < WM; ++i)
#pragma unroll
    for (int j = 0; j < WN; ++j) acc[i][j] = 0.0;

  auto load_tile = [&](int kt, double (&ra)[LA], double (&rb)[LB]) {
    const int klim = kend - kt;
#pragma unroll
    for (int s = 0; s < LA; ++s) {
      const bool ok = a_ok[s] && a_kk[s] < klim;
      ra[s] = gload(ok ? A + oa[s] : kZero);
      if constexpr (K1) {
        oa[s] += dA;  // single-level K: constant stride
      } else {
        ak2[s] += krem;
        const bool w = ak2[s] >= g.K2;
        ak2[s] -= w ? g.K2 : 0;
        oa[s] += w ? dAw : dA;
      }
    }
#pragma unroll
    for (int s = 0; s < LB; ++s) {
      const bool ok = b_ok[s] && b_kk[s] < klim;
      rb[s] = gload(ok ? B + ob[s] : kZero);
      if constexpr (K1) {
        ob[s] += dB;
      } else {
        bk2[s] += krem;
        const bool w = bk2[s] >= g.K2;
        bk2[s] -= w ? g.K2 : 0;
        ob[s] += w ? dBw : dB;
      }
    }
  };
  auto store_tile = [&](int buf, const double (&ra)[LA], const double (&rb)[LB]) {
#pragma unroll
    for (int s = 0; s < LA; ++s) {
      if constexpr (PA) {
        if (a_st[s]) As[buf][a_kk[s]][a_mm[s]] = ra[s];
      } else {
        As[buf][a_kk[s]][a_mm[s]] = ra[s];
      }
    }
#pragma unroll
    for (int s = 0; s < LB; ++s) Bs[buf][b_kk[s]][b_nn[s]] = rb[s];
  };
  // The fragments of K step ks + 4 are read from LDS while the MFMAs of step ks issue.
  auto compute = [&](int cur) {
    double fa[2][WM], fb[2][WN];
#pragma unroll
    for (int r = 0; r < WM; ++r) fa[0][r] = As[cur][lx][wm0 + r * 4 + ly];
#pragma unroll
    for (int c = 0; c < WN; ++c) fb[0][c] = Bs[cur][lx][wn0 + c * 16 + lb * 4 + ly];
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int h = (ks / 4) & 1;
      if (ks + 4 < BK) {
#pragma unroll
        for (int r = 0; r < WM; ++r) fa[h ^ 1][r] = As[cur][ks + 4 + lx][wm0 + r * 4 + ly];
#pragma unroll
        for (int c = 0; c < WN; ++c) fb[h ^ 1][c] = Bs[cur][ks + 4 + lx][wn0 + c * 16 + lb * 4 + ly];
      }
#pragma unroll
      for (int r = 0; r < WM; ++r)
#pragma unroll
        for (int c = 0; c < WN; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[h][r], fb[h][c], acc[r][c], 0, 0, 0);
    }
  };

  const int nkt = (kend - kbeg + BK - 1) / BK;
  double ra0[LA], rb0[LB];
  if constexpr (PF == 2) {
    // two K tiles of global loads in flight: register sets 0 and 1 alternate, LDS buffers
    // 0 and 1 alternate; tile t is in LDS buffer t % 2 when it is multiplied
    static_assert(NBUF == 2, "prefetch depth 2 needs two LDS buffers");
    // The loop body has no branch around its loads and stores: a tile past the end reads
    // only the zero word, and storing it is harmless, since the buffer it goes to is not read
    // in that phase. With such branches the compiler's wait counting merges paths on which
    // the older register set is still in flight, and then waits for every load in flight
    // before it issues the next tile's loads.
    double ra1[LA], rb1[LB];
    load_tile(kbeg, ra0, rb0);
    store_tile(0, ra0, rb0);
    load_tile(kbeg + BK, ra1, rb1);
    __syncthreads();
    for (int t = 0; t < nkt; t += 2) {
      load_tile(kbeg + (t + 2) * BK, ra0, rb0);
      compute(0);
      store_tile(1, ra1, rb1);  // tile t + 1; buffer 1 was last read before the previous barrier
      __syncthreads();
      if (t + 1 >= nkt) break;
      load_tile(kbeg + (t + 3) * BK, ra1, rb1);
      compute(1);
      store_tile(0, ra0, rb0);  // tile t + 2
      __syncthreads();
    }
  } else {
    if (nkt > 0) {
      load_tile(kbeg, ra0, rb0);
      store_tile(0, ra0, rb0);
    }
    __syncthreads();
    for (int t = 0; t < nkt; ++t) {
      const int cur = NBUF == 2 ? (t & 1) : 0;
      load_tile(kbeg + (t + 1) * BK, ra0, rb0);  // past the end: zeros, never stored
      compute(cur);
      if (NBUF == 1) __syncthreads();  // single buffer: every wave is done reading it
      if (t + 1 < nkt) store_tile(NBUF == 2 ? (cur ^ 1) : 0, ra0, rb0);
      __syncthreads();
    }
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

template <int WM, int WN, int WAVES_M, int WAVES_N, int BK, int NBUF, int PF, bool K1>
__global__ __launch_bounds__(NTHR) void gemm2_kernel(G2Args g) {
  __shared__ TileLds<4 * WM * WAVES_M, 16 * WN * WAVES_N, BK, NBUF> L;
  // Workgroups are dealt to the 8 XCDs round-robin by linear id; renumber them so that each
  // XCD (own L2) works through one contiguous range of (batch, m-tile, n-tile), where
  // neighbouring tiles share operand rows and columns.
  const int gx = gridDim.x, gy = gridDim.y;
  const int total = gx * gy * gridDim.z;
  const int lin = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  const int xcd = lin % 8, q = lin / 8, base = total / 8, rem = total % 8;
  const int tile = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + q;
  int bx, by, bz;
  tile_coords(tile, gx, gy, gridDim.z, g.batch_inner, bx, by, bz);
  gemm2_tile<WM, WN, WAVES_M, WAVES_N, BK, NBUF, PF, K1>(g, bx, by, bz, L);
}

// ---- Wide tile with LDS-direct operand loads ----
// The 64 x 128 tile of the wide variant (four waves of 32 x 64, K tile 16), whose operand tiles
// go from global memory straight into LDS (global_load_lds_dwordx4: each lane moves 16 bytes to
// the next 16 bytes of the wave's LDS window), without a register copy and an LDS store. Three
// LDS buffers hold tiles t, t + 1 and t + 2. For conflict-free fragment reads the 16-byte chunks
// of odd k rows are permuted: A rows pair up in one 1 KB window (row 2j + 1 at +512 B, chunk
// index XOR 4); B rows are 1 KB each (odd rows: chunk index XOR 8). Requirements (checked on
// the host): single-level indices, unit stride along M in A and along N in B, even M, N,
// strides and 16-byte aligned bases. Partial tiles read a 16-byte zero block.
__device__ const double kZero2[2] __attribute__((aligned(16))) = {0.0, 0.0};
constexpr int DBK = 16, DBM = 64, DBN = 128;
constexpr int DWM = 8, DWN = 4;  // 4-row and 16-column fragment groups per wave

__global__ __launch_bounds__(NTHR) void gemm2_dma_kernel(G2Args g) {
  __shared__ __attribute__((aligned(16))) double A0[DBK * DBM], A1[DBK * DBM], A2[DBK * DBM];
  __shared__ __attribute__((aligned(16))) double B0[DBK * DBN], B1[DBK * DBN], B2[DBK * DBN];
  typedef __attribute__((address_space(3))) void* lds_ptr;
  typedef const __attribute__((address_space(1))) void* glb_ptr;
  const int gx = gridDim.x, gy = gridDim.y;
  const int total = gx * gy * gridDim.z;
  const int lin = (blockIdx.z * gy + blockIdx.y) * gx + blockIdx.x;
  const int xcd = lin % 8, q = lin / 8, base = total / 8, rem = total % 8;
  const int tile = (xcd < rem ? xcd * (base + 1) : rem * (base + 1) + (xcd - rem) * base) + q;
  int bx, by, bz;
  tile_coords(tile, gx, gy, gridDim.z, g.batch_inner, bx, by, bz);
  const int split = bz / g.nbatch, bb = bz - split * g.nbatch;
  const int b1 = bb / g.nb2, b2 = bb - b1 * g.nb2;
  const double* A = g.A + b1 * g.sAb1 + b2 * g.sAb2;
  const double* B = g.B + b1 * g.sBb1 + b2 * g.sBb2;
  const int m0 = by * DBM, n0 = bx * DBN;
  const int kbeg = split * g.kchunk;
  const int kend = min(g.K, kbeg + g.kchunk);
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  // this lane's 16-byte chunks: A row pairs 2 wave, 2 wave + 1; B rows 4 wave .. 4 wave + 3
  int oa[2], ob[4], arow[2];
  bool mok[2], nok[4];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int hi = lane >> 5;
    arow[u] = 2 * (2 * wave + u) + hi;
    const int m = m0 + 2 * ((lane & 31) ^ (4 * hi));
    mok[u] = m < g.M;
    oa[u] = (mok[u] ? m : 0) + (kbeg + arow[u]) * (int)g.sAk2;
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = 4 * wave + u;
    const int n = n0 + 2 * (lane ^ (8 * (r & 1)));
    nok[u] = n < g.N;
    ob[u] = (nok[u] ? n : 0) + (kbeg + r) * (int)g.sBk2;
  }
  const int dA = DBK * (int)g.sAk2, dB = DBK * (int)g.sBk2;
  auto issue = [&](int kt, double* As, double* Bs) {
    const int klim = kend - kt;
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const double* src = (mok[u] && arow[u] < klim) ? A + oa[u] : kZero2;
      __builtin_amdgcn_global_load_lds((glb_ptr)src, (lds_ptr)(As + (2 * wave + u) * 128), 16, 0, 0);
      oa[u] += dA;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const double* src = (nok[u] && 4 * wave + u < klim) ? B + ob[u] : kZero2;
      __builtin_amdgcn_global_load_lds((glb_ptr)src, (lds_ptr)(Bs + (4 * wave + u) * 128), 16, 0, 0);
      ob[u] += dB;
    }
  };
  const int wm0 = (wave / 2) * (4 * DWM), wn0 = (wave % 2) * (16 * DWN);
  const int lx = lane / 16, lb = (lane / 4) % 4, ly = lane % 4;
  // element (k, m) of an A buffer sits at (k / 2) 128 + (k % 2) 64 + 2 ((m / 2) ^ 4 (k % 2)) + m % 2;
  // element (k, n) of a B buffer at k 128 + 2 ((n / 2) ^ 8 (k % 2)) + n % 2
  int offA[DWM], offB[DWN];
#pragma unroll
  for (int r = 0; r < DWM; ++r) offA[r] = (lx >> 1) * 128 + (lx & 1) * 64 + wm0 + ly + ((4 * r) ^ (8 * (lx & 1)));
#pragma unroll
  for (int c = 0; c < DWN; ++c) offB[c] = lx * 128 + wn0 + 4 * lb + ly + ((16 * c) ^ (16 * (lx & 1)));
  double acc[DWM][DWN];
#pragma unroll
  for (int i = 0; i < DWM; ++i)
#pragma unroll
    for (int j = 0; j < DWN; ++j) acc[i][j] = 0.0;
  auto compute = [&](const double* As, const double* Bs) {
    double fa[2][DWM], fb[2][DWN];
#pragma unroll
    for (int r = 0; r < DWM; ++r) fa[0][r] = As[offA[r]];
#pragma unroll
    for (int c = 0; c < DWN; ++c) fb[0][c] = Bs[offB[c]];
#pragma unroll
    for (int ks = 0; ks < DBK; ks += 4) {
      const int h = (ks / 4) & 1;
      if (ks + 4 < DBK) {
#pragma unroll
        for (int r = 0; r < DWM; ++r) fa[h ^ 1][r] = As[offA[r] + (ks + 4) * 64];
#pragma unroll
        for (int c = 0; c < DWN; ++c) fb[h ^ 1][c] = Bs[offB[c] + (ks + 4) * 128];
      }
#pragma unroll
      for (int r = 0; r < DWM; ++r)
#pragma unroll
        for (int c = 0; c < DWN; ++c)
          acc[r][c] = __builtin_amdgcn_mfma_f64_4x4x4f64(fa[h][r], fb[h][c], acc[r][c], 0, 0, 0);
    }
  };
  // Step t: wait for this wave's loads of tile t (those of tile t + 1, six per wave, may stay
  // in flight), then a barrier: every wave's tile t is in LDS and every wave is done with tile
  // t - 1, whose buffer then receives tile t + 2.
  auto step = [&](int t, const double* As, const double* Bs, double* An, double* Bn) {
    __builtin_amdgcn_s_waitcnt(0x0F76);  // vmcnt(6); expcnt and lgkmcnt unconstrained
    asm volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    asm volatile("" ::: "memory");
    issue(kbeg + (t + 2) * DBK, An, Bn);  // past the end: the zero block, never read
    compute(As, Bs);
  };
  const int nkt = (kend - kbeg + DBK - 1) / DBK;
  issue(kbeg, A0, B0);
  issue(kbeg + DBK, A1, B1);
  for (int t = 0; t < nkt; t += 3) {
    step(t, A0, B0, A2, B2);
    if (t + 1 >= nkt) break;
    step(t + 1, A1, B1, A0, B0);
    if (t + 2 >= nkt) break;
    step(t + 2, A2, B2, A1, B1);
  }
  // drain the loads still in flight (tiles past the end) before the workgroup's LDS is released
  __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
  // acc[r][c] at this lane is C[wm0 + 4r + lx][wn0 + 16c + 4lb + ly]
  if (g.ksplit > 1) {
    double* W = g.work + ((long)split * g.nbatch + bb) * (long)g.M * g.N;
#pragma unroll
    for (int r = 0; r < DWM; ++r) {
      const int m = m0 + wm0 + r * 4 + lx;
      if (m >= g.M) continue;
#pragma unroll
      for (int c = 0; c < DWN; ++c) {
        const int n = n0 + wn0 + c * 16 + lb * 4 + ly;
        if (n < g.N) W[(long)m * g.N + n] = acc[r][c];
      }
    }
    return;
  }
  double* C = g.C + b1 * g.sCb1 + b2 * g.sCb2;
#pragma unroll
  for (int r = 0; r < DWM; ++r) {
    const int m = m0 + wm0 + r * 4 + lx;
    if (m >= g.M) continue;
    const long crow = off2(m, g.M2, g.sCm1, g.sCm2);
#pragma unroll
    for (int c = 0; c < DWN; ++c) {
      const int n = n0 + wn0 + c * 16 + lb * 4 + ly;
      if (n >= g.N) continue;
      double* p = C + crow + off2(n, g.N2, g.sCn1, g.sCn2);
      double v = g.alpha * acc[r][c];
      if (g.beta != 0.0) v += g.beta * *p;
      *p = v;
    }
  }
}

// Many independent products in one persistent launch: workgroup w takes the tiles
// w, w + gridDim.x, ... of the concatenated tile lists (product i owns the tiles
// [prefix[i], prefix[i + 1])), so every workgroup ends after at most ceil(total / grid) tiles.
template <int WM, int WN, int WAVES_M, int WAVES_N, int BK, int NBUF, int PF>
__global__ __launch_bounds__(NTHR) void gemm2_grouped_kernel(const G2Args* gs, const int* prefix, int ngemm,
                                                             int total) {
  constexpr int BM = 4 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  __shared__ TileLds<BM, BN, BK, NBUF> L;
  for (int t = blockIdx.x; t < total; t += gridDim.x) {
    // the prefix sums are read through a global pointer (global, not flat, loads)
    const __attribute__((address_space(1))) int* pre = (const __attribute__((address_space(1))) int*)prefix;
    int lo = 0, hi = ngemm;
    while (hi - lo > 1) {
      const int mid = (lo + hi) / 2;
      if (pre[mid] <= t) lo = mid; else hi = mid;
    }
    const G2Args g = gs[lo];
    const int local = t - pre[lo];
    const int gx = (g.N + BN - 1) / BN, gy = (g.M + BM - 1) / BM;
    __syncthreads();  // the previous tile is done with the LDS buffers
    gemm2_tile<WM, WN, WAVES_M, WAVES_N, BK, NBUF, PF>(g, local % gx, (local / gx) % gy, local / (gx * gy), L);
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

template <int WM, int WN, int WAVES_M, int WAVES_N, int BK, int NBUF, int PF>
void launch(hipStream_t s, G2Args a, int nbatch) {
  constexpr int BM = 4 * WM * WAVES_M, BN = 16 * WN * WAVES_N;
  dim3 grid((a.N + BN - 1) / BN, (a.M + BM - 1) / BM, (unsigned)(nbatch * a.ksplit));
  require((long)grid.x * grid.y * grid.z < (1L << 31), IGA_EINVAL, "gemm2: grid too large");
  // a single-level K index (inner extent covering K) advances operands by a constant stride
  if (a.K2 >= a.K)
    gemm2_kernel<WM, WN, WAVES_M, WAVES_N, BK, NBUF, PF, true><<<grid, NTHR, 0, s>>>(a);
  else
    gemm2_kernel<WM, WN, WAVES_M, WAVES_N, BK, NBUF, PF, false><<<grid, NTHR, 0, s>>>(a);
}

}  // namespace

// Largest element offset of a two-level index over [0, ext) (nonnegative strides).
static long span(int ext, int inner, long s1, long s2) {
  if (ext <= 0) return 0;
  return (long)((ext - 1) / inner) * s1 + (long)(std::min(ext, inner) - 1) * s2;
}

// Validates d and fills the kernel's argument block (no split).
static G2Args make_args(const Gemm2& d) {
  require(d.M2 >= 1 && d.N2 >= 1 && d.K2 >= 1, IGA_EINVAL, "gemm2: inner extents must be >= 1");
  require(d.sAm1 >= 0 && d.sAm2 >= 0 && d.sAk1 >= 0 && d.sAk2 >= 0 && d.sBk1 >= 0 && d.sBk2 >= 0 &&
              d.sBn1 >= 0 && d.sBn2 >= 0,
          IGA_EINVAL, "gemm2: operand strides must be nonnegative");
  // the kernel addresses A and B with 32-bit element offsets from each batch's base
  const long kA = span(d.K, d.K2, d.sAk1, d.sAk2) + 64L * (d.sAk1 + d.sAk2);
  const long kB = span(d.K, d.K2, d.sBk1, d.sBk2) + 64L * (d.sBk1 + d.sBk2);
  require(span(d.M, d.M2, d.sAm1, d.sAm2) + kA < (1L << 31) && span(d.N, d.N2, d.sBn1, d.sBn2) + kB < (1L << 31),
          IGA_EINVAL, "gemm2: operand too large for 32-bit offsets");
  const long nb = (long)d.nb1 * d.nb2;
  require(nb <= 65535, IGA_EINVAL, "gemm2: batch too large");
  return G2Args{d.M, d.N, std::max(d.K, 0), d.M2, d.N2, d.K2, d.A, d.sAm1, d.sAm2, d.sAk1, d.sAk2, d.B, d.sBk1,
                d.sBk2, d.sBn1, d.sBn2, d.C, d.sCm1, d.sCm2, d.sCn1, d.sCn2, d.nb2, (int)nb, d.sAb1, d.sAb2,
                d.sBb1, d.sBb2, d.sCb1, d.sCb2, d.alpha, d.beta, 1, std::max(d.K, 0), nullptr,
                d.batch_inner ? 1 : 0};
}

// Output tile of each variant: 0: 64 x 64, 1: 32 x 128, 2: 16 x 256, 3: 128 x 32, 4: 64 x (32 WIDE_WN),
// 5: 80 x 64, 6: 64 x 96, 7: 96 x 64, 8: 24 x 128.
static void variant_tile(int v, int& BM, int& BN) {
  switch (v) {
    case 1: BM = 32; BN = 128; break;
    case 2: BM = 16; BN = 256; break;
    case 3: BM = 128; BN = 32; break;
    case 4: BM = 64; BN = 32 * IGA_WIDE_WN; break;
    case 5: BM = 80; BN = 64; break;
    case 6: BM = 64; BN = 96; break;
    case 7: BM = 96; BN = 64; break;
    case 8: BM = 24; BN = 128; break;
    default: BM = 64; BN = 64; break;
  }
}

int gemm2_variants() { return 9; }

static bool dma_eligible(const Gemm2& d);

int gemm2_pick(const Gemm2& d) {
  const long nb = (long)d.nb1 * d.nb2;
  if (d.M <= 16) return 2;
  // 17..24 rows (the blocks of the K core's middle factor, 18 to 25 ranks): a 24-row tile
  // instead of 32 rows of which a quarter or more would be padding
  if (d.M <= 24) return 8;
  if (d.M <= 32) return 1;
  if (d.N <= 32) return 3;
  if (d.M <= 64 && (long)((d.N + 32 * IGA_WIDE_WN - 1) / (32 * IGA_WIDE_WN)) * nb >= 512) return 4;
  if (d.M > 64 && d.M <= 80) return 5;  // one 80-row tile instead of 64 + 16
  // tall products with more than 64 columns (the interface stages of the local matvec, whose
  // columns are output ranks or (row, rank) pairs): a 128-wide column tile reads each row tile
  // of the long operand half as often as 64-wide tiles (measured 1.05-1.4x on those stages)
  // Without the LDS-direct loads a 96-wide tile runs about as fast per flop, so it is taken
  // where it pads the columns less (output ranks such as 74, 90 or 163: measured 1.04x on the
  // right-interface stage)
  if (d.M > 256 && d.N > 64) {
    const long w96 = (d.N + 95) / 96 * 96L, w128 = (d.N + 127) / 128 * 128L;
    return (w96 < w128 && !dma_eligible(d)) ? 6 : 4;
  }
  return 0;
}

size_t gemm2_desc_bytes() { return sizeof(G2Args); }

long gemm2_prepare(const Gemm2& d, int variant, void* host_desc) {
  G2Args a = make_args(d);
  std::memcpy(host_desc, &a, sizeof(G2Args));
  if (d.M <= 0 || d.N <= 0 || d.nb1 <= 0 || d.nb2 <= 0) return 0;
  int BM, BN;
  variant_tile(variant, BM, BN);
  return (long)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN) * a.nbatch;
}

template <int WM, int WN, int WAVES_M, int WAVES_N, int BK, int NBUF, int PF>
static void launch_grouped(hipStream_t s, const void* desc, const int* prefix, int ngemm, long total) {
  // persistent: a few workgroups per CU, each walking its share of the tiles
  const unsigned grid = (unsigned)std::min<long>(total, 1024);
  gemm2_grouped_kernel<WM, WN, WAVES_M, WAVES_N, BK, NBUF, PF>
      <<<grid, NTHR, 0, s>>>(static_cast<const G2Args*>(desc), prefix, ngemm, (int)total);
}

void gemm2_grouped(hipStream_t s, int variant, const void* dev_desc, const int* dev_prefix, int ngemm, long total) {
  if (ngemm <= 0 || total <= 0) return;
  require(total < (1L << 31), IGA_EINVAL, "gemm2_grouped: too many tiles");
  switch (variant) {
    case 2: launch_grouped<4, 4, 1, 4, 16, 2, IGA_PREFETCH>(s, dev_desc, dev_prefix, ngemm, total); break;
    case 1: launch_grouped<8, 2, 1, 4, 16, 2, IGA_PREFETCH>(s, dev_desc, dev_prefix, ngemm, total); break;
    case 3: launch_grouped<8, 2, 4, 1, 16, 2, IGA_PREFETCH>(s, dev_desc, dev_prefix, ngemm, total); break;
    case 4:
      launch_grouped<8, IGA_WIDE_WN, 2, 2, IGA_WIDE_BK, IGA_WIDE_NBUF, IGA_WIDE_PREFETCH>(s, dev_desc, dev_prefix,
                                                                                         ngemm, total);
      break;
    case 5: launch_grouped<10, 2, 2, 2, 16, 2, IGA_PREFETCH>(s, dev_desc, dev_prefix, ngemm, total); break;
    case 6: launch_grouped<8, 3, 2, 2, 16, 2, IGA_PREFETCH>(s, dev_desc, dev_prefix, ngemm, total); break;
    case 7: launch_grouped<12, 2, 2, 2, 16, 2, IGA_PREFETCH>(s, dev_desc, dev_prefix, ngemm, total); break;
    case 8: launch_grouped<6, 2, 1, 4, 16, 2, IGA_PREFETCH>(s, dev_desc, dev_prefix, ngemm, total); break;
    default: launch_grouped<8, 2, 2, 2, 16, 2, IGA_PREFETCH>(s, dev_desc, dev_prefix, ngemm, total); break;
  }
  IGA_HIP(hipGetLastError());
}

// The LDS-direct wide tile moves 16-byte chunks of two consecutive M (or N) elements: single-
// level indices, unit strides along M in A and N in B, even extents and strides, and 16-byte
// aligned operand bases.
static bool dma_eligible(const Gemm2& d) {
  auto even = [](long v) { return v % 2 == 0; };
  return d.K2 >= d.K && d.M2 >= d.M && d.N2 >= d.N && d.sAm2 == 1 && d.sBn2 == 1 && even(d.M) && even(d.N) &&
         even(d.sAk2) && even(d.sBk2) && even(d.sAb1) && even(d.sAb2) && even(d.sBb1) && even(d.sBb2) &&
         reinterpret_cast<uintptr_t>(d.A) % 16 == 0 && reinterpret_cast<uintptr_t>(d.B) % 16 == 0;
}

void gemm2(hipStream_t s, const Gemm2& d, double* work, size_t work_len) {
  if (d.M <= 0 || d.N <= 0 || d.nb1 <= 0 || d.nb2 <= 0) return;
  G2Args a = make_args(d);
  const long nb = a.nbatch;
  // tile shape by output shape
  const int variant = d.variant >= 0 ? d.variant : gemm2_pick(d);
  int BM, BN;
  variant_tile(variant, BM, BN);
  const long tiles = (long)((d.M + BM - 1) / BM) * ((d.N + BN - 1) / BN) * nb;
  // split K when the tiles cannot fill the chip (about four workgroups per CU) and the
  // contraction is long
  // long contraction (K >= 4096) whose tiles give fewer than ~16 workgroups per CU: split
  // into about 2048 workgroups and chunks of at most 8192, so that no workgroup runs one long
  // serial K loop while the chip idles
  constexpr int KALIGN = 48;  // split-K chunks are whole K tiles of every variant (12 or 16 deep)
  int want = 1;
  if (tiles < 512 && d.K >= 4 * KALIGN)
    want = (int)((1024 + tiles - 1) / tiles);
  else if (tiles < 4096 && d.K >= 4096)
    want = (int)std::max<long>((2048 + tiles - 1) / tiles, (d.K + 8191) / 8192);
  if (work && want > 1) {
    int ks = (int)std::min<long>(want, d.K / (2 * KALIGN));
    while (ks > 1 && (size_t)ks * nb * d.M * d.N > work_len) --ks;
    if (ks > 1) {
      a.ksplit = ks;
      a.kchunk = ((d.K + ks - 1) / ks + KALIGN - 1) / KALIGN * KALIGN;
      a.ksplit = (d.K + a.kchunk - 1) / a.kchunk;
      a.work = work;
    }
  }
  require((long)nb * a.ksplit <= 65535, IGA_EINVAL, "gemm2: batch too large");
  if (IGA_DMA && variant == 4 && IGA_WIDE_WN == 4 && dma_eligible(d)) {
    dim3 grid((a.N + DBN - 1) / DBN, (a.M + DBM - 1) / DBM, (unsigned)(nb * a.ksplit));
    require((long)grid.x * grid.y * grid.z < (1L << 31), IGA_EINVAL, "gemm2: grid too large");
    gemm2_dma_kernel<<<grid, NTHR, 0, s>>>(a);
  } else {
  switch (variant) {
    case 2: launch<4, 4, 1, 4, 16, 2, IGA_PREFETCH>(s, a, (int)nb); break;
    case 1: launch<8, 2, 1, 4, 16, 2, IGA_PREFETCH>(s, a, (int)nb); break;
    case 3: launch<8, 2, 4, 1, 16, 2, IGA_PREFETCH>(s, a, (int)nb); break;
    case 4: launch<8, IGA_WIDE_WN, 2, 2, IGA_WIDE_BK, IGA_WIDE_NBUF, IGA_WIDE_PREFETCH>(s, a, (int)nb); break;
    case 5: launch<10, 2, 2, 2, 16, 2, IGA_PREFETCH>(s, a, (int)nb); break;
    case 6: launch<8, 3, 2, 2, 16, 2, IGA_PREFETCH>(s, a, (int)nb); break;
    case 7: launch<12, 2, 2, 2, 16, 2, IGA_PREFETCH>(s, a, (int)nb); break;
    case 8: launch<6, 2, 1, 4, 16, 2, IGA_PREFETCH>(s, a, (int)nb); break;
    default: launch<8, 2, 2, 2, 16, 2, IGA_PREFETCH>(s, a, (int)nb); break;
  }
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
