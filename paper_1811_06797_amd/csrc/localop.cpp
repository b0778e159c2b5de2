// Projected local KKT operator (see localop.hpp) and the raw-buffer entry point.
#include "localop.hpp"

#include <algorithm>
#include <tuple>
#include <map>
#include <cstring>
#include <array>
#include <memory>
#include <unordered_map>
#include <vector>

#include "kernels.hpp"

namespace iga {

// An event from the context's reusable set (created on first use).
static hipEvent_t prof_event(iga_ctx* ctx) {
  if (ctx->prof_next == ctx->prof_events.size()) {
    hipEvent_t e;
    IGA_HIP(hipEventCreate(&e));
    ctx->prof_events.push_back(e);
  }
  return ctx->prof_events[ctx->prof_next++];
}

double band_nnz(int n, int p) {
  double s = 0;
  for (int i = 0; i < n; ++i) s += std::min(n - 1, i + p) - std::max(0, i - p) + 1;
  return s;
}

static double op_flops(const OpView& A, int r0o, int r0, int r1o, int r1, int ncol, double nnz_band) {
  // stage 1: 2 r0o r0 R0 n r1; stage 2: 2 r0o r1 (nonzero R0 x R1) nnz_band; stage 3: 2 r0o n R1 r1 r1o
  const double nz_blocks = A.flops_dense_factor * double(A.R0) * A.R1;
  return ncol * (2.0 * r0o * r0 * A.R0 * A.n * r1 + 2.0 * r0o * r1 * nz_blocks * nnz_band +
                 2.0 * r0o * A.n * A.R1 * (double)r1 * r1o);
}

double local_flops(const LocalOp& L) {
  const double nb = band_nnz(L.n, L.M.p);
  return op_flops(L.M, L.out0(), L.r0, L.out1(), L.r1, L.nblk, nb) +
         op_flops(L.K, L.out0(), L.r0, L.out1(), L.r1, L.kcols(), nb);
}

// Element-type plumbing of the staged apply: the FP64 and FP32 matrix-core GEMMs.
template <class T> struct Prec;
template <> struct Prec<double> {
  using G = k::Gemm2;
  static void gemm(hipStream_t s, const G& g, double* w, size_t n, bool) { k::gemm2(s, g, w, n); }
  static void zero(hipStream_t s, long n, double* y) { k::fill(s, n, 0.0, y); }
  static void band1(hipStream_t s, int n, int b, long nc, const double* A, const double* x, long ldx, double* y) {
    k::band_rank1(s, n, b, nc, A, x, ldx, y);
  }
  static void bandsm(hipStream_t s, int n, int b, int R0, int R1, long nc, const double* A, const double* x, long ldx,
                     long ldd, double* y) {
    k::band_small(s, n, b, R0, R1, nc, A, x, ldx, ldd, y);
  }
  static constexpr int prof_base = 0;
};
template <> struct Prec<float> {
  using G = k::Gemm2F;
  // FP32 storage; products in FP32 or, with bf16, on BF16 matrix cores
  static void gemm(hipStream_t s, const G& g, float* w, size_t n, bool bf16) {
    if (bf16)
      k::gemm2_bf16(s, g, w, n);
    else
      k::gemm2_f32(s, g, w, n);
  }
  static void zero(hipStream_t s, long n, float* y) { k::fill_f32(s, n, 0.0f, y); }
  static void band1(hipStream_t s, int n, int b, long nc, const float* A, const float* x, long ldx, float* y) {
    k::band_rank1_f32(s, n, b, nc, A, x, ldx, y);
  }
  static void bandsm(hipStream_t s, int n, int b, int R0, int R1, long nc, const float* A, const float* x, long ldx,
                     long ldd, float* y) {
    k::band_small_f32(s, n, b, R0, R1, nc, A, x, ldx, ldd, y);
  }
  static constexpr int prof_base = 2;
};

// One operator of the local matvec on matrix cores: for the ncol columns c of x
//   z[c][a'][i][b'] = sum PhiL[d][a'][a] A[d][i][i+o-p][g] x[c][a][i+o-p][b] PhiR[g][b'][b].
// Stage 1 writes t1[j + p][d][c][a'][b] (p zero slices on both ends of j), so that the
// banded stage is, for every row i, one dense GEMM over (o, d) whose B operand is the
// contiguous window of slices j = i-p .. i+p; one GEMM per nonzero rank block.
template <class T>
static void op_apply(iga_ctx* ctx, const OpView& A, const T* core, const T* relaid, const std::vector<RankBlock>& blocks,
                     const T* PhiL, const T* PhiR, int r0o, int r0, int r1, int r1o, int ncol, const T* x,
                     long xcs, T* z, long zcs, DevBuf<T>& t1, DevBuf<T>& t2, DevBuf<T>& wk,
                     LocalWork::PadKey& pad, int op_id, bool bf16 = false) {
  using G = typename Prec<T>::G;
  hipStream_t st = ctx->stream;
  const int n = A.n, p = A.p, b = 2 * p + 1, R0 = A.R0, R1 = A.R1;
  const long S2 = (long)r0o * r1;         // one (c) slab of (a', b)
  const long S1 = (long)ncol * S2;        // one (d) slab
  const long SJ = (long)R0 * S1;          // one j slice of t1
  t1.ensure(ctx, (size_t)(n + 2 * p) * SJ);
  t2.ensure(ctx, (size_t)n * R1 * S1);
  // the p zero slices at both ends of j are never written by stage 1: fill them once per layout
  if (p > 0 && (pad.gen != t1.gen() || pad.sj != SJ || pad.n != n || pad.p != p)) {
    Prec<T>::zero(st, p * SJ, t1.get());
    Prec<T>::zero(st, p * SJ, t1.get() + (long)(n + p) * SJ);
    pad.gen = t1.gen(); pad.sj = SJ; pad.n = n; pad.p = p;
  }
  // stage 1: one GEMM per column c with rows (d, a'): t1[j+p][d][c][a'][b] = sum_a PhiL[d][a'][a] x[c][a][j][b]
  G g1;
  g1.M = R0 * r0o; g1.N = n * r1; g1.N2 = r1; g1.K = r0;
  g1.A = PhiL; g1.sAm1 = (long)r0o * r0; g1.sAm2 = r0; g1.sAk2 = 1;
  g1.B = x; g1.sBk2 = (long)n * r1; g1.sBn1 = r1; g1.sBn2 = 1;
  g1.C = t1.get() + p * SJ; g1.M2 = r0o; g1.sCm1 = S1; g1.sCm2 = r1; g1.sCn1 = SJ; g1.sCn2 = 1;
  g1.nb1 = ncol; g1.sBb1 = xcs; g1.sCb1 = S2;
  Prec<T>::gemm(st, g1, nullptr, 0, bf16);
  // stage 2: per rank block, batched over rows i
  hipEvent_t pa = nullptr, pb = nullptr;
  if (ctx->prof_on) {
    pa = prof_event(ctx);
    pb = prof_event(ctx);
    IGA_HIP(hipEventRecord(pa, st));
  }
  const bool dense = blocks.size() == 1 && blocks[0].na == R0 && blocks[0].nb == R1;
  // a re-laid core: dense, or block-structured with few rank pairs (zeros included)
  const bool whole = relaid && (dense || (long)R0 * R1 <= kDenseRankPairs);
  if (whole && R0 == 1 && R1 == 1 && !bf16) {
    // a rank-1 core (the mass operator of a separable weight): a one-row GEMM would use one
    // sixteenth of a matrix-core tile, so the band combination of t1's slices runs as a
    // memory-bound stencil; the relaid core is [i][o]
    Prec<T>::band1(st, n, b, S1, relaid, t1.get(), SJ, t2.get());
  } else if (whole && R1 <= kSmallR1 && !bf16) {
    // few right ranks: a 16-row matrix-core tile would be mostly padding and its launch
    // overheads dominate, so the band sums run on the vector units
    Prec<T>::bandsm(st, n, b, R0, R1, S1, relaid, t1.get(), SJ, S1, t2.get());
  } else if (whole) {
    // core [i][o][d][g]: for row i the contraction index k = o R0 + d has constant strides
    // (R1 in the core, S1 in t1, whose slice i + o starts at (i + o) SJ = i SJ + o R0 S1)
    G g2;
    g2.M = R1; g2.N = (int)S1; g2.K = R0 * b;
    g2.A = relaid; g2.sAm2 = 1; g2.sAk2 = R1;
    g2.B = t1.get(); g2.sBk2 = S1; g2.sBn2 = 1;
    g2.C = t2.get(); g2.sCm2 = S1; g2.sCn2 = 1;
    g2.nb1 = n; g2.sAb1 = (long)b * R0 * R1; g2.sBb1 = SJ; g2.sCb1 = (long)R1 * S1;
    Prec<T>::gemm(st, g2, nullptr, 0, bf16);
  } else {
    for (const RankBlock& rb : blocks) {
      G g2;
      g2.M = rb.nb; g2.N = (int)S1; g2.K = rb.na * b; g2.K2 = rb.na;
      g2.A = core + (long)rb.a0 * n * b * R1 + rb.b0;
      g2.sAm2 = 1; g2.sAk1 = R1; g2.sAk2 = (long)n * b * R1;
      g2.B = t1.get() + rb.a0 * S1; g2.sBk1 = SJ; g2.sBk2 = S1; g2.sBn2 = 1;
      g2.C = t2.get() + rb.b0 * S1; g2.sCm2 = S1; g2.sCn2 = 1;
      g2.nb1 = n; g2.sAb1 = (long)b * R1; g2.sBb1 = SJ; g2.sCb1 = (long)R1 * S1;
      Prec<T>::gemm(st, g2, nullptr, 0, bf16);
    }
  }
  if (ctx->prof_on) {
    IGA_HIP(hipEventRecord(pb, st));
    double nz = 0;
    for (const RankBlock& rb : blocks) nz += (double)rb.na * rb.nb;
    ctx->prof.push_back({pa, pb, Prec<T>::prof_base + (bf16 ? 2 : 0) + op_id, (int)blocks.size(),
                         2.0 * r0o * r1 * ncol * nz * band_nnz(n, p)});
  }
  // stage 3: z[c][(a' i)][b'] = sum_{(g, b)} t2[i][g][c][a'][b] PhiR[g][b'][b]
  G g3;
  g3.M = r0o * n; g3.M2 = n; g3.N = r1o; g3.K = R1 * r1; g3.K2 = r1;
  g3.A = t2.get(); g3.sAm1 = r1; g3.sAm2 = (long)R1 * S1; g3.sAk1 = S1; g3.sAk2 = 1;
  g3.B = PhiR; g3.sBk1 = (long)r1o * r1; g3.sBk2 = 1; g3.sBn2 = r1;
  g3.C = z; g3.sCm1 = (long)n * r1o; g3.sCm2 = r1o; g3.sCn2 = 1;
  g3.nb1 = ncol; g3.sAb1 = S2; g3.sCb1 = zcs;
  const size_t wlen = (size_t)16 * ncol * r0o * n * r1o;
  wk.ensure(ctx, wlen);
  Prec<T>::gemm(st, g3, wk.get(), wlen, bf16);
}

void local_matvec(iga_ctx* ctx, const LocalOp& L, const double* x, double* y, LocalWork& w) {
  const long colsz = (long)L.r0 * L.n * L.r1;
  const int r0o = L.out0(), r1o = L.out1();
  const long osz = (long)r0o * L.n * r1o;  // one output column
  if (L.toff) {
    // general block structure: M on every block, K on its block ranges, table combination
    const int nz = L.nblk + L.kcols();
    w.z.ensure(ctx, (size_t)nz * osz);
    op_apply<double>(ctx, L.M, L.M.A, L.M.Ar, L.Mblocks, L.PhiL_M, L.PhiR_M, r0o, L.r0, L.r1, r1o, L.nblk, x,
                     colsz, w.z.get(), osz, w.tM, w.tM2, w.split, w.padM, 0);
    int pos = L.nblk;
    for (int j = 0; j < L.nkr; ++j) {
      op_apply<double>(ctx, L.K, L.K.A, L.K.Ar, L.Kblocks, L.PhiL_K, L.PhiR_K, r0o, L.r0, L.r1, r1o, L.kn[j],
                       x + L.kb[j] * colsz, colsz, w.z.get() + pos * osz, osz, w.tK, w.tK2, w.split, w.padK, 1);
      pos += L.kn[j];
    }
    k::combine_blocks(ctx->stream, osz, L.nblk, L.toff, L.src, L.tcoef, w.z.get(), y);
    return;
  }
  w.z.ensure(ctx, (size_t)5 * osz);
  op_apply<double>(ctx, L.M, L.M.A, L.M.Ar, L.Mblocks, L.PhiL_M, L.PhiR_M, r0o, L.r0, L.r1, r1o, 3, x, colsz, w.z.get(),
                   osz, w.tM, w.tM2, w.split, w.padM, 0);
  op_apply<double>(ctx, L.K, L.K.A, L.K.Ar, L.Kblocks, L.PhiL_K, L.PhiR_K, r0o, L.r0, L.r1, r1o, 2, x, 2 * colsz,
                   w.z.get() + 3 * osz, osz, w.tK, w.tK2, w.split, w.padK, 1);
  k::kkt_combine(ctx->stream, osz, L.coef, w.z.get(), w.z.get() + 3 * osz, y);
}

void local_matvec_f32(iga_ctx* ctx, const LocalOp& L, const float* x, float* y, LocalWork& w, bool bf16) {
  require(L.M.Af && L.K.Af && L.fPhiL_M && L.fPhiR_M && L.fPhiL_K && L.fPhiR_K, IGA_EINVAL,
          "local_matvec_f32: FP32 operands missing");
  require(L.toff == nullptr, IGA_EINVAL, "local_matvec_f32: the time-dependent system is FP64 only");
  const long colsz = (long)L.r0 * L.n * L.r1;
  const int r0o = L.out0(), r1o = L.out1();
  const long osz = (long)r0o * L.n * r1o;
  w.fz.ensure(ctx, (size_t)5 * osz);
  op_apply<float>(ctx, L.M, L.M.Af, L.M.Arf, L.Mblocks, L.fPhiL_M, L.fPhiR_M, r0o, L.r0, L.r1, r1o, 3, x, colsz,
                  w.fz.get(), osz, w.ftM, w.ftM2, w.fsplit, w.fpadM, 0, bf16);
  op_apply<float>(ctx, L.K, L.K.Af, L.K.Arf, L.Kblocks, L.fPhiL_K, L.fPhiR_K, r0o, L.r0, L.r1, r1o, 2, x, 2 * colsz,
                  w.fz.get() + 3 * osz, osz, w.ftK, w.ftK2, w.fsplit, w.fpadK, 1, bf16);
  k::kkt_combine_f32(ctx->stream, osz, L.coef, w.fz.get(), w.fz.get() + 3 * osz, y);
}

// ---- raw-buffer entry point (dense rank blocks) ----

namespace {
struct RawCache {
  IBuf loM1, hiM1, loM0, hiM0, loK1, hiK1, loK0, hiK0;
  int RM0 = -1, RM1 = -1, RK0 = -1, RK1 = -1;
  LocalWork w;
  FBuf fPhi[4], fM, fK, fx, fy;
  DBuf rM, rK;  // cores re-laid for the banded stage
  FBuf frM, frK;  // their FP32 copies (mixed-precision forms)
};
std::unordered_map<iga_ctx*, std::unique_ptr<RawCache>> g_raw;
RawCache& raw_cache(iga_ctx* ctx) {
  auto& p = g_raw[ctx];
  if (!p) p.reset(new RawCache());
  return *p;
}
void dense_ranges(iga_ctx* ctx, int R0, int R1, IBuf& lo1, IBuf& hi1, IBuf& lo0, IBuf& hi0) {
  std::vector<int> z1(R1, 0), h1(R1, R0), z0(R0, 0), h0(R0, R1);
  lo1.reset(ctx, R1); hi1.reset(ctx, R1); lo0.reset(ctx, R0); hi0.reset(ctx, R0);
  IGA_HIP(hipMemcpyAsync(lo1.get(), z1.data(), R1 * 4, hipMemcpyHostToDevice, ctx->stream));
  IGA_HIP(hipMemcpyAsync(hi1.get(), h1.data(), R1 * 4, hipMemcpyHostToDevice, ctx->stream));
  IGA_HIP(hipMemcpyAsync(lo0.get(), z0.data(), R0 * 4, hipMemcpyHostToDevice, ctx->stream));
  IGA_HIP(hipMemcpyAsync(hi0.get(), h0.data(), R0 * 4, hipMemcpyHostToDevice, ctx->stream));
  IGA_HIP(hipStreamSynchronize(ctx->stream));
}
}  // namespace

void release_raw_cache(iga_ctx* ctx) { g_raw.erase(ctx); }

double local_matvec_flops(int r0, int n, int r1, int p, int RM0, int RM1, int RK0, int RK1) {
  LocalOp L;
  L.r0 = r0; L.n = n; L.r1 = r1;
  L.M.R0 = RM0; L.M.R1 = RM1; L.M.n = n; L.M.p = p;
  L.K.R0 = RK0; L.K.R1 = RK1; L.K.n = n; L.K.p = p;
  return local_flops(L);
}

void local_matvec_impl(iga_ctx* ctx, int r0, int n, int r1, int p, int RM0, int RM1, int RK0, int RK1,
                       const double* PhiL_M, const double* PhiR_M, const double* PhiL_K,
                       const double* PhiR_K, const double* Mcore, const double* Kcore, double beta,
                       const double* x, double* y, int precision) {
  RawCache& C = raw_cache(ctx);
  if (C.RM0 != RM0 || C.RM1 != RM1) {
    dense_ranges(ctx, RM0, RM1, C.loM1, C.hiM1, C.loM0, C.hiM0);
    C.RM0 = RM0; C.RM1 = RM1;
  }
  if (C.RK0 != RK0 || C.RK1 != RK1) {
    dense_ranges(ctx, RK0, RK1, C.loK1, C.hiK1, C.loK0, C.hiK0);
    C.RK0 = RK0; C.RK1 = RK1;
  }
  LocalOp L;
  L.r0 = r0; L.n = n; L.r1 = r1;
  L.coef.m11 = beta;
  L.M.R0 = RM0; L.M.R1 = RM1; L.M.n = n; L.M.p = p; L.M.A = Mcore;
  L.M.lo_R1 = C.loM1.get(); L.M.hi_R1 = C.hiM1.get(); L.M.lo_R0 = C.loM0.get(); L.M.hi_R0 = C.hiM0.get();
  L.K.R0 = RK0; L.K.R1 = RK1; L.K.n = n; L.K.p = p; L.K.A = Kcore;
  L.K.lo_R1 = C.loK1.get(); L.K.hi_R1 = C.hiK1.get(); L.K.lo_R0 = C.loK0.get(); L.K.hi_R0 = C.hiK0.get();
  L.PhiL_M = PhiL_M; L.PhiR_M = PhiR_M; L.PhiL_K = PhiL_K; L.PhiR_K = PhiR_K;
  L.Mblocks = {RankBlock{0, RM0, 0, RM1}};
  L.Kblocks = {RankBlock{0, RK0, 0, RK1}};
  if (precision == IGA_FP64) {
    // cores re-laid as [n][2p+1][R0][R1] for the banded stage
    const int dimsM[4] = {RM0, n, 2 * p + 1, RM1}, dimsK[4] = {RK0, n, 2 * p + 1, RK1}, perm[4] = {1, 2, 0, 3};
    C.rM.ensure(ctx, (size_t)RM0 * n * (2 * p + 1) * RM1);
    C.rK.ensure(ctx, (size_t)RK0 * n * (2 * p + 1) * RK1);
    k::permute4(ctx->stream, Mcore, dimsM, perm, C.rM.get());
    k::permute4(ctx->stream, Kcore, dimsK, perm, C.rK.get());
    L.M.Ar = C.rM.get();
    L.K.Ar = C.rK.get();
    local_matvec(ctx, L, x, y, C.w);
    return;
  }
  // FP32 / BF16: convert every operand to FP32, contract (BF16 products round the operands
  // once more as they are staged), convert the result back
  hipStream_t st = ctx->stream;
  const int b = 2 * p + 1;
  const long szs[4] = {(long)RM0 * r0 * r0, (long)RM1 * r1 * r1, (long)RK0 * r0 * r0, (long)RK1 * r1 * r1};
  const double* src[4] = {PhiL_M, PhiR_M, PhiL_K, PhiR_K};
  for (int i = 0; i < 4; ++i) {
    C.fPhi[i].ensure(ctx, szs[i]);
    k::to_f32(st, szs[i], src[i], C.fPhi[i].get());
  }
  const long mz = (long)RM0 * n * b * RM1, kz = (long)RK0 * n * b * RK1, xz = L.size();
  C.fM.ensure(ctx, mz); C.fK.ensure(ctx, kz); C.fx.ensure(ctx, xz); C.fy.ensure(ctx, xz);
  k::to_f32(st, mz, Mcore, C.fM.get());
  k::to_f32(st, kz, Kcore, C.fK.get());
  k::to_f32(st, xz, x, C.fx.get());
  L.M.Af = C.fM.get(); L.K.Af = C.fK.get();
  {
    // re-laid cores, as in the FP64 form, converted to FP32
    const int dimsM[4] = {RM0, n, b, RM1}, dimsK[4] = {RK0, n, b, RK1}, perm[4] = {1, 2, 0, 3};
    C.rM.ensure(ctx, mz); C.rK.ensure(ctx, kz);
    C.frM.ensure(ctx, mz); C.frK.ensure(ctx, kz);
    k::permute4(st, Mcore, dimsM, perm, C.rM.get());
    k::permute4(st, Kcore, dimsK, perm, C.rK.get());
    k::to_f32(st, mz, C.rM.get(), C.frM.get());
    k::to_f32(st, kz, C.rK.get(), C.frK.get());
    L.M.Arf = C.frM.get(); L.K.Arf = C.frK.get();
  }
  L.fPhiL_M = C.fPhi[0].get(); L.fPhiR_M = C.fPhi[1].get();
  L.fPhiL_K = C.fPhi[2].get(); L.fPhiR_K = C.fPhi[3].get();
  local_matvec_f32(ctx, L, C.fx.get(), C.fy.get(), C.w, precision == IGA_BF16);
  k::to_f64(st, xz, C.fy.get(), y);
}

}  // namespace iga

// ---- batched local operators: many independent problems, one grouped launch per stage ----

namespace iga {

namespace {

struct BatchCache {
  DBuf ws;              // FP64 intermediates (t1, t2, z) of all problems
  FBuf fws;             // FP32 operand copies
  FBuf fws2;            // FP32 intermediates
  DBuf stage;           // device copy of the descriptor block (bytes, rounded up to doubles)
  std::vector<char> host;
  std::map<long, int> tuned;  // (precision, stage, size bucket) -> fastest tile variant
};
std::unordered_map<iga_ctx*, std::unique_ptr<BatchCache>> g_batch;

int log2_bucket(long x) {
  int b = 0;
  while ((1L << b) < x && b < 30) ++b;
  return b;
}

template <class T> struct GroupedOps;
template <> struct GroupedOps<double> {
  using G = k::Gemm2;
  static int pick(const G& g) { return k::gemm2_pick(g); }
  static int variants() { return k::gemm2_variants(); }
  static size_t bytes() { return k::gemm2_desc_bytes(); }
  static long prepare(const G& g, int v, void* h) { return k::gemm2_prepare(g, v, h); }
  static void launch(hipStream_t s, int v, const void* d, const int* pre, int n, long t) {
    k::gemm2_grouped(s, v, d, pre, n, t);
  }
  static void fill(hipStream_t s, int n, long m, const k::Segment* seg, double* b) { k::fill_segments(s, n, m, seg, b); }
  static void combine(hipStream_t s, int n, long m, const k::CombineItem* it, const double* z) {
    k::combine_grouped(s, n, m, it, z);
  }
  static constexpr int prec = 0;
};
template <> struct GroupedOps<float> {
  using G = k::Gemm2F;
  static int pick(const G& g) { return k::gemm2f_pick(g); }
  static int variants() { return 5; }
  static size_t bytes() { return k::gemm2f_desc_bytes(); }
  static long prepare(const G& g, int v, void* h) { return k::gemm2f_prepare(g, v, h); }
  static void launch(hipStream_t s, int v, const void* d, const int* pre, int n, long t) {
    k::gemm2f_grouped(s, v, d, pre, n, t);
  }
  static void fill(hipStream_t s, int n, long m, const k::Segment* seg, float* b) { k::fill_segments_f32(s, n, m, seg, b); }
  static void combine(hipStream_t s, int n, long m, const k::CombineItem* it, const float* z) {
    k::combine_grouped_f32(s, n, m, it, z);
  }
  static constexpr int prec = 1;
};

struct ProbPtrs {  // operands of one problem in the working precision
  const void* PhiL[2];
  const void* PhiR[2];
  const void* core[2];
  const void* x;
  void* y;
};

// Appends bytes to the host staging block at an aligned offset; returns the offset.
size_t stage_append(std::vector<char>& h, const void* src, size_t n) {
  size_t off = (h.size() + 255) / 256 * 256;
  h.resize(off + n);
  std::memcpy(h.data() + off, src, n);
  return off;
}

template <class T>
void batched_run(iga_ctx* ctx, const std::vector<BatchProblem>& P, const std::vector<ProbPtrs>& ptr,
                 DevBuf<T>& ws, BatchCache& C, bool autotune) {
  using Ops = GroupedOps<T>;
  using G = typename Ops::G;
  hipStream_t st = ctx->stream;
  const int np = (int)P.size();
  // workspace layout: per problem z (5 output columns), then per operator t1 and t2
  std::vector<long> zoff(np), t1off(2 * np), t2off(2 * np);
  long total = 0;
  for (int i = 0; i < np; ++i) {
    const BatchProblem& q = P[i];
    const long osz = (long)q.r0 * q.n * q.r1;
    zoff[i] = total;
    total += 5 * osz;
    for (int o = 0; o < 2; ++o) {
      const int ncol = o == 0 ? 3 : 2, R0 = o == 0 ? q.RM0 : q.RK0, R1 = o == 0 ? q.RM1 : q.RK1;
      const long S1 = (long)ncol * q.r0 * q.r1, SJ = (long)R0 * S1;
      t1off[2 * i + o] = total;
      total += (long)(q.n + 2 * q.p) * SJ;
      t2off[2 * i + o] = total;
      total += (long)q.n * R1 * S1;
    }
  }
  ws.ensure(ctx, (size_t)total);
  T* base = ws.get();
  // products of the three stages, and the pad segments / combine items
  std::vector<G> gemms[3];
  std::vector<k::Segment> segs;
  std::vector<k::CombineItem> comb;
  long maxseg = 0, maxe = 0;
  for (int i = 0; i < np; ++i) {
    const BatchProblem& q = P[i];
    const int n = q.n, p = q.p, b = 2 * p + 1, r0 = q.r0, r1 = q.r1;
    const long osz = (long)r0 * n * r1, colsz = osz;
    for (int o = 0; o < 2; ++o) {
      const int ncol = o == 0 ? 3 : 2, R0 = o == 0 ? q.RM0 : q.RK0, R1 = o == 0 ? q.RM1 : q.RK1;
      const long S2 = (long)r0 * r1, S1 = ncol * S2, SJ = (long)R0 * S1;
      T* t1 = base + t1off[2 * i + o];
      T* t2 = base + t2off[2 * i + o];
      const T* x = static_cast<const T*>(ptr[i].x);
      const long xcs = o == 0 ? colsz : 2 * colsz;  // K takes columns 0 and 2
      T* z = base + zoff[i] + (o == 0 ? 0 : 3 * osz);
      if (p > 0) {
        segs.push_back({t1off[2 * i + o], p * SJ});
        segs.push_back({t1off[2 * i + o] + (long)(n + p) * SJ, p * SJ});
        maxseg = std::max(maxseg, p * SJ);
      }
      G g1;
      g1.M = R0 * r0; g1.N = n * r1; g1.N2 = r1; g1.K = r0;
      g1.A = static_cast<const T*>(ptr[i].PhiL[o]); g1.sAm1 = (long)r0 * r0; g1.sAm2 = r0; g1.sAk2 = 1;
      g1.B = x; g1.sBk2 = (long)n * r1; g1.sBn1 = r1; g1.sBn2 = 1;
      g1.C = t1 + p * SJ; g1.M2 = r0; g1.sCm1 = S1; g1.sCm2 = r1; g1.sCn1 = SJ; g1.sCn2 = 1;
      g1.nb1 = ncol; g1.sBb1 = xcs; g1.sCb1 = S2;
      gemms[0].push_back(g1);
      G g2;
      g2.M = R1; g2.N = (int)S1; g2.K = R0 * b; g2.K2 = R0;
      g2.A = static_cast<const T*>(ptr[i].core[o]);
      g2.sAm2 = 1; g2.sAk1 = R1; g2.sAk2 = (long)n * b * R1;
      g2.B = t1; g2.sBk1 = SJ; g2.sBk2 = S1; g2.sBn2 = 1;
      g2.C = t2; g2.sCm2 = S1; g2.sCn2 = 1;
      g2.nb1 = n; g2.sAb1 = (long)b * R1; g2.sBb1 = SJ; g2.sCb1 = (long)R1 * S1;
      gemms[1].push_back(g2);
      G g3;
      g3.M = r0 * n; g3.M2 = n; g3.N = r1; g3.K = R1 * r1; g3.K2 = r1;
      g3.A = t2; g3.sAm1 = r1; g3.sAm2 = (long)R1 * S1; g3.sAk1 = S1; g3.sAk2 = 1;
      g3.B = static_cast<const T*>(ptr[i].PhiR[o]); g3.sBk1 = (long)r1 * r1; g3.sBk2 = 1; g3.sBn2 = r1;
      g3.C = z; g3.sCm1 = (long)n * r1; g3.sCm2 = r1; g3.sCn2 = 1;
      g3.nb1 = ncol; g3.sAb1 = S2; g3.sCb1 = osz;
      gemms[2].push_back(g3);
    }
    k::KktCoef cf;
    cf.m11 = q.beta;
    comb.push_back({zoff[i], osz, ptr[i].y, cf});
    maxe = std::max(maxe, osz);
  }
  auto key_of = [&](int s, const G& g) {
    return (long)Ops::prec * 100000000L + s * 1000000L + log2_bucket(g.M) * 10000L + log2_bucket(g.N) * 100L +
           log2_bucket((long)g.K * g.nb1 * g.nb2);
  };
  const size_t db = Ops::bytes();
  // stages the descriptor block of a list of products for one variant; returns (desc, prefix) offsets
  auto stage_group = [&](std::vector<char>& h, const std::vector<const G*>& list, int v, size_t& doff,
                         size_t& poff, long& tiles) {
    std::vector<char> d(db * list.size());
    std::vector<int> pre(list.size() + 1, 0);
    tiles = 0;
    for (size_t j = 0; j < list.size(); ++j) {
      pre[j] = (int)tiles;
      tiles += Ops::prepare(*list[j], v, d.data() + j * db);
    }
    pre[list.size()] = (int)tiles;
    doff = stage_append(h, d.data(), d.size());
    poff = stage_append(h, pre.data(), pre.size() * sizeof(int));
  };
  auto upload = [&](const std::vector<char>& h) -> const char* {
    C.stage.ensure(ctx, (h.size() + 7) / 8);
    IGA_HIP(hipMemcpyAsync(C.stage.get(), h.data(), h.size(), hipMemcpyHostToDevice, st));
    IGA_HIP(hipStreamSynchronize(st));
    return reinterpret_cast<const char*>(C.stage.get());
  };
  // pads, once per call (the intermediates are shared with other calls)
  {
    std::vector<char> h;
    const size_t so = segs.empty() ? 0 : stage_append(h, segs.data(), segs.size() * sizeof(k::Segment));
    if (!segs.empty()) {
      const char* d = upload(h);
      Ops::fill(st, (int)segs.size(), maxseg, reinterpret_cast<const k::Segment*>(d + so), base);
      IGA_HIP(hipStreamSynchronize(st));
    }
  }
  for (int s = 0; s < 3; ++s) {
    // buckets of this stage
    std::map<long, std::vector<const G*>> buckets;
    for (const G& g : gemms[s]) buckets[key_of(s, g)].push_back(&g);
    if (autotune) {
      for (auto& kv : buckets) {
        if (C.tuned.count(kv.first)) continue;
        float best = 1e30f;
        int bestv = Ops::pick(*kv.second[0]);
        for (int v = 0; v < Ops::variants(); ++v) {
          std::vector<char> h;
          size_t doff, poff;
          long tiles;
          stage_group(h, kv.second, v, doff, poff, tiles);
          const char* d = upload(h);
          hipEvent_t e0, e1;
          IGA_HIP(hipEventCreate(&e0));
          IGA_HIP(hipEventCreate(&e1));
          IGA_HIP(hipEventRecord(e0, st));
          Ops::launch(st, v, d + doff, reinterpret_cast<const int*>(d + poff), (int)kv.second.size(), tiles);
          IGA_HIP(hipEventRecord(e1, st));
          IGA_HIP(hipEventSynchronize(e1));
          float ms = 0.0f;
          IGA_HIP(hipEventElapsedTime(&ms, e0, e1));
          IGA_HIP(hipEventDestroy(e0));
          IGA_HIP(hipEventDestroy(e1));
          if (ms < best) { best = ms; bestv = v; }
        }
        C.tuned[kv.first] = bestv;
      }
    }
    // groups by variant: one grouped launch each
    std::map<int, std::vector<const G*>> groups;
    for (auto& kv : buckets) {
      auto it = C.tuned.find(kv.first);
      const int v = it != C.tuned.end() ? it->second : Ops::pick(*kv.second[0]);
      auto& dst = groups[v];
      dst.insert(dst.end(), kv.second.begin(), kv.second.end());
    }
    std::vector<char> h;
    std::vector<std::tuple<int, size_t, size_t, long, int>> launches;
    for (auto& kv : groups) {
      size_t doff, poff;
      long tiles;
      stage_group(h, kv.second, kv.first, doff, poff, tiles);
      launches.emplace_back(kv.first, doff, poff, tiles, (int)kv.second.size());
    }
    const char* d = upload(h);
    for (auto& L : launches)
      Ops::launch(st, std::get<0>(L), d + std::get<1>(L), reinterpret_cast<const int*>(d + std::get<2>(L)),
                  std::get<4>(L), std::get<3>(L));
    IGA_HIP(hipStreamSynchronize(st));  // the staging block is reused by the next stage
  }
  {
    std::vector<char> h;
    const size_t co = stage_append(h, comb.data(), comb.size() * sizeof(k::CombineItem));
    const char* d = upload(h);
    Ops::combine(st, (int)comb.size(), maxe, reinterpret_cast<const k::CombineItem*>(d + co), base);
    IGA_HIP(hipStreamSynchronize(st));
  }
}

}  // namespace

void release_batch_cache(iga_ctx* ctx) { g_batch.erase(ctx); }

void local_matvec_batched_impl(iga_ctx* ctx, const std::vector<BatchProblem>& P, int precision, bool autotune) {
  auto& cp = g_batch[ctx];
  if (!cp) cp.reset(new BatchCache());
  BatchCache& C = *cp;
  for (const BatchProblem& q : P) {
    require(q.r0 >= 1 && q.r1 >= 1 && q.n >= 1 && q.p >= 0 && q.RM0 >= 1 && q.RM1 >= 1 && q.RK0 >= 1 &&
                q.RK1 >= 1,
            IGA_EINVAL, "local_matvec_batched: bad sizes");
    require(q.PhiL_M && q.PhiR_M && q.PhiL_K && q.PhiR_K && q.Mcore && q.Kcore && q.x && q.y, IGA_EINVAL,
            "local_matvec_batched: NULL operand");
  }
  const int np = (int)P.size();
  std::vector<ProbPtrs> ptr(np);
  if (precision == IGA_FP64) {
    for (int i = 0; i < np; ++i) {
      const BatchProblem& q = P[i];
      ptr[i] = ProbPtrs{{q.PhiL_M, q.PhiL_K}, {q.PhiR_M, q.PhiR_K}, {q.Mcore, q.Kcore}, q.x, q.y};
    }
    batched_run<double>(ctx, P, ptr, C.ws, C, autotune);
    return;
  }
  // FP32: convert every operand in one grouped launch, contract, convert the results back
  hipStream_t st = ctx->stream;
  std::vector<long> off(np * 8 + 1, 0);
  std::vector<k::ConvSegment> in, out;
  long pos = 0, maxlen = 0;
  std::vector<std::array<long, 8>> at(np);
  for (int i = 0; i < np; ++i) {
    const BatchProblem& q = P[i];
    const int b = 2 * q.p + 1;
    const long len[8] = {(long)q.RM0 * q.r0 * q.r0, (long)q.RM1 * q.r1 * q.r1, (long)q.RK0 * q.r0 * q.r0,
                         (long)q.RK1 * q.r1 * q.r1, (long)q.RM0 * q.n * b * q.RM1, (long)q.RK0 * q.n * b * q.RK1,
                         3L * q.r0 * q.n * q.r1, 3L * q.r0 * q.n * q.r1};
    for (int j = 0; j < 8; ++j) {
      at[i][j] = pos;
      pos += (len[j] + 63) / 64 * 64;
      maxlen = std::max(maxlen, len[j]);
    }
  }
  C.fws.ensure(ctx, (size_t)pos);
  float* fb = C.fws.get();
  for (int i = 0; i < np; ++i) {
    const BatchProblem& q = P[i];
    const int b = 2 * q.p + 1;
    const double* src[7] = {q.PhiL_M, q.PhiR_M, q.PhiL_K, q.PhiR_K, q.Mcore, q.Kcore, q.x};
    const long len[7] = {(long)q.RM0 * q.r0 * q.r0, (long)q.RM1 * q.r1 * q.r1, (long)q.RK0 * q.r0 * q.r0,
                         (long)q.RK1 * q.r1 * q.r1, (long)q.RM0 * q.n * b * q.RM1, (long)q.RK0 * q.n * b * q.RK1,
                         3L * q.r0 * q.n * q.r1};
    for (int j = 0; j < 7; ++j) in.push_back({src[j], fb + at[i][j], len[j]});
    out.push_back({fb + at[i][7], q.y, 3L * q.r0 * q.n * q.r1});
    ptr[i] = ProbPtrs{{fb + at[i][0], fb + at[i][2]}, {fb + at[i][1], fb + at[i][3]}, {fb + at[i][4], fb + at[i][5]},
                      fb + at[i][6], fb + at[i][7]};
  }
  {
    std::vector<char> h;
    const size_t o = stage_append(h, in.data(), in.size() * sizeof(k::ConvSegment));
    C.stage.ensure(ctx, (h.size() + 7) / 8);
    IGA_HIP(hipMemcpyAsync(C.stage.get(), h.data(), h.size(), hipMemcpyHostToDevice, st));
    k::convert_segments(st, (int)in.size(), maxlen,
                        reinterpret_cast<const k::ConvSegment*>(reinterpret_cast<const char*>(C.stage.get()) + o), true);
    IGA_HIP(hipStreamSynchronize(st));
  }
  batched_run<float>(ctx, P, ptr, C.fws2, C, autotune);
  {
    std::vector<char> h;
    const size_t o = stage_append(h, out.data(), out.size() * sizeof(k::ConvSegment));
    C.stage.ensure(ctx, (h.size() + 7) / 8);
    IGA_HIP(hipMemcpyAsync(C.stage.get(), h.data(), h.size(), hipMemcpyHostToDevice, st));
    k::convert_segments(st, (int)out.size(), maxlen,
                        reinterpret_cast<const k::ConvSegment*>(reinterpret_cast<const char*>(C.stage.get()) + o), false);
    IGA_HIP(hipStreamSynchronize(st));
  }
}

}  // namespace iga
