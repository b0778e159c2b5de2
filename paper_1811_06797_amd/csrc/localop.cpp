// Projected local KKT operator (see localop.hpp) and the raw-buffer entry point.
#include "localop.hpp"

#include <algorithm>
#include <tuple>
#include <map>
#include <cstring>
#include <array>
#include <memory>
#include <mutex>
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
// Element counts of the intermediates of op_apply: t1 (with its p zero end slices), t2, and
// the split-K partials of stage 3.
static long op_t1_len(int n, int p, int R0, int r0o, int r1, int ncol) {
  return (long)(n + 2 * p) * R0 * ncol * r0o * r1;
}
static long op_t2_len(int n, int R1, int r0o, int r1, int ncol) { return (long)n * R1 * ncol * r0o * r1; }
static long op_split_len(int n, int r0o, int r1o, int ncol) { return 16L * ncol * r0o * n * r1o; }

// An operator core as the banded stage contracts it: element (d, i, o, g) -- input rank d,
// row i, band offset o (column j = i + o - p), output rank g -- at d s_in + g s_out + i s_row +
// o s_off of core. The usual orientation (input = left rank, output = right rank) has s_in =
// n b R1, s_out = 1, s_row = b R1, s_off = R1; the transposed one (used by the right interface
// update) swaps s_in and s_out. relaid is the core re-laid as [n][b][Rin][Rout] in this
// orientation (or null); blocks are its nonzero rank blocks (a0, na over input ranks, b0, nb
// over output ranks).
template <class T>
struct BandCore {
  int n = 0, p = 0, Rin = 0, Rout = 0;
  const T* core = nullptr;
  long s_in = 0, s_out = 0, s_row = 0, s_off = 0;
  const T* relaid = nullptr;
  const std::vector<RankBlock>* blocks = nullptr;
};

template <class T>
static BandCore<T> band_core(const OpView& A, const T* core, const T* relaid, const std::vector<RankBlock>& blocks) {
  BandCore<T> c;
  const int b = 2 * A.p + 1;
  c.n = A.n; c.p = A.p; c.Rin = A.R0; c.Rout = A.R1;
  c.core = core;
  c.s_in = (long)A.n * b * A.R1; c.s_out = 1; c.s_row = (long)b * A.R1; c.s_off = A.R1;
  c.relaid = relaid;
  c.blocks = &blocks;
  return c;
}

// Tile order of a banded-stage product (batch = row i). Neighbouring rows share 2p of their
// 2p + 1 slices of t1, the B operand, while each row has its own slice of the core, the A
// operand. Taking rows fastest keeps the shared t1 slices in L2 but re-reads the row's core
// slice for every column tile; that pays only while the core slice is small (measured at
// R = 80, b = 7, 358 KB per row: rows fastest doubled the fetched bytes, no faster).
template <class T>
static bool band_rows_inner(int b, int R0, int R1) {
  return (long)b * R0 * R1 * (long)sizeof(T) <= 64 * 1024;
}

// The banded stage on a padded input: out[i][g][c] = sum_{o, d} A(d, i, o, g) in[i + o][d][c] for
// c < S1, with in[j][d][c] at j SJ + d S1 + c (p zero slices at both ends of j) and out[i][g][c]
// at (i Rout + g) S1 + c.
template <class T>
static void band_stage(hipStream_t st, const BandCore<T>& A, const T* t1, long SJ, long S1, T* t2, bool bf16) {
  using G = typename Prec<T>::G;
  const int n = A.n, p = A.p, b = 2 * p + 1, R0 = A.Rin, R1 = A.Rout;
  const std::vector<RankBlock>& blocks = *A.blocks;
  const bool dense = blocks.size() == 1 && blocks[0].na == R0 && blocks[0].nb == R1;
  // a re-laid core: dense, or block-structured with few rank pairs (zeros included)
  const T* relaid = A.relaid;
  const bool whole = relaid && (dense || (long)R0 * R1 <= kDenseRankPairs);
  if (whole && R0 == 1 && R1 == 1 && !bf16) {
    // a rank-1 core (the mass operator of a separable weight): a one-row GEMM would use one
    // sixteenth of a matrix-core tile, so the band combination of t1's slices runs as a
    // memory-bound stencil; the relaid core is [i][o]
    Prec<T>::band1(st, n, b, S1, relaid, t1, SJ, t2);
  } else if (whole && R1 <= kSmallR1 && !bf16) {
    // few output ranks: a 16-row matrix-core tile would be mostly padding and its launch
    // overheads dominate, so the band sums run on the vector units
    Prec<T>::bandsm(st, n, b, R0, R1, S1, relaid, t1, SJ, S1, t2);
  } else if (whole) {
    // core [i][o][d][g]: for row i the contraction index k = o R0 + d has constant strides
    // (R1 in the core, S1 in t1, whose slice i + o starts at (i + o) SJ = i SJ + o R0 S1)
    G g2;
    g2.M = R1; g2.N = (int)S1; g2.K = R0 * b;
    g2.A = relaid; g2.sAm2 = 1; g2.sAk2 = R1;
    g2.B = t1; g2.sBk2 = S1; g2.sBn2 = 1;
    g2.C = t2; g2.sCm2 = S1; g2.sCn2 = 1;
    g2.nb1 = n; g2.sAb1 = (long)b * R0 * R1; g2.sBb1 = SJ; g2.sCb1 = (long)R1 * S1;
    g2.batch_inner = band_rows_inner<T>(b, R0, R1);
    Prec<T>::gemm(st, g2, nullptr, 0, bf16);
  } else {
    // one product per nonzero rank block, K = (o, d) two-level; the blocks partition the
    // output ranks (a dense core, or the block-diagonal middle core of K), so every row of t2
    // is written once
    for (const RankBlock& rb : blocks) {
      G g2;
      g2.M = rb.nb; g2.N = (int)S1; g2.K = rb.na * b; g2.K2 = rb.na;
      g2.A = A.core + rb.a0 * A.s_in + rb.b0 * A.s_out;
      g2.sAm2 = A.s_out; g2.sAk1 = A.s_off; g2.sAk2 = A.s_in;
      g2.B = t1 + rb.a0 * S1; g2.sBk1 = SJ; g2.sBk2 = S1; g2.sBn2 = 1;
      g2.C = t2 + rb.b0 * S1; g2.sCm2 = S1; g2.sCn2 = 1;
      g2.nb1 = n; g2.sAb1 = A.s_row; g2.sBb1 = SJ; g2.sCb1 = (long)R1 * S1;
      g2.batch_inner = band_rows_inner<T>(b, rb.na, rb.nb);
      Prec<T>::gemm(st, g2, nullptr, 0, bf16);
    }
  }
}

// Stages 1 and 2 on caller-provided intermediates t1 and t2 (see op_apply):
//   t1[j+p][d][c][a'][b] = sum_a PhiL[d][a'][a] x[c][a][j][b]
//   t2[i][g][c][a'][b]   = sum_{o,d} A(d, i, o, g) t1[i+o][d][c][a'][b]
// zero_pads fills t1's p zero end slices first (the caller knows whether they are in place);
// prof allows the event timing of the banded stage.
template <class T>
static void op_stage12(iga_ctx* ctx, const BandCore<T>& A, const T* PhiL, int r0o, int r0, int r1, int ncol,
                       const T* x, long xcs, T* t1, T* t2, bool zero_pads, int op_id, bool bf16, bool prof) {
  using G = typename Prec<T>::G;
  hipStream_t st = ctx->stream;
  const int n = A.n, p = A.p, b = 2 * p + 1, R0 = A.Rin, R1 = A.Rout;
  const std::vector<RankBlock>& blocks = *A.blocks;
  const long S2 = (long)r0o * r1;         // one (c) slab of (a', b)
  const long S1 = (long)ncol * S2;        // one (d) slab
  const long SJ = (long)R0 * S1;          // one j slice of t1
  // the p zero slices at both ends of j are never written by stage 1
  if (p > 0 && zero_pads) {
    Prec<T>::zero(st, p * SJ, t1);
    Prec<T>::zero(st, p * SJ, t1 + (long)(n + p) * SJ);
  }
  // stage 1: one GEMM per column c with rows (d, a'): t1[j+p][d][c][a'][b] = sum_a PhiL[d][a'][a] x[c][a][j][b]
  G g1;
  g1.M = R0 * r0o; g1.N = n * r1; g1.N2 = r1; g1.K = r0;
  g1.A = PhiL; g1.sAm1 = (long)r0o * r0; g1.sAm2 = r0; g1.sAk2 = 1;
  g1.B = x; g1.sBk2 = (long)n * r1; g1.sBn1 = r1; g1.sBn2 = 1;
  g1.C = t1 + p * SJ; g1.M2 = r0o; g1.sCm1 = S1; g1.sCm2 = r1; g1.sCn1 = SJ; g1.sCn2 = 1;
  g1.nb1 = ncol; g1.sBb1 = xcs; g1.sCb1 = S2;
  prof = prof && ctx->prof_on;
  hipEvent_t pa = nullptr, pb = nullptr;
  if (prof) {
    pa = prof_event(ctx);
    pb = prof_event(ctx);
    IGA_HIP(hipEventRecord(pa, st));
  }
  Prec<T>::gemm(st, g1, nullptr, 0, bf16);
  if (prof) {
    IGA_HIP(hipEventRecord(pb, st));
    iga_ctx::ProfRec rec{pa, pb, Prec<T>::prof_base + (bf16 ? 2 : 0) + op_id, 1,
                         2.0 * r0o * r0 * (double)R0 * n * r1 * ncol};
    rec.stage = 1;
    ctx->prof.push_back(rec);
  }
  // stage 2: per rank block, batched over rows i
  if (prof) {
    pa = prof_event(ctx);
    pb = prof_event(ctx);
    IGA_HIP(hipEventRecord(pa, st));
  }
  band_stage<T>(st, A, t1, SJ, S1, t2, bf16);
  if (prof) {
    IGA_HIP(hipEventRecord(pb, st));
    double nz = 0;
    for (const RankBlock& rb : blocks) nz += (double)rb.na * rb.nb;
    ctx->prof.push_back({pa, pb, Prec<T>::prof_base + (bf16 ? 2 : 0) + op_id, (int)blocks.size(),
                         2.0 * r0o * r1 * ncol * nz * band_nnz(n, p)});
  }
}

// The contraction itself, on caller-provided intermediates t1, t2 and wk (wlen elements).
template <class T>
static void op_apply_raw(iga_ctx* ctx, const OpView& A, const T* core, const T* relaid,
                         const std::vector<RankBlock>& blocks, const T* PhiL, const T* PhiR, int r0o, int r0, int r1,
                         int r1o, int ncol, const T* x, long xcs, T* z, long zcs, T* t1, T* t2, T* wk, size_t wlen,
                         bool zero_pads, int op_id, bool bf16, bool prof) {
  using G = typename Prec<T>::G;
  const int n = A.n, R1 = A.R1;
  const long S2 = (long)r0o * r1, S1 = (long)ncol * S2;
  op_stage12<T>(ctx, band_core<T>(A, core, relaid, blocks), PhiL, r0o, r0, r1, ncol, x, xcs, t1, t2, zero_pads,
                op_id, bf16, prof);
  // stage 3: z[c][(a' i)][b'] = sum_{(g, b)} t2[i][g][c][a'][b] PhiR[g][b'][b]
  G g3;
  g3.M = r0o * n; g3.M2 = n; g3.N = r1o; g3.K = R1 * r1; g3.K2 = r1;
  g3.A = t2; g3.sAm1 = r1; g3.sAm2 = (long)R1 * S1; g3.sAk1 = S1; g3.sAk2 = 1;
  g3.B = PhiR; g3.sBk1 = (long)r1o * r1; g3.sBk2 = 1; g3.sBn2 = r1;
  g3.C = z; g3.sCm1 = (long)n * r1o; g3.sCm2 = r1o; g3.sCn2 = 1;
  g3.nb1 = ncol; g3.sAb1 = S2; g3.sCb1 = zcs;
  prof = prof && ctx->prof_on;
  hipEvent_t pa = nullptr, pb = nullptr;
  if (prof) {
    pa = prof_event(ctx);
    pb = prof_event(ctx);
    IGA_HIP(hipEventRecord(pa, ctx->stream));
  }
  Prec<T>::gemm(ctx->stream, g3, wk, wlen, bf16);
  if (prof) {
    IGA_HIP(hipEventRecord(pb, ctx->stream));
    iga_ctx::ProfRec rec{pa, pb, Prec<T>::prof_base + (bf16 ? 2 : 0) + op_id, 1,
                         2.0 * r0o * n * (double)R1 * r1 * r1o * ncol};
    rec.stage = 3;
    ctx->prof.push_back(rec);
  }
}

// op_apply_raw on intermediates from the context pool (grown on demand); t1's zero end
// slices are filled once per layout.
template <class T>
static void op_apply(iga_ctx* ctx, const OpView& A, const T* core, const T* relaid, const std::vector<RankBlock>& blocks,
                     const T* PhiL, const T* PhiR, int r0o, int r0, int r1, int r1o, int ncol, const T* x,
                     long xcs, T* z, long zcs, DevBuf<T>& t1, DevBuf<T>& t2, DevBuf<T>& wk,
                     LocalWork::PadKey& pad, int op_id, bool bf16 = false) {
  const int n = A.n, p = A.p;
  const long SJ = (long)A.R0 * ncol * r0o * r1;
  t1.ensure(ctx, (size_t)op_t1_len(n, p, A.R0, r0o, r1, ncol));
  t2.ensure(ctx, (size_t)op_t2_len(n, A.R1, r0o, r1, ncol));
  const size_t wlen = (size_t)op_split_len(n, r0o, r1o, ncol);
  wk.ensure(ctx, wlen);
  const bool zero_pads = p > 0 && (pad.gen != t1.gen() || pad.sj != SJ || pad.n != n || pad.p != p);
  if (zero_pads) {
    pad.gen = t1.gen(); pad.sj = SJ; pad.n = n; pad.p = p;
  }
  op_apply_raw<T>(ctx, A, core, relaid, blocks, PhiL, PhiR, r0o, r0, r1, r1o, ncol, x, xcs, z, zcs, t1.get(),
                  t2.get(), wk.get(), wlen, zero_pads, op_id, bf16, true);
}

// ---- interface updates and one-column projections on the matrix cores ----

static std::vector<RankBlock> transposed_blocks(const std::vector<RankBlock>& blocks) {
  std::vector<RankBlock> t;
  t.reserve(blocks.size());
  for (const RankBlock& rb : blocks) t.push_back(RankBlock{rb.b0, rb.nb, rb.a0, rb.na});
  return t;
}

// Grows the workspace for stages 1-2 of one column and reports whether t1's zero end slices
// must be filled (a new buffer or another layout).
static bool iface_ensure(iga_ctx* ctx, IfaceWork& w, int n, int p, int Rin, int Rout, int r0o, int r1) {
  w.t1.ensure(ctx, (size_t)op_t1_len(n, p, Rin, r0o, r1, 1));
  w.t2.ensure(ctx, (size_t)op_t2_len(n, Rout, r0o, r1, 1));
  const long SJ = (long)Rin * r0o * r1;
  const bool zero = p > 0 && (w.pad.gen != w.t1.gen() || w.pad.sj != SJ || w.pad.n != n || w.pad.p != p);
  if (zero) {
    w.pad.gen = w.t1.gen(); w.pad.sj = SJ; w.pad.n = n; w.pad.p = p;
  }
  return zero;
}

void interface_left_mc(iga_ctx* ctx, const OpView& A, const std::vector<RankBlock>& blocks, const double* Phi,
                       const double* U, const double* V, int ru0, int ru1, int rv0, int rv1, double* out,
                       IfaceWork& w) {
  const int n = A.n;
  const bool zero = iface_ensure(ctx, w, n, A.p, A.R0, A.R1, ru0, rv1);
  // t2[i][g][a'][b] = sum_{o, d} A(d, i, o, g) sum_a Phi[d][a'][a] V[a][i+o-p][b]
  op_stage12<double>(ctx, band_core<double>(A, A.A, A.Ar, blocks), Phi, ru0, rv0, rv1, 1, V, 0, w.t1.get(),
                     w.t2.get(), zero, 0, false, false);
  // out[g][b'][b] = sum_{(a', i)} U[a'][i][b'] t2[i][g][a'][b]: one product per output rank g,
  // K = (a', i) two-level
  const long S1 = (long)ru0 * rv1;
  k::Gemm2 g;
  g.M = ru1; g.N = rv1; g.K = ru0 * n; g.K2 = n;
  g.A = U; g.sAm2 = 1; g.sAk1 = (long)n * ru1; g.sAk2 = ru1;
  g.B = w.t2.get(); g.sBk1 = rv1; g.sBk2 = (long)A.R1 * S1; g.sBn2 = 1;
  g.C = out; g.sCm2 = rv1; g.sCn2 = 1;
  g.nb1 = A.R1; g.sBb1 = S1; g.sCb1 = (long)ru1 * rv1;
  const size_t wlen = (size_t)16 * A.R1 * ru1 * rv1;
  w.split.ensure(ctx, wlen);
  k::gemm2(ctx->stream, g, w.split.get(), wlen);
}

void interface_right_mc(iga_ctx* ctx, const OpView& A, const double* relaidT, const std::vector<RankBlock>& blocks,
                        const double* Phi, const double* U, const double* V, int ru0, int ru1, int rv0, int rv1,
                        double* out, IfaceWork& w) {
  const int n = A.n, b = 2 * A.p + 1;
  // the core with its rank roles swapped: input rank g (right), output rank d (left)
  BandCore<double> c;
  c.n = n; c.p = A.p; c.Rin = A.R1; c.Rout = A.R0;
  c.core = A.A;
  c.s_in = 1; c.s_out = (long)n * b * A.R1; c.s_row = (long)b * A.R1; c.s_off = A.R1;
  c.relaid = relaidT;
  const std::vector<RankBlock> tb = transposed_blocks(blocks);
  c.blocks = &tb;
  // V^T[b][j][a] = V[a][j][b], so that stage 1 contracts Phi[g][b'][b] with it over b
  w.vt.ensure(ctx, (size_t)rv0 * n * rv1);
  {
    const int dims[4] = {1, rv0, n, rv1}, perm[4] = {0, 3, 2, 1};
    k::permute4(ctx->stream, V, dims, perm, w.vt.get());
  }
  const bool zero = iface_ensure(ctx, w, n, A.p, A.R1, A.R0, ru1, rv0);
  // t2[i][d][b'][a] = sum_{o, g} A(d, i, o, g) sum_b Phi[g][b'][b] V[a][i+o-p][b]
  op_stage12<double>(ctx, c, Phi, ru1, rv1, rv0, 1, w.vt.get(), 0, w.t1.get(), w.t2.get(), zero, 0, false, false);
  // out[d][a'][a] = sum_{(i, b')} U[a'][i][b'] t2[i][d][b'][a]: one product per output rank d,
  // K = (i, b') two-level, so that U is read along its unit-stride index b'
  const long S1 = (long)ru1 * rv0;
  k::Gemm2 g;
  g.M = ru0; g.N = rv0; g.K = n * ru1; g.K2 = ru1;
  g.A = U; g.sAm2 = (long)n * ru1; g.sAk1 = ru1; g.sAk2 = 1;
  g.B = w.t2.get(); g.sBk1 = (long)A.R0 * S1; g.sBk2 = rv0; g.sBn2 = 1;
  g.C = out; g.sCm2 = rv0; g.sCn2 = 1;
  g.nb1 = A.R0; g.sBb1 = S1; g.sCb1 = (long)ru0 * rv0;
  const size_t wlen = (size_t)16 * A.R0 * ru0 * rv0;
  w.split.ensure(ctx, wlen);
  k::gemm2(ctx->stream, g, w.split.get(), wlen);
}

void apply_one_mc(iga_ctx* ctx, const OpView& A, const std::vector<RankBlock>& blocks, const double* PhiL,
                  const double* PhiR, int r0o, int r0, int r1, int r1o, const double* x, double* z, IfaceWork& w) {
  const bool zero = iface_ensure(ctx, w, A.n, A.p, A.R0, A.R1, r0o, r1);
  const size_t wlen = (size_t)op_split_len(A.n, r0o, r1o, 1);
  w.split.ensure(ctx, wlen);
  op_apply_raw<double>(ctx, A, A.A, A.Ar, blocks, PhiL, PhiR, r0o, r0, r1, r1o, 1, x, 0, z, 0, w.t1.get(),
                       w.t2.get(), w.split.get(), wlen, zero, 0, false, false);
}

// ---- a TT-matrix applied to a full tensor, mode by mode on the matrix cores ----

// y = alpha A x + beta y, x and y full tensors [n0][n1][n2] (C order), A a TT-matrix with banded
// cores (eqs. M_kron, K_kron). A is the sum of the terms of its middle core's rank blocks (one
// for a dense middle core, the nine (k, l) terms of the stiffness operator); each term applies
// its three factor cores one mode at a time, with the mode being contracted moved outermost and
// padded with p zero slices, so that every mode product is the banded stage of the local matvec:
//   mode 0: Y0[i0][g1][(j1 j2)] = sum A0(0, i0, o, g1) x[i0+o-p][(j1 j2)]
//   mode 1: Y1[i1][g2][(i0 j2)] = sum A1(g1, i1, o, g2) Y0[i0][g1][i1+o-p][j2]
//   mode 2: Y2[i2][(i1 i0)]     = sum A2(g2, i2, o, 0)  Y1[i1][g2][i0][i2+o-p]
// and y[i0][i1][i2] += alpha Y2[i2][i1][i0].
void full_apply_mc(iga_ctx* ctx, const iga_ttop* A, const double* x, double* y, double alpha, double beta,
                   FullWork& w) {
  hipStream_t st = ctx->stream;
  const int n0 = A->n[0], n1 = A->n[1], n2 = A->n[2], p = A->p, b = 2 * p + 1;
  const long N = (long)n0 * n1 * n2;
  const OpCore& c0 = A->core[0];
  const OpCore& c1 = A->core[1];
  const OpCore& c2 = A->core[2];
  require(c0.R0 == 1 && c2.R1 == 1 && c0.blocks.size() == 1 && c2.blocks.size() == 1, IGA_EINVAL,
          "full_apply: outer cores must be single dense blocks");
  const std::vector<RankBlock>& terms = c1.blocks;
  int rmax = 1;
  for (const RankBlock& t : terms) rmax = std::max(rmax, std::max(t.na, t.nb));
  const int nmax = std::max(n0, std::max(n1, n2));
  const size_t big = (size_t)(nmax + 2 * p) * rmax * (N / std::min(n0, std::min(n1, n2)));
  w.p0.ensure(ctx, (size_t)(n0 + 2 * p) * n1 * n2);
  w.a.ensure(ctx, big);
  w.b.ensure(ctx, big);
  w.r2.ensure(ctx, (size_t)rmax * n2 * b);
  // x padded along mode 0
  const long C0 = (long)n1 * n2;
  k::fill(st, p * C0, 0.0, w.p0.get());
  k::fill(st, p * C0, 0.0, w.p0.get() + (long)(n0 + p) * C0);
  IGA_HIP(hipMemcpyAsync(w.p0.get() + p * C0, x, N * sizeof(double), hipMemcpyDeviceToDevice, st));
  for (size_t t = 0; t < terms.size(); ++t) {
    const RankBlock& tb = terms[t];
    const int na = tb.na, nb = tb.nb;
    // mode 0: core 0 restricted to columns [a0, a0 + na)
    {
      BandCore<double> c;
      const std::vector<RankBlock> one = {RankBlock{0, 1, 0, na}};
      c.n = n0; c.p = p; c.Rin = 1; c.Rout = na;
      c.core = c0.data.get() + tb.a0;
      c.s_in = (long)n0 * b * c0.R1; c.s_out = 1; c.s_row = (long)b * c0.R1; c.s_off = c0.R1;
      c.blocks = &one;
      band_stage<double>(st, c, w.p0.get(), C0, C0, w.a.get(), false);
    }
    // Y0 [i0][g1][j1][j2] -> P1 [j1 + p][g1][i0][j2]
    const long C1 = (long)n0 * n2, SJ1 = (long)na * C1;
    {
      const int dims[4] = {n0, na, n1, n2}, perm[4] = {2, 1, 0, 3};
      k::fill(st, p * SJ1, 0.0, w.b.get());
      k::fill(st, p * SJ1, 0.0, w.b.get() + (long)(n1 + p) * SJ1);
      k::permute4(st, w.a.get(), dims, perm, w.b.get() + p * SJ1);
    }
    // mode 1: the term's block of the middle core
    {
      BandCore<double> c;
      const std::vector<RankBlock> one = {RankBlock{0, na, 0, nb}};
      c.n = n1; c.p = p; c.Rin = na; c.Rout = nb;
      c.core = c1.data.get() + (long)tb.a0 * n1 * b * c1.R1 + tb.b0;
      c.s_in = (long)n1 * b * c1.R1; c.s_out = 1; c.s_row = (long)b * c1.R1; c.s_off = c1.R1;
      c.blocks = &one;
      band_stage<double>(st, c, w.b.get(), SJ1, C1, w.a.get(), false);
    }
    // Y1 [i1][g2][i0][j2] -> P2 [j2 + p][g2][i1][i0]
    const long C2 = (long)n1 * n0, SJ2 = (long)nb * C2;
    {
      const int dims[4] = {n1, nb, n0, n2}, perm[4] = {3, 1, 0, 2};
      k::fill(st, p * SJ2, 0.0, w.b.get());
      k::fill(st, p * SJ2, 0.0, w.b.get() + (long)(n2 + p) * SJ2);
      k::permute4(st, w.a.get(), dims, perm, w.b.get() + p * SJ2);
    }
    // mode 2: core 2 restricted to rows [b0, b0 + nb), re-laid as [n2][b][nb][1] (the rows are
    // contiguous), one output rank: the vector-unit banded stage
    {
      const int dims[4] = {nb, n2, b, 1}, perm[4] = {1, 2, 0, 3};
      k::permute4(st, c2.data.get() + (long)tb.b0 * n2 * b, dims, perm, w.r2.get());
      BandCore<double> c;
      const std::vector<RankBlock> one = {RankBlock{0, nb, 0, 1}};
      c.n = n2; c.p = p; c.Rin = nb; c.Rout = 1;
      c.core = c2.data.get() + (long)tb.b0 * n2 * b;
      c.s_in = (long)n2 * b; c.s_out = 1; c.s_row = b; c.s_off = 1;
      c.relaid = w.r2.get();
      c.blocks = &one;
      band_stage<double>(st, c, w.b.get(), SJ2, C2, w.a.get(), false);
    }
    // Y2 [i2][i1][i0] -> [i0][i1][i2], accumulated into y
    {
      const int dims[4] = {1, n2, n1, n0}, perm[4] = {0, 3, 2, 1};
      k::permute4(st, w.a.get(), dims, perm, w.b.get());
      k::axpby(st, N, alpha, w.b.get(), t == 0 ? beta : 1.0, y);
    }
  }
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
  const long colsz = (long)L.r0 * L.n * L.r1;
  const int r0o = L.out0(), r1o = L.out1();
  const long osz = (long)r0o * L.n * r1o;
  if (L.toff) {
    // general block structure (the time-dependent system), as in local_matvec
    const int nz = L.nblk + L.kcols();
    w.fz.ensure(ctx, (size_t)nz * osz);
    op_apply<float>(ctx, L.M, L.M.Af, L.M.Arf, L.Mblocks, L.fPhiL_M, L.fPhiR_M, r0o, L.r0, L.r1, r1o, L.nblk, x,
                    colsz, w.fz.get(), osz, w.ftM, w.ftM2, w.fsplit, w.fpadM, 0, bf16);
    int pos = L.nblk;
    for (int j = 0; j < L.nkr; ++j) {
      op_apply<float>(ctx, L.K, L.K.Af, L.K.Arf, L.Kblocks, L.fPhiL_K, L.fPhiR_K, r0o, L.r0, L.r1, r1o, L.kn[j],
                      x + L.kb[j] * colsz, colsz, w.fz.get() + pos * osz, osz, w.ftK, w.ftK2, w.fsplit, w.fpadK, 1,
                      bf16);
      pos += L.kn[j];
    }
    k::combine_blocks_f32(ctx->stream, osz, L.nblk, L.toff, L.src, L.tcoef, w.fz.get(), y);
    return;
  }
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
  LocalWork w;
  FBuf fPhi[4], fM, fK, fx, fy;
  DBuf rM, rK;  // cores re-laid for the banded stage
  FBuf frM, frK;  // their FP32 copies (mixed-precision forms)
};
// Per-context caches: the maps are shared by every host thread (each context is used by one
// thread at a time), so lookups and erasures take the lock.
std::mutex g_raw_mu;
std::unordered_map<iga_ctx*, std::unique_ptr<RawCache>> g_raw;
RawCache& raw_cache(iga_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_raw_mu);
  auto& p = g_raw[ctx];
  if (!p) p.reset(new RawCache());
  return *p;
}
}  // namespace

void release_raw_cache(iga_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_raw_mu);
  g_raw.erase(ctx);
}

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
  LocalOp L;
  L.r0 = r0; L.n = n; L.r1 = r1;
  L.coef.m11 = beta;
  L.M.R0 = RM0; L.M.R1 = RM1; L.M.n = n; L.M.p = p; L.M.A = Mcore;
  L.K.R0 = RK0; L.K.R1 = RK1; L.K.n = n; L.K.p = p; L.K.A = Kcore;
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

// Workspace of local_matvec_noalloc_impl in doubles, each part rounded up to 32 doubles (256
// bytes): the two re-laid cores, t1 and t2 of each operator, the five output columns and the
// split-K partials.
static long round32(long v) { return (v + 31) / 32 * 32; }
long local_matvec_noalloc_len(int r0, int n, int r1, int p, int RM0, int RM1, int RK0, int RK1) {
  const int b = 2 * p + 1;
  return round32((long)RM0 * n * b * RM1) + round32((long)RK0 * n * b * RK1) +
         round32(op_t1_len(n, p, RM0, r0, r1, 3)) + round32(op_t2_len(n, RM1, r0, r1, 3)) +
         round32(op_t1_len(n, p, RK0, r0, r1, 2)) + round32(op_t2_len(n, RK1, r0, r1, 2)) +
         round32(5L * r0 * n * r1) + round32(op_split_len(n, r0, r1, 3));
}

// local_matvec_impl in FP64 with every intermediate carved from ws (ws_len doubles, 256-byte
// aligned): the same kernels in the same order, no allocation, no event timing. The caller
// has checked ws_len >= local_matvec_noalloc_len.
void local_matvec_noalloc_impl(iga_ctx* ctx, int r0, int n, int r1, int p, int RM0, int RM1, int RK0, int RK1,
                               const double* PhiL_M, const double* PhiR_M, const double* PhiL_K,
                               const double* PhiR_K, const double* Mcore, const double* Kcore, double beta,
                               const double* x, double* y, double* ws, long ws_len) {
  require(local_matvec_noalloc_len(r0, n, r1, p, RM0, RM1, RK0, RK1) <= ws_len, IGA_EINVAL,
          "local_matvec_noalloc: workspace too small");
  hipStream_t st = ctx->stream;
  const int b = 2 * p + 1;
  double* cur = ws;
  auto take = [&](long len) {
    double* q = cur;
    cur += round32(len);
    return q;
  };
  double* rM = take((long)RM0 * n * b * RM1);
  double* rK = take((long)RK0 * n * b * RK1);
  double* tM = take(op_t1_len(n, p, RM0, r0, r1, 3));
  double* tM2 = take(op_t2_len(n, RM1, r0, r1, 3));
  double* tK = take(op_t1_len(n, p, RK0, r0, r1, 2));
  double* tK2 = take(op_t2_len(n, RK1, r0, r1, 2));
  double* z = take(5L * r0 * n * r1);
  const size_t wlen = (size_t)op_split_len(n, r0, r1, 3);
  double* split = take((long)wlen);
  LocalOp L;
  L.r0 = r0; L.n = n; L.r1 = r1;
  L.coef.m11 = beta;
  L.M.R0 = RM0; L.M.R1 = RM1; L.M.n = n; L.M.p = p; L.M.A = Mcore;
  L.K.R0 = RK0; L.K.R1 = RK1; L.K.n = n; L.K.p = p; L.K.A = Kcore;
  const std::vector<RankBlock> Mb = {RankBlock{0, RM0, 0, RM1}}, Kb = {RankBlock{0, RK0, 0, RK1}};
  const int dimsM[4] = {RM0, n, b, RM1}, dimsK[4] = {RK0, n, b, RK1}, perm[4] = {1, 2, 0, 3};
  k::permute4(st, Mcore, dimsM, perm, rM);
  k::permute4(st, Kcore, dimsK, perm, rK);
  const long colsz = (long)r0 * n * r1;
  // the scratch keeps what the last call left in it: the zero end slices of t1 are filled on
  // every call
  op_apply_raw<double>(ctx, L.M, Mcore, rM, Mb, PhiL_M, PhiR_M, r0, r0, r1, r1, 3, x, colsz, z, colsz, tM, tM2,
                       split, wlen, true, 0, false, false);
  op_apply_raw<double>(ctx, L.K, Kcore, rK, Kb, PhiL_K, PhiR_K, r0, r0, r1, r1, 2, x, 2 * colsz, z + 3 * colsz,
                       colsz, tK, tK2, split, (size_t)op_split_len(n, r0, r1, 2), true, 1, false, false);
  k::kkt_combine(st, colsz, L.coef, z, z + 3 * colsz, y);
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
std::mutex g_batch_mu;
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

void release_batch_cache(iga_ctx* ctx) {
  std::lock_guard<std::mutex> lk(g_batch_mu);
  g_batch.erase(ctx);
}

void local_matvec_batched_impl(iga_ctx* ctx, const std::vector<BatchProblem>& P, int precision, bool autotune) {
  BatchCache* cache;
  {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    auto& cp = g_batch[ctx];
    if (!cp) cp.reset(new BatchCache());
    cache = cp.get();
  }
  BatchCache& C = *cache;
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
