// The projected local KKT operator of one block-AMEn step (eq. KKT_red, tau = 1):
//   y = [M x0 + K x2 ; beta M x1 - M x2 ; K x0 - M x1]
// with M, K the reduced operators PhiL (x) A_d (x) PhiR of the two TT-matrices,
// optionally composed with a scaling of the unknowns (see KktCoef).
// The interfaces may be rectangular (test ranks r0o, r1o; trial ranks r0, r1).
#pragma once

#include <vector>

#include "common.hpp"
#include "kernels.hpp"
#include "ttops.hpp"

namespace iga {

// A block-structured operator core with at most this many rank pairs R0 R1 is contracted as one
// dense product over its re-laid form (zeros included) in the banded stage, not block by block.
constexpr long kDenseRankPairs = 1024;
// Re-laid cores with at most this many right ranks take the vector-unit banded stage.
constexpr int kSmallR1 = 16;

struct LocalOp {
  OpView M, K;
  std::vector<RankBlock> Mblocks, Kblocks;  // nonzero rank blocks of the two cores
  const double* PhiL_M = nullptr;  // [RM0][r0][r0]
  const double* PhiR_M = nullptr;  // [RM1][r1][r1]
  const double* PhiL_K = nullptr;
  const double* PhiR_K = nullptr;
  int r0 = 0, n = 0, r1 = 0;     // trial (input) ranks
  int r0o = -1, r1o = -1;        // test (output) ranks; -1: same as the trial ranks
  k::KktCoef coef;
  // FP32 copies for the mixed-precision form (null when unused)
  const float* fPhiL_M = nullptr;
  const float* fPhiR_M = nullptr;
  const float* fPhiL_K = nullptr;
  const float* fPhiR_K = nullptr;
  // General block structure (time-dependent system), null for the stationary 3 blocks:
  // M acts on all nblk blocks, K on the block ranges [kb[j], kb[j] + kn[j]), j < nkr, and
  // output block o = sum over its terms t of tcoef[t] z[src[t]], z = [M x_0 .. M x_{nblk-1},
  // K x of the ranges in order] (device tables toff [nblk + 1], src, tcoef).
  int nblk = 3;
  int nkr = 0, kb[2] = {0, 0}, kn[2] = {0, 0};
  const int* toff = nullptr;
  const int* src = nullptr;
  const double* tcoef = nullptr;
  int out0() const { return r0o < 0 ? r0 : r0o; }
  int out1() const { return r1o < 0 ? r1 : r1o; }
  long size() const { return (long)nblk * r0 * n * r1; }
  long out_size() const { return (long)nblk * out0() * n * out1(); }
  int kcols() const { return toff ? kn[0] + kn[1] : 2; }
};

struct LocalWork {
  DBuf tM, tK, tM2, tK2, z, split;  // split: split-K partials of the short-output stages
  // layout (generation of tM / tK, slice size, n, p) whose zero end slices are in place
  struct PadKey { unsigned gen = ~0u; long sj = -1; int n = -1, p = -1; } padM, padK, fpadM, fpadK;
  FBuf ftM, ftK, ftM2, ftK2, fz, fsplit, fx, fy;  // FP32 counterparts
};

// Workspace of the matrix-core interface updates and one-column projections.
struct IfaceWork {
  DBuf t1, t2, split, vt;
  LocalWork::PadKey pad;
};
// Left interface of core d + 1 from core d (Section 5, eqs. frame and ttlin):
//   out[g][b'][b] = sum U[a'][i][b'] Phi[d][a'][a] A[d][i][i+o-p][g] V[a][i+o-p][b],
// U: [ru0][n][ru1], V: [rv0][n][rv1], Phi: [R0][ru0][rv0], out: [R1][ru1][rv1]. A.Ar (the core
// re-laid as [n][2p+1][R0][R1]) may be null; blocks are the core's nonzero rank blocks.
void interface_left_mc(iga_ctx* ctx, const OpView& A, const std::vector<RankBlock>& blocks, const double* Phi,
                       const double* U, const double* V, int ru0, int ru1, int rv0, int rv1, double* out,
                       IfaceWork& w);
// Right interface of core d - 1 from core d:
//   out[d][a'][a] = sum U[a'][i][b'] Phi[g][b'][b] A[d][i][i+o-p][g] V[a][i+o-p][b],
// Phi: [R1][ru1][rv1], out: [R0][ru0][rv0]; relaidT (may be null) is the core re-laid as
// [n][2p+1][R1][R0].
void interface_right_mc(iga_ctx* ctx, const OpView& A, const double* relaidT, const std::vector<RankBlock>& blocks,
                        const double* Phi, const double* U, const double* V, int ru0, int ru1, int rv0, int rv1,
                        double* out, IfaceWork& w);
// One column of the projected operator: z[a'][i][b'] = sum PhiL[d][a'][a] A[d][i][i+o-p][g]
// x[a][i+o-p][b] PhiR[g][b'][b], x: [r0][n][r1], z: [r0o][n][r1o].
void apply_one_mc(iga_ctx* ctx, const OpView& A, const std::vector<RankBlock>& blocks, const double* PhiL,
                  const double* PhiR, int r0o, int r0, int r1, int r1o, const double* x, double* z, IfaceWork& w);

// Workspace of full_apply_mc.
struct FullWork {
  DBuf p0, a, b, r2;
};
// y = alpha A x + beta y for a TT-matrix A (banded cores) and full tensors x, y [n0][n1][n2],
// one mode at a time on the matrix cores.
void full_apply_mc(iga_ctx* ctx, const iga_ttop* A, const double* x, double* y, double alpha, double beta,
                   FullWork& w);

// y = A_loc x (FP64); x: [3][r0][n][r1], y: [3][r0o][n][r1o]
void local_matvec(iga_ctx* ctx, const LocalOp& L, const double* x, double* y, LocalWork& w);
// Same product on FP32 operands (x, y FP32; needs the f* fields and Af views), every
// contraction in FP32 or, with bf16, with its operands rounded to bfloat16 and FP32 accumulation.
void local_matvec_f32(iga_ctx* ctx, const LocalOp& L, const float* x, float* y, LocalWork& w, bool bf16 = false);
// One independent problem of the batched form (dense rank blocks, square interfaces).
struct BatchProblem {
  int r0, n, r1, p, RM0, RM1, RK0, RK1;
  const double *PhiL_M, *PhiR_M, *PhiL_K, *PhiR_K, *Mcore, *Kcore;
  double beta;
  const double* x;
  double* y;
};
// y_i = A_i x_i for every problem; each stage of all problems is one grouped matrix-core
// launch per tile variant (variants tuned per size bucket when autotune is set).
void local_matvec_batched_impl(iga_ctx* ctx, const std::vector<BatchProblem>& P, int precision, bool autotune);
void release_batch_cache(iga_ctx* ctx);

// Algorithmic flops of local_matvec: banded middle stage counted over the band's
// nonzero entries and over the nonzero rank blocks only.
double local_flops(const LocalOp& L);
double band_nnz(int n, int p);

}  // namespace iga
