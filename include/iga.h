/*
 * iga.h -- C ABI of the MI355X (gfx950) library for the low-rank tensor-train
 * method for isogeometric PDE-constrained optimisation (Buenger, Dolgov,
 * Stoll): TT assembly of the Galerkin mass and stiffness operators from a
 * B-spline geometry (Section 3), the KKT operator of the Poisson control
 * problem (Section 4, stationary reading) and its block-AMEn solver
 * (Section 5).
 *
 * Conventions
 * -----------
 * Status: every int-returning call returns IGA_OK (0) or a negative IGA_E*
 *   code; iga_last_error() then returns a thread-local message. A failed call
 *   leaves every handle it was given valid and allocates nothing the caller
 *   must free (out-handles stay NULL).
 * Ownership: every handle returned through an out-pointer is owned by the
 *   caller and released by its *_destroy; destroy(NULL) is a no-op. Inputs
 *   are never modified. Host arrays are copied before the call returns.
 * Memory: "dev" pointers are device memory of the context's GPU; "host"
 *   pointers are ordinary host memory.
 * Streams: all work is enqueued on the stream given to iga_ctx_create;
 *   calls that return host-visible results (ranks, norms, statistics)
 *   synchronise that stream.
 * Index order: C order (last index fastest). Three spatial directions.
 *   The solution space per direction d has degree p, N_d = n_d + 2
 *   B-splines on E_d = N_d - p uniform elements; n_d counts the free
 *   unknowns left after the Dirichlet boundary functions are omitted
 *   (Section 4). Full coefficient tensors are [n1][n2][n3].
 * Layouts:
 *   TT core          [r_{d-1}][n_d][r_d], r_0 = r_3 = 1        (eq. tt)
 *   block-TT core    [3][r_{d-1}][n_d][r_d] at the core holding the
 *                    component index l = (y, u, lambda), plain TT cores
 *                    elsewhere                                (eq. btt)
 *   TT-matrix core   banded [R_{d-1}][n_d][2p+1][R_d]: entry (i, o) is
 *                    column j = i + o - p of row i; entries with j outside
 *                    0..n_d-1 are zero.                 (eqs. M_kron, K_kron)
 */
#ifndef IGA_H
#define IGA_H

#ifdef __cplusplus
extern "C" {
#endif

#define IGA_OK 0
#define IGA_EINVAL (-1)  /* bad argument: sizes, degrees, tolerances, NULL */
#define IGA_ENOMEM (-2)  /* device allocation failed */
#define IGA_EHIP (-3)    /* a HIP runtime call failed */
#define IGA_EGEOM (-4)   /* det grad G <= 0 at an interpolation point: the map folds */
#define IGA_ENOCONV (-5) /* block AMEn stopped at nswp sweeps above tolerance */
#define IGA_ERANK (-6)   /* block AMEn stopped above tolerance with a solution rank at r_max */
#define IGA_ENUM (-7)    /* a non-finite value (NaN or Inf) arose: in an input, or in a local
                          residual or Krylov norm of block AMEn; no solution is returned */

#define IGA_FP64 0
#define IGA_FP32 1
#define IGA_MAX_TIME_STEPS 64  /* largest nt of iga_kkt_create_parabolic */
#define IGA_BF16 2

typedef struct iga_ctx iga_ctx;
typedef struct iga_tt iga_tt;     /* TT vector, 3 cores on the device        */
typedef struct iga_ttop iga_ttop; /* TT-matrix with banded cores             */
typedef struct iga_btt iga_btt;   /* block-TT holding (y, u, lambda)         */
typedef struct iga_kkt iga_kkt;   /* KKT operator built from M, K and beta   */

/* B-spline geometry map G = C : B (Section 2, eq. geometryMapping).
 * degree: geometry degree; ncp[d]: control points per direction;
 * knots[d]: host, open knot vector of length ncp[d] + degree + 1 on [0, 1];
 * ctrl: host, [3][ncp0][ncp1][ncp2], physical coordinates of the control points. */
typedef struct {
  int degree;
  int ncp[3];
  const double* knots[3];
  const double* ctrl;
} iga_geometry;

/* Options of the TT assembly (Section 3 and Section 6.1).
 * p_interp: degree of the weight-interpolation space (<= 0: 2p+1);
 * nquad: Gauss-Legendre points per element and direction (<= 0: 5);
 * weight_tol: relative Frobenius tolerance of the TT-SVD of each weight tensor
 *   (split as weight_tol / sqrt(2) per unfolding); 0 keeps all nonzero
 *   singular values (up to rounding);
 * weight_rmax: cap on each weight TT rank (<= 0: none). */
typedef struct {
  int p_interp;
  int nquad;
  double weight_tol;
  int weight_rmax;
} iga_assembly_opts;

/* Options of the block-AMEn solve (Section 5). Zero or negative fields take
 * the documented defaults.
 * nswp: maximum half-sweeps (default 20); r_max: cap on solution ranks
 * (default 256); kick_rank: residual-enrichment rank rho (default 4, -1 to
 * disable); local_tol: relative tolerance of each local solve (default tol/10);
 * local_maxit: maximum preconditioned GMRES iterations per local solve
 * (default 400); local_restart: GMRES restart length (default 40);
 * precision: IGA_FP64, or IGA_FP32 / IGA_BF16 for the mixed form (local contractions
 * in FP32, or with operands rounded to bfloat16 and FP32 accumulation, inside an FP64
 * iterative refinement of each local solve); init_rank: rank of the random
 * initial guess when x0 is NULL (default 2); seed: its seed; verbose: print
 * one line per half-sweep to stderr. */
typedef struct {
  int nswp;
  int r_max;
  int kick_rank;
  double local_tol;
  int local_maxit;
  int local_restart;
  int precision;
  int init_rank;
  unsigned long long seed;
  int verbose;
} iga_amen_opts;

/* Statistics of a solve; times in seconds from HIP events on the context stream. */
#define IGA_MAX_HISTORY 64
typedef struct {
  int half_sweeps;
  int converged;
  double max_local_residual;   /* of the last half-sweep, before its local solves */
  double residual;             /* ||A f - b|| / ||b|| of the returned solution (FP64, exact) */
  int ranks[2];                /* r_1, r_2 of the solution */
  long long local_solves;
  long long local_iterations;  /* preconditioned Krylov iterations, all local solves */
  long long local_matvecs;     /* FP64 projected local matvecs (each = 3 M + 2 K applications) */
  double local_matvec_flops;   /* algorithmic flops of those matvecs */
  double t_total;
  double t_local_matvec;       /* time inside the projected local matvec kernels */
  double t_precond;
  double t_krylov_other;
  double t_interfaces;
  double t_svd;                /* truncation steps: SVD, enrichment, next-core update (the
                                  local matvecs of the residual-based rank search are in
                                  t_local_matvec) */
  double t_residual;
  /* mixed form (precision IGA_FP32 or IGA_BF16): local matvecs with low-precision
   * contractions (FP32 or BF16 products, as chosen) inside the refinement's inner solves,
   * their algorithmic flops and time, and refinement steps (each followed by an FP64 local
   * residual); zero in the FP64 form */
  long long local_matvecs_fp32;
  double local_matvec_flops_fp32;
  double t_local_matvec_fp32;
  long long refinements;
  /* per half-sweep h < min(half_sweeps, IGA_MAX_HISTORY) (the quantities Section 6 reports):
   * the largest local residual of the half-sweep (measured before each local solve), the
   * solution ranks r_1, r_2 after it, and the number of stored solution entries
   * (sum_d r_{d-1} n_d r_d, the core holding the components counted nblk times) */
  double history_max_local_residual[IGA_MAX_HISTORY];
  int history_ranks[IGA_MAX_HISTORY][2];
  long long history_storage[IGA_MAX_HISTORY];
} iga_amen_stats;

/* Context on GPU `device`; hip_stream is a hipStream_t (NULL: the default stream). */
int iga_ctx_create(int device, void* hip_stream, iga_ctx** out);
void iga_ctx_destroy(iga_ctx* ctx);

/* Low-rank assembly of the mass and stiffness operators (Section 3):
 * evaluates omega = |det grad G| and Q = (grad G^T grad G)^{-1} omega on the
 * Greville grid of the interpolation space, compresses each of the seven
 * weight tensors (omega, q11, q12, q13, q22, q23, q33) by TT-SVD, solves the
 * collocation systems core by core (eq. weightEquationSolve), and integrates
 * the univariate factors M^(d)(w . beta~) and K_kl^(d)(v . beta~) by Gauss
 * quadrature (eqs. massMatrix1D, stiffnessFinal). M is returned as one
 * TT-matrix; K as the rank concatenation of its nine (k, l) terms (terms whose
 * weight vanishes are dropped). Boundary functions are omitted.
 * degree >= 1; n[d] >= 1; the geometry must be one-to-one (else IGA_EGEOM).
 * weight_ranks_out (nullable, host): [7][2] TT ranks (R1, R2) of the weights
 * in the order above; 0 for a weight that vanishes. */
int iga_assemble_factors(iga_ctx* ctx, const iga_geometry* geo, int degree, const int n[3],
                         const iga_assembly_opts* opts, iga_ttop** M, iga_ttop** K,
                         int* weight_ranks_out);

/* TT-matrix from host banded cores (layout above); R[0] = R[3] = 1. */
int iga_ttop_create(iga_ctx* ctx, int degree, const int n[3], const int R[4],
                    const double* const host_cores[3], iga_ttop** out);
/* Sizes: n[3], R[4], degree (any may be NULL). */
int iga_ttop_info(const iga_ttop* op, int* n, int* R, int* degree);
/* Copies banded core d to host [R_{d-1}][n_d][2p+1][R_d]. */
int iga_ttop_get_core(iga_ctx* ctx, const iga_ttop* op, int d, double* host_out);
void iga_ttop_destroy(iga_ttop* op);

/* TT of a full tensor [n0][n1][n2] (device, FP64, caller-owned, read only) by sequential
 * truncated SVDs (Section 5, eq. tt; the TT-SVD of the weight tensors in Section 3) with
 * relative Frobenius tolerance rel_tol (split as rel_tol / sqrt(2) per unfolding; 0 keeps
 * every nonzero singular value up to rounding). *out is owned by the caller
 * (iga_tt_destroy). Synchronises. */
int iga_tt_from_full(iga_ctx* ctx, const int n[3], const double* full, double rel_tol, iga_tt** out);

/* TT rounding (Section 5, eq. tt: the truncation applied to a TT vector): right-to-left
 * orthogonalisation, then left-to-right truncated SVDs of the unfoldings with the absolute
 * tolerance rel_tol ||in|| / sqrt(2) each, so that ||*out - in|| <= rel_tol ||in|| up to rounding
 * (rel_tol = 0 only removes exact rank deficiencies). The SVDs are those of the solver's
 * truncations. in is not modified; *out is new (iga_tt_destroy). IGA_EINVAL for a tolerance
 * outside [0, 1) or a TT of another context. Synchronises. */
int iga_tt_round(iga_ctx* ctx, const iga_tt* in, double rel_tol, iga_tt** out);

/* TT vectors. iga_tt_create copies host cores; iga_tt_wrap wraps caller-owned
 * device cores without copying (they must outlive the handle). r[0]=r[3]=1. */
int iga_tt_create(iga_ctx* ctx, const int n[3], const int r[4], const double* const host_cores[3],
                  iga_tt** out);
int iga_tt_wrap(iga_ctx* ctx, const int n[3], const int r[4], double* const dev_cores[3],
                iga_tt** out);
void iga_tt_destroy(iga_tt* t);
/* Sizes n[3] and ranks r[4] of a TT (r[0] = r[3] = 1). */
int iga_tt_info(const iga_tt* t, int n[3], int r[4]);
/* Copy core d, [r_d][n_d][r_{d+1}] (r_d n_d r_{d+1} doubles), to host memory. Synchronises. */
int iga_tt_get_core(iga_ctx* ctx, const iga_tt* t, int d, double* host_out);

/* Block-TT from host cores (layout above), component index at core ell_core. */
int iga_btt_create(iga_ctx* ctx, const int n[3], const int r[4], int ell_core,
                   const double* const host_cores[3], iga_btt** out);
int iga_btt_info(const iga_btt* x, int* n, int* r, int* ell_core);
/* Number of components (blocks) of x: 3 for the stationary system, 3 nt for the
 * time-dependent one; IGA_EINVAL for NULL. Core ell_core holds [nblk][r][n][r']. */
int iga_btt_blocks(const iga_btt* x);
int iga_btt_get_core(iga_ctx* ctx, const iga_btt* x, int d, double* host_out);
/* Expands the components into dev_out [nblk][n1][n2][n3] (tests, residuals). */
int iga_btt_to_full(iga_ctx* ctx, const iga_btt* x, double* dev_out);
void iga_btt_destroy(iga_btt* x);

/* KKT operator [[M,0,K],[0,beta M,-M],[K,-M,0]] of the stationary control
 * problem (eq. KKTSystem with one time step, tau = 1). beta > 0. M and K
 * must share n and degree and outlive the handle. */
int iga_kkt_create(iga_ctx* ctx, const iga_ttop* M, const iga_ttop* K, double beta, iga_kkt** out);

/* KKT operator of the time-dependent control problem (Section 4, eq. KKTSystem): implicit
 * Euler with nt steps of length tau (1 <= nt <= IGA_MAX_TIME_STEPS, tau > 0), y_0 = 0,
 *   [tau calM, 0, calK^T; 0, tau beta calM, -tau calM; calK, -tau calM, 0] [y; u; lambda]
 *     = [tau calM yhat; 0; 0],
 * calM = I_nt (x) M, calK = I_nt (x) tau K + C (x) M, C lower bidiagonal (1 on the diagonal,
 * -1 below), the desired state the same at every step. The time index is carried in the
 * block index of the solution: 3 nt blocks y_1..y_nt, u_1..u_nt, lambda_1..lambda_nt.
 * Accepted by iga_kkt_apply, iga_kkt_residual and iga_amen_solve (precision IGA_FP64);
 * the reduced-cost functions take stationary handles only. */
int iga_kkt_create_parabolic(iga_ctx* ctx, const iga_ttop* M, const iga_ttop* K, double beta, int nt,
                             double tau, iga_kkt** out);
/* Number of solution blocks of the system (3, or 3 nt); IGA_EINVAL for NULL. */
int iga_kkt_blocks(const iga_kkt* kkt);
void iga_kkt_destroy(iga_kkt* kkt);

/* y = A x exactly, without rounding: y has ranks (R^M_d + R^K_d) r_d and its
 * component index at the core of x (eqs. M_kron, K_kron, KKTSystem). */
int iga_kkt_apply(iga_ctx* ctx, const iga_kkt* kkt, const iga_btt* x, iga_btt** y);

/* ||A f - b|| / ||b|| with b = [M yhat; 0; 0] (time-dependent: [tau calM yhat; 0; 0]), in
 * FP64 on expanded vectors. */
int iga_kkt_residual(iga_ctx* ctx, const iga_kkt* kkt, const iga_tt* yhat, const iga_btt* f,
                     double* rel_residual);

/* Block-AMEn solve of A f = [M yhat; 0; 0] (Section 5): alternating sweeps
 * over the cores, each projecting the three block rows onto the frame of the
 * current solution (eq. KKT_red), solving the projected system by
 * preconditioned GMRES, enriching with a residual direction and moving the
 * component index by a truncated SVD (eqs. svd1, svd2). Stops when every local
 * residual of a half-sweep is <= tol (relative) or after nswp half-sweeps
 * (IGA_ENOCONV, or IGA_ERANK when a solution rank is at r_max; *sol is still returned).
 * A local residual or Krylov norm that is not finite (an iterate or input holding NaN or
 * Inf) ends the solve with IGA_ENUM and no solution.
 * x0 (nullable) is the initial guess.
 * stats (nullable) receives the statistics above. */
int iga_amen_solve(iga_ctx* ctx, const iga_kkt* kkt, const iga_tt* yhat, double tol,
                   const iga_amen_opts* opts, const iga_btt* x0, iga_btt** sol,
                   iga_amen_stats* stats);

/* SWITCHED OFF: returns IGA_EINVAL after checking its arguments (a run of 64 problems of
 * the batching workload through it faulted the GPU; the cause has not been found).
 * Batching form for whole solves: nprob independent block-AMEn solves, each exactly as
 * iga_amen_solve(ctx, kkts[i], yhats[i], tols[i], opts, NULL, &sols[i], &stats[i]), run
 * concurrently by nworkers (1..64) host threads. Each worker owns a stream and a workspace
 * on ctx's device for the duration of the call (default priority), so the solves' small
 * launches overlap on the GPU; each solve runs the same kernels in the same order as alone,
 * so results are those of the sequential calls. Every kkts[i] must live on ctx's device.
 * status[i] receives each solve's return code; sols[i] its solution (owned by the caller,
 * in ctx) for every status IGA_OK, IGA_ENOCONV or IGA_ERANK, else NULL. stats may be NULL
 * (else nprob entries). Returns IGA_OK, or the first failing problem's code when a solve
 * produced no solution. Memory: up to nworkers solves' workspaces at once. Synchronises. */
int iga_amen_solve_many(iga_ctx* ctx, int nprob, const iga_kkt* const* kkts, const iga_tt* const* yhats,
                        const double* tols, const iga_amen_opts* opts, int nworkers, iga_btt** sols,
                        iga_amen_stats* stats, int* status);

/* The projected local TT-matvec of one block-AMEn step (eq. KKT_red), on raw
 * device buffers: for l = 0..2 and A in {M, K}
 *   (A x_l)[a',i,b'] = sum PhiL_A[al][a'][a] A[al][i][i+o-p][be] x_l[a][i+o-p][b] PhiR_A[be][b'][b]
 * combined into y = [M x0 + K x2; beta M x1 - M x2; K x0 - M x1].
 * x, y: dev [3][r0][n][r1]; PhiL_*: dev [R_{d-1}][r0][r0]; PhiR_*: dev [R_d][r1][r1];
 * Mcore, Kcore: dev banded [R_{d-1}][n][2p+1][R_d] (dense in the rank indices).
 * precision: IGA_FP64, IGA_FP32 or IGA_BF16 (inputs are FP64; FP32 converts them to FP32
 * first, BF16 likewise and then rounds every contraction operand to bfloat16, accumulating
 * in FP32).
 * Enqueued on the context stream; returns immediately. */
int iga_local_matvec(iga_ctx* ctx, int r0, int n, int r1, int degree, int RM0, int RM1, int RK0,
                     int RK1, const double* PhiL_M, const double* PhiR_M, const double* PhiL_K,
                     const double* PhiR_K, const double* Mcore, const double* Kcore, double beta,
                     const double* x, double* y, int precision);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): iga_local_matvec in FP64 with no
 * allocation. Same arguments, layouts and result as iga_local_matvec with precision
 * IGA_FP64, the same kernels in the same order. Every intermediate (re-laid cores, the
 * three contraction stages, split-K partials) lives in one fixed device array of
 * IGA_NOALLOC_SCRATCH_BYTES per GPU, reserved when the library's code is loaded on that GPU
 * and held until the process ends; its address is looked up by iga_ctx_create. A shape whose
 * workspace exceeds the array returns IGA_EINVAL (the message gives the bytes needed). The
 * call makes no device allocation or free. All calls on one GPU share that GPU's array and
 * it keeps what the last call left: calls that overlap on one GPU (other streams or host
 * threads) race, so a caller must order them. Enqueued on the context stream; returns
 * immediately. */
#define IGA_NOALLOC_SCRATCH_BYTES (64L << 20)
int iga_local_matvec_noalloc(iga_ctx* ctx, int r0, int n, int r1, int degree, int RM0, int RM1, int RK0,
                             int RK1, const double* PhiL_M, const double* PhiR_M, const double* PhiL_K,
                             const double* PhiR_K, const double* Mcore, const double* Kcore, double beta,
                             const double* x, double* y);

/* Reduced cost of the control problem at a solution f = (y, u, lambda) of the KKT
 * system (Section 4, eq. optimization1 with time removed):
 *   J = 1/2 (y - yhat)^T M (y - yhat) + beta/2 u^T M u, in FP64 on expanded vectors. */
int iga_objective(iga_ctx* ctx, const iga_kkt* kkt, const iga_tt* yhat, const iga_btt* f, double* J);

/* Gradient of the reduced cost with respect to the desired-state coefficients: at the
 * optimum dJ/dyhat = -M (y - yhat) (derivative of the Lagrangian of Section 4 in yhat).
 * grad: device, [n0][n1][n2] FP64, caller-owned. Synchronises. */
int iga_grad_yhat(iga_ctx* ctx, const iga_kkt* kkt, const iga_tt* yhat, const iga_btt* f, double* grad);

/* Gradient of the reduced cost with respect to the geometry control points (the derivative
 * of the Lagrangian J + lambda^T (K y - M u) at f along the geometry). M and K depend on the
 * geometry through the weights omega and Q interpolated in the space of Section 3 (eqs.
 * weightEquationSystem, weightEquationSolve); the gradient is that of this discretisation
 * with untruncated weight tensors (weight_tol and weight_rmax of opts are not used; p_interp
 * and nquad are). geo, degree, n: as for iga_assemble_factors; f: the solution for the
 * operators assembled from geo (and beta). grad: host, [3][ncp0][ncp1][ncp2] FP64 (same
 * layout as geo->ctrl), caller-owned. Needs about 2 GB of device workspace plus the grid
 * arrays. Synchronises. */
int iga_grad_geometry(iga_ctx* ctx, const iga_geometry* geo, int degree, const int n[3],
                      const iga_assembly_opts* opts, double beta, const iga_tt* yhat, const iga_btt* f,
                      double* grad);

/* Batching form: the projected local TT-matvecs of many independent problems of uneven
 * sizes (each as in iga_local_matvec, eq. KKT_red) in one call. Each of the three
 * contraction stages of all problems is one persistent grouped launch per tile shape
 * (workgroups walk a shared list of tiles of all products); autotune != 0 times the tile
 * shapes on the first call for each size bucket and keeps the fastest for the context.
 * Results do not depend on the tile shape chosen. precision: IGA_FP64 or IGA_FP32 (operands
 * converted in one launch, contractions in FP32, results converted back). Operands as in
 * iga_local_matvec (device, FP64, caller-owned); y of different problems must not overlap.
 * Synchronises. */
typedef struct {
  int r0, n, r1, degree, RM0, RM1, RK0, RK1;
  const double* PhiL_M;
  const double* PhiR_M;
  const double* PhiL_K;
  const double* PhiR_K;
  const double* Mcore;
  const double* Kcore;
  double beta;
  const double* x;
  double* y;
} iga_local_problem;
int iga_local_matvec_batched(iga_ctx* ctx, int nprob, const iga_local_problem* probs, int precision,
                             int autotune);

/* Algorithmic flops of one iga_local_matvec call with these sizes. */
double iga_local_matvec_flops(int r0, int n, int r1, int degree, int RM0, int RM1, int RK0, int RK1);

/* Event timing of the three stages of the projected local TT-matvec (eq. KKT_red), chiefly
 * the banded (middle) stage, the contraction of the operator core with the band of
 * t1 = PhiL x, for measurement. Between iga_profile_start and iga_profile_stop every local
 * matvec on the context (inside iga_amen_solve or iga_local_matvec) records HIP event pairs on
 * the context stream around each stage, per operator and precision (index 0: M FP64, 1: K FP64,
 * 2: M FP32, 3: K FP32, 4: M BF16, 5: K BF16). stop synchronises the stream and returns:
 * stages (banded stages
 * timed), launches (kernel launches inside them: one per nonzero rank block of the core),
 * ms (summed event time) and flops (algorithmic flops: banded nonzeros times nonzero rank
 * blocks). out may be NULL. Calls on one context must not overlap. */
typedef struct {
  long stages[6];
  long launches[6];
  double ms[6];
  double flops[6];
  /* the same operators' other two stages: the left-interface product t1 = PhiL x and the
   * right-interface product with PhiR (summed event time and algorithmic flops) */
  double s1_ms[6];
  double s1_flops[6];
  double s3_ms[6];
  double s3_flops[6];
} iga_profile;
int iga_profile_start(iga_ctx* ctx);
int iga_profile_stop(iga_ctx* ctx, iga_profile* out);

/* Measured ceilings of the device for the roofline of the local TT-matvec (Section 5's
 * contractions run on the matrix cores; their operands stream from HBM). Runs six short
 * project-written probe kernels on the context stream and writes to out[6] (host memory,
 * caller-owned): TFLOP/s of v_mfma_f64_4x4x4_4b (the instruction of the FP64 contractions),
 * of v_mfma_f64_16x16x4, of v_mfma_f32_16x16x4 (FP32 form) and of v_mfma_f32_16x16x32_bf16
 * (BF16 form), each with 8 independent accumulators per wave and 8 workgroups per CU; then
 * GB/s of a device copy (bytes read plus written) and of a device read, over 512 MiB
 * buffers. Best of three timed launches each. Temporarily allocates 1 GiB of device memory
 * (IGA_ENOMEM if that fails) and about 5 MB from the context pool. Synchronises; takes about
 * 0.1 s. */
int iga_measure_peaks(iga_ctx* ctx, double* out);

const char* iga_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* IGA_H */
