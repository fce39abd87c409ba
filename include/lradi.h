/*
 * lradi.h -- C ABI of the MI355X (gfx950) implementation of the inexact
 * low-rank ADI iteration for large Sylvester equations
 *
 *     A X + X B = -f g^T,  A (n x n), B (m x m) sparse, f (n x r), g (m x r),
 *
 * as stated in eq. (sylv) and Algorithm 1 of Kuerschner, "Inexact linear solves
 * in the low-rank ADI iteration for large Sylvester equations".  The solution
 * is returned in factored form X ~ Z D Y^T with D = diag(gamma_1 I_r, ...,
 * gamma_k I_r) (Algorithm 1, output).  The generalized equation
 * A X C + M X B = -f g^T (eq. (gsylv)) and its Lyapunov case run on the same
 * engine (lradi_solve_gen, lradi_solve_lyap).  Shifts are real.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Dense blocks are row-major: an n x r block stores entry (i, c) at
 *    i*r + c.  Factor stacks Z, Y are k consecutive n x r (m x r) blocks.
 *  - "device" pointers are HIP device allocations (e.g. torch tensors on
 *    cuda:0); "host" pointers are ordinary memory.  Each argument states which.
 *  - Shifts: shiftsA[k] is added to A in the k-th A-side solve
 *    (A + shiftsA[k] I) z_k = w_{k-1} (beta_k of Algorithm 1); shiftsB[k] is
 *    added to B^T in the B-side solve (B^T + shiftsB[k] I) y_k = t_{k-1}
 *    (conj(alpha_k)).  gamma_k = -(shiftsA[k] + shiftsB[k]).  Arrays shorter
 *    than the number of steps are cycled.
 *  - Every call returns an int status (LRADI_OK = 0; negative = error,
 *    positive = warning with valid results).  No exception crosses the ABI.
 *    lradi_last_error() returns a message for the calling thread's last
 *    failing call.
 *  - All work of one context is issued on its HIP stream; calls on one context
 *    must not overlap (a context is not thread-safe).  Calls return after the
 *    stream has finished unless stated otherwise.
 */
#ifndef LRADI_H
#define LRADI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define LRADI_OK 0
#define LRADI_EINVAL (-1)      /* bad argument (shape, pointer, option)          */
#define LRADI_ENOMEM (-2)      /* device allocation failed / over HBM budget      */
#define LRADI_EHIP (-3)        /* a HIP runtime call failed                       */
#define LRADI_ENAN (-4)        /* NaN or Inf appeared in the iteration            */
#define LRADI_EBREAKDOWN (-5)  /* unrecoverable Krylov breakdown                  */
#define LRADI_ECANCELED (-6)   /* serving request cancelled before completion    */
#define LRADI_WNOCONV 1        /* kmax outer steps without reaching tau          */
#define LRADI_WINNER 2         /* some inner solve stopped at its iteration cap   */
#define LRADI_WGAP 3           /* converged in the computed residual, but the
                                  residual-gap estimate u_k + v_k of
                                  eq. (upd_resgap) ended above the budget epsilon
                                  of Thm 3 (clamps of eq. (bound_tols) overrode
                                  the admissible tolerances), so the true
                                  residual is not certified below 2 tol: it is
                                  only bounded by tol + (u_k + v_k)/||f g^T||.
                                  LRADI_WINNER takes precedence             */

/* ---- tolerance selections (Sec. 3.2) ---------------------------------- */
#define LRADI_SEL_RELATIVE 0   /* delta^A = rho*||w||, delta^B = rho*||t||        */
#define LRADI_SEL_FIXED 1      /* delta^A = delta^B = delta_fixed (Table 2 "fixed") */
#define LRADI_SEL_MID 2        /* eq. (simple_tols)                               */
#define LRADI_SEL_TIGHT_A 3    /* eq. (one_side): delta^A = delta_min              */
#define LRADI_SEL_TIGHT_B 4    /* mirror of eq. (one_side): delta^B = delta_min    */
#define LRADI_SEL_SYM 5        /* delta^A = delta^B: the largest equal pair on the
                                  boundary of eq. (ADI_relax1_prak)/(ADI_relax2_prak),
                                  clamped by eq. (bound_tols)                     */

/* ---- inner right preconditioners (opts.precond) ---------------------- */
#define LRADI_PRECOND_NONE 0
/* ILU(0) of A + s I in red-black order: rows 2-coloured so that every
 * off-diagonal entry joins a red and a black row; with S = [D_r E; F D_b]
 * (red first) it applies z_b = diag(T)^-1 (v_b - F D_r^-1 v_r),
 * T = D_b - F D_r^-1 E, refined by precond_sweeps Jacobi steps (or, with
 * precond_poly = 1, Chebyshev steps) on T, then z_r = D_r^-1 (v_r - E z_b).
 * Both half-steps are parallel over rows. */
#define LRADI_PRECOND_RBILU0 1

/* ---- arithmetic of the inner Krylov solves ---------------------------- */
#define LRADI_FP64 0           /* basis, SpMM and projections in FP64             */
#define LRADI_FP32_INNER 1     /* basis, SpMM and projections in FP32; residual
                                  factors, refinement residual, small least
                                  squares and all norms in FP64                  */

/* number of doubles per row of lradi_result_history() */
#define LRADI_HIST_COLS 16
/* columns: 0 k, 1 ||w_{k-1}t_{k-1}^T||/||fg^T|| (before the step),
 * 2 delta^A_k, 3 delta^B_k, 4 achieved ||r^A_k||, 5 achieved ||r^B_k||,
 * 6 inner block steps A, 7 inner block steps B, 8 u_k, 9 v_k,
 * 10 ||w_{k-1}||, 11 ||t_{k-1}||, 12 ||z_k||, 13 ||y_k||, 14 gamma_k,
 * 15 ||w_k t_k^T||/||fg^T|| (after the step)                               */

typedef struct lradi_ctx lradi_ctx;
typedef struct lradi_result lradi_result;

/* Compressed sparse row matrix, int32 indices, FP64 values, columns may be in
 * any order within a row.  Borrowed: the caller keeps ownership and keeps the
 * arrays alive for the duration of the call.  on_device = 1: the three
 * pointers are device pointers; 0: host pointers (copied in by the call). */
typedef struct {
  int32_t nrows, ncols;
  int64_t nnz;
  const int32_t* rowptr; /* nrows + 1 */
  const int32_t* colind; /* nnz */
  const double* val;     /* nnz */
  int32_t on_device;
} lradi_csr;

/* Options of one solve.  lradi_default_opts() fills the settings of the
 * paper's experiments (Sec. 4): tol 1e-8, delta_min = tol/20, delta_max =
 * 0.1, kmax = 50, xi = 1, back-looking mid selection; the dynamic
 * selections are evaluated in the balanced frame (rescale = 2), which keeps
 * the clamps of eq. (bound_tols) admissible when n and m differ a lot. */
typedef struct {
  double tol;          /* outer tau: stop when ||w t^T|| < tol*||f g^T||      */
  double eps;          /* absolute gap budget epsilon of Thm 3; <= 0 selects
                          tol*||f g^T||                                       */
  double delta_min;    /* eq. (bound_tols), absolute                          */
  double delta_max;    /* eq. (bound_tols), absolute                          */
  double xi;           /* safeguard constant of eqs. (ADI_relax*_prak)        */
  double delta_fixed;  /* LRADI_SEL_FIXED tolerance, absolute                 */
  double rho;          /* LRADI_SEL_RELATIVE factor                           */
  double fp32_floor;   /* FP32 inner: a restart cycle stops once its residual
                          estimate is below fp32_floor times its start        */
  int32_t kmax;        /* outer step budget (also enters the thresholds)      */
  int32_t selection;   /* LRADI_SEL_*                                         */
  int32_t backlook;    /* 1: eq. (ADI_relax2_prak), 0: eq. (ADI_relax1_prak)  */
  int32_t paper_abs;   /* 1: |.| of eq. (ADI_relax2_prak) as printed;
                          0: a spent budget gives delta_min                  */
  int32_t precision;   /* LRADI_FP64 or LRADI_FP32_INNER                      */
  int32_t restart;     /* block GMRES restart length m (blocks), 1..64        */
  int32_t max_inner;   /* cap on block Arnoldi steps per inner solve          */
  int32_t rescale;     /* 1: scale f, g to equal spectral norm (Sec. 4), the   *
                        * paper's frame.  2 (default): also evaluate the       *
                        * dynamic selections for the pair (s w, t/s) at equal  *
                        * norms and map them back (an extension: keeps         *
                        * delta_min admissible when the factor norms drift     *
                        * apart, so u_k + v_k stays within epsilon).  0: no    *
                        * rescaling                                           */
  int32_t b_is_transposed; /* 1: the B argument already holds B^T             */
  int32_t lookahead;   /* host scheduling depth (0 = synchronous), >= 0       */
  int32_t use_graph;   /* 1: capture one tick (inner step kernels, outer step
                          end, unfinished count) into a hipGraph per
                          look-ahead slot and replay it; captured again when
                          the set of systems changes.  Ignored with
                          profile = 1 or on the null stream               */
  int32_t profile;     /* 1: time the projection (Gram) and shifted-product
                          launches with HIP events and count their
                          algorithmic bytes (see lradi_profile_read)         */
  int32_t spmm_lanes;  /* shifted-product tiling: lanes per matrix row, each
                          owning r/lanes columns.  0: autotuned per matrix
                          shape (timed once per context, see
                          lradi_spmm_tune); -1: built-in rule without timing;
                          1, 2, 4: forced (must divide r)                    */
  int32_t precond;     /* right preconditioner of the inner block GMRES
                          (Sec. 3.2.4: right preconditioning keeps the
                          solver's residual the true inner residual):
                          LRADI_PRECOND_NONE or LRADI_PRECOND_RBILU0.  The
                          latter needs M = C = I and a bipartite sparsity
                          graph (else LRADI_EINVAL)                        */
  int32_t precond_sweeps; /* LRADI_PRECOND_RBILU0: Jacobi sweeps (Chebyshev
                          steps with precond_poly = 1) on the Schur
                          complement after the ILU(0) step, 0..64       */
  int32_t precond_pairs;  /* 1 (default): run the sweeps two per launch where
                          the black rows tile well (each tile's first sweep
                          also covers the rows its second one reads, kept in
                          workgroup memory): matrices of at least 32768 rows
                          whose tiles' regions stay within 1.6 times the
                          tiles (2-D stencils), in batches of at most 262144
                          black rows.  The results equal one sweep per
                          launch bit for bit.  0: one per launch           */
  int32_t precond_poly;   /* LRADI_PRECOND_RBILU0 with precond_sweeps > 0:
                          0 (default): the sweeps are Jacobi steps; 1:
                          Chebyshev steps (Golub-Varga semi-iteration on the
                          same splitting) over the interval that two
                          Gershgorin-type bounds give for the spectrum of
                          I - diag(T)^-1 T, recomputed per shift; they
                          assume that spectrum real, which holds when T is
                          diagonally similar to a symmetric matrix (e.g.
                          constant-coefficient upwind stencils); without
                          diagonal dominance (bound >= 1) the steps fall
                          back to Jacobi.  Same products with T per step;
                          paired as the sweeps (precond_pairs), with four
                          iterate blocks of the black rows instead of two
                          where pairs can run.  An extension, not in the
                          paper                                           */
  int32_t pad_;
} lradi_opts;

/* Per inner solve statistics (lradi_shifted_solve). */
typedef struct {
  int32_t steps;       /* block Arnoldi steps                                 */
  int32_t cycles;      /* restart cycles                                      */
  int32_t status;      /* 0 converged, 1 step cap hit, 2 breakdown, 3 NaN     */
  int32_t pad;
  double rnorm;        /* achieved ||W - (A + shift I) Z||_2 (FP64)           */
} lradi_inner_stats;

/* Kernel classes reported by lradi_profile_read. */
#define LRADI_PROF_GRAM 0      /* block projection V^T U (two launches per step)  */
#define LRADI_PROF_SPMM 1      /* shifted product U = (A + s I) V_j               */
#define LRADI_PROF_PRECOND 2   /* right preconditioner P_j = M V_j (sweeps + 2
                                  launches per step; bytes exclude the once-
                                  per-solve build of the Schur couplings)      */
#define LRADI_PROF_CLASSES 3

/* Accumulated measurements of one kernel class over the solves run with
 * opts.profile = 1 since the last lradi_profile_reset.  ms: summed
 * event-timed launch durations; bytes: summed algorithmic bytes (data the
 * method must read and write: basis blocks and candidate block for the
 * projection; values, indices, input and output block for the product). */
typedef struct {
  double ms;
  int64_t launches;
  int64_t bytes;
} lradi_kernel_profile;

void lradi_default_opts(lradi_opts* opts);
const char* lradi_strerror(int status);
const char* lradi_last_error(void);

/* Context: binds a device and a stream (NULL = a stream the context creates
 * and owns) and pools workspace.  device = HIP ordinal. */
int lradi_create(lradi_ctx** ctx, int device, void* hip_stream);
int lradi_destroy(lradi_ctx* ctx);

/* Size of the 2-D (dim = 2) or 3-D (dim = 3) upwind convection-diffusion
 * matrix on N^dim interior points (Sec. 4, eq. (ex:convdiff)). */
int lradi_convdiff_size(int dim, int N, int64_t* n, int64_t* nnz);

/* Fill caller-allocated host arrays rowptr (n+1), colind (nnz), val (nnz)
 * with A = -L_h of eq. (ex:convdiff): h = 1/(N+1), homogeneous Dirichlet,
 * lexicographic order with the first axis fastest, upwind first-order term,
 * ascending columns.  Values follow a fixed FP64 recipe (products and sums
 * rounded separately) so they are reproducible bit for bit.  omega: dim
 * doubles (host).  B^T of such a matrix is the matrix with -omega. */
int lradi_gen_convdiff(int dim, int N, const double* omega, int32_t* rowptr,
                       int32_t* colind, double* val);

/* Discretisations of the first-order term for lradi_gen_convdiff_scheme. */
#define LRADI_SCHEME_UPWIND 0  /* as lradi_gen_convdiff: real spectrum        */
#define LRADI_SCHEME_CENTRAL 1 /* central differences: coefficient of u at
                                  p - s_c is -ih2 - (w_c ih)/2, at p + s_c it is
                                  -ih2 + (w_c ih)/2, diagonal sum of 2 ih2
                                  (then negated); once the mesh Peclet number
                                  |w_c| h / 2 exceeds 1 the spectrum is complex
                                  (the non-symmetric case of Sec. 3.2.4 with
                                  complex shift parameters)                 */
/* lradi_gen_convdiff with the first-order term discretised by `scheme`;
 * same sizes, ordering and value recipe otherwise. */
int lradi_gen_convdiff_scheme(int dim, int N, const double* omega, int scheme, int32_t* rowptr,
                              int32_t* colind, double* val);

/* Y = (A + shift I) X for one n x r block (the shifted product used by every
 * inner Krylov step).  A: csr (host or device); X, Y: device, n x r
 * row-major, double when precision = LRADI_FP64, float when
 * LRADI_FP32_INNER (then A's values are used rounded to FP32).  1 <= r <= 8.
 * Returns after the stream finished. */
int lradi_spmm(lradi_ctx* ctx, const lradi_csr* A, double shift, const void* X,
               void* Y, int r, int precision);

/* Measurement helper for the shifted product: copies A to the device once,
 * then launches the product Y = (A + shift I) X reps times back to back and
 * returns the average launch time in milliseconds (HIP events on the
 * context's stream) and the algorithmic bytes of one launch (each nonzero's
 * value and column index once, X read once, Y written once; the row
 * structure, O(n / 32) slice starts in the product's layout, is not
 * counted).  lanes: the
 * tiling (1, 2, 4 lanes per row, dividing r), or 0 for the one the solver
 * would pick (lradi_spmm_tune). */
int lradi_spmm_bench(lradi_ctx* ctx, const lradi_csr* A, double shift, const void* X, void* Y,
                     int r, int precision, int lanes, int reps, double* avg_ms, int64_t* bytes);

/* Autotuner of the shifted-product tiling: times every admissible lanes per
 * row (1, 2, 4 dividing r) on A with r columns in the given precision and
 * returns the fastest in *lanes; the choice is cached in the context per
 * (n, nnz, r, precision) and reused by every later solve.  Products smaller
 * than 8 MiB of X are launch-bound and take the built-in rule untimed.  All
 * tilings give bitwise identical products. */
int lradi_spmm_tune(lradi_ctx* ctx, const lradi_csr* A, int r, int precision, int* lanes);

/* Solve nsys independent shifted block systems (A_s + shift_s I) Z_s = W_s
 * with block GMRES(m) plus FP64 iterative refinement until
 * ||W_s - (A_s + shift_s I) Z_s||_2 <= delta_s (absolute, spectral norm) --
 * the inner solves of Algorithm 1, eq. (gfadi_incsolves).  All systems run
 * in the same kernel launches.  A[s]: csr (host or device); W[s]: device,
 * n_s x r[s] doubles; Z[s]: device, n_s x r[s] doubles, overwritten (zero
 * initial guess).  shift, delta, r (1..8, at most n_s): host arrays of
 * nsys.  opts: precision, restart, max_inner, fp32_floor, precond,
 * precond_sweeps are used (NULL = defaults).  stats: host array of nsys, may
 * be NULL.  Warning LRADI_WINNER if a step cap was hit. */
int lradi_shifted_solve(lradi_ctx* ctx, int nsys, const lradi_csr* const* A,
                        const double* shift, const double* const* W, double* const* Z,
                        const int* r, const double* delta, const lradi_opts* opts,
                        lradi_inner_stats* stats);

/* Algorithm 1 (inexact LR-ADI) on A X + X B = -f g^T.  A: n x n csr, B: m x m
 * csr (B itself, or B^T when opts->b_is_transposed).  f, g: device, n x r and
 * m x r row-major doubles (not modified).  shiftsA/shiftsB: host, nshifts
 * doubles.  opts may be NULL (defaults).  *out receives a library-owned
 * result (free with lradi_result_free) also on LRADI_WNOCONV/LRADI_WINNER. */
int lradi_solve(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* B, const double* f,
                const double* g, int r, const double* shiftsA, const double* shiftsB,
                int nshifts, const lradi_opts* opts, lradi_result** out);

/* Algorithm 1 with M and C: A X C + M X B = -f g^T (eq. (gsylv)) by the
 * iteration of eq. (lradi_g): (A + beta_k M) z_k = w_{k-1},
 * w_k = w_{k-1} + gamma_k M z_k, (B + alpha_k C)^T y_k = t_{k-1},
 * t_k = t_{k-1} + gamma_k C^T y_k; the gap recursion of eq. (upd_resgap)
 * uses ||M z_k|| and ||C^T y_k||.  M (n x n) and C (m x m, or C^T when
 * opts->b_is_transposed) are csr matrices; either may be NULL (identity).
 * The inner systems are stored as pencils: the union pattern of A and M
 * with both value arrays, combined per shift inside the kernels.  Other
 * arguments as lradi_solve. */
int lradi_solve_gen(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* B, const lradi_csr* M,
                    const lradi_csr* C, const double* f, const double* g, int r,
                    const double* shiftsA, const double* shiftsB, int nshifts,
                    const lradi_opts* opts, lradi_result** out);

/* The Lyapunov case of eq. (gsylv) named with the related equations of
 * Sec. 3.2.4: A X M^T + M X A^T = -f f^T, i.e. B = A^T, C = M^T, g = f.
 * With alpha_k = beta_k = shifts[k] (added to A: (A + p_k M) z_k = w_{k-1})
 * the B-side system of eq. (lradi_g) is the A-side system and t_0 = w_0, so
 * one inner solve per step serves both sides: y_k = z_k, t_k = w_k,
 * gamma_k = -2 p_k and X = Z D Z^T.  The inner tolerance of a step is
 * min(delta^A, delta^B) of opts->selection (LRADI_SEL_SYM gives the largest
 * equal admissible pair); since r^B = r^A the gap recursion of
 * eq. (upd_resgap) gives u = v.  A: n x n csr; M: n x n csr or NULL
 * (identity); f: device, n x r row-major (not modified); shifts: host,
 * nshifts.  opts->b_is_transposed and opts->rescale have no effect (f and g
 * are one matrix).  The result's Y factor is Z (same device pointer, m = n);
 * its history rows repeat the A-side values in the B-side columns, with 0
 * B-side inner steps.  Errors as lradi_solve. */
int lradi_solve_lyap(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* M, const double* f, int r,
                     const double* shifts, int nshifts, const lradi_opts* opts, lradi_result** out);

/* One Sylvester problem for lradi_batch_solve and the serving loop. */
typedef struct {
  const lradi_csr* A;      /* n x n (host or device)                           */
  const lradi_csr* B;      /* m x m: B, or B^T when opts->b_is_transposed      */
  const double* f;         /* device, n x r row-major (not modified)           */
  const double* g;         /* device, m x r row-major (not modified)           */
  int32_t r;               /* 1..8, at most n and m                            */
  int32_t nshifts;
  const double* shiftsA;   /* host, nshifts (added to A)                       */
  const double* shiftsB;   /* host, nshifts (added to B^T)                     */
  double tol;              /* outer tau of this problem; <= 0 uses opts->tol.
                              opts->delta_min and opts->delta_fixed refer to
                              opts->tol and are scaled by tol / opts->tol     */
  const lradi_csr* M;      /* generalized equation A X C + M X B = -f g^T
                              (eq. (gsylv), iteration (lradi_g)): n x n, or
                              NULL for M = I                                  */
  const lradi_csr* C;      /* m x m (C^T when opts->b_is_transposed), or NULL
                              for C = I                                       */
  int32_t lyapunov;        /* nonzero: the Lyapunov case A X M^T + M X A^T =
                              -f f^T (B = A^T, C = M^T, g = f, shiftsB =
                              shiftsA; B, g, shiftsB, C are ignored and may
                              be NULL): one inner solve per step, Y = Z     */
  const double* shiftsA_im;  /* complex shifts: imaginary parts (host,
                              nshifts) of the shifts added to A, or NULL for
                              real shifts; see lradi_solve_complex          */
  const double* shiftsB_im;  /* imaginary parts of the shifts added to B^T  */
} lradi_problem;

/* Algorithm 1 with complex shift parameters in its complex form, the one
 * Sec. 3.2.4 keeps for non-symmetric problems whose shift sets contain
 * complex conjugate pairs (A, B, f, g real):
 *   (A + pA_k I) z_k = w_{k-1},  w_k = w_{k-1} + gamma_k z_k,
 *   (B^T + pB_k I) y_k = t_{k-1},  t_k = t_{k-1} + conj(gamma_k) y_k,
 *   gamma_k = -(pA_k + conj(pB_k)),  X ~ Z diag(gamma_k I_r) Y^*,
 * with pA_k = beta_k and pB_k = conj(alpha_k) of Algorithm 1.  Each inner
 * solve is the real form of the complex shifted system on the stacked block
 * [re; im] (2n rows); norms are those of the complex blocks (eq. (upd_resgap)
 * takes |gamma_k|).  The shifts come as real and imaginary parts (host
 * arrays of nshifts, cycled).  Needs r <= 4, no mass matrices and
 * opts->precond = LRADI_PRECOND_NONE (LRADI_EINVAL otherwise).  The result
 * is complex (lradi_result_is_complex): factor block k of Z is 2n x r with
 * the real parts in rows 0..n-1 and the imaginary parts in rows n..2n-1
 * (Y likewise, 2m x r), D holds (re, im) pairs of the gammas.  When the
 * shifts come in conjugate pairs and the step count completes every pair,
 * X is real up to rounding.  lradi_residual does not take complex factors.
 * Other arguments and errors as lradi_solve. */
int lradi_solve_complex(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* B, const double* f,
                        const double* g, int r, const double* shiftsA_re, const double* shiftsA_im,
                        const double* shiftsB_re, const double* shiftsB_im, int nshifts,
                        const lradi_opts* opts, lradi_result** out);

/* Algorithm 1 on nprob independent problems of uneven n, m, r advanced
 * together: every outer step of all unfinished problems runs in the same
 * kernel launches (the inner solves of all 2*nprob shifted systems share one
 * launch sequence per block Arnoldi step); finished problems leave the batch
 * at step boundaries.  opts is shared (its tol is the default per problem).
 * outs: caller array of nprob, each receives a library-owned result.  The
 * return value is the most severe status over the problems. */
int lradi_batch_solve(lradi_ctx* ctx, int nprob, const lradi_problem* probs,
                      const lradi_opts* opts, lradi_result** outs);

/* ---- serving: continuous batching over one context --------------------
 * A worker thread owned by the server admits queued problems whenever their
 * device footprint fits in hbm_budget bytes (and fewer than max_active are
 * in flight), advances every admitted problem one outer LR-ADI step per
 * iteration in shared kernel launches (as lradi_batch_solve), and completes
 * finished problems at step boundaries, so requests that arrive while
 * others run join as memory and slots free up.  Admission is first come,
 * first served.  While a server exists its context must not be used by the
 * caller.  submit / poll / cancel / stats may be called from any one thread. */
typedef struct lradi_server lradi_server;
typedef struct {
  int32_t active;          /* problems in flight                              */
  int32_t queued;          /* submitted, not yet admitted                     */
  int64_t completed;       /* finished (including failed and cancelled)       */
  int64_t steps;           /* scheduling rounds run by the worker             */
  int64_t bytes_in_use;    /* summed footprint of the problems in flight      */
  int64_t bytes_budget;
} lradi_server_counters;

/* max_active <= 0: no slot limit.  hbm_budget == 0: 80% of the device's
 * free memory at creation. */
int lradi_server_create(lradi_ctx* ctx, const lradi_opts* opts, int64_t hbm_budget,
                        int max_active, lradi_server** out);
/* Queue one problem.  The inputs are copied before the call returns (f, g
 * device, shifts host, matrices host or device).  *ticket identifies it.
 * LRADI_ENOMEM if the problem alone exceeds the budget (it is rejected). */
int lradi_server_submit(lradi_server* srv, const lradi_problem* prob, uint64_t* ticket);
/* 0: done, *out receives the result (caller frees it) and *latency_s the
 * time from submit to completion; 1: still pending; LRADI_EINVAL: unknown
 * ticket (or already collected). */
int lradi_server_poll(lradi_server* srv, uint64_t ticket, lradi_result** out, double* latency_s);
/* Cancel a queued or running request; it completes with LRADI_ECANCELED. */
int lradi_server_cancel(lradi_server* srv, uint64_t ticket);
int lradi_server_stats(lradi_server* srv, lradi_server_counters* out);
/* Stop the worker (running problems are cancelled) and free everything not
 * yet collected. */
int lradi_server_destroy(lradi_server* srv);

/* Scalars of a result: steps k, status, ||w_k t_k^T||/||f g^T||, ||f g^T||
 * (after the optional rescaling, which leaves f g^T unchanged). */
int lradi_result_info(const lradi_result* res, int* k, int* status, double* rel_res_comp,
                      double* norm_fg);
/* Device pointers (owned by the result) to Z (k x n x r), D (k gammas) and
 * Y (k x m x r); n, m, r may be NULL. */
int lradi_result_factors(const lradi_result* res, const double** Z, const double** D,
                         const double** Y, int* n, int* m, int* r);
/* Copy the factors to caller-owned host arrays of k*n*r, k and k*m*r
 * doubles (any may be NULL); complex results: k*2n*r, 2k and k*2m*r. */
int lradi_result_copy(const lradi_result* res, double* Z, double* D, double* Y);
/* 1 when the result holds complex factors (lradi_solve_complex). */
int lradi_result_is_complex(const lradi_result* res, int* is_complex);
/* Copy min(k, max_rows) history rows of LRADI_HIST_COLS doubles into rows
 * (host); returns the number of rows through *nrows. */
int lradi_result_history(const lradi_result* res, double* rows, int max_rows, int* nrows);
/* Wall time of the solve in seconds (host clock around the device work). */
int lradi_result_time(const lradi_result* res, double* seconds);
void lradi_result_free(lradi_result* res);

/* Read (host struct) or clear the per-context kernel measurements. */
int lradi_profile_read(lradi_ctx* ctx, int kernel_class, lradi_kernel_profile* out);
int lradi_profile_reset(lradi_ctx* ctx);

/* True scaled residual ||A Z D Y^T + Z D Y^T B + f g^T||_2 / ||f g^T||_2 of
 * a factored solution (Sec. 4 estimates it after termination with eigs on
 * R^T R; here Golub-Kahan-Lanczos bidiagonalisation with full
 * reorthogonalisation of R applied implicitly, FP64).  A, B as in
 * lradi_solve (B^T when b_is_transposed); f, g, Z (k x n x r), Y (k x m x r):
 * device; D: host, k gammas. */
int lradi_residual(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* B,
                   int b_is_transposed, const double* f, const double* g, int r,
                   const double* Z, const double* D, const double* Y, int k,
                   double* rel_true_res);

/* The same for the generalized equation: ||A X C + M X B + f g^T||_2 /
 * ||f g^T||_2 with X = Z D Y^T; M, C csr (C^T when b_is_transposed) or NULL
 * for the identity. */
int lradi_residual_gen(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* B, const lradi_csr* M,
                       const lradi_csr* C, int b_is_transposed, const double* f, const double* g,
                       int r, const double* Z, const double* D, const double* Y, int k,
                       double* rel_true_res);

/* ---- callers that cannot allocate -------------------------------------
 * For callers that must not allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 *
 * lradi_residual_noalloc computes what lradi_residual (b_is_transposed = 0,
 * M = C = I) computes, with the same kernels and the same arithmetic, but
 * makes no device allocation (no hipMalloc / hipFree, no allocating library
 * call): its Lanczos bases, partial sums and scalars live in a scratch array
 * of lradi_residual_noalloc_limit() bytes (64 MiB) that the library holds on
 * every device it runs on from module load until the process ends.  The
 * caller passes every input on the device: A (n x n) and its transpose At,
 * B (m x m) and its transpose Bt, all csr with on_device = 1 (int32 indices,
 * FP64 values, valid structure: not checked here); f, g, Z, Y as in
 * lradi_residual (device); D: host, k gammas (copied into the scratch).
 * Inputs whose workspace exceeds the scratch (it grows with (n + m) times
 * 2 k r, e.g. n = m = 4096 with k r = 120 fits, the 2-D 256^2 / 192^2
 * configuration at k r = 164 does not) are rejected with LRADI_EINVAL and a
 * message naming the sizes.  Calls on one device share its scratch array,
 * which keeps the last call's contents; the library serialises them with a
 * per-device lock, and the call returns after its stream finished.  A
 * context must have been created on the device first (lradi_create looks
 * up the scratch address there). */
int lradi_residual_noalloc(lradi_ctx* ctx, const lradi_csr* A, const lradi_csr* At,
                           const lradi_csr* B, const lradi_csr* Bt, const double* f,
                           const double* g, int r, const double* Z, const double* D,
                           const double* Y, int k, double* rel_true_res);
/* Size in bytes of the scratch array of lradi_residual_noalloc. */
int64_t lradi_residual_noalloc_limit(void);
/* Number of device allocations the library has made in this process
 * (diagnostics: lets a caller check that a call allocated nothing). */
int64_t lradi_alloc_count(void);

#ifdef __cplusplus
}
#endif
#endif /* LRADI_H */
