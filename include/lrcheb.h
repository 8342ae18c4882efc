/*
 * lrcheb.h - C ABI of the low-rank ChebyshevT solver for parameter-dependent
 * matrix equations on AMD Instinct MI355X (gfx950).
 *
 * The library solves the matrix equation of one Newton step on a parameter
 * subset (Benner, Richter, Weinhandl, arXiv 2008.10275, Sec. 3.4,
 * eq. newton_matrix1, written generically):
 *
 *     sum_{i<q} K_i X D_i = F,      D_i = diag(d[i, :]),  X, F in R^{n x m},
 *
 * with X kept in low-rank form U diag(s) V^T.  The iteration is the
 * preconditioned Chebyshev method with truncation ("ChebyshevT", Sec. 4.1 and
 * Sec. 5.1), the preconditioner is the operator at the subset's centre
 * parameters (Sec. 4.2), factorised once (Sec. 5 uses a permuted LU), and
 * Algorithm 1 (Sec. 4.1) drives one Newton step per subset from the upper
 * median parameter's solution (Sec. 3.3).
 *
 * Conventions for every call:
 *  - Host arrays passed in are copied; the library never keeps or frees caller
 *    memory.  Pointers named *_dev are device pointers owned by the caller.
 *  - Dense host matrices are column-major (Fortran order) unless stated.
 *  - Device factors are row-major: element (row i, column j) at p[i * ld + j].
 *  - Status: 0 success; LRC_ENOTCONV (> 0) is a warning (the result is valid,
 *    the best iterate is kept); negative values are errors, with a message
 *    available from lrc_last_error().  No call aborts the process.
 *  - Work is enqueued on the context's stream; calls that return host data
 *    synchronise that stream.  One context per host thread.
 */
#ifndef LRCHEB_H
#define LRCHEB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lrc_ctx_s* lrc_ctx;
typedef struct lrc_ops_s* lrc_ops;
typedef struct lrc_prob_s* lrc_prob;
typedef int lrc_status;

enum {
  LRC_OK = 0,
  LRC_ENOTCONV = 1,    /* tolerance not reached within the iteration limits */
  LRC_EINVAL = -1,     /* invalid argument (message says which)              */
  LRC_ENOMEM = -2,     /* device or host allocation failed                   */
  LRC_EDEVICE = -3,    /* HIP runtime error (message holds the HIP string)   */
  LRC_ESINGULAR = -4,  /* zero or non-finite pivot in the preconditioner LU  */
  LRC_EBREAKDOWN = -5, /* Cholesky breakdown not recoverable by a shift      */
  LRC_ECALLBACK = -6   /* a user callback returned non-zero                  */
};

/* precision of the iteration.  LRC_MIXED_FP32: fp32 ChebyshevT on the
 * correction equation inside fp64 iterative refinement.  LRC_MIXED_FP32_DIR:
 * one ChebyshevT whose iterate and residual (SpMM and truncation) are fp64
 * while the preconditioner solves and the direction updates run in fp32.
 * LRC_MIXED_BF16GRAM: LRC_MIXED_FP32 whose fp32 truncations take their first
 * CholeskyQR pass on bf16 Gram products (operands rounded to bf16, fp32
 * accumulation, a preset shift of 1e-2 on the equilibrated Gram), the second
 * pass in fp32; the fp64 residual and refinement decide the accuracy. */
enum { LRC_FP64 = 0, LRC_MIXED_FP32 = 1, LRC_MIXED_FP32_DIR = 2, LRC_MIXED_BF16GRAM = 3 };
/* low-rank solver of the update equation (Sec. 4.1 names both): the
 * preconditioned Chebyshev iteration with truncation, or GMREST, restarted
 * GMRES with truncation on the left-preconditioned operator in the Frobenius
 * inner product (fp64 only; needs no spectrum interval; restart = the
 * Krylov dimension of a cycle; iters counts Arnoldi steps). */
enum { LRC_SOLVER_CHEBYSHEV = 0, LRC_SOLVER_GMREST = 1 };
/* form of the Chebyshev recurrence (both are the same polynomial iteration;
 * they differ only in where the truncation errors enter).
 * LRC_CHEB_DIRECTION: a direction D is kept, D <- T(a D + b P^-1 R), and the
 * iterate is updated by S <- T(S + D): two truncations per update.
 * LRC_CHEB_THREE_TERM: the three-term recurrence of the Chebyshev polynomials
 * on the iterates, S_{k+1} <- T((1 + a) S_k - a S_{k-1} + b P^-1 R_k), one
 * truncation of up to 2 rank_cap + rank(R) columns per update; every
 * precision takes it (with LRC_MIXED_FP32_DIR the fp32 solve P^-1 R is
 * widened to fp64 for the fp64 update).  Needs 2 rank_cap + rank_cap <= 128. */
enum { LRC_CHEB_DIRECTION = 0, LRC_CHEB_THREE_TERM = 1 };
/* initial guess of lrc_solve: none; the upper-median column's solution x~
 * as the fixed term X0 = x~ 1^T; given factors as the fixed term X0.  The
 * guess stays a separate exact term (X = X0 + S) so that truncation errors
 * are relative to the small correction S, not to X.
 * LRC_INIT_GIVEN_JUDGED: the given X0 (for instance a surrogate's prediction)
 * is judged column by column against the median guess x~ 1^T, which is
 * computed as for LRC_INIT_MEDIAN: column j keeps the guess whose fp64
 * residual ||(F - L(X0))_j|| is smaller, so X0 = [U0 | x~] diag(s0, 1)
 * [diag(w) V0 | 1 - w]^T with w_j in {0, 1}; lrc_info.median_fallback_cols
 * counts the columns where the median guess won.
 * LRC_INIT_NEWTON: the given X0 is the linearisation point of a Newton step
 * and F is already that step's right-hand side B (eq. newton_matrix1): S
 * solves L(S) = F and the solution is X = X0 + S (Sec. 3.4,
 * eq. matrix_nextiterate1); residuals are those of the Newton equation,
 * ||F - L(S)||. */
enum { LRC_INIT_ZERO = 0, LRC_INIT_MEDIAN = 1, LRC_INIT_GIVEN = 2, LRC_INIT_GIVEN_JUDGED = 3,
       LRC_INIT_NEWTON = 4 };

typedef struct {
  int rank_cap;        /* R: maximum rank of every truncated quantity           */
  double trunc_tol;    /* relative Frobenius tail of every truncation (eps)     */
  double res_tol;      /* stop at ||F - L(X)||_F <= res_tol * ||F||_F           */
  int max_iter;        /* total Chebyshev updates (all restarts, all refinements) */
  int restart;         /* restart the recurrence every `restart` updates, in [1, 64] */
  double cheb_c;       /* half-width of the spectrum interval (<= 0: from lrc_prob_spectrum) */
  double cheb_d;       /* centre of the spectrum interval                       */
  int precision;       /* LRC_FP64, LRC_MIXED_FP32 or LRC_MIXED_FP32_DIR          */
  int refine_max;      /* mixed: maximum fp64 refinement steps                  */
  double inner_tol;    /* mixed: residual reduction asked of each fp32 inner solve
                          (default 1e-4)                                         */
  int init;            /* LRC_INIT_*                                            */
  double median_tol;   /* relative residual of the median-parameter solve (the
                          accuracy eps_N of Sec. 3.1; default 1e-6 as in Sec. 5) */
  int verify_fp64;     /* 1: finish with the entry-wise fp64 residual           */
  int eager;           /* 1: launch every step directly instead of replaying the
                          captured HIP graphs of the iterations (same arithmetic) */
  double inner_trunc_tol; /* truncation tolerance of the fp32 steps (<= 0: for
                          LRC_MIXED_FP32 max(trunc_tol, 1e-2 * inner_tol), for
                          LRC_MIXED_FP32_DIR max(trunc_tol, 1e-6))                 */
  double res_ref;      /* reference norm of the residual tests (> 0), replacing
                          ||F||_F: stop at ||resid||_F <= res_tol * res_ref,
                          relres = ||resid||_F / res_ref, max_col_relres per
                          column against res_ref / sqrt(m); 0: ||F||_F and
                          ||F_j|| (the Newton driver passes ||b|| sqrt(m))    */
  int solver;          /* LRC_SOLVER_CHEBYSHEV (default) or LRC_SOLVER_GMREST   */
  int recurrence;      /* LRC_CHEB_DIRECTION (default) or LRC_CHEB_THREE_TERM   */
} lrc_opts;

typedef struct {
  int rank;              /* rank of the correction S (X = X0 + S)                */
  int rank_x0;           /* rank of the fixed initial term X0                    */
  int iters;             /* Chebyshev updates of the iterate (all stages)        */
  int prec_applies;      /* preconditioner applications (matrix solves)          */
  int refinements;       /* fp64 refinement steps (mixed precision)              */
  int median_iters;      /* iterations of the median-parameter solve             */
  double relres;         /* ||F - L(X)||_F / ||F||_F, fp64 entry-wise if verified */
  double relres_est;     /* same quantity from the last truncated residual       */
  double max_col_relres; /* max_j ||(F - L(X))_j|| / ||F_j|| (fp64 entry-wise)   */
  double seconds_setup;  /* factorisation of the preconditioner (host + upload)  */
  double seconds_solve;  /* lrc_solve wall time                                  */
  int info_flags;        /* bit 0: shifted Cholesky used; bit 1: breakdown; bit 2: eigen
                            not converged; bit 4: the median solve stopped above its
                            tolerance (its iterate kept as the guess, since it still
                            reduces the column's residual); bit 5: the median solve
                            failed (non-finite or no reduction) and the zero guess
                            was used instead                                       */
  int status;            /* this problem's outcome: LRC_OK or LRC_ENOTCONV       */
  int newton_steps;      /* Newton steps of the median problem (Algorithm 1 driver) */
  int median_fallback_cols; /* LRC_INIT_GIVEN_JUDGED: columns where the median guess
                            replaced the given one                                 */
} lrc_info;

/* Default options (rank cap 20, tol 1e-8, res_tol 1e-8, restart 6, fp64). */
void lrc_opts_default(lrc_opts* opts);

/* --------------------------------------------------------------- context
 * device: HIP device index.  stream: a hipStream_t borrowed from the caller
 * (NULL = the null stream); it must outlive the context. */
lrc_status lrc_create(lrc_ctx* ctx, int device, void* stream);
void lrc_destroy(lrc_ctx ctx);
const char* lrc_last_error(lrc_ctx ctx);
/* Replace the stream used by later calls (borrowed). */
lrc_status lrc_set_stream(lrc_ctx ctx, void* stream);

/* --------------------------------------------------------------- operators
 * q square operators K_i (n x n) in CSR: rowptr[i] (n+1, int64, starting at 0
 * and ending at nnz_i), col[i] (nnz_i, int32, ascending inside a row, in
 * [0, n)), val[i] (nnz_i doubles).  Copied to the device in fp64 and fp32.
 * Errors: LRC_EINVAL for malformed CSR or q outside [1, 8]. */
lrc_status lrc_ops_create(lrc_ctx ctx, int64_t n, int q, const int64_t* const* rowptr,
                          const int32_t* const* col, const double* const* val, lrc_ops* ops);
/* New values for operator i on the same pattern (a new linearisation point). */
lrc_status lrc_ops_update_values(lrc_ops ops, int i, const double* val);
void lrc_ops_destroy(lrc_ops ops);
/* W_i = K_i U for all i (device, row-major).  dtype 0: fp64, 1: fp32.
 * U: n x r with ld ldu; W: q blocks of n x r with ld ldw, block i at
 * W + i * n * ldw.  ldu, ldw multiples of 8, r <= min(ldu, ldw) <= 256; U and W
 * 16-byte aligned (LRC_EINVAL otherwise).  Columns of W past r are not written.
 * dtype | LRC_SPMM_SKIP_EMPTY: only the rows of W_i whose row of K_i holds
 * entries are computed and written (the others are left untouched: the caller
 * keeps them zero); this is the form the solver's own products use, since
 * K_1, K_2 of the paper's structure live on the solid part only. */
enum { LRC_SPMM_SKIP_EMPTY = 4 };
lrc_status lrc_ops_spmm_dev(lrc_ops ops, int dtype, int r, const void* U_dev, int ldu,
                            void* W_dev, int ldw);
/* SpMM autotuning for this operator set at width r (dtype 0/1): times every
 * candidate launch shape (columns per lane 1/2/4/8, 2/4/8 waves per
 * workgroup, grid caps 2048/8192/32768) on the device at widths r, r/2 and
 * r/4 (a launch planned for capacity r runs at the device rank, below it) and
 * caches the fastest in total in the context for (precision, n, q, nnz, r);
 * every later SpMM of that shape (solver steps included) uses it, and the
 * solver tunes on first use anyway.  cfg (may be NULL) receives {columns per
 * lane, waves, grid cap}; times_us (may be NULL) {best, default shape}: the
 * microseconds per launch summed over the timed widths.  Results do
 * not depend on the shape: each row is summed in the same order by one lane
 * group whatever the choice. */
lrc_status lrc_ops_spmm_tune(lrc_ops ops, int dtype, int r, int cfg[3], double times_us[2]);
/* lrc_ops_spmm_dev with an explicit launch shape cfg = {columns per lane (1, 2,
 * 4 or 8; 0 = default), waves per workgroup (1..8), grid cap (>= 1)};
 * LRC_EINVAL for a shape that cannot cover r (r / columns per lane > 64). */
lrc_status lrc_ops_spmm_shape_dev(lrc_ops ops, int dtype, int r, const void* U_dev, int ldu,
                                  void* W_dev, int ldw, const int cfg[3]);

/* --------------------------------------------------------------- problem
 * One subset: m parameter columns, the table d (q x m, column-major, i.e.
 * d[i + q*j] = diag(D_i)[j]) and F = FU diag(Fs) FV^T of rank rF
 * (FU: n x rF, FV: m x rF, column-major; Fs NULL means ones).
 * The operators must outlive the problem. */
lrc_status lrc_prob_create(lrc_ops ops, int64_t m, const double* d, int rF, const double* FU,
                           const double* Fs, const double* FV, lrc_prob* prob);
void lrc_prob_destroy(lrc_prob prob);
/* Factorise P = sum_i dbar_i K_i (dbar: q values, NULL = arithmetic means of the
 * rows of d), the centre preconditioner of Sec. 4.2.  kind LRC_PREC_LU: the
 * exact factorisation Sec. 5 uses (nested-dissection ordering + multifrontal
 * LU without pivoting on the host, inverted supernode blocks uploaded for the
 * level-scheduled GPU solves; leaf_size: nodes per nested-dissection leaf,
 * <= 0: the default, 64).  kind LRC_PREC_ILU0: the incomplete LU without
 * fill on P's pattern (for operators whose exact factors do not fit), applied
 * by one launch per level of its triangular solves; leaf_size is ignored.
 * lrc_prob_spectrum's interval holds for the exact kind only: with ILU(0)
 * give cheb_c / cheb_d or use LRC_SOLVER_GMREST.  LRC_ESINGULAR on a zero or
 * non-finite pivot. */
enum { LRC_PREC_LU = 0, LRC_PREC_ILU0 = 1 };
lrc_status lrc_prob_precondition(lrc_prob prob, const double* dbar, int leaf_size, int kind);
/* Interval [d - c, d + c] enclosing the preconditioned spectra: the smallest
 * interval holding 1 and every ratio d[i, j] / dbar_i (valid when K_0 + K_0^T
 * and K_1..K_{q-1} are positive semi-definite). */
lrc_status lrc_prob_spectrum(lrc_prob prob, double* c, double* d);
/* Statistics of the factorisation: out[0] supernodes, [1] forward levels,
 * [2] backward levels, [3] max front, [4] stored block entries,
 * [5] host ordering s, [6] host factor s, [7] upload s.  For ILU(0): [0]
 * rows, [1], [2] the levels of its two triangular solves, [3] 1, [4] stored
 * entries of L\U, [5], [6] 0, [7] upload s. */
lrc_status lrc_prob_precond_stats(lrc_prob prob, double out[8]);
/* Z = P^{-1} R on device columns (row-major n x k, k <= 64). dtype 0/1. */
lrc_status lrc_prob_prec_apply_dev(lrc_prob prob, int dtype, int k, const void* R_dev, int ldr,
                                   void* Z_dev, int ldz);

/* Solve.  init = LRC_INIT_GIVEN uses X0 = U0 diag(s0) V0^T (host, column-major,
 * rank r0; s0 NULL = ones) as the fixed initial term; LRC_INIT_MEDIAN solves the
 * upper-median parameter problem (Sec. 3.3) and uses X0 = x~ 1^T; the correction
 * S with L(S) = F - L(X0) is computed by ChebyshevT.  info may be NULL. */
lrc_status lrc_solve(lrc_prob prob, const lrc_opts* opts, int r0, const double* U0,
                     const double* s0, const double* V0, lrc_info* info);
/* lrc_solve with the initial term X0 = U0 diag(s0) V0^T given as device
 * factors (row-major fp64: U0 n x r0 with ld ldu, V0 m x r0 with ld ldv; s0
 * host, NULL = ones), e.g. a surrogate's prediction that never leaves the
 * GPU.  opts->init must be LRC_INIT_GIVEN and r0 in [1, 64]; the factors are
 * copied before the call returns. */
lrc_status lrc_solve_x0_dev(lrc_prob prob, const lrc_opts* opts, int r0, const double* U0_dev,
                            int ldu, const double* s0, const double* V0_dev, int ldv,
                            lrc_info* info);
/* Batched solve of K preconditioned problems of one context (Algorithm 1
 * treats the parameter subsets independently, so their Newton steps can run
 * together).  Same options and results as K calls of lrc_solve with
 * opts->init LRC_INIT_MEDIAN or LRC_INIT_ZERO (LRC_INIT_GIVEN is refused);
 * opts->restart must be in [1, 64] (as for lrc_solve): a restart cycle of the
 * ChebyshevT recurrence for all problems is captured once as two HIP graphs
 * (its two halves) and replayed until every problem has converged or
 * stopped, each step being one launch over all problems, with finished
 * problems skipped on the device; the host reads the problems' states after
 * the first half when their measured rates say that they all stop within it.  Problems
 * may differ in m, F, the operator values and the preconditioner; problems
 * whose factorisations share one supernode structure (same sparsity pattern)
 * share each preconditioner launch as well.  infos (K entries, may be NULL)
 * receives per-problem results, infos[k].status its outcome.  Returns the
 * worst per-problem status, or an error (nothing solved) for invalid input. */
lrc_status lrc_solve_batched(lrc_prob* probs, int K, const lrc_opts* opts, lrc_info* infos);
/* Solution X = [U0 | U] diag([s0, s]) [V0 | V]^T as host arrays (column-major):
 * pass NULL pointers to query *rank (total columns).  U: n x rank, V: m x rank. */
lrc_status lrc_get_solution(lrc_prob prob, int* rank, double* U, double* s, double* V);
/* Entry-wise fp64 residual of the current solution: ||F - L(X)||_F / ||F||_F and
 * per-column norms ||(F - L(X))_j|| (colres: m values, may be NULL). */
lrc_status lrc_residual(lrc_prob prob, double* relres, double* colres);

/* Truncation T_{R,eps}(A diag(c) B^T) of device factors (row-major fp64 or fp32:
 * dtype 0/1; dtype 2: fp32 factors whose first CholeskyQR pass runs on bf16
 * Gram products, as the fp32 steps of LRC_MIXED_BF16GRAM do): A n x k (ld
 * lda), B m x k (ld ldb), c (k host doubles).  Outputs:
 * U (n x rank, ld ldu), V (m x rank, ld ldv) device; s (host, rank values);
 * k <= 128, rank_cap <= 64.  CholeskyQR2 on both factors + fp64 SVD of the core. */
lrc_status lrc_truncate_dev(lrc_ctx ctx, int dtype, int64_t n, int64_t m, int k,
                            const void* A_dev, int lda, const double* c, const void* B_dev,
                            int ldb, int rank_cap, double tol, void* U_dev, int ldu,
                            double* s, void* V_dev, int ldv, int* rank);

/* Same truncation with B's last k - k1 columns row-scaled: the product is
 * A diag(c) [B1 | diag(w) B2]^T with B1 = B[:, :k1], B2 = B[:, k1:k], and A is
 * handled as the two blocks A[:, :k1], A[:, k1:].  This is the structure of
 * the factored residual's V side, [V_F | D_i V_S] (Sec. 3.4).  w_dev: m device
 * doubles.  0 <= k1 < k. */
lrc_status lrc_truncate_scaled_dev(lrc_ctx ctx, int dtype, int64_t n, int64_t m, int k, int k1,
                                   const void* A_dev, int lda, const double* c, const void* B_dev,
                                   int ldb, const double* w_dev, int rank_cap, double tol,
                                   void* U_dev, int ldu, double* s, void* V_dev, int ldv, int* rank);

/* lrc_truncate_dev without any allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, results and errors as
 * lrc_truncate_dev.  Its workspace is one fixed 64 MiB device array per GPU,
 * held until the process ends, instead of a per-call allocation: n + m <=
 * 32768 rows always fit (fp64 or fp32); a larger shape returns LRC_EINVAL
 * with the bytes it would need.  Every call on one GPU uses that same array
 * and leaves its contents behind (the call clears what must start at zero),
 * so calls that overlap on one GPU, from two streams or two threads, race:
 * the caller serialises them.  LRC_EINVAL while kernel timing
 * (lrc_profile_enable) is on, since timing allocates.  The call synchronises
 * its stream to return s and rank. */
lrc_status lrc_truncate_noalloc_dev(lrc_ctx ctx, int dtype, int64_t n, int64_t m, int k,
                                    const void* A_dev, int lda, const double* c,
                                    const void* B_dev, int ldb, int rank_cap, double tol,
                                    void* U_dev, int ldu, double* s, void* V_dev, int ldv,
                                    int* rank);

/* --------------------------------------------------------------- surrogate
 * Learned initial guess (not in the paper; the initial guess is the upper
 * median's solution, Sec. 3.3): a perceptron d0 -> d1 -> d2 -> d3 with exact
 * erf GELU after the two hidden layers, mapping parameters (mu, lambda) to
 * coefficients on a snapshot (POD) basis.  bf16 weights and activations, fp32
 * accumulation on MFMA, fp32 master weights and Adam.  Sizes: d0 <= 32,
 * d1, d2 in {32, 64}, d3 <= 32.  params: the d1 d0 + d1 + d2 d1 + d2 + d3 d2 +
 * d3 initial values packed as W1, b1, W2, b2, W3, b3 (W row-major, out x in).
 * Device arrays (row-major fp64): X (B x d0, raw parameters), T (B x d3, raw
 * coefficients), Y (B x d3).  The scaling starts as the identity (inputs taken
 * as already in [-1, 1], targets as already standardised); lrc_mlp_fit_scaling
 * sets it from data: inputs mapped affinely from their range onto [-1, 1],
 * targets standardised per column (mean, population deviation).  The loss is
 * the mean squared error over B x d3 standardised entries.  B <= 4096. */
typedef struct lrc_mlp_s* lrc_mlp;
lrc_status lrc_mlp_create(lrc_ctx ctx, const int sizes[4], const float* params, lrc_mlp* mlp);
void lrc_mlp_destroy(lrc_mlp mlp);
lrc_status lrc_mlp_fit_scaling(lrc_mlp mlp, int B, const double* X_dev, const double* T_dev);
/* One forward and backward pass without an update: *loss and the packed
 * gradients (host, same layout as params; either may be NULL). */
lrc_status lrc_mlp_grad(lrc_mlp mlp, int B, const double* X_dev, const double* T_dev, float* loss,
                        float* grads);
/* `steps` full-batch Adam steps (bias-corrected); loss_hist (host, steps
 * values, may be NULL) receives the loss before each step. */
lrc_status lrc_mlp_train(lrc_mlp mlp, int B, const double* X_dev, const double* T_dev, int steps,
                         float lr, float beta1, float beta2, float eps, float* loss_hist);
/* Y = network(X) in coefficient units (unstandardised). */
lrc_status lrc_mlp_predict(lrc_mlp mlp, int B, const double* X_dev, double* Y_dev);
/* Current fp32 master parameters (packed like params). */
lrc_status lrc_mlp_get_params(lrc_mlp mlp, float* params);

/* --------------------------------------------------------------- timing
 * Per-kernel-class timing with HIP events recorded on the stream each kernel
 * is launched on (process-wide, not thread-safe).  A class is a kernel family
 * and its arithmetic type ("spmm.f32", "gram.f64", ...; lrc_profile_class_name).
 * lrc_profile_enable(mode): 0 stops recording (the record is kept); 1 clears
 * the record and brackets every launch with two event records; 2 clears and,
 * in addition, copies the device-resident widths each launch reads (4-byte
 * device-to-device copies before the first event, so outside the bracket)
 * so that its algorithmic work can be totalled.  LRC_EINVAL for another mode.
 * lrc_profile_read synchronises the recorded events and fills, for classes
 * c < ncls (any array may be NULL): ms[c] summed kernel time, count[c]
 * launches, work[c] summed algorithmic work of the launches recorded in mode
 * 2 and unit[c] its unit (0 no model, 1 HBM bytes, 2 flops).  Returns the
 * number of classes. */
lrc_status lrc_profile_enable(int mode);
int lrc_profile_read(int ncls, double* ms, int* count, double* work, int* unit);
const char* lrc_profile_class_name(int c);

/* --------------------------------------------------------------- Algorithm 1
 * Linearisation callback.  stage 0 (Newton, Sec. 3.4): at the point x (n
 * values) write the values of the Jacobian's operators J_i(x) into val_out[i]
 * (nnz_i values on operator i's fixed pattern, prefilled with the current
 * values: leave untouched to keep them) and the factors of the Newton step's
 * right-hand side B_k(x) = BU BV^T (eq. rhs_matrix1): column j of B_k(x) is
 * the nonlinear residual b - g(x, p_j) of the subset's parameter column j.
 * stage 1 (fixed point, Sec. 5.3, eq. picard_matrix1): the operators of the
 * fixed-point linearisation at x and the right-hand side b 1^T of the
 * equation for X itself.  *rB in [1, 8] columns: BU is n x rB (column-major,
 * ld n), BV m_k x rB (column-major, ld m_k), where m_k is the subset's size
 * and its columns are those of d starting at the subset's offset.  *bnorm
 * receives ||b||_2, the load vector's norm, against which residuals are
 * reported relative (||residual_j|| / ||b||).  Returns 0, or non-zero to abort
 * the driver with LRC_ECALLBACK. */
typedef int (*lrc_linearize_fn)(void* user, int k, int stage, const double* x,
                                double* const* val_out, int* rB, double* BU, double* BV,
                                double* bnorm);

/* Algorithm 1 (Sec. 4.1).  Split the m parameter columns of d (q x m,
 * column-major) into K consecutive subsets (sizes: K values, NULL = eq.
 * clustering1 of Sec. 3.3: floor(m / K) each, the remainder on the last),
 * and for every subset k:
 *   1. Newton on the upper-median column (Sec. 3.3, 0-based offset
 *      floor(m_k / 2)) starting from x~^{k-1} (x_init, NULL = zero, for k = 0):
 *      at each iterate x the callback gives J(x) and B_k(x); the step
 *      A(x, p_med) dx = B_k(x) e_med is solved on the GPU (preconditioned
 *      vector Chebyshev to opts->median_tol relative) until
 *      ||B_k(x) e_med||_2 <= eps_newton (absolute, as Sec. 4.1), at most
 *      newton_max steps; the last callback's point is x~^k;
 *   2. the centre preconditioner is factorised for J(x~^k) (re-factorised
 *      whenever an iterate changes the operator values);
 *   3. picard = 0: one low-rank Newton step L(S) = B_k(x~^k) with
 *      X^k = x~^k 1^T + S (LRC_INIT_NEWTON); picard = 1: the fixed-point
 *      variant, X^k solves L_F(X) = b 1^T directly from zero with the stage-1
 *      operators (eq. picard_matrix1).
 * cb NULL: the operators are linear (J = K) and B_k(x) = f 1^T - L(x 1^T),
 * with f (n values) the load vector; f is ignored when cb is given.
 * kind: the preconditioner (LRC_PREC_LU or LRC_PREC_ILU0) of every subset.
 * Results: out[k] receives the subset's problem (owned by the caller, free
 * with lrc_prob_destroy; its solution is X^k); info[k] (may be NULL) its
 * statistics, relative to ||b|| sqrt(m_k); sizes_out (K values, may be NULL)
 * the subset sizes used.  Returns the worst per-subset status. */
lrc_status lrc_newton_subsets(lrc_ops ops, int64_t m, const double* d, int K,
                              const int64_t* sizes, const double* f, const double* x_init,
                              lrc_linearize_fn cb, void* user, double eps_newton,
                              int newton_max, int picard, int kind, const lrc_opts* opts,
                              lrc_prob* out, lrc_info* info, int64_t* sizes_out);

/* --------------------------------------------------------------- theta-scheme
 * Time stepping of one parameter subset (Sec. 4.3, eq. timedep_matrix1) for
 * the linear problem M X'(t) + L(X) = b(t) 1^T with the theta-scheme: step i
 * solves L_theta(X^i) = F_i with L_theta(X) = (1/dt) M X + theta L(X) (the
 * q-term solver on K'_0 = M/dt + theta K_0, K'_i = theta K_i, same table d)
 * and F_i = theta b^i 1^T + (1 - theta) b^{i-1} 1^T + (1/dt) M X^{i-1}
 * - (1 - theta) G, through lrc_solve with the median initial term, so that
 * X^i = x~^i 1^T + S^i.  history 0: G = L(X^{i-1}) exactly (rank q times the
 * iterate's); history 1: G = L(x~^{i-1} 1^T), rank <= q (the paper's
 * approximation of the previous step's residual term; equal for theta = 1).
 * M: n x n CSR (rowptr n + 1 int64, col int32 sorted, values), copied.
 * b: n x (steps + 1) column-major, b(t_0) .. b(t_steps).  X(t_0) = U0
 * diag(s0) V0^T (host column-major, rank r0 in [0, 64]; r0 = 0: zero).
 * theta in (0, 1], dt > 0, q <= 6.  The preconditioner of L_theta (centre
 * parameters) is factorised once.  out receives the last step's problem
 * (its solution is X^steps; free with lrc_prob_destroy); info (steps entries,
 * may be NULL) each step's statistics.  LRC_EINVAL when a step's F_i would
 * exceed rank 64 (lower rank_cap or use history 1).  Returns the worst
 * per-step status. */
lrc_status lrc_theta_scheme(lrc_ops ops, const int64_t* M_rowptr, const int32_t* M_col,
                            const double* M_val, int64_t m, const double* d, int steps,
                            const double* b, int r0, const double* U0, const double* s0,
                            const double* V0, double theta, double dt, int history,
                            const lrc_opts* opts, lrc_prob* out, lrc_info* info);

#ifdef __cplusplus
}
#endif

#endif /* LRCHEB_H */
