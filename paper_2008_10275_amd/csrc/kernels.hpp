// Launchers of the HIP kernels (gfx950).  All launches are asynchronous on the
// given stream.  Ranks / column counts that only the device knows are passed as
// device pointers (nullptr + a constant otherwise), so that the host never has
// to synchronise to size a launch: grids are sized by capacities.
#pragma once
#include "common.hpp"
#include "prof.hpp"

namespace lrc {

// Batched launches: `dev` holds one argument struct per item (blockIdx.z), and
// items whose `done` flag is set do nothing.  dev == nullptr: a single item
// with the by-value arguments.
template <class A>
struct Batched {
  const A* dev = nullptr;
  const int* done = nullptr;
  int n = 1;
};

// ----------------------------------------------------------------- sparse
// One CSR operator on the device (int32 row pointers and columns).
template <class T>
struct DevCsr {
  const int* rowptr;
  const int* col;
  const T* val;
  int64_t n;
  int64_t nnz;
  int maxrow;   // most entries in one row
  const int* rows;   // the rows that hold entries, ascending (nullptr: every row does)
  int64_t nrows;     // their number (n when rows is nullptr)
  // the same entries in a padded column-major layout over those nrows rows
  // (entry u of visited row x at u * nrows + x; padding: the row's first
  // column with value 0), ew entries per row; ew = 0: none (CSR only)
  const int* ecol;
  const T* eval;
  int ew;
};

constexpr int kMaxOps = 8;

// W_i = K_i * U for i < q  (U: n x r row-major with ld ldu; W_i rows of ld ldw).
// r is read from r_dev when non-null (else r_const); rcap bounds it.
template <class T>
void launch_spmm(const DevCsr<T>* ops, int q, const T* U, int ldu, const int* r_dev,
                 int r_const, int rcap, T* const* W, int ldw, int cpl, hipStream_t s);
template <class T>
struct SpmmArgs {
  DevCsr<T> op[kMaxOps];
  T* W[kMaxOps];
  const T* U;
  const int* r_dev;
  int r_const;
  int q;
  int ldu;
  int ldw;
  int wpad;   // 1: W's columns past the rank, up to 16 bytes, may be overwritten (zeros)
  int skip_empty;   // 1: only the operators' non-empty rows are visited and written
                    // (W's other rows are zero from the buffer's set-up and stay so)
};
template <class T>
struct SpmmLaunch {
  SpmmArgs<T> a;
  int cpl = 4;     // columns per lane (as requested)
  int nv = 1;      // 16-byte vectors per lane
  int lpr = 1;     // lanes per row
  int waves = 4;   // waves per workgroup
  int blocks = 1;
  int q = 1;
  bool wide = false;   // an operator's padded copy is wider than 9 entries
  Work work;
};
// Launch shape of the SpMM: columns per lane (0: the dtype's default), waves
// per workgroup, and the cap on the grid (rows beyond it are strided).
struct SpmmCfg {
  int cpl = 0;
  int waves = 4;
  int max_blocks = 8192;
};
template <class T>
// skip_empty: visit only the operators' non-empty rows (their row lists), for
// product buffers whose other rows are zero from their set-up
SpmmLaunch<T> make_spmm(const DevCsr<T>* ops, int q, const T* U, int ldu, const int* r_dev,
                        int r_const, int rcap, T* const* W, int ldw, SpmmCfg cfg,
                        bool skip_empty = false);
template <class T>
void enqueue_spmm(const SpmmLaunch<T>& l, Batched<SpmmArgs<T>> b, hipStream_t s);

// Level-scheduled supernodal triangular solves (data from nd_factor).
// Source of one staged front row.  Forward: R row `src` (or none when < 0)
// plus `na` contribution rows listed from asm_src[a0].  Backward: y row `src`
// when >= 0, else x row -src - 1 (a boundary row); na = 0.
struct GatherRow {
  int src;
  int na;
  int64_t a0;
};
struct LevelTasks {
  const int2* tasks;   // product: (supernode, first output row) per 16-row task
  int count;
  const int2* rows;    // (supernode, front row) per staged row
  int nrows;
  const GatherRow* grows;   // gather source of every staged row (in staging order)
  int nin_max;         // longest product input (ns forward, ns + nb backward)
  int direct;          // the products read their inputs at the source (no gather):
                       // every backward level, forward levels without contributions
  double blk;          // nonzero dense block entries the level's products read
  int64_t in_rows;     // staged rows the products read (per column)
  int64_t out_rows;    // rows the products write (per column)
  int ilu_off;         // ILU(0): the level's rows start here in the level row list
  int64_t ilu_nnz;     // ILU(0): entries of the level's rows in its triangle
  int64_t z_rows;      // backward: rows of the solution Z the products write
};

template <class T>
struct PrecDev {
  int64_t n;
  const int* perm;
  const int* j0;
  const int* ns;
  const int* nb;
  const int64_t* fw_off;
  const int64_t* bw_off;
  const int64_t* front_off;
  const int64_t* cb_off;
  const int64_t* asm_ptr;
  const int64_t* asm_src;
  const int64_t* bnd_off;
  const int* bnd;
  const T* fw;
  const T* bw;
  const int64_t* soff_fwd;   // staging row offset of each supernode in its forward level
  const int64_t* soff_bwd;   // ... in its backward level
  const int* leaf;           // 1: the supernode has no children, so no front reads
                             // its rows of the permuted solution x (backward)
  // kind 1 (ILU(0)): L\U on the pattern of P (values: the item's fw), the
  // diagonal positions and the rows of the levels (forward, backward)
  int kind;
  const int* irp;
  const int* icol;
  const int* idiag;
  const int* irows_f;
  const int* irows_b;
};

// Z = P^{-1} R  (R, Z: n x k row-major; k read from k_dev or k_const, <= kcap <= 64).
// ws_y, ws_x: n x ldw scratch; ws_cb: (contribution rows) x ldw scratch;
// ws_stage: (largest level's front rows) x ldw scratch.
template <class T>
void launch_prec_apply(const PrecDev<T>& P, const std::vector<LevelTasks>& fwd,
                       const std::vector<LevelTasks>& bwd, const T* R, int ldr, T* Z, int ldz,
                       const int* k_dev, int k_const, int kcap, T* ws_y, T* ws_x, T* ws_cb,
                       T* ws_stage, int ldw, hipStream_t s);
// The per-item operands of a batched apply: items share the supernode
// structure (and the level tasks) of `P` and bring their own factor values.
template <class T>
struct PrecItem {
  const T* fw;
  const T* bw;
  const T* R;
  int ldr;
  T* Z;
  int ldz;
  const int* k_dev;
  int k_const;
  T* y;
  T* x;
  T* cb;
  T* stage;
  // when set (exact-LU kind only), the solution rows go here in fp64 instead
  // of to Z: a solve computed in fp32 feeds an fp64 consumer without a copy
  double* Z64 = nullptr;
};
// kterms: the widths of every item the launch covers, for the work model
// (nullptr: the single item `it`)
template <class T>
void enqueue_prec_apply(const PrecDev<T>& P, const std::vector<LevelTasks>& fwd,
                        const std::vector<LevelTasks>& bwd, const PrecItem<T>& it,
                        Batched<PrecItem<T>> b, int kcap, int ldw, hipStream_t s,
                        const std::vector<WTerm>* kterms = nullptr);
// Host checks of one item's operands (capacity, 16-byte rows and alignment).
template <class T>
void check_prec_item(const PrecItem<T>& it, int kcap, int ldw);

// ----------------------------------------------------------------- dense tall-skinny
// Partial Gram products G = X^T X for up to two operands in one launch; the
// partials (one upper-triangular kcap x kcap block per workgroup, fp32 or fp64
// accumulation per `T`) are then reduced in fp64 into G (kcap x kcap, full).
template <class T>
struct GramJob {
  BlockView<T> X;
  int64_t rows;
  double* G;       // output kcap x kcap (row-major, symmetric fill)
  int* kout;       // optional: receives the total width
};
template <class T>
void launch_gram(const GramJob<T>* jobs, int njobs, int kcap, double* ws_partial,
                 size_t ws_bytes, int* info, hipStream_t s);
template <class T>
struct GramArgs {
  BlockView<T> X[2];
  int64_t rows[2];
  int nwg0;          // workgroups of job 0; the rest belong to job 1
  int nwg1;
  T* partial;        // one partial per workgroup
};
template <class T>
struct GramRedArgs {
  GramArgs<T> g;
  double* G0;
  double* G1;
  int kcap;
  int* k0;
  int* k1;
  int* info;
};
// Host-built arguments of one Gram launch pair (partials, reduction).
template <class T>
struct GramLaunch {
  GramArgs<T> g;
  GramRedArgs<T> r;
  int njobs = 1;
  int grid = 0;      // partial workgroups
  int kb = 0;        // host bound of the width (selects the tile class)
  bool sc1 = false;  // second operand row-scaled
  bool bf16 = false; // fp32 operands rounded to bf16 on load, bf16 MFMA, fp32 accumulation
  Work work;
};
template <class T>
GramLaunch<T> make_gram(const GramJob<T>* jobs, int njobs, int kcap, double* ws_partial,
                        size_t ws_bytes, int* info);
template <class T>
void enqueue_gram(const GramLaunch<T>& l, Batched<GramArgs<T>> bg, Batched<GramRedArgs<T>> br,
                  hipStream_t s);
size_t gram_workspace_bytes(int64_t rows_a, int64_t rows_b, int kcap, bool fp64);

// Y = X * M  with X a block view (rows x k), M (k x r) fp64 row-major with ld kcapM,
// Y (rows x r) row-major ld ldy.  k, r read from device.
template <class T>
struct TsmmJob {
  BlockView<T> X;
  int64_t rows;
  const double* M;
  int ldm;
  const int* r_dev;
  T* Y;
  int ldy;
};
template <class T>
void launch_tsmm(const TsmmJob<T>* jobs, int njobs, int kcap, int rcap, hipStream_t s);
template <class T>
struct TsmmArgs {
  TsmmJob<T> job[2];
  int nwg0, nwg1;
};
template <class T>
struct TsmmLaunch {
  TsmmArgs<T> a;
  int grid = 0;
  int kb = 0;        // host bound of the input width (selects the register class)
  int rb = 0;        // host bound of the output width
  bool sc1 = false;
  bool tri = false;  // M upper triangular: the products skip its zero blocks
  Work work;
};
template <class T>
TsmmLaunch<T> make_tsmm(const TsmmJob<T>* jobs, int njobs, int kcap, int rcap, bool tri = false);
template <class T>
void enqueue_tsmm(const TsmmLaunch<T>& l, Batched<TsmmArgs<T>> b, hipStream_t s);

// ----------------------------------------------------------------- small fp64 (one workgroup)
// State of one truncation on the device (all k x k blocks have ld = kcap).
struct TruncState {
  double* G[2];      // Gram matrices (A side, B side)
  double* R1[2];     // first-pass Cholesky factors (with column scaling)
  double* T1[2];     // R1^{-1}
  double* R2[2];     // second-pass factors
  double* R2i[2];    // R2^{-1}
  double* M;         // core
  double* H;         // Q of the pivoted QR of the core (k x kj)
  double* VM;        // Y: rotations of the one-sided Jacobi on R^T (kj x kj)
  double* W;         // R of the pivoted QR (kj x k, original column order), then U_M = Q Y
  double* VP;        // V_M: unit right singular vectors of the core (k x kj)
  double* XA;        // R2A^{-1} U_M(:, order)   (k x r, ld kcap)
  double* XB;        // R2B^{-1} V_M(:, order)
  int* order;        // singular directions by decreasing sigma
  double* lam;       // singular values of the core (kj values, Jacobi order)
  int* piv;          // pivot order of the QR (diagnostic)
  int* kj;           // numerical rank kept by the QR (Jacobi dimension)
  double* rot;       // rotation log (c, s) per round and pair
  int* rounds;       // number of logged rounds (-1: Y written by the Jacobi kernel)
  int* k;            // total width (A and B have the same column count)
  int* info;         // bit 0: shifted Cholesky, 1: breakdown, 2: Jacobi not converged, 3: capacity
};

struct CholArgs {
  TruncState st;
  int pass;
  int kcap;
  double eps;
  double shift0;     // diagonal shift of the first attempt (equilibrated Gram)
};
// Pivoted Householder QR of the core, stopped once the trailing block's
// Frobenius norm is below 1e-3 of the truncation's tail budget
// (max(tol ||M||_F, abs_tol)).
struct QrArgs {
  TruncState st;
  int kcap;
  double tol;
  double abs_tol;    // absolute tail budget of the truncation (0: none)
  double data_eps;   // relative precision of the truncated factors (fp32: 1e-7, fp64: 0):
                     // the QR also stops once the trailing block is below data_eps ||M||_F
};
struct JacArgs {
  TruncState st;
  int kcap;
  int max_rounds;
  double tol;        // truncation tolerance (unused by the rotations: they go to rounding level)
  double abs_tol;
};
struct RepArgs {
  TruncState st;
  int kcap;
};
struct SelArgs {
  TruncState st;
  int kcap;
  int rank_cap;
  double tol;
  double abs_tol;    // the tail may also reach this absolute Frobenius norm
  double* s_out;
  int* rank_out;
  double* norm_out;
};
// C = op(A) diag(mid) op(B)[:, colperm] diag(colscale), all k x k (or k x r
// output columns), fp64, ld kcap.
struct SmallGemm {
  const double* A;
  const double* B;
  double* C;
  const int* colperm;        // optional
  const double* colscale;    // optional (per output column)
  const int* ncols_dev;      // optional: output columns (default k)
  int transA, transB;
  int use_core;              // mid = core coefficients
  const int* rowperm;        // optional: output row i goes to row rowperm[i]
  const int* inner_dev;      // optional: contraction length (default k)
};
struct SmallGemmArgs {
  SmallGemm g[2];
  CoreView core;
  const int* k;
  int kcap;
  int njobs;
};

void enqueue_chol(const CholArgs& a, Batched<CholArgs> b, hipStream_t s);
void enqueue_qrcp(const QrArgs& a, Batched<QrArgs> b, hipStream_t s);
void enqueue_jacobi(const JacArgs& a, Batched<JacArgs> b, hipStream_t s);
void enqueue_replay(const RepArgs& a, Batched<RepArgs> b, hipStream_t s);
void enqueue_select(const SelArgs& a, Batched<SelArgs> b, hipStream_t s);
SmallGemmArgs make_small_gemm(const SmallGemm* jobs, int njobs, CoreView core, const int* k,
                              int kcap);
void enqueue_small_gemm(const SmallGemmArgs& a, Batched<SmallGemmArgs> b, hipStream_t s);
// the two products before the core SVD (R_A R_B, M) and the two after it
// (U_M = Q Y; XA / XB)
void make_core_gemms(const TruncState& st, const CoreView& core, int kcap, SmallGemmArgs* out);
void make_finish_gemms(const TruncState& st, int kcap, const int* rank_out, SmallGemmArgs* out);

// ----------------------------------------------------------------- batch control
// Convergence state of one item of a lockstep batch of ChebyshevT solves.
struct BCtl {
  const double* norm;   // the item's residual norm (device)
  double target;        // absolute residual target
  double best;          // best residual so far (stagnation test)
  double last;          // last residual read
  int iters;            // updates done
  int max_iter;
  int stall;            // consecutive checks without a 30% gain over `best`
  int stall_limit;
  int state;            // 0 running, 1 converged, 2 stopped (limit, stagnation, non-finite)
  int pad;
};
// After a residual: reads every running item's norm, counts the update when
// `after_update`, and sets done[j] once item j converged or must stop.
void launch_batch_check(BCtl* ctl, int* done, int nb, int after_update, hipStream_t s);

// ----------------------------------------------------------------- residual (fp64)
// Per-column squared norms of  R = A B^T  (A: n x K view, B: m x K view scaled by
// the core).  colsq: m doubles (output).
void launch_residual_fp64(const BlockView<double>& A, int64_t n, const BlockView<double>& B,
                          CoreView core, int64_t m, int kcap, double* colsq, double* ws,
                          size_t ws_bytes, hipStream_t s);
size_t residual_workspace_bytes(int64_t n, int64_t m);

// ----------------------------------------------------------------- vectors
template <class Tin, class Tout>
void launch_cast(const Tin* x, int ldx, Tout* y, int ldy, int64_t rows, const int* cols_dev,
                 int cols_const, int colcap, hipStream_t s);
// Lockstep single-column Chebyshev solves (the median-parameter systems).
// Vectors are column 0 of n x 8 row-major blocks.
struct MedItem {
  const double* f;      // n: right-hand side column
  const double* W;      // q blocks of n x 8: K_t x (block t at W + t * n * 8)
  const double* coef;   // q: the median parameter's diagonal entries d_t
  double* x;            // iterate
  double* dl;           // last step
  double* r;            // residual f - sum_t coef_t K_t x
  const double* z;      // preconditioned residual
  double* part;         // med_partials() partial sums of r^2
  float* r32;           // non-null: fp32 copy of r for an fp32 preconditioner solve,
  const float* z32;     // whose result z32 replaces z (both n x 8, column 0)
  int64_t n;
  int q;
};
struct MedCtl {
  double target;        // absolute residual target
  double c, dc;         // spectrum half-width and centre
  double rho, alpha, beta;
  double norm;          // last residual norm
  int iters, max_iter;
  int state;            // 0 running, 1 converged, 2 stopped
  int pad;
};
int med_partials();
void launch_med_update(const MedItem* items, const MedCtl* ctl, const int* done, int nb,
                       int64_t nmax, hipStream_t s);
void launch_med_resid(const MedItem* items, const int* done, int nb, hipStream_t s);
void launch_med_check(const MedItem* items, MedCtl* ctl, int* done, int nb, int after_update,
                      hipStream_t s);
void launch_fill(double* p, int64_t count, double v, hipStream_t s);
// One item of a batched factor copy with a precision change.
template <class Tin, class Tout>
struct CastItem {
  const Tin* U;
  const Tin* V;
  const double* s;
  const int* r;
  Tout* U2;
  Tout* V2;
  double* s2;
  int* r2;
  int ldu, ldv, ldu2, ldv2;
  int64_t n, m;
  int colcap;        // columns the destination holds
};
template <class Tin, class Tout>
void launch_cast_lr(const CastItem<Tin, Tout>* items, const int* done, int nb, int64_t rows_max,
                    int colcap, hipStream_t s);
void launch_copy_cols(const double* src, int lds, double* dst, int ldd, int64_t rows, int cols,
                      hipStream_t s);

}  // namespace lrc
