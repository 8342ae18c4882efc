// Launchers of the HIP kernels (gfx950).  All launches are asynchronous on the
// given stream.  Ranks / column counts that only the device knows are passed as
// device pointers (nullptr + a constant otherwise), so that the host never has
// to synchronise to size a launch: grids are sized by capacities.
#pragma once
#include "common.hpp"

namespace lrc {

// ----------------------------------------------------------------- sparse
// One CSR operator on the device (int32 row pointers and columns).
template <class T>
struct DevCsr {
  const int* rowptr;
  const int* col;
  const T* val;
  int64_t n;
  int64_t nnz;
};

constexpr int kMaxOps = 8;

// W_i = K_i * U for i < q  (U: n x r row-major with ld ldu; W_i rows of ld ldw).
// r is read from r_dev when non-null (else r_const); rcap bounds it.
template <class T>
void launch_spmm(const DevCsr<T>* ops, int q, const T* U, int ldu, const int* r_dev,
                 int r_const, int rcap, T* const* W, int ldw, int cpl, hipStream_t s);

// Level-scheduled supernodal triangular solves (data from nd_factor).
struct LevelTasks {
  const int2* tasks;   // product: (supernode, first output row) per workgroup (16 rows)
  int count;
  const int2* rows;    // gather: (supernode, front row) per staged row
  int nrows;
  double blk;          // dense block entries the level's products read
  int64_t in_rows;     // staged rows the products read (per column)
  int64_t out_rows;    // rows the products write (per column)
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
};

// Z = P^{-1} R  (R, Z: n x k row-major; k read from k_dev or k_const, <= kcap <= 64).
// ws_y, ws_x: n x ldw scratch; ws_cb: (contribution rows) x ldw scratch;
// ws_stage: (largest level's front rows) x ldw scratch.
template <class T>
void launch_prec_apply(const PrecDev<T>& P, const std::vector<LevelTasks>& fwd,
                       const std::vector<LevelTasks>& bwd, const T* R, int ldr, T* Z, int ldz,
                       const int* k_dev, int k_const, int kcap, T* ws_y, T* ws_x, T* ws_cb,
                       T* ws_stage, int ldw, hipStream_t s);

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

// ----------------------------------------------------------------- small fp64 (one workgroup)
// State of one truncation on the device (all k x k blocks have ld = kcap).
struct TruncState {
  double* G[2];      // Gram matrices (A side, B side)
  double* R1[2];     // first-pass Cholesky factors (with column scaling)
  double* T1[2];     // R1^{-1}
  double* R2[2];     // second-pass factors
  double* R2i[2];    // R2^{-1}
  double* M;         // core
  double* H;         // M^T M
  double* VM;        // eigenvectors Y of the preconditioned Gram R R^T (kj x kj)
  double* W;         // pivoted Cholesky factor R, then M V (columns ~ sigma_j u_j)
  double* VP;        // V = Pi R^T Y (k x kj, column norms sqrt(lambda_j))
  double* XA;        // R2A^{-1} U_M(:, :r)   (k x r, ld kcap)
  double* XB;        // R2B^{-1} V_M(:, :r)
  int* order;        // columns by decreasing sigma
  double* invsig;    // 1 / ||W_j|| in that order
  double* invnu;     // 1 / ||VP_j|| in that order
  double* lam;       // eigenvalues of R R^T from the Jacobi rounds (kj values)
  int* piv;          // pivot order of the Cholesky of M^T M
  int* kj;           // numerical rank found by that Cholesky (Jacobi dimension)
  double* rot;       // rotation log (c, s) per round and pair
  int* rounds;       // number of logged rounds
  int* k;            // total width (A and B have the same column count)
  int* info;         // bit 0: shifted Cholesky, 1: breakdown, 2: Jacobi not converged, 3: capacity
};

void launch_chol(TruncState st, int pass, int kcap, double eps_gram, hipStream_t s);
void launch_core_jacobi(TruncState st, CoreView core, int kcap, int max_rounds, double tol,
                        hipStream_t s);
void launch_jacobi_replay(TruncState st, int kcap, hipStream_t s);
void launch_trunc_finish(TruncState st, int kcap, int rank_cap, double tol, double* s_out,
                         int* rank_out, double* norm_out, hipStream_t s);

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
// out[j] = sum over rows of x[j]^2 per column, fp64 (rows x cols) -> host-visible buffer
void launch_sumsq(const double* x, int64_t n, double* out, hipStream_t s);
void launch_vec_resid(const double* f, double* const* W, const double* coef, int q, int64_t n,
                      double* r, hipStream_t s);
void launch_vec_cheb_update(double* x, double* dl, const double* z, int64_t n, double alpha,
                            double beta, hipStream_t s);
void launch_fill(double* p, int64_t count, double v, hipStream_t s);
void launch_copy_cols(const double* src, int lds, double* dst, int ldd, int64_t rows, int cols,
                      hipStream_t s);

}  // namespace lrc
