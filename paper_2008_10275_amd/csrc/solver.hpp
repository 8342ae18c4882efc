// Solver core: operators, preconditioner, truncation engine and the
// ChebyshevT iteration (host orchestration of the HIP kernels).
#pragma once
#include <array>
#include <chrono>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/lrcheb.h"
#include "host/ilu0.h"
#include "host/ndfact.h"
#include "kernels.hpp"

namespace lrc {

constexpr int kTruncCap = 128;   // max concatenated columns of a truncation
// Right-hand side and residual truncations drop directions whose total weight
// stays below this fraction of the absolute residual target: they cannot move
// the result by more than that.
constexpr double kResFloor = 1e-3;
constexpr int kPrecCols = 64;    // max right-hand sides per preconditioner apply

struct Ctx {
  void* handle = nullptr;        // the lrc_ctx that owns this context
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  double* pinned = nullptr;      // small host-visible readback buffer
  int* pinned_i = nullptr;
  // tuned SpMM launch shapes per (element size, n, q, nnz, width)
  std::map<std::array<int64_t, 5>, SpmmCfg> spmm_cache;
  void sync() { LRC_HIP(hipStreamSynchronize(stream)); }
};

struct Ops {
  Ctx* ctx = nullptr;
  int64_t n = 0;
  int q = 0;
  std::vector<CsrHost> host;
  std::vector<DevBuf> rowptr, col, val64, val32;
  std::vector<DevBuf> rowlist;   // per operator: its non-empty rows (empty when all are)
  // padded (ELL) copy of stencil-like operators: slot -> CSR entry (-1: padding)
  std::vector<std::vector<int64_t>> emap;
  std::vector<DevBuf> ecol, eval64, eval32;
  std::vector<DevCsr<double>> d64;
  std::vector<DevCsr<float>> d32;
  void upload_values(int i);
};

// factor of the preconditioner on the device: supernodal exact LU (kind 0)
// or ILU(0) on the pattern of P (kind 1)
struct Prec {
  int kind = 0;
  Ilu0 ilu;             // kind 1: host copy of the incomplete factor
  DevBuf irp, icol, idiag, irows_f, irows_b, ilu64, ilu32;
  SupernodalFactor F;   // host copy (blocks freed after upload)
  DevBuf perm, j0, ns, nb, fw_off, bw_off, front_off, cb_off, asm_ptr, asm_src, bnd_off, bnd, leaf;
  DevBuf fw64, bw64, fw32, bw32;
  DevBuf fwd_tasks, bwd_tasks, soff_fwd, soff_bwd, grows;
  std::vector<LevelTasks> fwd, bwd;
  int64_t stage_rows = 0;
  PrecDev<double> p64;
  PrecDev<float> p32;
  int64_t cb_rows = 0;
  double seconds_upload = 0.0;
  template <class T> const PrecDev<T>& dev() const;
};
template <> inline const PrecDev<double>& Prec::dev<double>() const { return p64; }
template <> inline const PrecDev<float>& Prec::dev<float>() const { return p32; }

// Low-rank factor U diag(s) V^T on the device, rank held on the device.
template <class T>
struct LR {
  int64_t n = 0, m = 0;
  int cap = 0, ld = 0;
  DevBuf U, V, s, rank;
  void alloc(int64_t n_, int64_t m_, int cap_, hipStream_t st);
  T* u() const { return U.as<T>(); }
  T* v() const { return V.as<T>(); }
  double* sv() const { return s.as<double>(); }
  int* r() const { return rank.as<int>(); }
};

// Host-built arguments of every launch of one truncation, in launch order.
template <class T>
struct TruncPlan {
  GramLaunch<T> g1;
  CholArgs c1;
  TsmmLaunch<T> t1;
  GramLaunch<T> g2;
  CholArgs c2;
  SmallGemmArgs core[2];
  QrArgs qr;
  JacArgs jac;
  RepArgs rep;
  SmallGemmArgs fin;
  SelArgs sel;
  SmallGemmArgs xab;
  TsmmLaunch<T> t2;
};
// Per-item device copies of a batch of plans, one array per launch.  All
// default (dev == nullptr): the single truncation of the plan itself.
template <class T>
struct TruncBatch {
  Batched<GramArgs<T>> g1, g2;
  Batched<GramRedArgs<T>> r1, r2;
  Batched<CholArgs> c1, c2;
  Batched<TsmmArgs<T>> t1, t2;
  Batched<SmallGemmArgs> core[2], fin, xab;
  Batched<QrArgs> qr;
  Batched<JacArgs> jac;
  Batched<RepArgs> rep;
  Batched<SelArgs> sel;
};
template <class T>
void enqueue_trunc(const TruncPlan<T>& p, const TruncBatch<T>& b, hipStream_t s);
// The launch shape of a batch: every grid covers the largest item.
template <class T>
TruncPlan<T> merge_plans(const std::vector<TruncPlan<T>>& v);
// Uploads the per-item arguments into `buf` (reallocated when too small) and
// returns the batch view with the given per-item done flags.
template <class T>
TruncBatch<T> upload_plans(const std::vector<TruncPlan<T>>& v, const int* done, DevBuf& buf,
                           hipStream_t s);

// Workspace + state of the truncation T_{R,eps}(A diag(c) B^T).
template <class T>
struct Truncator {
  int kcap = 0, ldq = 0, max_rounds = 0;
  int64_t nmax = 0, mmax = 0;
  DevBuf ws;                      // owned workspace (alloc); empty when bound
  double* arena = nullptr;        // k x k blocks (zeroed at set-up)
  int* ints_p = nullptr;          // integer state (zeroed at set-up)
  double* gws = nullptr;          // Gram partial sums
  T* qa = nullptr;                // first-pass factor of the A side (nmax x kcap)
  T* qb = nullptr;                // first-pass factor of the B side (mmax x kcap)
  size_t arena_bytes = 0, ints_bytes = 0, gram_bytes = 0;
  bool bf16 = false;              // first CholeskyQR pass on bf16 Gram products (fp32 only)
  TruncState st{};
  // owns a workspace for nmax_ x mmax_ rows (grow-only)
  void alloc(int64_t nmax_, int64_t mmax_, hipStream_t s);
  // uses `bytes` of caller memory at `mem` instead (nothing is allocated)
  void bind(void* mem, size_t bytes, int64_t nmax_, int64_t mmax_, hipStream_t s);
  void carve(void* base, int64_t nmax_, int64_t mmax_);
  // outputs may alias input blocks; s_out/rank_out/norm_out are device pointers
  void run(const BlockView<T>& A, int64_t n, const BlockView<T>& B, int64_t m,
           const CoreView& core, int rank_cap, double tol, T* Uout, int ldu, T* Vout, int ldv,
           double* s_out, int* rank_out, double* norm_out, hipStream_t s);
  TruncPlan<T> plan(const BlockView<T>& A, int64_t n, const BlockView<T>& B, int64_t m,
                    const CoreView& core, int rank_cap, double tol, T* Uout, int ldu, T* Vout,
                    int ldv, double* s_out, int* rank_out, double* norm_out,
                    double abs_tol = 0.0) const;
};

// Bytes of the workspace of a truncation with nmax + mmax rows.
template <class T>
size_t trunc_workspace_bytes(int64_t nmax, int64_t mmax);

struct Prob;

// State and workspace of one ChebyshevT solve in precision T of L(S) = B, and
// the launch arguments of its steps (the lockstep driver runs them).
template <class T>
struct Cheb {
  Prob* P = nullptr;
  int cap = 0;
  LR<T> S, D, R;
  DevBuf W, Z, py, px, pcb, pst, norm;
  Truncator<T> tr;
  void alloc(Prob* p, int cap_);
  // truncation tolerance of the steps; norms go to norm[0] residual,
  // norm[1] direction, norm[2] iterate, norm[3] refinement, norm[4] rhs
  double tol = 0.0;
  SpmmLaunch<T> spmm_plan(const T* U, int ldu, const int* r_dev) const;
  // rank_cap <= 0: the solve's cap
  // abs_tol: directions whose total weight stays below it are dropped as well
  // X: the iterate the residual is taken of (nullptr: S; the SpMM of X must
  // have written W)
  TruncPlan<T> resid_plan(const LR<T>& B, double* norm_dev, double tol, int rank_cap = 0,
                          double abs_tol = 0.0, const LR<T>* X = nullptr) const;
  TruncPlan<T> dstart_plan(double dc) const;
  TruncPlan<T> supd_plan() const;
  TruncPlan<T> dstep_plan(double alpha, double beta) const;
  // three-term update out = T(a X + b Y + g Z R_V^T) (Y == nullptr: no Y
  // term); out may be Y, whose factors the truncation has read before it
  // writes its result
  TruncPlan<T> upd3_plan(const LR<T>& X, double a, const LR<T>* Y, double b, double g,
                         const LR<T>& out) const;
  PrecItem<T> prec_item() const;
};

struct SolveRun;

struct Prob {
  Prob();
  ~Prob();
  Prob(const Prob&) = delete;
  Prob& operator=(const Prob&) = delete;
  Ops* ops = nullptr;
  Ctx* ctx = nullptr;
  int64_t m = 0;
  std::vector<double> d;          // q x m column-major
  DevBuf d_rows;                  // q rows of m doubles (row i = diag(D_i))
  int rF = 0;
  std::vector<double> FU, Fs, FV; // host copies (column-major)
  double fnorm = 0.0;             // ||F||_F
  std::vector<double> dbar;
  std::unique_ptr<Prec> prec;
  double seconds_setup = 0.0;
  // solution: X = X0 + S (fp64 factors)
  LR<double> X0, S;
  int rank_x0 = 0, rank_s = 0;
  // the last solve's residual convention: X0 is a linearisation point that
  // L(S) = F does not include (LRC_INIT_NEWTON), and the reference norm
  bool newton_point = false;
  double ref = 0.0;
  LR<double> F64;                  // F as a device LR (fp64)
  // workspaces kept between solves (reallocated only when a shape changes)
  std::unique_ptr<SolveRun> run;
  DevBuf res_w0, res_ws, res_colsq, res_tmp;   // fp64 residual scratch
  const double* drow(int i) const { return d_rows.as<double>() + size_t(i) * m; }
};

// Grow-only device buffer.
inline void ensure(DevBuf& b, size_t bytes) {
  if (b.bytes < bytes) b.alloc(bytes);
}
// Median-column solve workspace (column 0 of n x 8 blocks).
struct MedWork {
  DevBuf f, coef, x, dl, r, z, W, py, px, pcb, pst, part, r32, z32;
};

// SpMM autotuning (tune.cpp): time every candidate launch shape of the fused
// SpMM of `o` at width `rcap`; spmm_config returns the cached choice, tuning
// on the first request.
struct SpmmTuneResult {
  SpmmCfg best;
  double best_us = 0.0;
  double default_us = 0.0;
  int tried = 0;
};
template <class T>
SpmmTuneResult tune_spmm(const Ops& o, int rcap);
template <class T>
SpmmCfg spmm_config(const Ops& o, int rcap);

// helpers
void log_line(const char* phase, int it, double norm, double ref);   // LRC_LOG set: one JSON line
template <class Tin, class Tout>
void cast_lr(const LR<Tin>& a, LR<Tout>& b, hipStream_t s);
template <class T>
BlockView<T> view1(const T* p, int ld, const int* wdev, int wconst, const double* rowscale = nullptr);

double residual_fp64(Prob& P, const LR<double>& X0, int r0, const LR<double>& S, double* colres);
// ChebyshevT-preconditioned solve of the median column's system
// A(d[:, jmed]) x = rhs of a preconditioned problem to relative residual
// `tol` (the lockstep driver's median phase on one problem); returns the
// iterations and the MedCtl state (1 converged, 2 stopped).
int median_column_solve(Prob& P, const std::vector<double>& rhs, double tol, bool eager,
                        std::vector<double>& x, int* iters);
// Device fp64 SpMM W_i = K_i x of one vector (n x q, column-major on the host).
void ops_apply_vector(Ops& o, const std::vector<double>& x, std::vector<double>& W);
// Device fp64 SpMM of a host block X (n x w column-major, w <= 64): W holds the
// q products K_i X one after another, each n x w column-major.
void ops_apply_block(Ops& o, const std::vector<double>& X, int w, std::vector<double>& W);

// Initial term given as device factors (row-major fp64).
struct X0Dev {
  const double* U;
  int ldu;
  const double* V;
  int ldv;
};

lrc_status solve_problem(Prob& P, const lrc_opts& o, int r0, const double* U0, const double* s0,
                         const double* V0, lrc_info* info, const X0Dev* xd = nullptr);

// One solve split into set-up (spectrum bounds, workspaces, the median
// column's system), the iterative phases (run by `lockstep` for one or many
// problems: median solve, right-hand side B = F - L(X0), ChebyshevT with
// refinement) and the report.
struct SolveRun {
  Prob* P = nullptr;
  std::chrono::steady_clock::time_point t0;
  double c = 0.0, dc = 0.0;
  int cap = 0, inner_cap = 0, max_iter = 0, refine_max = 0;
  double target = 0.0, rhs_tol = 0.0, inner_trunc_tol = 0.0;
  double ref = 0.0;     // reference norm of the residual tests (||F||_F or opts.res_ref)
  // LRC_INIT_NEWTON: X0 is the linearisation point and B = F (not F - L(X0))
  bool newton_point = false;
  // LRC_INIT_GIVEN_JUDGED: the given guess, judged against the median's per column
  bool judged = false;
  LR<double> Xg;
  int rank_g = 0;
  lrc_info inf{};
  std::unique_ptr<Cheb<double>> c64;
  std::unique_ptr<Cheb<float>> c32;
  LR<double> B64, E64;
  LR<float> Bin;
  int flags = 0, iters = 0, papp = 0, refinements = 0;
  bool conv = false;
  MedWork med;          // median-column workspace
  DevBuf rhs_w0;        // K_i X0 for the right-hand side
  double last = 0.0;
  // median column (init LRC_INIT_MEDIAN): index, interval, right-hand side, coefficients
  int jmed = -1;
  double cm = 0.0, dm = 0.0, median_tol = 0.0;
  std::vector<double> fmed, coefmed;
  void prepare(Prob& P_, const lrc_opts& o, int r0, const double* U0, const double* s0,
               const double* V0, const X0Dev* xd = nullptr);
  // X0 = x 1^T from the median solve; state: 1 converged, 2 stopped (norm:
  // the final residual norm, fnorm: ||f_med||)
  void set_median_x0(const double* x, int iters, int state = 1, double norm = 0.0,
                     double fnorm = 1.0);
  // LRC_INIT_GIVEN_JUDGED: X0 from the given and the median guess column by column
  void judge_guess();
  TruncPlan<double> rhs_plan(const lrc_opts& o, double* const* W0) const;
  lrc_status finish(const lrc_opts& o, lrc_info* info);
  // mixed precision pieces
  void alloc_mixed();
  void accumulate_plan_inputs(hipStream_t s);
  TruncPlan<double> accumulate_plan(const lrc_opts& o) const;
};

// The iterative phases of prepared solves in lockstep: every step is one
// launch over all of them, finished problems are skipped on the device, and
// the iterations are replayed from captured HIP graphs (opts.eager: launched
// directly instead).  Runs on a stream of its own, synchronised with the
// problems' context stream at both ends.
void lockstep(std::vector<SolveRun*>& runs, const lrc_opts& o);

// GMREST on a prepared fp64 run whose right-hand side B64 is built: restarted
// truncated GMRES in place of the ChebyshevT recurrence (gmrest.cpp).
void gmrest_solve(SolveRun& run, const lrc_opts& o, hipStream_t s);

std::vector<lrc_status> solve_batched(const std::vector<Prob*>& probs, const lrc_opts& o,
                                      lrc_info* infos);

}  // namespace lrc
