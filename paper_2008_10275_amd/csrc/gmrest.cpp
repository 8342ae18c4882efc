// GMREST: restarted GMRES with truncation for L(S) = B, the paper's second
// low-rank solver next to ChebyshevT (Sec. 2.2 and Sec. 4.1; its algorithm is
// in the companion paper and not printed).  Reading: restarted GMRES(l) on the
// left-preconditioned operator Z -> P^-1 L(Z) (P on the left factor, Sec. 4.2)
// in the Frobenius inner product, every Krylov matrix kept in low-rank form
// and truncated after each operation:
//   R = T(B - L(S)), stop if ||R|| <= tau ||F||  (explicit, at every restart)
//   V_1 = T(P^-1 R) / beta
//   for j: W = T(P^-1 T(L(V_j))); modified Gram-Schmidt W = T(W - h_ij V_i);
//          h_{j+1,j} = ||W||; Givens rotations on H; V_{j+1} = W / h_{j+1,j}
//   S = T(S + y_j V_j) one term at a time.
// Every operator product, preconditioner solve, truncation and the Gram
// products behind the inner products run in the HIP kernels; the host keeps
// the (l + 1) x l Hessenberg matrix and reads one pair of small Gram matrices
// per inner product.
#include <cmath>
#include <vector>

#include "solver.hpp"

namespace lrc {
namespace {

template <class T>
void add_blk(BlockView<T>& v, const T* p, int ld, const int* wdev) {
  LRC_CHECK(v.nb < kMaxBlocks, ST_EINVAL, "gmrest: too many blocks");
  const int b = v.nb++;
  v.ptr[b] = p;
  v.ld[b] = ld;
  v.wdev[b] = wdev;
  v.wconst[b] = 0;
  v.rowscale[b] = nullptr;
  v.cap[b] = ld;
}
void add_cor(CoreView& c, const double* s, double coef, const int* wdev) {
  const int b = c.nb++;
  c.s[b] = s;
  c.coef[b] = coef;
  c.wdev[b] = wdev;
  c.wconst[b] = 0;
}

struct Gmrest {
  SolveRun& run;
  Prob& P;
  Cheb<double>& C;
  hipStream_t s;
  int64_t n, m;
  int q, cap, ld;
  double tol;
  std::vector<LR<double>> V;   // Krylov basis (unscaled; basis i is scale[i] * V[i])
  LR<double> LV, Wk;
  DevBuf G, gws, ints;
  size_t gws_bytes = 0;

  Gmrest(SolveRun& r, int restart, hipStream_t st)
      : run(r), P(*r.P), C(*r.c64), s(st) {
    n = P.ops->n;
    m = P.m;
    q = P.ops->q;
    cap = C.cap;
    ld = ld_for(cap);
    V.resize(restart + 1);
    for (auto& v : V) v.alloc(n, m, cap, s);
    LV.alloc(n, m, cap, s);
    Wk.alloc(n, m, cap, s);
    G.alloc(size_t(2) * kTruncCap * kTruncCap * 8);
    gws_bytes = gram_workspace_bytes(n, m, kTruncCap, true);
    gws.alloc(gws_bytes);
    ints.alloc(64);
    LRC_HIP(hipMemsetAsync(ints.p, 0, 64, s));
  }

  void trunc(const BlockView<double>& A, const BlockView<double>& B, const CoreView& c,
             LR<double>& out, int slot) {
    enqueue_trunc(C.tr.plan(A, n, B, m, c, cap, tol, out.u(), out.ld, out.v(), out.ld, out.sv(),
                            out.r(), C.norm.as<double>() + slot),
                  TruncBatch<double>(), s);
  }
  double read_norm(int slot) {
    double v = 0.0;
    LRC_HIP(hipMemcpyAsync(&v, C.norm.as<double>() + slot, 8, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipStreamSynchronize(s));
    return v;
  }
  // out = T(coef L(X))
  void apply_L(const LR<double>& X, double coef, LR<double>& out) {
    enqueue_spmm(C.spmm_plan(X.u(), X.ld, X.r()), Batched<SpmmArgs<double>>(), s);
    BlockView<double> A{}, B{};
    CoreView c{};
    for (int i = 0; i < q; ++i) {
      add_blk(A, C.W.as<double>() + size_t(i) * n * ld, ld, X.r());
      add_blk(B, X.v(), X.ld, X.r());
      B.rowscale[B.nb - 1] = P.drow(i);
      add_cor(c, X.sv(), coef, X.r());
    }
    trunc(A, B, c, out, 5);
  }
  // out = T(P^-1 X) (P on the left factor)
  void apply_prec(const LR<double>& X, LR<double>& out, int slot) {
    const PrecDev<double>& pd = P.prec->dev<double>();
    PrecItem<double> it{pd.fw, pd.bw, X.u(), X.ld, C.Z.as<double>(), ld, X.r(), 0,
                        C.py.as<double>(), C.px.as<double>(), C.pcb.as<double>(),
                        C.pst.as<double>()};
    enqueue_prec_apply(pd, P.prec->fwd, P.prec->bwd, it, Batched<PrecItem<double>>(), cap, ld, s);
    ++run.papp;
    BlockView<double> A{}, B{};
    CoreView c{};
    add_blk(A, C.Z.as<double>(), ld, X.r());
    add_blk(B, X.v(), X.ld, X.r());
    add_cor(c, X.sv(), 1.0, X.r());
    trunc(A, B, c, out, slot);
  }
  // <X, Y>_F from the Gram matrices of [X_U | Y_U] and [X_V | Y_V]
  double inner(const LR<double>& X, const LR<double>& Y) {
    BlockView<double> A{}, B{};
    add_blk(A, X.u(), X.ld, X.r());
    add_blk(A, Y.u(), Y.ld, Y.r());
    add_blk(B, X.v(), X.ld, X.r());
    add_blk(B, Y.v(), Y.ld, Y.r());
    double* Gu = G.as<double>();
    double* Gv = Gu + size_t(kTruncCap) * kTruncCap;
    GramJob<double> jobs[2] = {{A, n, Gu, nullptr}, {B, m, Gv, nullptr}};
    enqueue_gram(make_gram<double>(jobs, 2, kTruncCap, gws.as<double>(), gws_bytes,
                                   ints.as<int>()),
                 Batched<GramArgs<double>>(), Batched<GramRedArgs<double>>(), s);
    std::vector<double> g(size_t(2) * kTruncCap * kTruncCap), sx(64), sy(64);
    int rx = 0, ry = 0;
    LRC_HIP(hipMemcpyAsync(g.data(), G.p, g.size() * 8, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(&rx, X.r(), 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(&ry, Y.r(), 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(sx.data(), X.sv(), size_t(X.cap) * 8, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(sy.data(), Y.sv(), size_t(Y.cap) * 8, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipStreamSynchronize(s));
    const double* gu = g.data();
    const double* gv = gu + size_t(kTruncCap) * kTruncCap;
    double acc = 0.0;
    for (int a = 0; a < rx; ++a)
      for (int b = 0; b < ry; ++b) {
        const size_t e = size_t(a) * kTruncCap + rx + b;
        acc += sx[a] * sy[b] * gu[e] * gv[e];
      }
    return acc;
  }
  // out = T(a X + b Y) (out may be Y)
  void axpby(double a, const LR<double>& X, double b, const LR<double>& Y, LR<double>& out,
             int slot) {
    BlockView<double> A{}, B{};
    CoreView c{};
    add_blk(A, Y.u(), Y.ld, Y.r());
    add_blk(A, X.u(), X.ld, X.r());
    add_blk(B, Y.v(), Y.ld, Y.r());
    add_blk(B, X.v(), X.ld, X.r());
    add_cor(c, Y.sv(), b, Y.r());
    add_cor(c, X.sv(), a, X.r());
    trunc(A, B, c, out, slot);
  }

  void solve(const lrc_opts& o) {
    tol = o.trunc_tol;
    C.tol = tol;
    const int l = o.restart;
    const double target = run.target;
    const int max_iter = run.max_iter;
    LR<double>& S = C.S;
    LRC_HIP(hipMemsetAsync(S.rank.p, 0, 16, s));   // S = 0
    int iters = 0;
    run.conv = false;
    std::vector<double> H(size_t(l + 1) * l), g(l + 1), cs(l), sn(l), y, scale(l + 1);
    auto h = [&](int i, int j) -> double& { return H[size_t(i) * l + j]; };
    for (;;) {
      enqueue_spmm(C.spmm_plan(S.u(), S.ld, S.r()), Batched<SpmmArgs<double>>(), s);
      enqueue_trunc(C.resid_plan(run.B64, C.norm.as<double>(), tol, 0, kResFloor * target),
                    TruncBatch<double>(), s);
      const double nr = read_norm(0);
      run.last = nr;
      log_line("gmrest", iters, nr, run.ref);
      if (!std::isfinite(nr)) break;
      if (nr <= target) {
        run.conv = true;
        break;
      }
      if (iters >= max_iter) break;
      apply_prec(C.R, V[0], 6);
      const double beta = read_norm(6);
      if (!(beta > 0.0)) break;
      scale[0] = 1.0 / beta;
      const double cyc_tol = beta * target / nr;
      std::fill(H.begin(), H.end(), 0.0);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int kept = 0;
      for (int j = 0; j < l; ++j) {
        apply_L(V[j], scale[j], LV);
        apply_prec(LV, Wk, 7);
        for (int i = 0; i <= j; ++i) {
          h(i, j) = scale[i] * inner(V[i], Wk);
          axpby(-h(i, j) * scale[i], V[i], 1.0, Wk, Wk, 7);
        }
        const double hn = read_norm(7);
        h(j + 1, j) = hn;
        ++iters;
        for (int i = 0; i < j; ++i) {
          const double t = cs[i] * h(i, j) + sn[i] * h(i + 1, j);
          h(i + 1, j) = -sn[i] * h(i, j) + cs[i] * h(i + 1, j);
          h(i, j) = t;
        }
        const double rho = std::hypot(h(j, j), h(j + 1, j));
        cs[j] = rho > 0 ? h(j, j) / rho : 1.0;
        sn[j] = rho > 0 ? h(j + 1, j) / rho : 0.0;
        h(j, j) = rho;
        h(j + 1, j) = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        kept = j + 1;
        const double est = std::fabs(g[j + 1]);
        if (est <= cyc_tol || !(hn > 0.0) || iters >= max_iter || j == l - 1) break;
        std::swap(V[j + 1], Wk);
        scale[j + 1] = 1.0 / hn;
      }
      // back substitution of the triangular least-squares problem
      y.assign(kept, 0.0);
      for (int i = kept - 1; i >= 0; --i) {
        double acc = g[i];
        for (int k = i + 1; k < kept; ++k) acc -= h(i, k) * y[k];
        y[i] = h(i, i) != 0.0 ? acc / h(i, i) : 0.0;
      }
      for (int j = 0; j < kept; ++j) axpby(y[j] * scale[j], V[j], 1.0, S, S, 2);
    }
    run.iters = iters;
  }
};

}  // namespace

void gmrest_solve(SolveRun& run, const lrc_opts& o, hipStream_t s) {
  LRC_CHECK(run.c64 != nullptr, ST_EINVAL, "gmrest: solve not prepared");
  Gmrest g(run, o.restart, s);
  g.solve(o);
}

}  // namespace lrc
