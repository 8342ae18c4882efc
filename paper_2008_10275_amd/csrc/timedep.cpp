// Theta-scheme time stepping over one parameter subset (lrc_theta_scheme).
//
// Linear stand-in of the time-dependent problem of Sec. 4.3: per column j,
// M x_j' + A_j x_j = b(t) with A_j = sum_i d[i, j] K_i.  Step i solves the
// matrix equation of eq. timedep_matrix1 with the generic q-term solver:
// L_theta(X) = (1/dt) M X + theta L(X), i.e. operators K'_0 = M/dt + theta K_0
// and K'_i = theta K_i on the same parameter table, and the right-hand side
//   F_i = theta b^i 1^T + (1 - theta) b^{i-1} 1^T + (1/dt) M X^{i-1}
//         - (1 - theta) G,
// G = L(X^{i-1}) (exact history) or L(x~^{i-1} 1^T) (rank <= q, the paper's
// approximation of the previous step's residual term).  Each step runs the
// median column's solve and the low-rank update like lrc_solve with the
// median initial term, X^i = x~^i 1^T + S^i.  The products with M and the K_i
// of the previous iterate's factors run on the GPU (fp64 SpMM); the
// preconditioner of L_theta is factorised once and kept for every step.
#include <algorithm>
#include <cmath>
#include <string>

#include "handles.hpp"

using namespace lrc;

namespace {

// a A + b B on the union pattern (both n x n host CSR, sorted columns)
CsrHost axpby(double a, const CsrHost& A, double b, const CsrHost& B) {
  CsrHost C;
  C.n = A.n;
  C.rowptr.assign(A.n + 1, 0);
  for (int64_t r = 0; r < A.n; ++r) {
    int64_t p = A.rowptr[r], pe = A.rowptr[r + 1], s = B.rowptr[r], se = B.rowptr[r + 1];
    while (p < pe || s < se) {
      const int32_t ca = p < pe ? A.col[p] : INT32_MAX, cb = s < se ? B.col[s] : INT32_MAX;
      const int32_t c = std::min(ca, cb);
      double v = 0.0;
      if (ca == c) v += a * A.val[p++];
      if (cb == c) v += b * B.val[s++];
      C.col.push_back(c);
      C.val.push_back(v);
    }
    C.rowptr[r + 1] = int64_t(C.col.size());
  }
  return C;
}

CsrHost scaled(double a, const CsrHost& A) {
  CsrHost C = A;
  for (double& v : C.val) v *= a;
  return C;
}

lrc_ops make_ops(lrc_ctx ctx, int64_t n, const std::vector<CsrHost>& K) {
  const int q = int(K.size());
  std::vector<const int64_t*> rp(q);
  std::vector<const int32_t*> cl(q);
  std::vector<const double*> vl(q);
  for (int i = 0; i < q; ++i) {
    rp[i] = K[i].rowptr.data();
    cl[i] = K[i].col.data();
    vl[i] = K[i].val.data();
  }
  lrc_ops o = nullptr;
  const lrc_status st = lrc_ops_create(ctx, n, q, rp.data(), cl.data(), vl.data(), &o);
  if (st != LRC_OK) throw Error(st, lrc_last_error(ctx));
  return o;
}

}  // namespace

extern "C" lrc_status lrc_theta_scheme(lrc_ops ops, const int64_t* M_rowptr, const int32_t* M_col,
                                       const double* M_val, int64_t m, const double* d, int steps,
                                       const double* b, int r0, const double* U0,
                                       const double* s0, const double* V0, double theta, double dt,
                                       int history, const lrc_opts* opts, lrc_prob* out,
                                       lrc_info* info) {
  if (!ops || !opts || !out || !d || !b || !M_rowptr) return LRC_EINVAL;
  Ops& base = ops->o;
  return guarded(base.ctx, [&]() -> lrc_status {
    const int q = base.q;
    const int64_t n = base.n;
    LRC_CHECK(steps >= 1 && m >= 1, ST_EINVAL, "theta_scheme: need steps >= 1 and m >= 1");
    LRC_CHECK(theta > 0.0 && theta <= 1.0 && dt > 0.0 && std::isfinite(dt), ST_EINVAL,
              "theta_scheme: need theta in (0, 1] and dt > 0");
    LRC_CHECK(history == 0 || history == 1, ST_EINVAL, "theta_scheme: history must be 0 or 1");
    LRC_CHECK(q + 2 <= kMaxOps, ST_EINVAL, "theta_scheme: at most 6 operators");
    LRC_CHECK(r0 >= 0 && r0 <= 64 && (r0 == 0 || (U0 && V0)), ST_EINVAL,
              "theta_scheme: initial value factors missing or rank outside [0, 64]");
    *out = nullptr;
    lrc_ctx_s* cx = static_cast<lrc_ctx_s*>(base.ctx->handle);
    CsrHost M;
    M.n = n;
    M.rowptr.assign(M_rowptr, M_rowptr + n + 1);
    LRC_CHECK(M.rowptr[0] == 0 && M.rowptr[n] >= 0, ST_EINVAL, "theta_scheme: bad mass rowptr");
    M.col.assign(M_col, M_col + M.rowptr[n]);
    M.val.assign(M_val, M_val + M.rowptr[n]);
    // operators of the step's equation and of its right-hand side
    std::vector<CsrHost> Kt, Kh;
    Kt.push_back(axpby(1.0 / dt, M, theta, base.host[0]));
    for (int i = 1; i < q; ++i) Kt.push_back(scaled(theta, base.host[i]));
    // history blocks: [M/dt - (1-theta) K_0, -(1-theta) K_1.., M/dt, -(1-theta) K_0]
    Kh.push_back(axpby(1.0 / dt, M, -(1.0 - theta), base.host[0]));
    for (int i = 1; i < q; ++i) Kh.push_back(scaled(-(1.0 - theta), base.host[i]));
    Kh.push_back(scaled(1.0 / dt, M));
    Kh.push_back(scaled(-(1.0 - theta), base.host[0]));
    std::unique_ptr<lrc_ops_s> ot(make_ops(cx, n, Kt)), oh(make_ops(cx, n, Kh));
    // the previous iterate X^{i-1} = XU diag(Xs) XV^T (host, column-major)
    int rX = r0;
    std::vector<double> XU(U0, U0 + size_t(n) * r0), XV(V0, V0 + size_t(m) * r0), Xs(r0, 1.0);
    if (s0) std::copy(s0, s0 + r0, Xs.begin());
    const int jmed = int(m / 2);
    std::vector<double> xt(n, 0.0);   // x~^{i-1}: the median column of X^0, then the median solve
    for (int a = 0; a < rX; ++a)
      for (int64_t r = 0; r < n; ++r) xt[r] += XU[size_t(a) * n + r] * Xs[a] * XV[size_t(a) * m + jmed];
    std::unique_ptr<lrc_prob_s> prev;
    lrc_status worst = LRC_OK;
    for (int it = 1; it <= steps; ++it) {
      // GPU products of the history operators with [XU | x~]
      const int w = rX + 1;
      std::vector<double> blk(size_t(n) * w);
      std::copy(XU.begin(), XU.end(), blk.begin());
      std::copy(xt.begin(), xt.end(), blk.begin() + size_t(n) * rX);
      std::vector<double> W;
      ops_apply_block(oh->o, blk, w, W);
      auto Wcol = [&](int op, int a) { return W.data() + (size_t(op) * w + a) * n; };
      // F_i factors
      std::vector<double> FU, FV, Fs;
      auto add = [&](const double* u, double sv, const double* v, double vscale_row_i) {
        FU.insert(FU.end(), u, u + n);
        Fs.push_back(sv);
        for (int64_t j = 0; j < m; ++j) {
          const double dj = vscale_row_i < 0 ? 1.0 : d[size_t(j) * q + int(vscale_row_i)];
          FV.push_back(v ? v[j] * dj : dj);
        }
      };
      std::vector<double> bb(n);
      for (int64_t r = 0; r < n; ++r)
        bb[r] = theta * b[size_t(it) * n + r] + (1.0 - theta) * b[size_t(it - 1) * n + r];
      add(bb.data(), 1.0, nullptr, -1);
      if (history == 0) {
        // (1/dt) M X - (1 - theta) L(X): q blocks of the previous factors
        for (int i = 0; i < (theta < 1.0 ? q : 1); ++i)
          for (int a = 0; a < rX; ++a)
            add(Wcol(i, a), Xs[a], XV.data() + size_t(a) * m, i == 0 ? -1 : i);
      } else {
        // (1/dt) M X exactly, -(1 - theta) L(x~ 1^T) of rank <= q
        for (int a = 0; a < rX; ++a) add(Wcol(q, a), Xs[a], XV.data() + size_t(a) * m, -1);
        if (theta < 1.0) {
          add(Wcol(q + 1, rX), 1.0, nullptr, -1);
          for (int i = 1; i < q; ++i) add(Wcol(i, rX), 1.0, nullptr, i);
        }
      }
      const int rF = int(Fs.size());
      LRC_CHECK(rF <= 64, ST_EINVAL,
                "theta_scheme: right-hand side rank " + std::to_string(rF) +
                    " exceeds 64 (lower rank_cap or use the median history)");
      lrc_prob tmp = nullptr;
      lrc_status st = lrc_prob_create(ot.get(), m, d, rF, FU.data(), Fs.data(), FV.data(), &tmp);
      if (st != LRC_OK) return st;
      std::unique_ptr<lrc_prob_s> pb(tmp);
      if (prev && prev->p.prec) {
        pb->p.prec = std::move(prev->p.prec);
        pb->p.seconds_setup = prev->p.seconds_setup;
      } else {
        st = lrc_prob_precondition(pb.get(), nullptr, 0, LRC_PREC_LU);
        if (st != LRC_OK) return st;
      }
      lrc_opts o = *opts;
      o.init = LRC_INIT_MEDIAN;
      lrc_info inf{};
      st = lrc_solve(pb.get(), &o, 0, nullptr, nullptr, nullptr, &inf);
      if (st < 0) return st;
      worst = std::max(worst, st);
      if (info) info[it - 1] = inf;
      // X^i on the host for the next step; x~^i from the median term
      int r = 0;
      st = lrc_get_solution(pb.get(), &r, nullptr, nullptr, nullptr);
      if (st != LRC_OK) return st;
      rX = r;
      XU.assign(size_t(n) * r, 0.0);
      XV.assign(size_t(m) * r, 0.0);
      Xs.assign(r, 0.0);
      if (r > 0) {
        st = lrc_get_solution(pb.get(), &r, XU.data(), Xs.data(), XV.data());
        if (st != LRC_OK) return st;
      }
      std::fill(xt.begin(), xt.end(), 0.0);
      const int nmed = inf.rank_x0 > 0 ? inf.rank_x0 : r;   // median term, else the median column
      for (int a = 0; a < nmed; ++a)
        for (int64_t i = 0; i < n; ++i)
          xt[i] += XU[size_t(a) * n + i] * Xs[a] * XV[size_t(a) * m + jmed];
      prev = std::move(pb);
    }
    prev->owned_ops = std::move(ot);
    *out = prev.release();
    return worst;
  });
}
