// Host orchestration of the low-rank ChebyshevT solve (see solver.hpp).
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>

namespace lrc {

using clk = std::chrono::steady_clock;
static double secs_since(clk::time_point a) {
  return std::chrono::duration<double>(clk::now() - a).count();
}

// One JSON line per residual check on stderr when LRC_LOG is set.
static bool log_enabled() {
  static const bool on = std::getenv("LRC_LOG") != nullptr;
  return on;
}
void log_line(const char* phase, int it, double norm, double ref) {
  if (!log_enabled()) return;
  std::fprintf(stderr, "{\"phase\": \"%s\", \"iter\": %d, \"norm\": %.6e, \"rel\": %.6e}\n",
               phase, it, norm, ref > 0 ? norm / ref : 0.0);
}

// ------------------------------------------------------------------ Ops
void Ops::upload_values(int i) {
  const auto& h = host[i];
  std::vector<float> v32(h.val.begin(), h.val.end());
  hipStream_t s = ctx->stream;
  LRC_HIP(hipMemcpyAsync(val64[i].p, h.val.data(), h.val.size() * 8, hipMemcpyHostToDevice, s));
  LRC_HIP(hipMemcpyAsync(val32[i].p, v32.data(), v32.size() * 4, hipMemcpyHostToDevice, s));
  if (size_t(i) < emap.size() && !emap[i].empty()) {
    const auto& mp = emap[i];
    std::vector<double> e64(mp.size());
    std::vector<float> e32(mp.size());
    for (size_t e = 0; e < mp.size(); ++e) {
      e64[e] = mp[e] >= 0 ? h.val[size_t(mp[e])] : 0.0;
      e32[e] = float(e64[e]);
    }
    LRC_HIP(hipMemcpyAsync(eval64[i].p, e64.data(), e64.size() * 8, hipMemcpyHostToDevice, s));
    LRC_HIP(hipMemcpyAsync(eval32[i].p, e32.data(), e32.size() * 4, hipMemcpyHostToDevice, s));
    LRC_HIP(hipStreamSynchronize(s));   // e64, e32 are temporaries
  }
  LRC_HIP(hipStreamSynchronize(s));   // v32 is a temporary
}

// ------------------------------------------------------------------ LR
template <class T>
void LR<T>::alloc(int64_t n_, int64_t m_, int cap_, hipStream_t st) {
  n = n_;
  m = m_;
  cap = std::max(cap_, 1);
  ld = ld_for(cap);
  U.alloc(size_t(std::max<int64_t>(n, 1)) * ld * sizeof(T));
  V.alloc(size_t(std::max<int64_t>(m, 1)) * ld * sizeof(T));
  s.alloc(size_t(std::max(cap, 8)) * sizeof(double));
  rank.alloc(16);
  LRC_HIP(hipMemsetAsync(rank.p, 0, 16, st));
  LRC_HIP(hipMemsetAsync(s.p, 0, s.bytes, st));
}
template struct LR<double>;
template struct LR<float>;

template <class T>
BlockView<T> view1(const T* p, int ld, const int* wdev, int wconst, const double* rowscale) {
  BlockView<T> v{};
  v.nb = 1;
  v.ptr[0] = p;
  v.ld[0] = ld;
  v.wdev[0] = wdev;
  v.wconst[0] = wconst;
  v.rowscale[0] = rowscale;
  v.cap[0] = wdev ? ld : wconst;
  return v;
}
template BlockView<double> view1(const double*, int, const int*, int, const double*);
template BlockView<float> view1(const float*, int, const int*, int, const double*);

template <class T>
static void add_block(BlockView<T>& v, const T* p, int ld, const int* wdev, int wconst,
                      const double* rowscale = nullptr) {
  LRC_CHECK(v.nb < kMaxBlocks, ST_EINVAL, "too many factor blocks (increase kMaxBlocks)");
  const int b = v.nb++;
  v.ptr[b] = p;
  v.ld[b] = ld;
  v.wdev[b] = wdev;
  v.wconst[b] = wconst;
  v.rowscale[b] = rowscale;
  v.cap[b] = wdev ? ld : wconst;
}

static void add_core(CoreView& c, const double* s, double coef, const int* wdev, int wconst) {
  LRC_CHECK(c.nb < kMaxBlocks, ST_EINVAL, "too many core blocks");
  const int b = c.nb++;
  c.s[b] = s;
  c.coef[b] = coef;
  c.wdev[b] = wdev;
  c.wconst[b] = wconst;
}

// ------------------------------------------------------------------ Truncator
// Workspace of a truncation with row capacities nmax (A side) and mmax (B
// side): the k x k arena, the Jacobi rotation log, the integer state, the Gram
// partial sums and the first-pass factors Q1A, Q1B.  Offsets are 256-byte
// aligned inside one block.
struct TruncLayout {
  size_t arena, rot, ints, gram, qa, qb, total;
};
template <class T>
static TruncLayout trunc_layout(int64_t nmax, int64_t mmax) {
  auto al = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t kk = size_t(kTruncCap) * kTruncCap;
  const int rounds = 30 * (kTruncCap - 1);
  TruncLayout l{};
  size_t off = 0;
  // arena of the k x k blocks: 10 per-side blocks + M, H, VM, W, VP, XA, XB + lam
  l.arena = off; off += al((17 * kk + size_t(kTruncCap)) * sizeof(double));
  l.rot = off;   off += al(size_t(rounds) * 64 * 2 * sizeof(double));
  l.ints = off;  off += al((2 * kTruncCap + 16) * sizeof(int));
  l.gram = off;  off += al(gram_workspace_bytes(nmax, mmax, kTruncCap, sizeof(T) == 8));
  l.qa = off;    off += al(size_t(std::max<int64_t>(nmax, 1)) * kTruncCap * sizeof(T));
  l.qb = off;    off += al(size_t(std::max<int64_t>(mmax, 1)) * kTruncCap * sizeof(T));
  l.total = off;
  return l;
}
template <class T>
size_t trunc_workspace_bytes(int64_t nmax, int64_t mmax) {
  return trunc_layout<T>(nmax, mmax).total;
}
template size_t trunc_workspace_bytes<double>(int64_t, int64_t);
template size_t trunc_workspace_bytes<float>(int64_t, int64_t);

template <class T>
void Truncator<T>::carve(void* base, int64_t nmax_, int64_t mmax_) {
  nmax = nmax_;
  mmax = mmax_;
  kcap = kTruncCap;
  ldq = kTruncCap;
  max_rounds = 30 * (kcap - 1);
  const TruncLayout l = trunc_layout<T>(nmax, mmax);
  unsigned char* b0 = static_cast<unsigned char*>(base);
  const size_t kk = size_t(kcap) * kcap;
  double* b = reinterpret_cast<double*>(b0 + l.arena);
  arena = b;
  arena_bytes = l.rot - l.arena;
  for (int x = 0; x < 2; ++x) {
    st.G[x] = b; b += kk;
    st.R1[x] = b; b += kk;
    st.T1[x] = b; b += kk;
    st.R2[x] = b; b += kk;
    st.R2i[x] = b; b += kk;
  }
  st.M = b; b += kk;
  st.H = b; b += kk;
  st.VM = b; b += kk;
  st.W = b; b += kk;
  st.VP = b; b += kk;
  st.XA = b; b += kk;
  st.XB = b; b += kk;
  st.lam = b; b += kcap;
  st.rot = reinterpret_cast<double*>(b0 + l.rot);
  int* ib = reinterpret_cast<int*>(b0 + l.ints);
  ints_p = ib;
  ints_bytes = l.gram - l.ints;
  st.order = ib;
  st.piv = ib + kcap;
  st.rounds = ib + 2 * kcap;
  st.k = ib + 2 * kcap + 1;
  st.info = ib + 2 * kcap + 2;
  st.kj = ib + 2 * kcap + 3;
  gws = reinterpret_cast<double*>(b0 + l.gram);
  gram_bytes = l.qa - l.gram;
  qa = reinterpret_cast<T*>(b0 + l.qa);
  qb = reinterpret_cast<T*>(b0 + l.qb);
}

template <class T>
void Truncator<T>::alloc(int64_t nmax_, int64_t mmax_, hipStream_t s) {
  if (nmax_ <= nmax && mmax_ <= mmax && ws.p) return;
  const int64_t nn = std::max(nmax, nmax_), mm = std::max(mmax, mmax_);
  ws.alloc(trunc_workspace_bytes<T>(nn, mm));
  carve(ws.p, nn, mm);
  LRC_HIP(hipMemsetAsync(arena, 0, arena_bytes, s));
  LRC_HIP(hipMemsetAsync(ints_p, 0, ints_bytes, s));
}

template <class T>
void Truncator<T>::bind(void* mem, size_t bytes, int64_t nmax_, int64_t mmax_, hipStream_t s) {
  LRC_CHECK(trunc_workspace_bytes<T>(nmax_, mmax_) <= bytes, ST_EINVAL,
            "truncation: bound workspace too small");
  carve(mem, nmax_, mmax_);
  // cleared with a kernel (not a memset node), so the call stays capturable
  launch_fill(arena, int64_t(arena_bytes / 8), 0.0, s);
  launch_fill(reinterpret_cast<double*>(ints_p), int64_t(ints_bytes / 8), 0.0, s);
}

template <class T>
TruncPlan<T> Truncator<T>::plan(const BlockView<T>& A, int64_t n, const BlockView<T>& B,
                                int64_t m, const CoreView& core, int rank_cap, double tol,
                                T* Uout, int ldu, T* Vout, int ldv, double* s_out, int* rank_out,
                                double* norm_out, double abs_tol) const {
  LRC_CHECK(n <= nmax && m <= mmax, ST_EINVAL, "truncation workspace too small");
  LRC_CHECK(rank_cap >= 1 && rank_cap <= 64 && rank_cap <= ldu && rank_cap <= ldv, ST_EINVAL,
            "truncation: rank cap must be in [1, 64] and fit the output leading dimensions");
  const double eps = sizeof(T) == 8 ? 1e-14 : 1e-6;
  TruncPlan<T> p;
  GramJob<T> g1[2] = {{A, n, st.G[0], st.k}, {B, m, st.G[1], nullptr}};
  p.g1 = make_gram<T>(g1, 2, kcap, gws, gram_bytes, st.info);
  // bf16 first pass (fp32 operands only): the Gram carries relative errors of
  // a few 2^-9 per entry, so its Cholesky starts from a preset shift of 1e-2
  // (on the unit diagonal) and takes the pivot threshold of bf16 rounding;
  // the fp32 second pass restores orthogonality
  const bool b16 = bf16 && sizeof(T) == 4;
  p.g1.bf16 = b16;
  p.c1 = CholArgs{st, 1, kcap, b16 ? 4e-3 : eps, b16 ? 1e-2 : 0.0};
  TsmmJob<T> t1[2] = {{A, n, st.T1[0], kcap, st.k, qa, ldq}, {B, m, st.T1[1], kcap, st.k, qb, ldq}};
  // the first pass writes st.k <= min(kcap, width bound) columns
  // (T1 = D R1^{-1} is upper triangular)
  p.t1 = make_tsmm<T>(t1, 2, kcap, std::min(kcap, std::max(view_cap(A), view_cap(B))), true);
  BlockView<T> va = view1<T>(qa, ldq, st.k, 0), vb = view1<T>(qb, ldq, st.k, 0);
  va.cap[0] = vb.cap[0] = std::min(kcap, std::max(view_cap(A), view_cap(B)));
  GramJob<T> g2[2] = {{va, n, st.G[0], nullptr}, {vb, m, st.G[1], nullptr}};
  p.g2 = make_gram<T>(g2, 2, kcap, gws, gram_bytes, st.info);
  p.c2 = CholArgs{st, 2, kcap, eps, 0.0};
  make_core_gemms(st, core, kcap, p.core);
  p.qr = QrArgs{st, kcap, tol, abs_tol, sizeof(T) == 4 ? 1e-7 : 0.0};
  p.jac = JacArgs{st, kcap, max_rounds, tol, abs_tol};
  p.rep = RepArgs{st, kcap};
  SmallGemmArgs fin[2];
  make_finish_gemms(st, kcap, rank_out, fin);
  p.fin = fin[0];
  p.xab = fin[1];
  p.sel = SelArgs{st, kcap, rank_cap, tol, abs_tol, s_out, rank_out, norm_out};
  TsmmJob<T> t2[2] = {{va, n, st.XA, kcap, rank_out, Uout, ldu},
                      {vb, m, st.XB, kcap, rank_out, Vout, ldv}};
  p.t2 = make_tsmm<T>(t2, 2, kcap, rank_cap);
  return p;
}

template <class T>
void enqueue_trunc(const TruncPlan<T>& p, const TruncBatch<T>& b, hipStream_t s) {
  enqueue_gram(p.g1, b.g1, b.r1, s);
  enqueue_chol(p.c1, b.c1, s);
  enqueue_tsmm(p.t1, b.t1, s);
  enqueue_gram(p.g2, b.g2, b.r2, s);
  enqueue_chol(p.c2, b.c2, s);
  for (int i = 0; i < 2; ++i) enqueue_small_gemm(p.core[i], b.core[i], s);
  enqueue_qrcp(p.qr, b.qr, s);
  enqueue_jacobi(p.jac, b.jac, s);
  enqueue_replay(p.rep, b.rep, s);
  enqueue_small_gemm(p.fin, b.fin, s);
  enqueue_select(p.sel, b.sel, s);
  enqueue_small_gemm(p.xab, b.xab, s);
  enqueue_tsmm(p.t2, b.t2, s);
  // diagnostics (eager launches only): width, Jacobi dimension and rounds of
  // the first item's truncation, one JSON line each on stderr
  static const bool stats = std::getenv("LRC_TRUNC_STATS") != nullptr;
  if (stats) {
    int h[3] = {0, 0, 0};
    LRC_HIP(hipMemcpyAsync(&h[0], p.jac.st.k, 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(&h[1], p.jac.st.kj, 8, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipStreamSynchronize(s));
    std::fprintf(stderr, "{\"tstat\": [%d, %d, %d, %d]}\n", int(sizeof(T)), h[0], h[1], h[2]);
  }
}

template <class T>
static void merge_gram(GramLaunch<T>& a, const GramLaunch<T>& b) {
  LRC_CHECK(a.sc1 == b.sc1 && a.njobs == b.njobs, ST_EINVAL,
            "batched truncation: items differ in operand structure");
  a.grid = std::max(a.grid, b.grid);
  a.kb = std::max(a.kb, b.kb);
}
template <class T>
static void merge_tsmm(TsmmLaunch<T>& a, const TsmmLaunch<T>& b) {
  LRC_CHECK(a.sc1 == b.sc1 && a.tri == b.tri, ST_EINVAL,
            "batched truncation: items differ in operand structure");
  a.grid = std::max(a.grid, b.grid);
  a.kb = std::max(a.kb, b.kb);
  a.rb = std::max(a.rb, b.rb);
}

template <class T>
TruncPlan<T> merge_plans(const std::vector<TruncPlan<T>>& v) {
  LRC_CHECK(!v.empty(), ST_EINVAL, "batched truncation: no items");
  TruncPlan<T> p = v[0];
  std::vector<Work> w1, w2, w3, w4;
  for (const auto& x : v) {
    w1.push_back(x.g1.work);
    w2.push_back(x.g2.work);
    w3.push_back(x.t1.work);
    w4.push_back(x.t2.work);
  }
  p.g1.work = combine_work(w1);
  p.g2.work = combine_work(w2);
  p.t1.work = combine_work(w3);
  p.t2.work = combine_work(w4);
  for (size_t i = 1; i < v.size(); ++i) {
    merge_gram(p.g1, v[i].g1);
    merge_gram(p.g2, v[i].g2);
    merge_tsmm(p.t1, v[i].t1);
    merge_tsmm(p.t2, v[i].t2);
    for (int j = 0; j < 2; ++j)
      LRC_CHECK(p.core[j].njobs == v[i].core[j].njobs, ST_EINVAL, "batched truncation: jobs differ");
  }
  return p;
}

// Appends one launch's per-item arguments (256-byte aligned) to the host image
// of the argument buffer whose device base is `base`.
template <class A, class Get>
static Batched<A> put(std::vector<unsigned char>& h, size_t& off, size_t nb, const int* done,
                      const char* base, Get get) {
  off = (off + 255) / 256 * 256;
  const size_t at = off;
  off += nb * sizeof(A);
  if (h.size() < off) h.resize(off);
  for (size_t i = 0; i < nb; ++i) {
    const A& a = get(i);
    std::memcpy(h.data() + at + i * sizeof(A), &a, sizeof(A));
  }
  Batched<A> b;
  b.dev = reinterpret_cast<const A*>(base + at);
  b.done = done;
  b.n = int(nb);
  return b;
}

template <class T>
TruncBatch<T> upload_plans(const std::vector<TruncPlan<T>>& v, const int* done, DevBuf& buf,
                           hipStream_t s) {
  const size_t nb = v.size();
  const size_t per = sizeof(GramArgs<T>) * 2 + sizeof(GramRedArgs<T>) * 2 + sizeof(CholArgs) * 2 +
                     sizeof(TsmmArgs<T>) * 2 + sizeof(SmallGemmArgs) * 4 + sizeof(QrArgs) +
                     sizeof(JacArgs) + sizeof(RepArgs) + sizeof(SelArgs);
  const size_t need = nb * per + 20 * 256;
  if (buf.bytes < need) buf.alloc(need);
  const char* base = reinterpret_cast<const char*>(buf.p);
  std::vector<unsigned char> h;
  size_t off = 0;
  TruncBatch<T> b;
#define LRC_PUT(field, expr, type) \
  b.field = put<type>(h, off, nb, done, base, [&](size_t i) -> const type& { return v[i].expr; })
  LRC_PUT(g1, g1.g, GramArgs<T>);
  LRC_PUT(r1, g1.r, GramRedArgs<T>);
  LRC_PUT(c1, c1, CholArgs);
  LRC_PUT(t1, t1.a, TsmmArgs<T>);
  LRC_PUT(g2, g2.g, GramArgs<T>);
  LRC_PUT(r2, g2.r, GramRedArgs<T>);
  LRC_PUT(c2, c2, CholArgs);
  for (int j = 0; j < 2; ++j) LRC_PUT(core[j], core[j], SmallGemmArgs);
  LRC_PUT(qr, qr, QrArgs);
  LRC_PUT(jac, jac, JacArgs);
  LRC_PUT(rep, rep, RepArgs);
  LRC_PUT(fin, fin, SmallGemmArgs);
  LRC_PUT(sel, sel, SelArgs);
  LRC_PUT(xab, xab, SmallGemmArgs);
  LRC_PUT(t2, t2.a, TsmmArgs<T>);
#undef LRC_PUT
  LRC_CHECK(off <= buf.bytes, ST_EINVAL, "batched truncation: argument buffer layout");
  LRC_HIP(hipMemcpyAsync(buf.p, h.data(), off, hipMemcpyHostToDevice, s));
  LRC_HIP(hipStreamSynchronize(s));   // h is a temporary
  return b;
}

template void enqueue_trunc<double>(const TruncPlan<double>&, const TruncBatch<double>&, hipStream_t);
template void enqueue_trunc<float>(const TruncPlan<float>&, const TruncBatch<float>&, hipStream_t);
template TruncPlan<double> merge_plans<double>(const std::vector<TruncPlan<double>>&);
template TruncPlan<float> merge_plans<float>(const std::vector<TruncPlan<float>>&);
template TruncBatch<double> upload_plans<double>(const std::vector<TruncPlan<double>>&, const int*,
                                                 DevBuf&, hipStream_t);
template TruncBatch<float> upload_plans<float>(const std::vector<TruncPlan<float>>&, const int*,
                                               DevBuf&, hipStream_t);

template <class T>
void Truncator<T>::run(const BlockView<T>& A, int64_t n, const BlockView<T>& B, int64_t m,
                       const CoreView& core, int rank_cap, double tol, T* Uout, int ldu,
                       T* Vout, int ldv, double* s_out, int* rank_out, double* norm_out,
                       hipStream_t s) {
  enqueue_trunc(plan(A, n, B, m, core, rank_cap, tol, Uout, ldu, Vout, ldv, s_out, rank_out,
                     norm_out),
                TruncBatch<T>(), s);
  if (log_enabled()) {
    int hk[6] = {0, 0, 0, 0, 0, 0};
    double hn = 0.0;
    LRC_HIP(hipMemcpyAsync(&hk[4], st.kj, 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(&hk[5], st.kj + 1, 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(&hk[0], st.k, 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(&hk[1], rank_out, 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(&hk[2], st.info, 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(&hk[3], st.rounds, 4, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipMemcpyAsync(&hn, norm_out, 8, hipMemcpyDeviceToHost, s));
    LRC_HIP(hipStreamSynchronize(s));
    std::fprintf(stderr, "{\"trunc\": %d, \"k\": %d, \"kj\": %d, \"rank\": %d, \"norm\": %.9e, \"info\": %d, \"rounds\": %d, \"jacobi_rounds\": %d}\n",
                 int(sizeof(T)), hk[0], hk[4], hk[1], hn, hk[2], hk[3], hk[5]);
    if (hk[0] > 0 && hk[4] == 0) {
      // diagnostics of a truncation whose core came out empty
      const int kk = hk[0];
      std::vector<double> buf(size_t(kcap) * kcap);
      auto diag = [&](const double* dp, const char* name) {
        LRC_HIP(hipMemcpy(buf.data(), dp, buf.size() * 8, hipMemcpyDeviceToHost));
        double mn = 1e300, mx = -1e300;
        int nan = 0;
        for (int i = 0; i < kk; ++i) {
          const double v = buf[size_t(i) * kcap + i];
          if (!(v == v)) ++nan;
          else { mn = std::min(mn, v); mx = std::max(mx, v); }
        }
        std::fprintf(stderr, "  %s diag: min %.3e max %.3e nan %d  (0,1)=%.3e\n", name, mn, mx, nan,
                     kk > 1 ? buf[1] : 0.0);
      };
      diag(st.G[0], "G_A(pass2)");
      diag(st.G[1], "G_B(pass2)");
      diag(st.R1[0], "R_A");
      diag(st.R1[1], "R_B");
      diag(st.R2[0], "R2_A");
      diag(st.R2[1], "R2_B");
      diag(st.M, "M");
      diag(st.H, "H");
      {
        LRC_HIP(hipMemcpy(buf.data(), st.T1[0], buf.size() * 8, hipMemcpyDeviceToHost));
        int nan = 0, big = 0;
        for (int i = 0; i < kk; ++i)
          for (int j = 0; j < kk; ++j) {
            const double v = buf[size_t(i) * kcap + j];
            if (!(v == v)) ++nan;
            else if (std::fabs(v) > 1e30) ++big;
          }
        std::fprintf(stderr, "  T1_A: nan %d big %d\n", nan, big);
        std::vector<T> q(size_t(n) * ldq);
        LRC_HIP(hipMemcpy(q.data(), qa, q.size() * sizeof(T), hipMemcpyDeviceToHost));
        std::vector<int> colnan(kk, 0);
        for (int64_t i = 0; i < n; ++i)
          for (int j = 0; j < kk; ++j)
            if (!(q[size_t(i) * ldq + j] == q[size_t(i) * ldq + j])) ++colnan[j];
        std::fprintf(stderr, "  Q1_A nan per column:");
        for (int j = 0; j < kk; ++j) std::fprintf(stderr, " %d", colnan[j]);
        std::fprintf(stderr, "\n");
      }
    }
  }
}
template struct Truncator<double>;
template struct Truncator<float>;

// ------------------------------------------------------------------ ChebyshevT
template <class T> static const std::vector<DevCsr<T>>& ops_dev(const Ops& o);
template <> const std::vector<DevCsr<double>>& ops_dev<double>(const Ops& o) { return o.d64; }
template <> const std::vector<DevCsr<float>>& ops_dev<float>(const Ops& o) { return o.d32; }

template <class T>
void Cheb<T>::alloc(Prob* p, int cap_) {
  P = p;
  cap = cap_;
  hipStream_t s = P->ctx->stream;
  const int64_t n = P->ops->n, m = P->m;
  S.alloc(n, m, cap, s);
  D.alloc(n, m, cap, s);
  R.alloc(n, m, cap, s);
  const int ld = ld_for(cap);
  W.alloc(size_t(P->ops->q) * n * ld * sizeof(T));
  // the SpMM of the iterate visits only the operators' non-empty rows: the
  // other rows of W stay the zeros written here
  LRC_HIP(hipMemsetAsync(W.p, 0, W.bytes, s));
  Z.alloc(size_t(n) * ld * sizeof(T));
  py.alloc(size_t(n) * ld * sizeof(T));
  px.alloc(size_t(n) * ld * sizeof(T));
  const int64_t cbr = P->prec ? P->prec->cb_rows : 0;
  const int64_t str = P->prec ? P->prec->stage_rows : 0;
  pcb.alloc(size_t(std::max<int64_t>(cbr, 1)) * ld * sizeof(T));
  pst.alloc(size_t(std::max<int64_t>(str, 1)) * ld * sizeof(T));
  norm.alloc(64);
  tr.alloc(n, m, s);
}

template <class T>
SpmmLaunch<T> Cheb<T>::spmm_plan(const T* U, int ldu, const int* r_dev) const {
  const Ops& o = *P->ops;
  const int ld = ld_for(cap);
  T* Wp[kMaxOps];
  for (int i = 0; i < o.q; ++i) Wp[i] = W.as<T>() + size_t(i) * o.n * ld;
  return make_spmm<T>(ops_dev<T>(o).data(), o.q, U, ldu, r_dev, 0, cap, Wp, ld,
                      spmm_config<T>(o, cap), true);
}

// R = T(B - sum_i K_i S D_i): blocks [B | K_0 S | ... ] and [B_V | D_0 S_V | ...]
template <class T>
TruncPlan<T> Cheb<T>::resid_plan(const LR<T>& B, double* norm_dev, double tol_, int rank_cap,
                                 double abs_tol, const LR<T>* X) const {
  const Ops& o = *P->ops;
  const LR<T>& S = X ? *X : this->S;
  const int ld = ld_for(cap);
  BlockView<T> A{}, Bv{};
  CoreView c{};
  add_block(A, B.u(), B.ld, B.r(), 0);
  add_block(Bv, B.v(), B.ld, B.r(), 0);
  add_core(c, B.sv(), 1.0, B.r(), 0);
  for (int i = 0; i < o.q; ++i) {
    add_block(A, W.as<T>() + size_t(i) * o.n * ld, ld, S.r(), 0);
    add_block(Bv, S.v(), S.ld, S.r(), 0, P->drow(i));
    add_core(c, S.sv(), -1.0, S.r(), 0);
  }
  return tr.plan(A, o.n, Bv, P->m, c, rank_cap > 0 ? std::min(rank_cap, cap) : cap, tol_, R.u(),
                 R.ld, R.v(), R.ld, R.sv(), R.r(), norm_dev, abs_tol);
}

// D = T(Z R_V^T / dc) with Z = P^{-1} R_U diag(s_R)
template <class T>
TruncPlan<T> Cheb<T>::dstart_plan(double dc) const {
  const int ld = ld_for(cap);
  BlockView<T> A = view1<T>(Z.as<T>(), ld, R.r(), 0);
  BlockView<T> Bv = view1<T>(R.v(), R.ld, R.r(), 0);
  CoreView cv{};
  add_core(cv, R.sv(), 1.0 / dc, R.r(), 0);
  return tr.plan(A, P->ops->n, Bv, P->m, cv, cap, tol, D.u(), D.ld, D.v(), D.ld, D.sv(), D.r(),
                 norm.as<double>() + 1);
}

// S = T(S + D)
template <class T>
TruncPlan<T> Cheb<T>::supd_plan() const {
  BlockView<T> A{}, Bv{};
  CoreView cv{};
  add_block(A, S.u(), S.ld, S.r(), 0);
  add_block(A, D.u(), D.ld, D.r(), 0);
  add_block(Bv, S.v(), S.ld, S.r(), 0);
  add_block(Bv, D.v(), D.ld, D.r(), 0);
  add_core(cv, S.sv(), 1.0, S.r(), 0);
  add_core(cv, D.sv(), 1.0, D.r(), 0);
  return tr.plan(A, P->ops->n, Bv, P->m, cv, cap, tol, S.u(), S.ld, S.v(), S.ld, S.sv(), S.r(),
                 norm.as<double>() + 2);
}

// D = T(alpha D + beta Z R_V^T)
template <class T>
TruncPlan<T> Cheb<T>::dstep_plan(double alpha, double beta) const {
  const int ld = ld_for(cap);
  BlockView<T> A{}, Bv{};
  CoreView cv{};
  add_block(A, D.u(), D.ld, D.r(), 0);
  add_block(A, Z.as<T>(), ld, R.r(), 0);
  add_block(Bv, D.v(), D.ld, D.r(), 0);
  add_block(Bv, R.v(), R.ld, R.r(), 0);
  add_core(cv, D.sv(), alpha, D.r(), 0);
  add_core(cv, R.sv(), beta, R.r(), 0);
  return tr.plan(A, P->ops->n, Bv, P->m, cv, cap, tol, D.u(), D.ld, D.v(), D.ld, D.sv(), D.r(),
                 norm.as<double>() + 1);
}

// out = T(a X + b Y + g Z R_V^T), Z = P^{-1} R_U (the three-term update)
template <class T>
TruncPlan<T> Cheb<T>::upd3_plan(const LR<T>& X, double a, const LR<T>* Y, double b, double g,
                                const LR<T>& out) const {
  const int ld = ld_for(cap);
  BlockView<T> A{}, Bv{};
  CoreView cv{};
  add_block(A, X.u(), X.ld, X.r(), 0);
  add_block(Bv, X.v(), X.ld, X.r(), 0);
  add_core(cv, X.sv(), a, X.r(), 0);
  if (Y) {
    add_block(A, Y->u(), Y->ld, Y->r(), 0);
    add_block(Bv, Y->v(), Y->ld, Y->r(), 0);
    add_core(cv, Y->sv(), b, Y->r(), 0);
  }
  add_block(A, Z.as<T>(), ld, R.r(), 0);
  add_block(Bv, R.v(), R.ld, R.r(), 0);
  add_core(cv, R.sv(), g, R.r(), 0);
  return tr.plan(A, P->ops->n, Bv, P->m, cv, cap, tol, out.u(), out.ld, out.v(), out.ld,
                 out.sv(), out.r(), norm.as<double>() + 2);
}

// Z = P^{-1} R_U
template <class T>
PrecItem<T> Cheb<T>::prec_item() const {
  const PrecDev<T>& pd = P->prec->dev<T>();
  return PrecItem<T>{pd.fw, pd.bw, R.u(), R.ld, Z.as<T>(), ld_for(cap), R.r(), 0,
                     py.as<T>(), px.as<T>(), pcb.as<T>(), pst.as<T>()};
}

template struct Cheb<double>;
template struct Cheb<float>;

// ------------------------------------------------------------------ helpers
static void upload_lr(LR<double>& X, int r, const double* Uh, const double* sh, const double* Vh,
                      hipStream_t s) {
  // host column-major -> device row-major
  std::vector<double> u(size_t(X.n) * X.ld, 0.0), v(size_t(X.m) * X.ld, 0.0),
      sv(size_t(std::max(X.cap, 8)), 0.0);
  for (int j = 0; j < r; ++j) {
    for (int64_t i = 0; i < X.n; ++i) u[size_t(i) * X.ld + j] = Uh[size_t(j) * X.n + i];
    for (int64_t i = 0; i < X.m; ++i) v[size_t(i) * X.ld + j] = Vh[size_t(j) * X.m + i];
    sv[j] = sh ? sh[j] : 1.0;
  }
  LRC_HIP(hipMemcpyAsync(X.U.p, u.data(), u.size() * 8, hipMemcpyHostToDevice, s));
  LRC_HIP(hipMemcpyAsync(X.V.p, v.data(), v.size() * 8, hipMemcpyHostToDevice, s));
  LRC_HIP(hipMemcpyAsync(X.s.p, sv.data(), sv.size() * 8, hipMemcpyHostToDevice, s));
  LRC_HIP(hipMemcpyAsync(X.rank.p, &r, sizeof(int), hipMemcpyHostToDevice, s));
  LRC_HIP(hipStreamSynchronize(s));
}

template <class Tin, class Tout>
void cast_lr(const LR<Tin>& a, LR<Tout>& b, hipStream_t s) {
  const int cap = std::min(a.cap, b.cap);
  launch_cast<Tin, Tout>(a.u(), a.ld, b.u(), b.ld, a.n, a.r(), 0, cap, s);
  launch_cast<Tin, Tout>(a.v(), a.ld, b.v(), b.ld, a.m, a.r(), 0, cap, s);
  LRC_HIP(hipMemcpyAsync(b.s.p, a.s.p, size_t(cap) * 8, hipMemcpyDeviceToDevice, s));
  LRC_HIP(hipMemcpyAsync(b.rank.p, a.rank.p, sizeof(int), hipMemcpyDeviceToDevice, s));
}
template void cast_lr<double, float>(const LR<double>&, LR<float>&, hipStream_t);
template void cast_lr<float, double>(const LR<float>&, LR<double>&, hipStream_t);
template void cast_lr<double, double>(const LR<double>&, LR<double>&, hipStream_t);
template void cast_lr<float, float>(const LR<float>&, LR<float>&, hipStream_t);

static int read_rank(Ctx& ctx, const int* r) {
  LRC_HIP(hipMemcpyAsync(ctx.pinned_i, r, sizeof(int), hipMemcpyDeviceToHost, ctx.stream));
  ctx.sync();
  return ctx.pinned_i[0];
}

// Entry-wise fp64 residual of X = X0 + S.
double residual_fp64(Prob& P, const LR<double>& X0, int r0, const LR<double>& S, double* colres) {
  Ctx& ctx = *P.ctx;
  hipStream_t s = ctx.stream;
  const Ops& o = *P.ops;
  const int64_t n = o.n, m = P.m;
  const int ld0 = X0.ld, lds = S.ld;
  ensure(P.res_w0, size_t(o.q) * n * ld0 * 8);
  ensure(P.res_ws, size_t(o.q) * n * lds * 8);
  DevBuf& W0 = P.res_w0;
  DevBuf& WS = P.res_ws;
  double* W0p[kMaxOps];
  double* WSp[kMaxOps];
  for (int i = 0; i < o.q; ++i) {
    W0p[i] = W0.as<double>() + size_t(i) * n * ld0;
    WSp[i] = WS.as<double>() + size_t(i) * n * lds;
  }
  if (r0 > 0)
    enqueue_spmm(make_spmm<double>(o.d64.data(), o.q, X0.u(), ld0, X0.r(), 0, X0.cap, W0p, ld0,
                                   spmm_config<double>(o, X0.cap)),
                 Batched<SpmmArgs<double>>(), s);
  enqueue_spmm(make_spmm<double>(o.d64.data(), o.q, S.u(), lds, S.r(), 0, S.cap, WSp, lds,
                                 spmm_config<double>(o, S.cap)),
               Batched<SpmmArgs<double>>(), s);
  BlockView<double> A{}, B{};
  CoreView c{};
  add_block(A, P.F64.u(), P.F64.ld, P.F64.r(), 0);
  add_block(B, P.F64.v(), P.F64.ld, P.F64.r(), 0);
  add_core(c, P.F64.sv(), 1.0, P.F64.r(), 0);
  for (int i = 0; i < o.q; ++i) {
    if (r0 > 0) {
      add_block(A, W0p[i], ld0, X0.r(), 0);
      add_block(B, X0.v(), ld0, X0.r(), 0, P.drow(i));
      add_core(c, X0.sv(), -1.0, X0.r(), 0);
    }
    add_block(A, WSp[i], lds, S.r(), 0);
    add_block(B, S.v(), lds, S.r(), 0, P.drow(i));
    add_core(c, S.sv(), -1.0, S.r(), 0);
  }
  // the blocks' host-side width bounds are the factors' rank caps (their
  // leading dimensions round those up to 8)
  for (int b = 0; b < A.nb; ++b) {
    const int cb = b == 0 ? P.rF : (r0 > 0 && (b - 1) % 2 == 0) ? X0.cap : S.cap;
    A.cap[b] = B.cap[b] = std::min(A.cap[b], cb);
  }
  LRC_CHECK(P.rF + o.q * ((r0 > 0 ? X0.cap : 0) + S.cap) <= 192, ST_EINVAL,
            "fp64 residual: more than 192 concatenated columns");
  ensure(P.res_colsq, size_t(m) * 8);
  const size_t wsb = residual_workspace_bytes(n, m);
  ensure(P.res_tmp, wsb);
  DevBuf& colsq = P.res_colsq;
  DevBuf& ws = P.res_tmp;
  // the exact concatenated width picks the residual's tile shape
  const int width = P.rF + o.q * ((r0 > 0 ? read_rank(ctx, X0.r()) : 0) + read_rank(ctx, S.r()));
  launch_residual_fp64(A, n, B, c, m, width, colsq.as<double>(), ws.as<double>(), wsb, s);
  std::vector<double> h(m);
  LRC_HIP(hipMemcpyAsync(h.data(), colsq.p, size_t(m) * 8, hipMemcpyDeviceToHost, s));
  ctx.sync();
  double tot = 0.0;
  for (int64_t j = 0; j < m; ++j) {
    tot += h[j];
    if (colres) colres[j] = std::sqrt(std::max(h[j], 0.0));
  }
  return std::sqrt(tot);
}

// ------------------------------------------------------------------ solve
template <class T>
static void reset_lr(LR<T>& X, int64_t n, int64_t m, int cap, hipStream_t s) {
  if (X.U.p && X.n == n && X.m == m && X.cap == cap) {
    LRC_HIP(hipMemsetAsync(X.rank.p, 0, 16, s));
    LRC_HIP(hipMemsetAsync(X.s.p, 0, X.s.bytes, s));
  } else {
    X.alloc(n, m, cap, s);
  }
}

template <class T>
static void ensure_cheb(std::unique_ptr<Cheb<T>>& c, Prob* P, int cap) {
  if (!c || c->P != P || c->cap != cap || c->S.n != P->ops->n || c->S.m != P->m) {
    c = std::make_unique<Cheb<T>>();
    c->alloc(P, cap);
    return;
  }
  if (!c->S.U.p) c->S.alloc(P->ops->n, P->m, cap, P->ctx->stream);   // handed to the problem
  // the preconditioner may have been refactorised since (other level sizes)
  const size_t ld = size_t(ld_for(cap)) * sizeof(T);
  ensure(c->pcb, size_t(std::max<int64_t>(P->prec->cb_rows, 1)) * ld);
  ensure(c->pst, size_t(std::max<int64_t>(P->prec->stage_rows, 1)) * ld);
}

Prob::Prob() = default;
Prob::~Prob() = default;

void SolveRun::prepare(Prob& P_, const lrc_opts& o, int r0, const double* U0, const double* s0,
                       const double* V0, const X0Dev* xd) {
  t0 = clk::now();
  P = &P_;
  flags = iters = papp = refinements = 0;
  conv = false;
  last = 0.0;
  Prob& Pr = *P;
  hipStream_t s = Pr.ctx->stream;
  const Ops& op = *Pr.ops;
  const int64_t n = op.n, m = Pr.m;
  LRC_CHECK(Pr.prec != nullptr, ST_EINVAL, "lrc_solve: call lrc_prob_precondition first");
  LRC_CHECK(o.rank_cap >= 1 && o.rank_cap <= kPrecCols, ST_EINVAL,
            "lrc_solve: rank_cap must be in [1, 64]");
  LRC_CHECK(o.trunc_tol >= 0.0 && o.res_tol >= 0.0, ST_EINVAL, "lrc_solve: negative tolerance");
  LRC_CHECK(o.restart >= 1 && o.restart <= 64, ST_EINVAL,
            "lrc_solve: restart must be in [1, 64] (one restart cycle is one graph)");
  c = o.cheb_c;
  dc = o.cheb_d;
  if (!(c > 0.0) || !(dc > 0.0)) {
    double lo = 1.0, hi = 1.0;
    for (int64_t j = 0; j < m; ++j)
      for (int i = 0; i < op.q; ++i) {
        const double rt = Pr.d[size_t(j) * op.q + i] / Pr.dbar[i];
        lo = std::min(lo, rt);
        hi = std::max(hi, rt);
      }
    c = 0.5 * (hi - lo);
    dc = 0.5 * (hi + lo);
  }
  c = std::max(c, 1e-12 * dc);
  inf = lrc_info{};
  LRC_CHECK(o.init >= LRC_INIT_ZERO && o.init <= LRC_INIT_NEWTON, ST_EINVAL,
            "lrc_solve: unknown init");
  ref = o.res_ref > 0.0 ? o.res_ref : Pr.fnorm;
  newton_point = o.init == LRC_INIT_NEWTON;
  judged = o.init == LRC_INIT_GIVEN_JUDGED;
  rank_g = 0;
  // fixed initial term X0
  Pr.rank_x0 = 0;
  jmed = -1;
  if (o.init == LRC_INIT_MEDIAN || judged) {
    // upper-median column (Sec. 3.3): its system A(d_jmed) x = F e_jmed is
    // solved by the lockstep driver; its own, much narrower, spectrum interval
    jmed = int(m / 2);
    double lo = 1.0, hi = 1.0;
    for (int i = 0; i < op.q; ++i) {
      const double rt = Pr.d[size_t(jmed) * op.q + i] / Pr.dbar[i];
      lo = std::min(lo, rt);
      hi = std::max(hi, rt);
    }
    cm = std::max(0.5 * (hi - lo), 1e-3 * 0.5 * (hi + lo));
    dm = 0.5 * (hi + lo);
    fmed.assign(n, 0.0);
    for (int a = 0; a < Pr.rF; ++a) {
      const double w = Pr.Fs[a] * Pr.FV[size_t(a) * m + jmed];
      for (int64_t i = 0; i < n; ++i) fmed[i] += w * Pr.FU[size_t(a) * n + i];
    }
    coefmed.resize(op.q);
    for (int i = 0; i < op.q; ++i) coefmed[i] = Pr.d[size_t(jmed) * op.q + i];
    median_tol = o.median_tol > 0 ? o.median_tol : 1e-6;
  }
  if ((o.init == LRC_INIT_GIVEN || judged || newton_point) && r0 > 0) {
    LRC_CHECK(r0 <= 64, ST_EINVAL, "lrc_solve: initial rank at most 64");
    LR<double>& G = judged ? Xg : Pr.X0;
    reset_lr(G, n, m, r0, s);
    if (xd) {
      // device factors (row-major fp64): copied, the core from the host
      LRC_CHECK(xd->U && xd->V && xd->ldu >= r0 && xd->ldv >= r0, ST_EINVAL,
                "lrc_solve_x0_dev: U0 and V0 device factors with ld >= r0 required");
      launch_copy_cols(xd->U, xd->ldu, G.u(), G.ld, n, r0, s);
      launch_copy_cols(xd->V, xd->ldv, G.v(), G.ld, m, r0, s);
      std::vector<double> sv(size_t(std::max(G.cap, 8)), 0.0);
      for (int j = 0; j < r0; ++j) sv[j] = s0 ? s0[j] : 1.0;
      LRC_HIP(hipMemcpyAsync(G.s.p, sv.data(), sv.size() * 8, hipMemcpyHostToDevice, s));
      LRC_HIP(hipMemcpyAsync(G.rank.p, &r0, sizeof(int), hipMemcpyHostToDevice, s));
      LRC_HIP(hipStreamSynchronize(s));   // sv is a temporary
    } else {
      LRC_CHECK(U0 && V0, ST_EINVAL, "lrc_solve: U0 and V0 required for a given initial term");
      upload_lr(G, r0, U0, s0, V0, s);
    }
    if (judged) rank_g = r0;
    else Pr.rank_x0 = r0;
  } else if (o.init != LRC_INIT_MEDIAN) {
    LRC_CHECK(!judged, ST_EINVAL, "lrc_solve: LRC_INIT_GIVEN_JUDGED needs a given term");
    reset_lr(Pr.X0, n, m, 1, s);
  }
  cap = o.rank_cap;
  // room left for the right-hand side in the residual concatenation
  // [B | K_0 S | ... | K_{q-1} S] of at most 128 columns
  const int room = std::max(8, kTruncCap - op.q * cap);
  const int bcap = std::min(std::min(64, room), std::max(Pr.rF + op.q,
                                                         o.init == LRC_INIT_GIVEN || judged ? 64 : 1));
  ensure_cheb(c64, P, cap);
  reset_lr(B64, n, m, bcap, s);
  max_iter = o.max_iter > 0 ? o.max_iter : 200;
  // mixed precision: the inner correction's own cap keeps [rhs | K_i E] within 128 columns
  inner_cap = std::max(1, std::min(cap, (kTruncCap - cap) / op.q));
  target = o.res_tol * ref;
  refine_max = o.refine_max > 0 ? o.refine_max : 8;
  rhs_tol = std::max(o.trunc_tol, 0.1 * (o.inner_tol > 0 ? o.inner_tol : 1e-5));
  // the fp32 inner solve needs no truncation finer than its own target (and
  // fp32 data resolves nothing much finer): by default 1e-2 * inner_tol
  inner_trunc_tol = o.inner_trunc_tol > 0
                        ? o.inner_trunc_tol
                        : std::max(o.trunc_tol, o.precision == LRC_MIXED_FP32_DIR
                                                    ? 1e-6
                                                    : 1e-2 * (o.inner_tol > 0 ? o.inner_tol : 1e-3));
  LRC_CHECK(o.precision == LRC_FP64 || o.precision == LRC_MIXED_FP32 ||
                o.precision == LRC_MIXED_FP32_DIR || o.precision == LRC_MIXED_BF16GRAM,
            ST_EINVAL, "lrc_solve: unknown precision");
  LRC_CHECK(o.recurrence == LRC_CHEB_DIRECTION || o.recurrence == LRC_CHEB_THREE_TERM, ST_EINVAL,
            "lrc_solve: unknown recurrence");
  LRC_CHECK(o.recurrence != LRC_CHEB_THREE_TERM || 3 * ld_for(cap) <= kTruncCap, ST_EINVAL,
            "lrc_solve: the three-term recurrence needs 3 * rank_cap <= 128");
  LRC_CHECK(o.solver == LRC_SOLVER_CHEBYSHEV ||
                (o.solver == LRC_SOLVER_GMREST && o.precision == LRC_FP64),
            ST_EINVAL, "lrc_solve: unknown solver (GMREST runs in fp64)");
  if (o.precision == LRC_MIXED_FP32 || o.precision == LRC_MIXED_BF16GRAM) {
    alloc_mixed();
    c32->tr.bf16 = o.precision == LRC_MIXED_BF16GRAM;
  }
  if (o.precision == LRC_MIXED_FP32_DIR) ensure_cheb(c32, P, cap);   // fp32 direction and Z
}

// X0 = x 1^T from the median column's solution x (column 0 of an n x 8 block)
void SolveRun::set_median_x0(const double* x, int iters, int state, double norm, double fnorm) {
  Prob& Pr = *P;
  hipStream_t s = Pr.ctx->stream;
  const int64_t n = Pr.ops->n, m = Pr.m;
  reset_lr(Pr.X0, n, m, 1, s);
  inf.median_iters = iters;
  if (state != 1) {
    // the median solve stopped above its tolerance: its iterate is still the
    // better guess if it reduced the column's residual below ||f_med||
    // (the zero guess's); otherwise (non-finite, no reduction) X0 = 0
    flags |= 16;
    if (!(std::isfinite(norm) && norm < fnorm)) {
      flags |= 32;
      Pr.rank_x0 = 0;
      return;
    }
  }
  launch_copy_cols(x, 8, Pr.X0.u(), Pr.X0.ld, n, 1, s);
  std::vector<double> ones(size_t(m) * Pr.X0.ld, 0.0);
  for (int64_t j = 0; j < m; ++j) ones[size_t(j) * Pr.X0.ld] = 1.0;
  const double one = 1.0;
  const int r1 = 1;
  LRC_HIP(hipMemcpyAsync(Pr.X0.V.p, ones.data(), ones.size() * 8, hipMemcpyHostToDevice, s));
  LRC_HIP(hipMemcpyAsync(Pr.X0.s.p, &one, 8, hipMemcpyHostToDevice, s));
  LRC_HIP(hipMemcpyAsync(Pr.X0.rank.p, &r1, 4, hipMemcpyHostToDevice, s));
  LRC_HIP(hipStreamSynchronize(s));   // `ones` is a temporary
  Pr.rank_x0 = 1;
}

void SolveRun::judge_guess() {
  Prob& Pr = *P;
  Ctx& ctx = *Pr.ctx;
  hipStream_t s = ctx.stream;
  const int64_t n = Pr.ops->n, m = Pr.m;
  LR<double> none;
  none.alloc(n, m, 1, s);   // rank 0
  // fp64 per-column residuals of both guesses (the median's may be zero)
  std::vector<double> cmed(m), cgiv(m);
  residual_fp64(Pr, Pr.X0, Pr.rank_x0, none, cmed.data());
  residual_fp64(Pr, Xg, rank_g, none, cgiv.data());
  std::vector<char> w(m);
  int fb = 0;
  for (int64_t j = 0; j < m; ++j) {
    w[j] = cgiv[j] <= cmed[j] ? 1 : 0;
    fb += w[j] ? 0 : 1;
  }
  inf.median_fallback_cols = fb;
  if (fb == 0) {
    std::swap(Pr.X0, Xg);
    Pr.rank_x0 = rank_g;
    return;
  }
  // X0 = [Ug | x~] diag(s_g, 1) [diag(w) Vg | 1 - w]^T (the x~ column only
  // when the median solve produced one)
  const int rm = Pr.rank_x0;   // 0 or 1
  const int r = rank_g + rm;
  LR<double> X;
  X.alloc(n, m, r, s);
  launch_copy_cols(Xg.u(), Xg.ld, X.u(), X.ld, n, rank_g, s);
  if (rm) launch_copy_cols(Pr.X0.u(), Pr.X0.ld, X.u() + rank_g, X.ld, n, 1, s);
  std::vector<double> vg(size_t(m) * Xg.ld), sg(size_t(std::max(Xg.cap, 8)));
  LRC_HIP(hipMemcpyAsync(vg.data(), Xg.V.p, vg.size() * 8, hipMemcpyDeviceToHost, s));
  LRC_HIP(hipMemcpyAsync(sg.data(), Xg.s.p, sg.size() * 8, hipMemcpyDeviceToHost, s));
  LRC_HIP(hipStreamSynchronize(s));
  std::vector<double> v(size_t(m) * X.ld, 0.0), sv(size_t(std::max(X.cap, 8)), 0.0);
  for (int64_t j = 0; j < m; ++j) {
    for (int a = 0; a < rank_g; ++a) v[size_t(j) * X.ld + a] = w[j] ? vg[size_t(j) * Xg.ld + a] : 0.0;
    if (rm) v[size_t(j) * X.ld + rank_g] = w[j] ? 0.0 : 1.0;
  }
  for (int a = 0; a < rank_g; ++a) sv[a] = sg[a];
  if (rm) sv[rank_g] = 1.0;
  LRC_HIP(hipMemcpyAsync(X.V.p, v.data(), v.size() * 8, hipMemcpyHostToDevice, s));
  LRC_HIP(hipMemcpyAsync(X.s.p, sv.data(), sv.size() * 8, hipMemcpyHostToDevice, s));
  LRC_HIP(hipMemcpyAsync(X.rank.p, &r, sizeof(int), hipMemcpyHostToDevice, s));
  LRC_HIP(hipStreamSynchronize(s));   // v and sv are temporaries
  std::swap(Pr.X0, X);
  Pr.rank_x0 = r;
}

// Right-hand side B = F - L(X0), truncated to the rhs capacity at a tolerance
// far below the solver's: blocks [F_U | K_i X0_U] and [F_V | D_i X0_V].
TruncPlan<double> SolveRun::rhs_plan(const lrc_opts& o, double* const* W0) const {
  const Prob& Pr = *P;
  const Ops& op = *Pr.ops;
  const LR<double>& X0 = Pr.X0;
  BlockView<double> A{}, B{};
  CoreView cv{};
  add_block(A, Pr.F64.u(), Pr.F64.ld, Pr.F64.r(), 0);
  add_block(B, Pr.F64.v(), Pr.F64.ld, Pr.F64.r(), 0);
  add_core(cv, Pr.F64.sv(), 1.0, Pr.F64.r(), 0);
  for (int i = 0; i < op.q; ++i) {
    add_block(A, W0[i], X0.ld, X0.r(), 0);
    add_block(B, X0.v(), X0.ld, X0.r(), 0, Pr.drow(i));
    add_core(cv, X0.sv(), -1.0, X0.r(), 0);
  }
  // B is kept to 1e-14 of its norm, but directions whose total weight stays
  // below 1e-3 of the final residual target are dropped: they cannot move the
  // result's residual by more than that
  const int rcap = std::min(B64.cap, 64);
  return c64->tr.plan(A, op.n, B, Pr.m, cv, rcap, std::min(1e-14, o.trunc_tol * 1e-3), B64.u(),
                      B64.ld, B64.v(), B64.ld, B64.sv(), B64.r(), c64->norm.as<double>() + 4,
                      kResFloor * target);
}

void SolveRun::alloc_mixed() {
  hipStream_t s = P->ctx->stream;
  const int64_t n = P->ops->n, m = P->m;
  ensure_cheb(c32, P, inner_cap);
  reset_lr(Bin, n, m, inner_cap, s);   // the outer residual is truncated to inner_cap
  reset_lr(E64, n, m, inner_cap, s);
  LRC_HIP(hipMemsetAsync(c64->S.rank.p, 0, 16, s));
}

// S64 <- T(S64 + E64), E64 = fp64 copy of the inner correction
void SolveRun::accumulate_plan_inputs(hipStream_t s) {
  cast_lr<float, double>(c32->S, E64, s);
}
TruncPlan<double> SolveRun::accumulate_plan(const lrc_opts& o) const {
  const LR<double>& S64 = c64->S;
  BlockView<double> A{}, Bv{};
  CoreView cv{};
  add_block(A, S64.u(), S64.ld, S64.r(), 0);
  add_block(A, E64.u(), E64.ld, E64.r(), 0);
  add_block(Bv, S64.v(), S64.ld, S64.r(), 0);
  add_block(Bv, E64.v(), E64.ld, E64.r(), 0);
  add_core(cv, S64.sv(), 1.0, S64.r(), 0);
  add_core(cv, E64.sv(), 1.0, E64.r(), 0);
  return c64->tr.plan(A, P->ops->n, Bv, P->m, cv, cap, o.trunc_tol, S64.u(), S64.ld, S64.v(),
                      S64.ld, S64.sv(), S64.r(), c64->norm.as<double>() + 3);
}

lrc_status SolveRun::finish(const lrc_opts& o, lrc_info* info) {
  Prob& Pr = *P;
  Ctx& ctx = *Pr.ctx;
  const int64_t n = Pr.ops->n, m = Pr.m;
  // the solution takes the iterate's buffers; the iterate gets the previous
  // solution's (reused next time when the shapes agree)
  std::swap(Pr.S, c64->S);
  if (c64->S.U.p && (c64->S.cap != c64->cap || c64->S.n != n || c64->S.m != m)) c64->S = LR<double>();
  Pr.rank_s = read_rank(ctx, Pr.S.r());
  inf.rank = Pr.rank_s;
  inf.rank_x0 = Pr.rank_x0;
  inf.iters = iters;
  inf.prec_applies = papp;
  inf.refinements = refinements;
  inf.relres_est = last / ref;
  inf.relres = inf.relres_est;
  inf.info_flags = flags;
  Pr.newton_point = newton_point;
  Pr.ref = ref;
  if (flags & 8)
    throw Error(ST_EINVAL, "truncation capacity exceeded: more than 128 concatenated columns "
                           "(reduce rank_cap or the rank of the right-hand side)");
  if (o.verify_fp64) {
    std::vector<double> col(m);
    const double nr = residual_fp64(Pr, Pr.X0, newton_point ? 0 : Pr.rank_x0, Pr.S, col.data());
    inf.relres = nr / ref;
    // per-column relative residuals against ||F_j||, with G = FU^T FU
    std::vector<double> g(size_t(Pr.rF) * Pr.rF, 0.0);
    for (int a = 0; a < Pr.rF; ++a)
      for (int b = 0; b < Pr.rF; ++b) {
        double acc = 0.0;
        for (int64_t i = 0; i < n; ++i) acc += Pr.FU[size_t(a) * n + i] * Pr.FU[size_t(b) * n + i];
        g[size_t(a) * Pr.rF + b] = acc;
      }
    double mx = 0.0;
    for (int64_t j = 0; j < m && o.res_ref > 0.0; ++j)
      mx = std::max(mx, col[j] * std::sqrt(double(m)) / ref);
    for (int64_t j = 0; j < m && !(o.res_ref > 0.0); ++j) {
      double fj = 0.0;
      for (int a = 0; a < Pr.rF; ++a)
        for (int b = 0; b < Pr.rF; ++b)
          fj += Pr.FV[size_t(a) * m + j] * Pr.Fs[a] * g[size_t(a) * Pr.rF + b] * Pr.Fs[b] *
                Pr.FV[size_t(b) * m + j];
      if (fj > 0) mx = std::max(mx, col[j] / std::sqrt(fj));
    }
    inf.max_col_relres = mx;
  }
  inf.seconds_setup = Pr.seconds_setup;
  inf.seconds_solve = secs_since(t0);
  const bool ok = conv && (!o.verify_fp64 || inf.relres <= o.res_tol);
  inf.status = ok ? ST_OK : ST_NOTCONV;
  if (info) *info = inf;
  return ok ? ST_OK : ST_NOTCONV;
}

lrc_status solve_problem(Prob& P, const lrc_opts& o, int r0, const double* U0, const double* s0,
                         const double* V0, lrc_info* info, const X0Dev* xd) {
  const auto t0 = clk::now();
  if (!P.run) P.run = std::make_unique<SolveRun>();
  SolveRun& run = *P.run;
  run.prepare(P, o, r0, U0, s0, V0, xd);
  const double tp = secs_since(t0);
  std::vector<SolveRun*> one{&run};
  lockstep(one, o);
  const double tl = secs_since(t0);
  const lrc_status st = run.finish(o, info);
  if (log_enabled())
    std::fprintf(stderr, "{\"solve_s\": {\"prepare\": %.5f, \"lockstep\": %.5f, \"finish\": %.5f}}\n",
                 tp, tl - tp, secs_since(t0) - tl);
  return st;
}

}  // namespace lrc
