// Lockstep execution of the iterative phases of one or many solves (parameter
// subsets, each with its own linearisation point; a single solve is a batch of
// one): every step is one launch whose grid's z dimension runs over the
// problems, per-problem arguments come from device arrays built once per call
// site, finished problems are skipped through device-side done flags, and the
// iterations (a restart cycle of ChebyshevT, a few steps of the median-column
// solve) are captured into HIP graphs that the host replays until every
// problem has stopped.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>

#include "solver.hpp"

namespace lrc {

namespace {

bool log_on() {
  static const bool on = std::getenv("LRC_LOG") != nullptr;
  return on;
}

// Uploads one launch's per-item argument structs.
template <class A>
Batched<A> upload_items(const std::vector<A>& v, const int* done, DevBuf& buf, hipStream_t s) {
  const size_t bytes = v.size() * sizeof(A);
  if (buf.bytes < bytes) buf.alloc(bytes);
  LRC_HIP(hipMemcpyAsync(buf.p, v.data(), bytes, hipMemcpyHostToDevice, s));
  LRC_HIP(hipStreamSynchronize(s));   // v may be a temporary
  Batched<A> b;
  b.dev = buf.as<A>();
  b.done = done;
  b.n = int(v.size());
  return b;
}

template <class T>
SpmmLaunch<T> merge_spmm(const std::vector<SpmmLaunch<T>>& v) {
  SpmmLaunch<T> l = v[0];
  std::vector<Work> ws;
  for (const auto& x : v) ws.push_back(x.work);
  l.work = combine_work(ws);
  for (const auto& x : v) {
    LRC_CHECK(x.cpl == l.cpl && x.lpr == l.lpr && x.waves == l.waves, ST_EINVAL,
              "batched solve: problems differ in the SpMM launch shape");
    l.blocks = std::max(l.blocks, x.blocks);
    l.q = std::max(l.q, x.q);
  }
  return l;
}

// True when two factorisations have the same supernode structure, so that
// one set of level tasks serves both.
bool same_structure(const SupernodalFactor& a, const SupernodalFactor& b) {
  return a.n == b.n && a.nsn == b.nsn && a.perm == b.perm && a.j0 == b.j0 && a.ns == b.ns &&
         a.nb == b.nb && a.bnd_off == b.bnd_off && a.bnd == b.bnd && a.fw_off == b.fw_off &&
         a.bw_off == b.bw_off && a.front_off == b.front_off && a.cb_off == b.cb_off &&
         a.asm_ptr == b.asm_ptr && a.asm_src == b.asm_src && a.height == b.height;
}

struct GraphExec {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  GraphExec() = default;
  GraphExec(const GraphExec&) = delete;
  GraphExec& operator=(const GraphExec&) = delete;
  ~GraphExec() { reset(); }
  void reset() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    x = nullptr;
    g = nullptr;
  }
};

// Profiling is suspended while a stream is captured (event pairs would be
// recorded into the graph) and restored on every exit path.
struct CaptureGuard {
  hipStream_t s;
  bool active = false;
  explicit CaptureGuard(hipStream_t s_) : s(s_) {
    // thread-local mode: only this thread's unsafe calls end the capture
    LRC_HIP(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    profiler().suspended++;
    active = true;
  }
  hipGraph_t end() {
    hipGraph_t g = nullptr;
    active = false;
    profiler().suspended--;
    LRC_HIP(hipStreamEndCapture(s, &g));
    return g;
  }
  ~CaptureGuard() {
    if (!active) return;
    profiler().suspended--;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(s, &g) == hipSuccess && g) (void)hipGraphDestroy(g);
  }
};


// Preconditioner applies of a batch: one launch per level for all items when
// their factorisations share the supernode structure, else one per item.
template <class T>
struct PrecBatch {
  std::vector<const Prec*> pre;
  std::vector<PrecItem<T>> items;
  bool shared = true;
  Batched<PrecItem<T>> all;
  std::vector<Batched<PrecItem<T>>> one;
  int kcap = 1, ldw = 8;
  void setup(const std::vector<const Prec*>& p, const std::vector<PrecItem<T>>& it,
             const int* done, int kcap_, int ldw_, DevBuf& buf, hipStream_t s) {
    pre = p;
    items = it;
    kcap = kcap_;
    ldw = ldw_;
    for (auto* x : pre)
      if (x->kind != pre[0]->kind ||
          (x->kind == 0 ? !same_structure(x->F, pre[0]->F)
                        : (x->ilu.rowptr != pre[0]->ilu.rowptr || x->ilu.col != pre[0]->ilu.col)))
        shared = false;
    for (const auto& x : items) check_prec_item(x, kcap, ldw);
    all = upload_items(items, done, buf, s);
    one.clear();
    if (!shared)
      for (size_t j = 0; j < items.size(); ++j) {
        Batched<PrecItem<T>> b;
        b.dev = all.dev + j;
        b.done = done + j;
        b.n = 1;
        one.push_back(b);
      }
  }
  void enqueue(hipStream_t s) const {
    if (shared) {
      std::vector<WTerm> kt;
      for (const auto& x : items) kt.push_back(WTerm{x.k_dev, x.k_const});
      enqueue_prec_apply<T>(pre[0]->dev<T>(), pre[0]->fwd, pre[0]->bwd, items[0], all, kcap, ldw, s,
                            &kt);
    } else {
      for (size_t j = 0; j < items.size(); ++j)
        enqueue_prec_apply<T>(pre[j]->dev<T>(), pre[j]->fwd, pre[j]->bwd, items[j], one[j], kcap,
                              ldw, s);
    }
  }
};

// Replays `steps` from a captured graph (captured on first use), or launches
// them directly when eager.
struct Replay {
  GraphExec graph;
  bool eager = false;
  template <class F>
  void run(hipStream_t s, int cls, F steps) {
    if (eager) {
      steps();
      return;
    }
    if (!graph.x) {
      const auto t0 = std::chrono::steady_clock::now();
      CaptureGuard cg(s);
      steps();
      graph.g = cg.end();
      const auto t1 = std::chrono::steady_clock::now();
      LRC_HIP(hipGraphInstantiate(&graph.x, graph.g, nullptr, nullptr, 0));
      if (log_on())
        std::fprintf(stderr, "{\"graph_capture_s\": %.5f, \"instantiate_s\": %.5f}\n",
                     std::chrono::duration<double>(t1 - t0).count(),
                     std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count());
    }
    ProfScope ps(cls, s);
    LRC_HIP(hipGraphLaunch(graph.x, s));
  }
  // Captures and instantiates the graph on stream cs without launching it
  // (a later run() on any stream launches it); nothing in eager mode.
  template <class F>
  void prepare(hipStream_t cs, F steps) {
    if (eager || graph.x) return;
    const auto t0 = std::chrono::steady_clock::now();
    CaptureGuard cg(cs);
    steps();
    graph.g = cg.end();
    const auto t1 = std::chrono::steady_clock::now();
    LRC_HIP(hipGraphInstantiate(&graph.x, graph.g, nullptr, nullptr, 0));
    if (log_on())
      std::fprintf(stderr, "{\"graph_capture_s\": %.5f, \"instantiate_s\": %.5f, \"ahead\": 1}\n",
                   std::chrono::duration<double>(t1 - t0).count(),
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t1).count());
  }
};

// A restart cycle replayed as two graphs, steps [0, half) and [half, cycle).
// At a cycle's start both halves are launched back to back, unless the
// residual rates measured so far say that every running item stops within
// the first half: then the host checks after it, so that the second half's
// updates, which every finished item would still launch and skip, are not
// run.  `step_range(k0, k1)` enqueues steps [k0, k1) of a cycle; the two
// halves together enqueue exactly one cycle.
struct HalfCycles {
  Replay a, b;
  int cycle = 1, half = 1, pos = 0;
  std::vector<double> pnorm;
  std::vector<int> piters;
  void setup(int cycle_, bool eager, int nb) {
    cycle = std::max(cycle_, 1);
    half = (cycle + 1) / 2;
    a.eager = b.eager = eager;
    pnorm.assign(nb, -1.0);
    piters.assign(nb, 0);
  }
  template <class F>
  void prepare(hipStream_t cs, F step_range) {
    a.prepare(cs, [&]() { step_range(0, half); });
    if (half < cycle) b.prepare(cs, [&]() { step_range(half, cycle); });
  }
  void restart() {
    pos = 0;
    std::fill(pnorm.begin(), pnorm.end(), -1.0);
    std::fill(piters.begin(), piters.end(), 0);
  }
  // the largest number of updates a running item still needs, from its
  // residual's rate since the previous check (a whole cycle when unknown)
  double need(const std::vector<BCtl>& h) {
    double worst = 0.0;
    for (size_t j = 0; j < h.size(); ++j) {
      if (h[j].state != 0) continue;
      double nd = cycle;
      const int di = h[j].iters - piters[j];
      if (pnorm[j] > 0.0 && di > 0 && h[j].last > h[j].target) {
        const double rate = std::pow(h[j].last / pnorm[j], 1.0 / di);
        if (rate > 0.0 && rate < 0.95)
          nd = std::ceil(std::log(h[j].target / h[j].last) / std::log(rate));
      }
      worst = std::max(worst, nd);
      pnorm[j] = h[j].last;
      piters[j] = h[j].iters;
    }
    return worst;
  }
  template <class F>
  void run(hipStream_t s, int cls, const std::vector<BCtl>& h, F step_range) {
    const double nd = need(h);
    if (pos == 0) {
      a.run(s, cls, [&]() { step_range(0, half); });
      if (half == cycle) return;
      if (nd > half) {
        b.run(s, cls, [&]() { step_range(half, cycle); });
      } else {
        pos = half;
      }
    } else {
      b.run(s, cls, [&]() { step_range(half, cycle); });
      pos = 0;
    }
  }
};

// ------------------------------------------------------------------ median columns
// Preconditioned Chebyshev on the median parameter's single column, for every
// item at once; a few iterations per graph replay.
struct MedianBatch {
  static constexpr int kIterPerReplay = 4;
  Replay rep1;   // a single update, for the last ones
  int nb = 0;
  hipStream_t s = nullptr;
  std::vector<MedWork*> b;
  std::vector<std::unique_ptr<DevBuf>> bufs;
  DevBuf items, ctl, done;
  std::vector<MedCtl> hctl;
  int64_t nmax = 0;
  SpmmLaunch<double> sp0;
  Batched<SpmmArgs<double>> spB;
  PrecBatch<double> pb;
  PrecBatch<float> pb32;
  bool f32 = false;
  Replay rep;

  DevBuf& newbuf() {
    bufs.push_back(std::make_unique<DevBuf>());
    return *bufs.back();
  }

  // seed: hand each item's solution to its run as the fixed term X0 = x 1^T.
  // f32prec: the preconditioner solves run on the fp32 factors (the
  // residual, the iterate and the steps stay fp64, so the iteration still
  // converges to the fp64 solution; an inexact but fixed preconditioner only
  // moves the rate, by ~1e-7 relative), for the mixed-precision forms.
  // overlap: host work run once while the first replay executes on the GPU
  // (it must not use stream s_)
  void solve(std::vector<SolveRun*>& run, hipStream_t s_, bool eager, bool seed = true,
             bool f32prec = false, const std::function<void()>& overlap = {}) {
    f32 = f32prec;
    s = s_;
    nb = int(run.size());
    rep.eager = eager;
    rep1.eager = eager;
    std::vector<MedItem> hi(nb);
    std::vector<SpmmLaunch<double>> sl;
    std::vector<SpmmArgs<double>> sa;
    std::vector<PrecItem<double>> pi;
    std::vector<PrecItem<float>> pi32;
    std::vector<const Prec*> pre;
    hctl.assign(nb, MedCtl{});
    for (int j = 0; j < nb; ++j) {
      SolveRun& r = *run[j];
      const Prob& P = *r.P;
      const Ops& op = *P.ops;
      const int64_t n = op.n;
      nmax = std::max(nmax, n);
      MedWork& x = r.med;
      b.push_back(&x);
      const size_t col = size_t(n) * 8 * 8;
      ensure(x.f, r.fmed.size() * 8);
      ensure(x.coef, r.coefmed.size() * 8);
      LRC_HIP(hipMemcpyAsync(x.f.p, r.fmed.data(), r.fmed.size() * 8, hipMemcpyHostToDevice, s));
      LRC_HIP(hipMemcpyAsync(x.coef.p, r.coefmed.data(), r.coefmed.size() * 8,
                             hipMemcpyHostToDevice, s));
      for (DevBuf* d : {&x.x, &x.dl, &x.r, &x.z, &x.py, &x.px}) {
        ensure(*d, col);
        LRC_HIP(hipMemsetAsync(d->p, 0, col, s));
      }
      // the median SpMM visits only non-empty operator rows: a fresh product
      // buffer starts as zeros and its other rows stay so
      const bool fresh_w = x.W.bytes < col * op.q;
      ensure(x.W, col * op.q);
      if (fresh_w) LRC_HIP(hipMemsetAsync(x.W.p, 0, x.W.bytes, s));
      ensure(x.pcb, size_t(std::max<int64_t>(P.prec->cb_rows, 1)) * 8 * 8);
      ensure(x.pst, size_t(std::max<int64_t>(P.prec->stage_rows, 1)) * 8 * 8);
      ensure(x.part, size_t(med_partials()) * 8);
      if (f32) {
        ensure(x.r32, size_t(n) * 8 * 4);
        ensure(x.z32, size_t(n) * 8 * 4);
        LRC_HIP(hipMemsetAsync(x.r32.p, 0, x.r32.bytes, s));
        LRC_HIP(hipMemsetAsync(x.z32.p, 0, x.z32.bytes, s));
      }
      hi[j] = MedItem{x.f.as<double>(), x.W.as<double>(), x.coef.as<double>(), x.x.as<double>(),
                      x.dl.as<double>(), x.r.as<double>(), x.z.as<double>(),
                      x.part.as<double>(), f32 ? x.r32.as<float>() : nullptr,
                      f32 ? x.z32.as<float>() : nullptr, n, op.q};
      double* Wp[kMaxOps];
      for (int i = 0; i < op.q; ++i) Wp[i] = x.W.as<double>() + size_t(i) * n * 8;
      sl.push_back(make_spmm<double>(op.d64.data(), op.q, x.x.as<double>(), 8, nullptr, 1, 1, Wp,
                                     8, spmm_config<double>(op, 1), true));
      sa.push_back(sl.back().a);
      pi.push_back(PrecItem<double>{P.prec->p64.fw, P.prec->p64.bw, x.r.as<double>(), 8,
                                    x.z.as<double>(), 8, nullptr, 1, x.py.as<double>(),
                                    x.px.as<double>(), x.pcb.as<double>(), x.pst.as<double>()});
      // fp32 work rows of ld 8 fit the fp64 buffers sized for ld 8
      pi32.push_back(PrecItem<float>{P.prec->p32.fw, P.prec->p32.bw, x.r32.as<float>(), 8,
                                     x.z32.as<float>(), 8, nullptr, 1, x.py.as<float>(),
                                     x.px.as<float>(), x.pcb.as<float>(), x.pst.as<float>()});
      pre.push_back(P.prec.get());
      double fn = 0.0;
      for (double v : r.fmed) fn += v * v;
      MedCtl& c = hctl[j];
      c.target = r.median_tol * std::sqrt(fn);
      c.c = r.cm;
      c.dc = r.dm;
      c.max_iter = 1000;
    }
    items.alloc(size_t(nb) * sizeof(MedItem));
    LRC_HIP(hipMemcpyAsync(items.p, hi.data(), hi.size() * sizeof(MedItem), hipMemcpyHostToDevice, s));
    ctl.alloc(size_t(nb) * sizeof(MedCtl));
    LRC_HIP(hipMemcpyAsync(ctl.p, hctl.data(), hctl.size() * sizeof(MedCtl), hipMemcpyHostToDevice, s));
    done.alloc(size_t(nb) * sizeof(int));
    LRC_HIP(hipMemsetAsync(done.p, 0, done.bytes, s));
    const int* dn = done.as<int>();
    sp0 = merge_spmm(sl);
    spB = upload_items(sa, dn, newbuf(), s);
    if (f32)
      pb32.setup(pre, pi32, dn, 1, 8, newbuf(), s);
    else
      pb.setup(pre, pi, dn, 1, 8, newbuf(), s);
    const MedItem* it = items.as<MedItem>();
    MedCtl* ct = ctl.as<MedCtl>();
    int* dd = done.as<int>();
    // residual of x = 0, then iterations
    enqueue_spmm(sp0, spB, s);
    launch_med_resid(it, dd, nb, s);
    launch_med_check(it, ct, dd, nb, 0, s);
    bool overlapped = false;
    std::vector<double> norm0(nb, 0.0);
    auto iterations = [&](int count) {
      for (int k = 0; k < count; ++k) {
        if (f32)
          pb32.enqueue(s);
        else
          pb.enqueue(s);
        launch_med_update(it, ct, dd, nb, nmax, s);
        enqueue_spmm(sp0, spB, s);
        launch_med_resid(it, dd, nb, s);
        launch_med_check(it, ct, dd, nb, 1, s);
      }
    };
    while (true) {
      LRC_HIP(hipMemcpyAsync(hctl.data(), ctl.p, hctl.size() * sizeof(MedCtl),
                             hipMemcpyDeviceToHost, s));
      LRC_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (const auto& c : hctl) all = all && c.state != 0;
      if (all) break;
      // After the first replay the observed rate of each running item gives
      // the updates it still needs; when every item needs at most two, single
      // updates are replayed: an update of a finished item still costs its
      // ~45 launches of early exits (about a quarter of a millisecond)
      double need_max = 0.0;
      for (int j = 0; j < nb; ++j) {
        const MedCtl& c = hctl[j];
        if (c.iters == 0) norm0[j] = c.norm;
        if (c.state != 0) continue;
        double need = kIterPerReplay;
        if (c.iters > 0 && norm0[j] > 0.0) {
          const double rate = std::pow(c.norm / norm0[j], 1.0 / c.iters);
          if (rate > 0.0 && rate < 0.95 && c.norm > c.target)
            need = std::ceil(std::log(c.target / c.norm) / std::log(rate));
        }
        need_max = std::max(need_max, need);
      }
      if (need_max <= 2.0)
        rep1.run(s, kcls(K_GRAPH, false), [&]() { iterations(1); });
      else
        rep.run(s, kcls(K_GRAPH, false), [&]() { iterations(kIterPerReplay); });
      if (overlap && !overlapped) {
        overlapped = true;
        // one more update is queued before the host work, so that the GPU
        // keeps working while the host is busy; an item already finished
        // skips it, one still running would have taken it next anyway
        rep1.run(s, kcls(K_GRAPH, false), [&]() { iterations(1); });
        overlap();
      }
    }
    if (overlap && !overlapped) overlap();
    for (int j = 0; j < nb && seed; ++j) {
      double fn = 0.0;
      for (double v : run[j]->fmed) fn += v * v;
      run[j]->set_median_x0(b[j]->x.as<double>(), hctl[j].iters, hctl[j].state, hctl[j].norm,
                            std::sqrt(fn));
    }
    if (log_on())
      for (int j = 0; j < nb; ++j)
        std::fprintf(stderr, "{\"median\": %d, \"iters\": %d, \"norm\": %.6e, \"state\": %d}\n", j,
                     hctl[j].iters, hctl[j].norm, hctl[j].state);
  }
};

// ------------------------------------------------------------------ ChebyshevT
// Lockstep ChebyshevT over the items' Cheb<T> objects (one per problem).
template <class T>
struct BatchCheb {
  std::vector<Cheb<T>*> it;
  std::vector<const LR<T>*> B;
  std::vector<double> c, dc;
  int cycle = 6;
  hipStream_t s = nullptr;
  int nb = 0;
  DevBuf done, ctl;
  std::vector<BCtl> hctl;
  // uploaded per-site arguments (alive as long as the graph)
  std::vector<std::unique_ptr<DevBuf>> bufs;
  SpmmLaunch<T> spmm0;
  Batched<SpmmArgs<T>> spmmB;
  PrecBatch<T> pb;
  TruncPlan<T> resid0, dstart0, supd0;
  TruncBatch<T> residB, dstartB, supdB;
  std::vector<TruncPlan<T>> dstep0;
  std::vector<TruncBatch<T>> dstepB;
  // three-term form: the iterate alternates between S (0) and the buffer of
  // D (1), which the direction form needs and this form does not; the SpMM
  // and the residual exist for either, the update per step of the cycle
  bool three = false;
  SpmmLaunch<T> spmm1;
  Batched<SpmmArgs<T>> spmmB1;
  TruncPlan<T> resid1;
  TruncBatch<T> residB1;
  std::vector<TruncPlan<T>> u30;
  std::vector<TruncBatch<T>> u3B;
  DevBuf back;       // per item: copy of D's buffer into S (odd cycles)
  int64_t rows_max = 0;
  Replay rep;        // its eager flag only: the cycle runs as two halves
  HalfCycles hc;

  DevBuf& newbuf() {
    bufs.push_back(std::make_unique<DevBuf>());
    return *bufs.back();
  }

  // res_abs: per item, the absolute floor of the residual's truncation
  void setup(const std::vector<Cheb<T>*>& items, const std::vector<const LR<T>*>& rhs,
             const std::vector<double>& c_, const std::vector<double>& dc_, double tol,
             const std::vector<double>& res_abs, int cycle_, bool eager, hipStream_t s_,
             bool three_ = false) {
    it = items;
    B = rhs;
    c = c_;
    dc = dc_;
    cycle = cycle_;
    s = s_;
    three = three_;
    rep.eager = eager;
    nb = int(it.size());
    done.alloc(size_t(nb) * sizeof(int));
    ctl.alloc(size_t(nb) * sizeof(BCtl));
    hctl.assign(nb, BCtl{});
    const int* dn = done.as<int>();
    for (auto* x : it) {
      LRC_CHECK(x->cap == it[0]->cap, ST_EINVAL, "batched solve: problems differ in rank_cap");
      x->tol = tol;
    }
    // SpMM of the iterate (residual)
    {
      std::vector<SpmmLaunch<T>> v;
      std::vector<SpmmArgs<T>> a;
      for (auto* x : it) {
        v.push_back(x->spmm_plan(x->S.u(), x->S.ld, x->S.r()));
        a.push_back(v.back().a);
      }
      spmm0 = merge_spmm(v);
      spmmB = upload_items(a, dn, newbuf(), s);
    }
    {
      std::vector<PrecItem<T>> a;
      std::vector<const Prec*> pre;
      for (auto* x : it) {
        a.push_back(x->prec_item());
        pre.push_back(x->P->prec.get());
      }
      pb.setup(pre, a, dn, it[0]->cap, ld_for(it[0]->cap), newbuf(), s);
    }
    auto site = [&](auto make, TruncPlan<T>& p0, TruncBatch<T>& bt) {
      std::vector<TruncPlan<T>> v;
      for (int j = 0; j < nb; ++j) v.push_back(make(j));
      p0 = merge_plans(v);
      bt = upload_plans(v, dn, newbuf(), s);
    };
    site([&](int j) {
      return it[j]->resid_plan(*B[j], it[j]->norm.template as<double>(), tol, 0, res_abs[j]);
    }, resid0, residB);
    if (three) {
      setup_three(tol, res_abs, site);
      return;
    }
    site([&](int j) { return it[j]->dstart_plan(dc[j]); }, dstart0, dstartB);
    site([&](int j) { return it[j]->supd_plan(); }, supd0, supdB);
    // D updates of a cycle: the coefficients follow rho_0 = c/dc,
    // rho_{k+1} = 1 / (2 dc/c - rho_k) for every item
    std::vector<double> rho(nb);
    for (int j = 0; j < nb; ++j) rho[j] = c[j] / dc[j];
    dstep0.resize(std::max(cycle - 1, 0));
    dstepB.resize(std::max(cycle - 1, 0));
    for (int k = 0; k + 1 < cycle; ++k) {
      std::vector<double> rn(nb);
      for (int j = 0; j < nb; ++j) rn[j] = 1.0 / (2.0 * dc[j] / c[j] - rho[j]);
      site([&](int j) { return it[j]->dstep_plan(rn[j] * rho[j], 2.0 * rn[j] / c[j]); },
           dstep0[k], dstepB[k]);
      rho = rn;
    }
  }

  // The three-term sites: SpMM and residual of the iterate in D's buffer,
  // and per step k of a cycle the update of the iterate in buffer k % 2 (and
  // its predecessor in the other) into buffer (k + 1) % 2:
  //   k = 0:  T(S + P^-1 R / dc)
  //   k > 0:  T((1 + rn rho) X_k - rn rho X_{k-1} + (2 rn / c) P^-1 R),
  //           rn = 1 / (2 dc / c - rho), rho <- rn, from rho = c / dc.
  // A cycle of odd length ends in D's buffer and is copied back into S, so
  // that every cycle starts from S.
  template <class Site>
  void setup_three(double tol, const std::vector<double>& res_abs, Site& site) {
    const int* dn = done.template as<int>();
    for (auto* x : it)
      LRC_CHECK(3 * x->S.ld <= kTruncCap, ST_EINVAL,
                "three-term recurrence: 3 * rank_cap must not exceed 128 columns");
    {
      std::vector<SpmmLaunch<T>> v;
      std::vector<SpmmArgs<T>> a;
      for (auto* x : it) {
        v.push_back(x->spmm_plan(x->D.u(), x->D.ld, x->D.r()));
        a.push_back(v.back().a);
      }
      spmm1 = merge_spmm(v);
      spmmB1 = upload_items(a, dn, newbuf(), s);
    }
    site([&](int j) {
      return it[j]->resid_plan(*B[j], it[j]->norm.template as<double>(), tol, 0, res_abs[j],
                               &it[j]->D);
    }, resid1, residB1);
    std::vector<double> rho(nb);
    for (int j = 0; j < nb; ++j) rho[j] = c[j] / dc[j];
    u30.resize(cycle);
    u3B.resize(cycle);
    for (int k = 0; k < cycle; ++k) {
      std::vector<double> a(nb, 1.0), b(nb, 0.0), g(nb);
      for (int j = 0; j < nb; ++j) {
        if (k == 0) {
          g[j] = 1.0 / dc[j];
          continue;
        }
        const double rn = 1.0 / (2.0 * dc[j] / c[j] - rho[j]);
        a[j] = 1.0 + rn * rho[j];
        b[j] = -rn * rho[j];
        g[j] = 2.0 * rn / c[j];
        rho[j] = rn;
      }
      site([&](int j) {
        Cheb<T>& x = *it[j];
        const LR<T>& X = (k & 1) ? x.D : x.S;
        const LR<T>& Y = (k & 1) ? x.S : x.D;
        return x.upd3_plan(X, a[j], k == 0 ? nullptr : &Y, b[j], g[j], Y);
      }, u30[k], u3B[k]);
    }
    if (cycle & 1) {
      std::vector<CastItem<T, T>> v;
      for (auto* x : it) {
        v.push_back(CastItem<T, T>{x->D.u(), x->D.v(), x->D.sv(), x->D.r(), x->S.u(), x->S.v(),
                                   x->S.sv(), x->S.r(), x->D.ld, x->D.ld, x->S.ld, x->S.ld,
                                   x->S.n, x->S.m, x->S.cap});
        rows_max = std::max(rows_max, x->S.n + x->S.m);
      }
      upload_items(v, dn, back, s);
    }
  }

  // capture the cycle's graphs on the set-up stream, then run on `main`
  void prepare_on(hipStream_t main) {
    hc.setup(cycle, rep.eager, nb);
    hc.prepare(s, [&](int k0, int k1) { steps(k0, k1); });
    s = main;
  }

  void resid(int after_update, int buf = 0) {
    enqueue_spmm(buf ? spmm1 : spmm0, buf ? spmmB1 : spmmB, s);
    enqueue_trunc(buf ? resid1 : resid0, buf ? residB1 : residB, s);
    launch_batch_check(ctl.as<BCtl>(), done.as<int>(), nb, after_update, s);
  }

  // After the run: an item that stopped at step k of a cycle (k = (iters - 1)
  // mod cycle) of the three-term form holds its iterate in D's buffer when k
  // is even; it is copied into S, where the callers read the solution.
  void three_back() {
    if (!three) return;
    for (int j = 0; j < nb; ++j) {
      const int t = hctl[j].iters;
      if (t >= 1 && ((t - 1) % cycle) % 2 == 0) cast_lr<T, T>(it[j]->D, it[j]->S, s);
    }
  }

  // Steps [k0, k1) of a restart cycle.  Direction form: step 0 starts with
  // D = T(P^-1 R / dc); step k updates S = T(S + D), takes the residual and,
  // before the next step, the direction D = T(alpha D + beta P^-1 R).
  // Three-term form: step k is the update of setup_three and the residual.
  void steps(int k0, int k1) {
    if (three) {
      for (int k = k0; k < k1; ++k) {
        pb.enqueue(s);
        enqueue_trunc(u30[k], u3B[k], s);
        resid(1, (k + 1) & 1);
      }
      if (k1 == cycle && (cycle & 1))
        launch_cast_lr(back.as<CastItem<T, T>>(), done.as<int>(), nb, rows_max, it[0]->S.cap, s);
      return;
    }
    for (int k = k0; k < k1; ++k) {
      if (k == 0) {
        pb.enqueue(s);
        enqueue_trunc(dstart0, dstartB, s);
      }
      enqueue_trunc(supd0, supdB, s);
      resid(1);
      if (k + 1 == cycle) break;
      pb.enqueue(s);
      enqueue_trunc(dstep0[k], dstepB[k], s);
    }
  }

  // Runs the lockstep iteration.  Items with init_done[j] set do nothing.
  // With S = 0 the first residual is the right-hand side itself: when
  // `r0_norm` is given (its Frobenius norm per item) and every B fits R, R is
  // a copy of B instead of a truncation of [B].
  void run(const std::vector<int>& init_done, const std::vector<double>& target,
           const std::vector<int>& max_iter, int stall_limit,
           const std::vector<double>* r0_norm = nullptr) {
    bool copy = r0_norm != nullptr;
    for (int j = 0; j < nb; ++j) copy = copy && B[j]->cap <= it[j]->R.cap;
    std::vector<int> dn(init_done);
    for (int j = 0; j < nb; ++j) {
      BCtl& h = hctl[j];
      h = BCtl{};
      h.norm = it[j]->norm.template as<double>();
      h.target = target[j];
      h.max_iter = max_iter[j];
      h.stall_limit = stall_limit;
      h.state = init_done[j] ? 2 : 0;
      LRC_HIP(hipMemsetAsync(it[j]->S.rank.p, 0, 16, s));
      LRC_HIP(hipMemsetAsync(it[j]->D.rank.p, 0, 16, s));
      if (copy && !init_done[j]) {
        // the checks of the first residual, as the device does them
        const double nr = (*r0_norm)[j];
        h.last = h.best = nr;
        if (!std::isfinite(nr)) h.state = 2;
        else if (nr <= h.target) h.state = 1;
        else if (h.max_iter <= 0) h.state = 2;
        if (h.state) dn[j] = 1;
        cast_lr<T, T>(*B[j], it[j]->R, s);
      }
    }
    LRC_HIP(hipMemcpyAsync(ctl.p, hctl.data(), size_t(nb) * sizeof(BCtl), hipMemcpyHostToDevice,
                           s));
    LRC_HIP(hipMemcpyAsync(done.p, dn.data(), size_t(nb) * sizeof(int), hipMemcpyHostToDevice,
                           s));
    if (!copy) resid(0);
    if (int(hc.pnorm.size()) != nb) hc.setup(cycle, rep.eager, nb);
    hc.restart();
    while (true) {
      LRC_HIP(hipMemcpyAsync(hctl.data(), ctl.p, size_t(nb) * sizeof(BCtl),
                             hipMemcpyDeviceToHost, s));
      LRC_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (const auto& h : hctl) all = all && h.state != 0;
      if (all) break;
      hc.run(s, kcls(K_GRAPH, is_f32<T>()), hctl, [&](int k0, int k1) { steps(k0, k1); });
    }
    three_back();
    if (log_on())
      for (int j = 0; j < nb; ++j)
        std::fprintf(stderr,
                     "{\"cheb\": %d, \"item\": %d, \"iters\": %d, \"norm\": %.6e, \"state\": %d}\n",
                     int(sizeof(T)), j, hctl[j].iters, hctl[j].last, hctl[j].state);
  }
};

// ------------------------------------------------------------------ mixed directions
// One ChebyshevT with an fp64 iterate S and fp64 residual R (SpMM and
// truncation), and fp32 preconditioner solves Z = P^{-1} R and directions D:
// R is copied to fp32 for the solve and the direction update, D back to fp64
// for the iterate update.  Same lockstep and graph machinery as BatchCheb.
struct BatchDir {
  std::vector<SolveRun*> run;
  int nb = 0, cycle = 6, cap = 0;
  hipStream_t s = nullptr;
  DevBuf done, ctl, castR, castD;
  std::vector<BCtl> hctl;
  std::vector<std::unique_ptr<DevBuf>> bufs;
  int64_t rows_max = 0;
  SpmmLaunch<double> sp0;
  Batched<SpmmArgs<double>> spB;
  PrecBatch<float> pb;
  TruncPlan<double> resid0, supd0;
  TruncBatch<double> residB, supdB;
  TruncPlan<float> dstart0;
  TruncBatch<float> dstartB;
  std::vector<TruncPlan<float>> dstep0;
  std::vector<TruncBatch<float>> dstepB;
  // three-term form (as in BatchCheb): fp64 iterate alternating between S and
  // D's buffer, the fp32 solve P^-1 R widened to fp64 before each update
  bool three = false;
  SpmmLaunch<double> sp1;
  Batched<SpmmArgs<double>> spB1;
  TruncPlan<double> resid1;
  TruncBatch<double> residB1;
  std::vector<TruncPlan<double>> u30;
  std::vector<TruncBatch<double>> u3B;
  DevBuf castZ, zscr, back;
  bool all_lu = true;   // every item's preconditioner is the exact LU
  bool zcast = false;   // some item's solve (ILU(0)) writes fp32 Z: widen it
  Replay rep;        // its eager flag only: the cycle runs as two halves
  HalfCycles hc;

  DevBuf& newbuf() {
    bufs.push_back(std::make_unique<DevBuf>());
    return *bufs.back();
  }

  void setup(std::vector<SolveRun*>& r, const lrc_opts& o, bool eager, hipStream_t s_) {
    run = r;
    nb = int(run.size());
    s = s_;
    cycle = o.restart;
    three = o.recurrence == LRC_CHEB_THREE_TERM;
    all_lu = true;
    for (auto* x : run) all_lu = all_lu && x->P->prec->kind == 0;
    rep.eager = eager;
    cap = run[0]->cap;
    done.alloc(size_t(nb) * sizeof(int));
    ctl.alloc(size_t(nb) * sizeof(BCtl));
    hctl.assign(nb, BCtl{});
    const int* dn = done.as<int>();
    std::vector<SpmmLaunch<double>> sl;
    std::vector<SpmmArgs<double>> sa;
    std::vector<PrecItem<float>> pi;
    std::vector<const Prec*> pre;
    std::vector<CastItem<double, float>> cr;
    std::vector<CastItem<float, double>> cd;
    for (auto* x : run) {
      Cheb<double>& C = *x->c64;
      Cheb<float>& F = *x->c32;
      LRC_CHECK(x->cap == cap, ST_EINVAL, "batched solve: problems differ in rank_cap");
      C.tol = o.trunc_tol;
      F.tol = x->inner_trunc_tol;
      rows_max = std::max(rows_max, x->P->ops->n + x->P->m);
      sl.push_back(C.spmm_plan(C.S.u(), C.S.ld, C.S.r()));
      sa.push_back(sl.back().a);
      pi.push_back(F.prec_item());
      // three-term form, exact LU throughout: the fp32 solve writes fp64 Z
      // directly (ILU(0) reads its own Z rows back, so a batch holding it
      // keeps fp32 Z and widens it)
      if (three && all_lu) pi.back().Z64 = C.Z.as<double>();
      pre.push_back(x->P->prec.get());
      cr.push_back(CastItem<double, float>{C.R.u(), C.R.v(), C.R.sv(), C.R.r(), F.R.u(), F.R.v(),
                                           F.R.sv(), F.R.r(), C.R.ld, C.R.ld, F.R.ld, F.R.ld,
                                           C.R.n, C.R.m, std::min(C.R.cap, F.R.cap)});
      cd.push_back(CastItem<float, double>{F.D.u(), F.D.v(), F.D.sv(), F.D.r(), C.D.u(), C.D.v(),
                                           C.D.sv(), C.D.r(), F.D.ld, F.D.ld, C.D.ld, C.D.ld,
                                           F.D.n, F.D.m, std::min(F.D.cap, C.D.cap)});
    }
    sp0 = merge_spmm(sl);
    spB = upload_items(sa, dn, newbuf(), s);
    pb.setup(pre, pi, dn, cap, ld_for(cap), newbuf(), s);
    upload_items(cr, dn, castR, s);
    upload_items(cd, dn, castD, s);
    auto site64 = [&](auto make, TruncPlan<double>& p0, TruncBatch<double>& bt) {
      std::vector<TruncPlan<double>> v;
      for (int j = 0; j < nb; ++j) v.push_back(make(j));
      p0 = merge_plans(v);
      bt = upload_plans(v, dn, newbuf(), s);
    };
    auto site32 = [&](auto make, TruncPlan<float>& p0, TruncBatch<float>& bt) {
      std::vector<TruncPlan<float>> v;
      for (int j = 0; j < nb; ++j) v.push_back(make(j));
      p0 = merge_plans(v);
      bt = upload_plans(v, dn, newbuf(), s);
    };
    site64([&](int j) {
      Cheb<double>& C = *run[j]->c64;
      return C.resid_plan(run[j]->B64, C.norm.as<double>(), o.trunc_tol, 0,
                          kResFloor * run[j]->target);
    }, resid0, residB);
    if (three) {
      setup_three(o, site64);
      return;
    }
    site64([&](int j) { return run[j]->c64->supd_plan(); }, supd0, supdB);
    site32([&](int j) { return run[j]->c32->dstart_plan(run[j]->dc); }, dstart0, dstartB);
    std::vector<double> rho(nb);
    for (int j = 0; j < nb; ++j) rho[j] = run[j]->c / run[j]->dc;
    dstep0.resize(std::max(cycle - 1, 0));
    dstepB.resize(std::max(cycle - 1, 0));
    for (int k = 0; k + 1 < cycle; ++k) {
      std::vector<double> rn(nb);
      for (int j = 0; j < nb; ++j) rn[j] = 1.0 / (2.0 * run[j]->dc / run[j]->c - rho[j]);
      site32([&](int j) {
        return run[j]->c32->dstep_plan(rn[j] * rho[j], 2.0 * rn[j] / run[j]->c);
      }, dstep0[k], dstepB[k]);
      rho = rn;
    }
  }

  template <class Site>
  void setup_three(const lrc_opts& o, Site& site64) {
    const int* dn = done.as<int>();
    LRC_CHECK(3 * ld_for(cap) <= kTruncCap, ST_EINVAL,
              "three-term recurrence: 3 * rank_cap must not exceed 128 columns");
    std::vector<SpmmLaunch<double>> sl;
    std::vector<SpmmArgs<double>> sa;
    std::vector<CastItem<float, double>> cz;
    std::vector<CastItem<double, double>> cb;
    zscr.alloc(size_t(nb) * (64 * sizeof(double) + 16));
    for (int j = 0; j < nb; ++j) {
      Cheb<double>& C = *run[j]->c64;
      Cheb<float>& F = *run[j]->c32;
      sl.push_back(C.spmm_plan(C.D.u(), C.D.ld, C.D.r()));
      sa.push_back(sl.back().a);
      // Z only (m = 0 rows of V); its core and rank copies land in scratch
      double* zs = zscr.as<double>() + size_t(j) * 66;
      cz.push_back(CastItem<float, double>{F.Z.as<float>(), nullptr, F.R.sv(), F.R.r(),
                                           C.Z.as<double>(), nullptr, zs,
                                           reinterpret_cast<int*>(zs + 64), ld_for(cap), 0,
                                           ld_for(cap), 0, C.R.n, 0, cap});
      cb.push_back(CastItem<double, double>{C.D.u(), C.D.v(), C.D.sv(), C.D.r(), C.S.u(),
                                            C.S.v(), C.S.sv(), C.S.r(), C.D.ld, C.D.ld, C.S.ld,
                                            C.S.ld, C.S.n, C.S.m, C.S.cap});
    }
    sp1 = merge_spmm(sl);
    spB1 = upload_items(sa, dn, newbuf(), s);
    zcast = !all_lu;
    if (zcast) upload_items(cz, dn, castZ, s);
    if (cycle & 1) upload_items(cb, dn, back, s);
    site64([&](int j) {
      Cheb<double>& C = *run[j]->c64;
      return C.resid_plan(run[j]->B64, C.norm.as<double>(), o.trunc_tol, 0,
                          kResFloor * run[j]->target, &C.D);
    }, resid1, residB1);
    std::vector<double> rho(nb);
    for (int j = 0; j < nb; ++j) rho[j] = run[j]->c / run[j]->dc;
    u30.resize(cycle);
    u3B.resize(cycle);
    for (int k = 0; k < cycle; ++k) {
      std::vector<double> a(nb, 1.0), b(nb, 0.0), g(nb);
      for (int j = 0; j < nb; ++j) {
        const double cj = run[j]->c, dj = run[j]->dc;
        if (k == 0) {
          g[j] = 1.0 / dj;
          continue;
        }
        const double rn = 1.0 / (2.0 * dj / cj - rho[j]);
        a[j] = 1.0 + rn * rho[j];
        b[j] = -rn * rho[j];
        g[j] = 2.0 * rn / cj;
        rho[j] = rn;
      }
      site64([&](int j) {
        Cheb<double>& C = *run[j]->c64;
        const LR<double>& X = (k & 1) ? C.D : C.S;
        const LR<double>& Y = (k & 1) ? C.S : C.D;
        return C.upd3_plan(X, a[j], k == 0 ? nullptr : &Y, b[j], g[j], Y);
      }, u30[k], u3B[k]);
    }
  }

  void cast_r() {
    launch_cast_lr(castR.as<CastItem<double, float>>(), done.as<int>(), nb, rows_max, cap, s);
  }
  void cast_d() {
    launch_cast_lr(castD.as<CastItem<float, double>>(), done.as<int>(), nb, rows_max, cap, s);
  }
  void prepare_on(hipStream_t main) {
    hc.setup(cycle, rep.eager, nb);
    hc.prepare(s, [&](int k0, int k1) { steps(k0, k1); });
    s = main;
  }

  void resid(int after_update, int buf = 0) {
    enqueue_spmm(buf ? sp1 : sp0, buf ? spB1 : spB, s);
    enqueue_trunc(buf ? resid1 : resid0, buf ? residB1 : residB, s);
    launch_batch_check(ctl.as<BCtl>(), done.as<int>(), nb, after_update, s);
    cast_r();
  }
  // steps [k0, k1) of a cycle
  void steps(int k0, int k1) {
    if (three) {
      for (int k = k0; k < k1; ++k) {
        pb.enqueue(s);
        if (zcast)
          launch_cast_lr(castZ.as<CastItem<float, double>>(), done.as<int>(), nb, rows_max, cap,
                         s);
        enqueue_trunc(u30[k], u3B[k], s);
        resid(1, (k + 1) & 1);
      }
      if (k1 == cycle && (cycle & 1))
        launch_cast_lr(back.as<CastItem<double, double>>(), done.as<int>(), nb, rows_max, cap, s);
      return;
    }
    for (int k = k0; k < k1; ++k) {
      if (k == 0) {
        pb.enqueue(s);
        enqueue_trunc(dstart0, dstartB, s);
        cast_d();
      }
      enqueue_trunc(supd0, supdB, s);
      resid(1);
      if (k + 1 == cycle) break;
      pb.enqueue(s);
      enqueue_trunc(dstep0[k], dstepB[k], s);
      cast_d();
    }
  }

  void solve(const std::vector<double>& r0_norm) {
    bool copy = true;
    for (auto* x : run) copy = copy && x->B64.cap <= x->c64->R.cap;
    std::vector<int> dn(nb, 0);
    for (int j = 0; j < nb; ++j) {
      SolveRun& x = *run[j];
      BCtl& h = hctl[j];
      h = BCtl{};
      h.norm = x.c64->norm.as<double>();
      h.target = x.target;
      h.max_iter = x.max_iter;
      h.stall_limit = 1 << 30;
      for (DevBuf* rk : {&x.c64->S.rank, &x.c64->D.rank, &x.c32->D.rank})
        LRC_HIP(hipMemsetAsync(rk->p, 0, 16, s));
      if (copy) {
        const double nr = r0_norm[j];
        h.last = h.best = nr;
        if (!std::isfinite(nr)) h.state = 2;
        else if (nr <= h.target) h.state = 1;
        else if (h.max_iter <= 0) h.state = 2;
        if (h.state) dn[j] = 1;
        cast_lr<double, double>(x.B64, x.c64->R, s);
      }
    }
    LRC_HIP(hipMemcpyAsync(ctl.p, hctl.data(), size_t(nb) * sizeof(BCtl), hipMemcpyHostToDevice, s));
    LRC_HIP(hipMemcpyAsync(done.p, dn.data(), size_t(nb) * sizeof(int), hipMemcpyHostToDevice, s));
    if (copy) cast_r();
    else resid(0);
    if (int(hc.pnorm.size()) != nb) hc.setup(cycle, rep.eager, nb);
    hc.restart();
    while (true) {
      LRC_HIP(hipMemcpyAsync(hctl.data(), ctl.p, size_t(nb) * sizeof(BCtl),
                             hipMemcpyDeviceToHost, s));
      LRC_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (const auto& h : hctl) all = all && h.state != 0;
      if (all) break;
      hc.run(s, kcls(K_GRAPH, false), hctl, [&](int k0, int k1) { steps(k0, k1); });
    }
    // an item that stopped at an even step k of a cycle holds its iterate in
    // D's buffer (see BatchCheb::three_back)
    if (three)
      for (int j = 0; j < nb; ++j) {
        const int t = hctl[j].iters;
        if (t >= 1 && ((t - 1) % cycle) % 2 == 0) cast_lr<double, double>(run[j]->c64->D,
                                                                            run[j]->c64->S, s);
      }
  }
};

int read_info(const int* p, hipStream_t s) {
  int v = 0;
  LRC_HIP(hipMemcpyAsync(&v, p, sizeof(int), hipMemcpyDeviceToHost, s));
  LRC_HIP(hipStreamSynchronize(s));
  return v;
}

// A stream of the library's own for the lockstep phase: graphs cannot be
// captured from the legacy default stream, which callers often pass.
struct OwnStream {
  hipStream_t s = nullptr;
  OwnStream() { LRC_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking)); }
  OwnStream(const OwnStream&) = delete;
  OwnStream& operator=(const OwnStream&) = delete;
  ~OwnStream() {
    if (s) {
      (void)hipStreamSynchronize(s);
      (void)hipStreamDestroy(s);
    }
  }
};

// B = F - L(X0) for every item with an initial term (one SpMM + one
// truncation launch for all of them); F itself otherwise.
void build_rhs(std::vector<SolveRun*>& run, const lrc_opts& o, hipStream_t s) {
  const int nb = int(run.size());
  std::vector<int> hd(nb, 1);
  bool any = false;
  for (int j = 0; j < nb; ++j) {
    SolveRun& r = *run[j];
    if (r.P->rank_x0 == 0 || r.newton_point) {
      LRC_CHECK(r.P->rF <= r.B64.cap, ST_EINVAL,
                "right-hand side rank exceeds the room left by q * rank_cap in 128 columns");
      cast_lr<double, double>(r.P->F64, r.B64, s);
    } else {
      hd[j] = 0;
      any = true;
    }
  }
  if (!any) return;
  DevBuf done = upload(hd, s);
  std::vector<SpmmLaunch<double>> sl;
  std::vector<SpmmArgs<double>> sa;
  std::vector<TruncPlan<double>> tp;
  for (int j = 0; j < nb; ++j) {
    SolveRun& r = *run[j];
    const Prob& P = *r.P;
    const Ops& op = *P.ops;
    const LR<double>& X0 = P.X0;
    ensure(r.rhs_w0, size_t(op.q) * op.n * X0.ld * 8);
    double* Wp[kMaxOps];
    for (int i = 0; i < op.q; ++i) Wp[i] = r.rhs_w0.as<double>() + size_t(i) * op.n * X0.ld;
    sl.push_back(make_spmm<double>(op.d64.data(), op.q, X0.u(), X0.ld, X0.r(), 0, X0.cap, Wp,
                                   X0.ld, spmm_config<double>(op, X0.cap)));
    sa.push_back(sl.back().a);
    tp.push_back(r.rhs_plan(o, Wp));
  }
  DevBuf sb, tb;
  enqueue_spmm(merge_spmm(sl), upload_items(sa, done.as<int>(), sb, s), s);
  enqueue_trunc(merge_plans(tp), upload_plans(tp, done.as<int>(), tb, s), s);
  LRC_HIP(hipStreamSynchronize(s));   // the temporaries above are released on return
}

}  // namespace

int median_column_solve(Prob& P, const std::vector<double>& rhs, double tol, bool eager,
                        std::vector<double>& x, int* iters) {
  LRC_CHECK(P.prec != nullptr, ST_EINVAL, "median solve: the problem has no preconditioner");
  const Ops& op = *P.ops;
  const int64_t n = op.n, m = P.m;
  LRC_CHECK(int64_t(rhs.size()) == n, ST_EINVAL, "median solve: right-hand side length");
  SolveRun r;
  r.P = &P;
  r.jmed = int(m / 2);
  double lo = 1.0, hi = 1.0;
  for (int i = 0; i < op.q; ++i) {
    const double rt = P.d[size_t(r.jmed) * op.q + i] / P.dbar[i];
    lo = std::min(lo, rt);
    hi = std::max(hi, rt);
  }
  r.cm = std::max(0.5 * (hi - lo), 1e-3 * 0.5 * (hi + lo));
  r.dm = 0.5 * (hi + lo);
  r.fmed = rhs;
  r.coefmed.resize(op.q);
  for (int i = 0; i < op.q; ++i) r.coefmed[i] = P.d[size_t(r.jmed) * op.q + i];
  r.median_tol = tol;
  Ctx& cx = *P.ctx;
  cx.sync();
  int state = 0;
  {
    OwnStream own;
    MedianBatch mb;
    std::vector<SolveRun*> v{&r};
    mb.solve(v, own.s, eager, false);
    DevBuf xc(size_t(n) * 8);
    launch_copy_cols(r.med.x.as<double>(), 8, xc.as<double>(), 1, n, 1, own.s);
    x.resize(n);
    LRC_HIP(hipMemcpyAsync(x.data(), xc.p, size_t(n) * 8, hipMemcpyDeviceToHost, own.s));
    LRC_HIP(hipStreamSynchronize(own.s));
    if (iters) *iters = mb.hctl[0].iters;
    state = mb.hctl[0].state;
  }
  return state;
}

void ops_apply_block(Ops& o, const std::vector<double>& X, int w, std::vector<double>& W) {
  const int64_t n = o.n;
  LRC_CHECK(w >= 1 && w <= 64 && int64_t(X.size()) == n * w, ST_EINVAL,
            "operator apply: block shape");
  hipStream_t s = o.ctx->stream;
  const int ld = ld_for(w);
  std::vector<double> xb(size_t(n) * ld, 0.0);
  for (int a = 0; a < w; ++a)
    for (int64_t i = 0; i < n; ++i) xb[size_t(i) * ld + a] = X[size_t(a) * n + i];
  DevBuf xd = upload(xb, s), wd(size_t(o.q) * n * ld * 8);
  double* Wp[kMaxOps];
  for (int i = 0; i < o.q; ++i) Wp[i] = wd.as<double>() + size_t(i) * n * ld;
  enqueue_spmm(make_spmm<double>(o.d64.data(), o.q, xd.as<double>(), ld, nullptr, w, w, Wp, ld,
                                 spmm_config<double>(o, w)),
               Batched<SpmmArgs<double>>(), s);
  std::vector<double> h(size_t(o.q) * n * ld);
  LRC_HIP(hipMemcpyAsync(h.data(), wd.p, h.size() * 8, hipMemcpyDeviceToHost, s));
  LRC_HIP(hipStreamSynchronize(s));
  W.assign(size_t(o.q) * n * w, 0.0);
  for (int i = 0; i < o.q; ++i)
    for (int a = 0; a < w; ++a)
      for (int64_t r = 0; r < n; ++r)
        W[(size_t(i) * w + a) * n + r] = h[(size_t(i) * n + r) * ld + a];
}

void ops_apply_vector(Ops& o, const std::vector<double>& x, std::vector<double>& W) {
  ops_apply_block(o, x, 1, W);
}

// The fp64 iterative refinement's outer sites (residual SpMM and truncation,
// accumulation of the correction) and its fp32 inner ChebyshevT, built like
// the other forms' phase: plans, uploads and graphs on the given stream,
// which may be a second one while the median iterations run.
struct RefineSetup {
  DevBuf odone, octl;
  std::vector<BCtl> ho;
  std::vector<int> hd;
  std::vector<std::unique_ptr<DevBuf>> bufs;
  SpmmLaunch<double> sp0;
  Batched<SpmmArgs<double>> spB;
  TruncPlan<double> res0, acc0;
  TruncBatch<double> resB, accB;
  BatchCheb<float> bc;
  void setup(std::vector<SolveRun*>& run, const lrc_opts& o, const std::vector<double>& c,
             const std::vector<double>& dc, const std::vector<double>& tgt, bool eager,
             hipStream_t s) {
    const int nb = int(run.size());
    odone.alloc(size_t(nb) * sizeof(int));
    octl.alloc(size_t(nb) * sizeof(BCtl));
    ho.assign(nb, BCtl{});
    hd.assign(nb, 0);
    for (int j = 0; j < nb; ++j) {
      ho[j] = BCtl{};
      ho[j].norm = run[j]->c64->norm.as<double>();
      ho[j].target = tgt[j];
      ho[j].max_iter = 1 << 30;
      ho[j].stall_limit = 1 << 30;
    }
    LRC_HIP(hipMemcpyAsync(octl.p, ho.data(), size_t(nb) * sizeof(BCtl), hipMemcpyHostToDevice, s));
    LRC_HIP(hipMemcpyAsync(odone.p, hd.data(), size_t(nb) * sizeof(int), hipMemcpyHostToDevice, s));
    auto nbuf = [&]() -> DevBuf& {
      bufs.push_back(std::make_unique<DevBuf>());
      return *bufs.back();
    };
    const int* od = odone.as<int>();
    // outer residual (fp64, truncated at the inner solve's accuracy) and accumulation sites
    {
      std::vector<SpmmLaunch<double>> v;
      std::vector<SpmmArgs<double>> a;
      std::vector<TruncPlan<double>> vr, va;
      for (auto* r : run) {
        Cheb<double>& C = *r->c64;
        v.push_back(C.spmm_plan(C.S.u(), C.S.ld, C.S.r()));
        a.push_back(v.back().a);
        // truncated straight to the inner solve's cap: its first residual
        vr.push_back(C.resid_plan(r->B64, C.norm.as<double>(), r->rhs_tol, r->inner_cap));
        va.push_back(r->accumulate_plan(o));
      }
      sp0 = merge_spmm(v);
      spB = upload_items(a, od, nbuf(), s);
      res0 = merge_plans(vr);
      resB = upload_plans(vr, od, nbuf(), s);
      acc0 = merge_plans(va);
      accB = upload_plans(va, od, nbuf(), s);
    }
    {
      std::vector<Cheb<float>*> items;
      std::vector<const LR<float>*> rhs;
      for (auto* r : run) {
        items.push_back(r->c32.get());
        rhs.push_back(&r->Bin);
      }
      bc.setup(items, rhs, c, dc, run[0]->inner_trunc_tol, std::vector<double>(nb, 0.0),
               o.restart, eager, s, o.recurrence == LRC_CHEB_THREE_TERM);
    }
  }
  void prepare_on(hipStream_t main) { bc.prepare_on(main); }
};

void lockstep(std::vector<SolveRun*>& run, const lrc_opts& o) {
  const int nb = int(run.size());
  LRC_CHECK(nb >= 1, ST_EINVAL, "lockstep: no problems");
  Ctx& cx = *run[0]->P->ctx;
  for (auto* r : run)
    LRC_CHECK(r->P->ctx == run[0]->P->ctx, ST_EINVAL,
              "lrc_solve_batched: all problems must belong to one context");
  const bool eager = o.eager != 0;
  cx.sync();
  OwnStream own;
  hipStream_t s = own.s;
  const auto t_start = std::chrono::steady_clock::now();
  auto since = [&]() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  };
  std::vector<double> c(nb), dc(nb), tgt(nb);
  std::vector<int> mi(nb);
  for (int j = 0; j < nb; ++j) {
    c[j] = run[j]->c;
    dc[j] = run[j]->dc;
    tgt[j] = run[j]->target;
    mi[j] = run[j]->max_iter;
  }
  // The ChebyshevT phase's plans, uploads and graph depend only on buffers
  // and scalars fixed before the median solve: for the fp64 iteration and
  // the fp32-solve form they are built on a second stream while the median
  // iterations run on the GPU, and the graph is then launched on s.
  OwnStream aux;
  std::unique_ptr<BatchDir> bd;
  std::unique_ptr<BatchCheb<double>> bc64;
  std::unique_ptr<RefineSetup> rsu;
  std::vector<Cheb<double>*> items64;
  std::vector<const LR<double>*> rhs64;
  std::vector<double> res_abs;
  auto cheb_setup = [&]() {
    const auto t0 = std::chrono::steady_clock::now();
    if (o.precision == LRC_MIXED_FP32_DIR) {
      bd = std::make_unique<BatchDir>();
      bd->setup(run, o, eager, aux.s);
      bd->prepare_on(s);
    } else if (o.precision == LRC_FP64 && o.solver == LRC_SOLVER_CHEBYSHEV) {
      for (auto* r : run) {
        items64.push_back(r->c64.get());
        rhs64.push_back(&r->B64);
        res_abs.push_back(kResFloor * r->target);
      }
      bc64 = std::make_unique<BatchCheb<double>>();
      bc64->setup(items64, rhs64, c, dc, o.trunc_tol, res_abs, o.restart, eager, aux.s,
                  o.recurrence == LRC_CHEB_THREE_TERM);
      bc64->prepare_on(s);
    } else if (o.precision == LRC_MIXED_FP32 || o.precision == LRC_MIXED_BF16GRAM) {
      rsu = std::make_unique<RefineSetup>();
      rsu->setup(run, o, c, dc, tgt, eager, aux.s);
      rsu->prepare_on(s);
    }
    if (log_on())
      std::fprintf(stderr, "{\"cheb_setup_s\": %.5f}\n",
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
  };
  bool cheb_ready = false;
  // the SpMM tuner times its candidates on an idle GPU: its first call for
  // the iterate's capacity happens here, before the median iterations run
  for (auto* r : run) {
    (void)spmm_config<double>(*r->P->ops, r->cap);
    if (o.precision == LRC_MIXED_FP32 || o.precision == LRC_MIXED_BF16GRAM)
      (void)spmm_config<float>(*r->P->ops, r->cap);
  }
  // 1. median-parameter columns (init LRC_INIT_MEDIAN)
  {
    std::vector<SolveRun*> med;
    for (auto* r : run)
      if (r->jmed >= 0) med.push_back(r);
    if (!med.empty()) {
      MedianBatch mb;
      mb.solve(med, s, eager, true, o.precision != LRC_FP64, [&]() {
        cheb_setup();
        cheb_ready = true;
      });
      LRC_HIP(hipStreamSynchronize(s));
      cx.sync();
    }
  }
  if (!cheb_ready) cheb_setup();
  // judged initial terms: the given guess against the median's, per column
  for (auto* r : run)
    if (r->judged) r->judge_guess();
  const double t_median = since();
  // 2. right-hand sides B = F - L(X0)
  build_rhs(run, o, s);
  const double t_rhs = since();
  // 3. ChebyshevT (fp64), or fp32 ChebyshevT inside fp64 refinement
  // ||B||: from the right-hand side's truncation, or ||F|| when B = F
  std::vector<double> bn(nb);
  for (int j = 0; j < nb; ++j) {
    if (run[j]->P->rank_x0 == 0 || run[j]->newton_point) {
      bn[j] = run[j]->P->fnorm;
    } else {
      LRC_HIP(hipMemcpyAsync(&bn[j], run[j]->c64->norm.as<double>() + 4, 8,
                             hipMemcpyDeviceToHost, s));
    }
  }
  LRC_HIP(hipStreamSynchronize(s));
  if (o.precision == LRC_MIXED_FP32_DIR) {
    bd->solve(bn);
    for (int j = 0; j < nb; ++j) {
      run[j]->iters = bd->hctl[j].iters;
      run[j]->papp = bd->hctl[j].iters;
      run[j]->conv = bd->hctl[j].state == 1;
      run[j]->last = bd->hctl[j].last;
      run[j]->flags |= read_info(run[j]->c64->tr.st.info, s);
      run[j]->flags |= read_info(run[j]->c32->tr.st.info, s);
    }
  } else if (o.precision == LRC_FP64 && o.solver == LRC_SOLVER_GMREST) {
    for (int j = 0; j < nb; ++j) {
      gmrest_solve(*run[j], o, s);
      run[j]->flags |= read_info(run[j]->c64->tr.st.info, s);
    }
  } else if (o.precision == LRC_FP64) {
    BatchCheb<double>& bc = *bc64;
    bc.run(std::vector<int>(nb, 0), tgt, mi, 1 << 30, &bn);
    for (int j = 0; j < nb; ++j) {
      run[j]->iters = bc.hctl[j].iters;
      run[j]->papp = bc.hctl[j].iters;
      run[j]->conv = bc.hctl[j].state == 1;
      run[j]->last = bc.hctl[j].last;
      run[j]->flags |= read_info(run[j]->c64->tr.st.info, s);
    }
  } else {
    RefineSetup& R = *rsu;
    DevBuf& odone = R.odone;
    DevBuf& octl = R.octl;
    std::vector<BCtl>& ho = R.ho;
    std::vector<int>& hd = R.hd;
    const SpmmLaunch<double>& sp0 = R.sp0;
    const Batched<SpmmArgs<double>>& spB = R.spB;
    const TruncPlan<double>& res0 = R.res0;
    const TruncPlan<double>& acc0 = R.acc0;
    const TruncBatch<double>& resB = R.resB;
    const TruncBatch<double>& accB = R.accB;
    BatchCheb<float>& bc = R.bc;
    const double itol = o.inner_tol > 0 ? o.inner_tol : 1e-3;
    while (true) {
      enqueue_spmm(sp0, spB, s);
      enqueue_trunc(res0, resB, s);
      launch_batch_check(octl.as<BCtl>(), odone.as<int>(), nb, 0, s);
      LRC_HIP(hipMemcpyAsync(ho.data(), octl.p, size_t(nb) * sizeof(BCtl), hipMemcpyDeviceToHost, s));
      LRC_HIP(hipStreamSynchronize(s));
      // refinement and iteration limits are the host's to apply
      bool any = false;
      std::vector<int> idone(nb, 1), imax(nb, 0);
      std::vector<double> itgt(nb, 0.0);
      for (int j = 0; j < nb; ++j) {
        SolveRun& r = *run[j];
        if (hd[j]) continue;
        r.last = ho[j].last;
        log_line("refine64", r.refinements, r.last, r.P->fnorm);
        if (ho[j].state != 0) {
          r.conv = ho[j].state == 1;
          hd[j] = 1;
        } else if (r.refinements >= r.refine_max || r.iters >= r.max_iter) {
          hd[j] = 1;
        } else {
          // inner solve: to its relative tolerance, to half the outer target,
          // or until the fp32 residual stagnates at its rounding floor
          idone[j] = 0;
          imax[j] = r.max_iter - r.iters;
          itgt[j] = std::max(itol * r.last, 0.5 * r.target);
          any = true;
        }
      }
      LRC_HIP(hipMemcpyAsync(odone.p, hd.data(), size_t(nb) * sizeof(int), hipMemcpyHostToDevice,
                             s));
      if (!any) break;
      std::vector<double> r0n(nb, 0.0);
      for (int j = 0; j < nb; ++j) {
        r0n[j] = run[j]->last;
        if (!idone[j]) cast_lr<double, float>(run[j]->c64->R, run[j]->Bin, s);
      }
      bc.run(idone, itgt, imax, 2, &r0n);
      for (int j = 0; j < nb; ++j) {
        if (idone[j]) continue;
        run[j]->iters += bc.hctl[j].iters;
        run[j]->papp += bc.hctl[j].iters;
        ++run[j]->refinements;
        run[j]->accumulate_plan_inputs(s);
      }
      enqueue_trunc(acc0, accB, s);
    }
    for (int j = 0; j < nb; ++j) {
      run[j]->flags |= read_info(run[j]->c64->tr.st.info, s);
      run[j]->flags |= read_info(run[j]->c32->tr.st.info, s);
    }
  }
  LRC_HIP(hipStreamSynchronize(s));
  if (log_on())
    std::fprintf(stderr,
                 "{\"lockstep_s\": {\"items\": %d, \"median\": %.4f, \"rhs\": %.4f, \"cheb\": %.4f}}\n",
                 nb, t_median, t_rhs - t_median, since() - t_rhs);
}

std::vector<lrc_status> solve_batched(const std::vector<Prob*>& probs, const lrc_opts& o,
                                      lrc_info* infos) {
  const int nb = int(probs.size());
  LRC_CHECK(nb >= 1, ST_EINVAL, "lrc_solve_batched: no problems");
  std::vector<SolveRun*> ptr(nb);
  for (int j = 0; j < nb; ++j) {
    Prob& P = *probs[j];
    if (!P.run) P.run = std::make_unique<SolveRun>();
    P.run->prepare(P, o, 0, nullptr, nullptr, nullptr);
    ptr[j] = P.run.get();
  }
  lockstep(ptr, o);
  std::vector<lrc_status> st(nb);
  for (int j = 0; j < nb; ++j) st[j] = ptr[j]->finish(o, infos ? infos + j : nullptr);
  return st;
}

}  // namespace lrc
