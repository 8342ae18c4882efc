// Lockstep solves of several problems (parameter subsets, each with its own
// linearisation point): every step of the ChebyshevT iteration is one launch
// whose grid's z dimension runs over the problems, per-problem arguments come
// from device arrays built once per call site, finished problems are skipped
// through device-side done flags, and one restart cycle is captured into a
// HIP graph that the host replays until every problem has stopped.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>

#include "solver.hpp"

namespace lrc {

namespace {

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
  for (const auto& x : v) {
    LRC_CHECK(x.cpl == l.cpl && x.lpr == l.lpr, ST_EINVAL,
              "batched solve: problems differ in the factor capacity");
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
         a.asm_ptr == b.asm_ptr && a.asm_src == b.asm_src;
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
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    const hipError_t q = hipStreamIsCapturing(s, &cs);
    const hipError_t e = hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) {
      char msg[256];
      std::snprintf(msg, sizeof msg,
                    "hipStreamBeginCapture: %s (stream %p, is-capturing query %s, status %d)",
                    hipGetErrorString(e), static_cast<void*>(s), hipGetErrorName(q), int(cs));
      throw Error(ST_EDEVICE, msg);
    }
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
  bool shared_prec = true;
  PrecItem<T> prec0{};
  Batched<PrecItem<T>> precB;
  std::vector<Batched<PrecItem<T>>> precOne;   // per item when the structures differ
  TruncPlan<T> resid0, dstart0, supd0;
  TruncBatch<T> residB, dstartB, supdB;
  std::vector<TruncPlan<T>> dstep0;
  std::vector<TruncBatch<T>> dstepB;
  GraphExec graph;

  DevBuf& newbuf() {
    bufs.push_back(std::make_unique<DevBuf>());
    return *bufs.back();
  }

  void setup(const std::vector<Cheb<T>*>& items, const std::vector<const LR<T>*>& rhs,
             const std::vector<double>& c_, const std::vector<double>& dc_, double tol,
             int cycle_, hipStream_t s_) {
    it = items;
    B = rhs;
    c = c_;
    dc = dc_;
    cycle = cycle_;
    s = s_;
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
    // preconditioner: one batched apply when all structures agree
    {
      std::vector<PrecItem<T>> a;
      for (auto* x : it) a.push_back(x->prec_item());
      prec0 = a[0];
      for (auto* x : it)
        if (!same_structure(x->P->prec->F, it[0]->P->prec->F)) shared_prec = false;
      DevBuf& pb = newbuf();
      precB = upload_items(a, dn, pb, s);
      if (!shared_prec)
        for (int j = 0; j < nb; ++j) {
          Batched<PrecItem<T>> b;
          b.dev = pb.as<PrecItem<T>>() + j;
          b.done = dn + j;
          b.n = 1;
          precOne.push_back(b);
        }
    }
    auto site = [&](auto make, TruncPlan<T>& p0, TruncBatch<T>& b) {
      std::vector<TruncPlan<T>> v;
      for (int j = 0; j < nb; ++j) v.push_back(make(j));
      p0 = merge_plans(v);
      b = upload_plans(v, dn, newbuf(), s);
    };
    site([&](int j) { return it[j]->resid_plan(*B[j], it[j]->norm.template as<double>(), tol); },
         resid0, residB);
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

  void precond() {
    if (shared_prec) {
      const Prec& P0 = *it[0]->P->prec;
      enqueue_prec_apply<T>(P0.dev<T>(), P0.fwd, P0.bwd, prec0, precB, it[0]->cap,
                            ld_for(it[0]->cap), s);
    } else {
      for (int j = 0; j < nb; ++j) {
        const Prec& Pj = *it[j]->P->prec;
        enqueue_prec_apply<T>(Pj.dev<T>(), Pj.fwd, Pj.bwd, it[j]->prec_item(), precOne[j],
                              it[j]->cap, ld_for(it[j]->cap), s);
      }
    }
  }

  void resid(int after_update) {
    enqueue_spmm(spmm0, spmmB, s);
    enqueue_trunc(resid0, residB, s);
    launch_batch_check(ctl.as<BCtl>(), done.as<int>(), nb, after_update, s);
  }

  void cycle_steps() {
    precond();
    enqueue_trunc(dstart0, dstartB, s);
    for (int k = 0; k < cycle; ++k) {
      enqueue_trunc(supd0, supdB, s);
      resid(1);
      if (k + 1 == cycle) break;
      precond();
      enqueue_trunc(dstep0[k], dstepB[k], s);
    }
  }

  void capture() {
    graph.reset();
    CaptureGuard cg(s);
    cycle_steps();
    graph.g = cg.end();
    LRC_HIP(hipGraphInstantiate(&graph.x, graph.g, nullptr, nullptr, 0));
  }

  // Runs the lockstep iteration.  Items with init_done[j] set do nothing.
  // target/max_iter/stall_limit per item; returns the final control states.
  void run(const std::vector<int>& init_done, const std::vector<double>& target,
           const std::vector<int>& max_iter, int stall_limit) {
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
    }
    LRC_HIP(hipMemcpyAsync(ctl.p, hctl.data(), size_t(nb) * sizeof(BCtl), hipMemcpyHostToDevice,
                           s));
    LRC_HIP(hipMemcpyAsync(done.p, init_done.data(), size_t(nb) * sizeof(int),
                           hipMemcpyHostToDevice, s));
    resid(0);
    if (!graph.x) capture();
    while (true) {
      LRC_HIP(hipMemcpyAsync(hctl.data(), ctl.p, size_t(nb) * sizeof(BCtl),
                             hipMemcpyDeviceToHost, s));
      LRC_HIP(hipStreamSynchronize(s));
      bool all = true;
      for (const auto& h : hctl) all = all && h.state != 0;
      if (all) break;
      ProfScope ps(kcls(K_GRAPH, is_f32<T>()), s);
      LRC_HIP(hipGraphLaunch(graph.x, s));
    }
    if (log_on())
      for (int j = 0; j < nb; ++j)
        std::fprintf(stderr,
                     "{\"batch\": %d, \"item\": %d, \"iters\": %d, \"norm\": %.6e, \"state\": %d}\n",
                     int(sizeof(T)), j, hctl[j].iters, hctl[j].last, hctl[j].state);
  }

  static bool log_on() {
    static const bool on = std::getenv("LRC_LOG") != nullptr;
    return on;
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

}  // namespace

std::vector<lrc_status> solve_batched(const std::vector<Prob*>& probs, const lrc_opts& o,
                                      lrc_info* infos) {
  const int nb = int(probs.size());
  LRC_CHECK(nb >= 1, ST_EINVAL, "lrc_solve_batched: no problems");
  LRC_CHECK(o.restart >= 1 && o.restart <= 64, ST_EINVAL,
            "lrc_solve_batched: restart must be in [1, 64] (one cycle is one graph)");
  Ctx& cx = *probs[0]->ctx;
  for (auto* P : probs)
    LRC_CHECK(P->ctx == probs[0]->ctx, ST_EINVAL,
              "lrc_solve_batched: all problems must belong to one context");
  std::vector<SolveRun> run(nb);
  for (int j = 0; j < nb; ++j) run[j].prepare(*probs[j], o, 0, nullptr, nullptr, nullptr);
  for (auto& r : run)
    if (o.precision != LRC_FP64) r.alloc_mixed();
  cx.sync();
  OwnStream own;
  hipStream_t s = own.s;
  std::vector<double> c(nb), dc(nb), tgt(nb);
  std::vector<int> mi(nb);
  for (int j = 0; j < nb; ++j) {
    c[j] = std::max(run[j].c, 1e-12 * run[j].dc);
    dc[j] = run[j].dc;
    tgt[j] = run[j].target;
    mi[j] = run[j].max_iter;
  }
  if (o.precision == LRC_FP64) {
    BatchCheb<double> bc;
    std::vector<Cheb<double>*> items;
    std::vector<const LR<double>*> rhs;
    for (auto& r : run) {
      items.push_back(r.c64.get());
      rhs.push_back(&r.B64);
    }
    bc.setup(items, rhs, c, dc, o.trunc_tol, o.restart, s);
    bc.run(std::vector<int>(nb, 0), tgt, mi, 1 << 30);
    for (int j = 0; j < nb; ++j) {
      run[j].iters = bc.hctl[j].iters;
      run[j].papp = bc.hctl[j].iters;
      run[j].conv = bc.hctl[j].state == 1;
      run[j].last = bc.hctl[j].last;
      run[j].flags |= read_info(run[j].c64->tr.st.info, s);
    }
  } else {
    // fp32 inner ChebyshevT in lockstep, wrapped in lockstep fp64 refinement
    DevBuf odone(size_t(nb) * sizeof(int)), octl(size_t(nb) * sizeof(BCtl));
    std::vector<BCtl> ho(nb);
    std::vector<int> hd(nb, 0);
    for (int j = 0; j < nb; ++j) {
      ho[j] = BCtl{};
      ho[j].norm = run[j].c64->norm.as<double>();
      ho[j].target = tgt[j];
      ho[j].max_iter = 1 << 30;
      ho[j].stall_limit = 1 << 30;
    }
    LRC_HIP(hipMemcpyAsync(octl.p, ho.data(), size_t(nb) * sizeof(BCtl), hipMemcpyHostToDevice, s));
    LRC_HIP(hipMemcpyAsync(odone.p, hd.data(), size_t(nb) * sizeof(int), hipMemcpyHostToDevice, s));
    std::vector<std::unique_ptr<DevBuf>> bufs;
    auto nbuf = [&]() -> DevBuf& {
      bufs.push_back(std::make_unique<DevBuf>());
      return *bufs.back();
    };
    const int* od = odone.as<int>();
    // outer residual (fp64, truncated at the inner solve's accuracy) and accumulation sites
    SpmmLaunch<double> sp0;
    Batched<SpmmArgs<double>> spB;
    TruncPlan<double> res0, acc0;
    TruncBatch<double> resB, accB;
    {
      std::vector<SpmmLaunch<double>> v;
      std::vector<SpmmArgs<double>> a;
      std::vector<TruncPlan<double>> vr, va;
      for (auto& r : run) {
        Cheb<double>& C = *r.c64;
        v.push_back(C.spmm_plan(C.S.u(), C.S.ld, C.S.r()));
        a.push_back(v.back().a);
        vr.push_back(C.resid_plan(r.B64, C.norm.as<double>(), r.rhs_tol));
        va.push_back(r.accumulate_plan(o));
      }
      sp0 = merge_spmm(v);
      spB = upload_items(a, od, nbuf(), s);
      res0 = merge_plans(vr);
      resB = upload_plans(vr, od, nbuf(), s);
      acc0 = merge_plans(va);
      accB = upload_plans(va, od, nbuf(), s);
    }
    BatchCheb<float> bc;
    {
      std::vector<Cheb<float>*> items;
      std::vector<const LR<float>*> rhs;
      for (auto& r : run) {
        items.push_back(r.c32.get());
        rhs.push_back(&r.Bin);
      }
      bc.setup(items, rhs, c, dc, o.trunc_tol, o.restart, s);
    }
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
        SolveRun& r = run[j];
        if (ho[j].state == 0 && hd[j] == 0) {
          r.last = ho[j].last;
          log_line("refine64", r.refinements, r.last, r.P->fnorm);
          if (r.refinements >= r.refine_max || r.iters >= r.max_iter) {
            hd[j] = 1;
            continue;
          }
          idone[j] = 0;
          imax[j] = r.max_iter - r.iters;
          itgt[j] = std::max(itol * r.last, 0.5 * r.target);
          any = true;
        } else if (hd[j] == 0) {
          r.last = ho[j].last;
          r.conv = ho[j].state == 1;
          hd[j] = 1;
        }
      }
      LRC_HIP(hipMemcpyAsync(odone.p, hd.data(), size_t(nb) * sizeof(int), hipMemcpyHostToDevice,
                             s));
      if (!any) break;
      for (int j = 0; j < nb; ++j)
        if (!idone[j]) cast_lr<double, float>(run[j].c64->R, run[j].Bin, s);
      bc.run(idone, itgt, imax, 2);
      for (int j = 0; j < nb; ++j) {
        if (idone[j]) continue;
        run[j].iters += bc.hctl[j].iters;
        run[j].papp += bc.hctl[j].iters;
        ++run[j].refinements;
        run[j].accumulate_plan_inputs(s);
      }
      enqueue_trunc(acc0, accB, s);
    }
    for (int j = 0; j < nb; ++j) {
      run[j].flags |= read_info(run[j].c64->tr.st.info, s);
      run[j].flags |= read_info(run[j].c32->tr.st.info, s);
    }
  }
  LRC_HIP(hipStreamSynchronize(s));
  std::vector<lrc_status> st(nb);
  for (int j = 0; j < nb; ++j) st[j] = run[j].finish(o, infos ? infos + j : nullptr);
  return st;
}

}  // namespace lrc
