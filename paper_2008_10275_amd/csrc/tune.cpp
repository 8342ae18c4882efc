// Autotuner of the fused CSR SpMM launch shape.  For one operator set, factor
// width and precision it times every candidate (columns per lane, waves per
// workgroup, grid cap) on the device with HIP events at the width and at half
// and a quarter of it, and keeps the fastest in total;
// results are cached in the context per (precision, n, q, nnz, width), so
// operator sets of the same shape (e.g. the subsets of one Newton step) share
// one tuning.  The arithmetic of every row is the same for all shapes (one
// lane group sums the row's nonzeros in order), so the choice never changes
// results.
#include <algorithm>

#include "solver.hpp"

namespace lrc {

namespace {

template <class T> const std::vector<DevCsr<T>>& dev_ops(const Ops& o);
template <> const std::vector<DevCsr<double>>& dev_ops<double>(const Ops& o) { return o.d64; }
template <> const std::vector<DevCsr<float>>& dev_ops<float>(const Ops& o) { return o.d32; }

std::array<int64_t, 5> key_of(const Ops& o, int rcap, int es) {
  int64_t nnz = 0;
  for (const auto& c : o.d64) nnz += c.nnz;
  return {es, o.n, o.q, nnz, rcap};
}

}  // namespace

template <class T>
SpmmTuneResult tune_spmm(const Ops& o, int rcap) {
  LRC_CHECK(rcap >= 1 && rcap <= 64 * 8, ST_EINVAL, "spmm tune: bad width");
  Ctx& cx = *o.ctx;
  hipStream_t s = cx.stream;
  const int ld = round_up(rcap, 8);
  DevBuf U(size_t(o.n) * ld * sizeof(T)), W(size_t(o.q) * o.n * ld * sizeof(T));
  LRC_HIP(hipMemsetAsync(U.p, 0, U.bytes, s));
  T* Wp[kMaxOps];
  for (int i = 0; i < o.q; ++i) Wp[i] = W.as<T>() + size_t(i) * o.n * ld;
  SpmmCfg def;
  std::vector<SpmmCfg> cand{def};
  constexpr int VW = 16 / int(sizeof(T));
  for (int cpl : {1, 2, 4, 8}) {
    // shapes are 16-byte vectors per lane: skip requests that map to the same
    if (cpl > 1 && cpl < VW) continue;
    if (ceil_div(ceil_div(rcap, VW), std::max(1, cpl / VW)) > 64 || (cpl > VW && cpl > rcap)) continue;
    for (int waves : {2, 4, 8})
      for (int mb : {2048, 8192, 32768}) cand.push_back(SpmmCfg{cpl, waves, mb});
  }
  hipEvent_t e0, e1;
  LRC_HIP(hipEventCreate(&e0));
  LRC_HIP(hipEventCreate(&e1));
  profiler().suspended++;
  SpmmTuneResult res;
  res.best_us = 1e30;
  // A launch planned for capacity rcap runs at the device width, which sits
  // anywhere below it (the rank of the iterate grows towards the solution's):
  // every shape is scored by its summed time at rcap / 4, rcap / 2 and rcap.
  std::vector<int> widths{rcap};
  for (int w : {rcap / 2, rcap / 4})
    if (w >= 1 && w != widths.back()) widths.push_back(w);
  auto time_us = [&](const SpmmCfg& cfg, int w) {
    const SpmmLaunch<T> l =
        make_spmm<T>(dev_ops<T>(o).data(), o.q, U.as<T>(), ld, nullptr, w, rcap, Wp, ld, cfg,
                     true);
    enqueue_spmm(l, Batched<SpmmArgs<T>>(), s);   // warm-up
    constexpr int reps = 5;
    LRC_HIP(hipEventRecord(e0, s));
    for (int k = 0; k < reps; ++k) enqueue_spmm(l, Batched<SpmmArgs<T>>(), s);
    LRC_HIP(hipEventRecord(e1, s));
    LRC_HIP(hipEventSynchronize(e1));
    float ms = 0.0f;
    LRC_HIP(hipEventElapsedTime(&ms, e0, e1));
    return 1e3 * ms / reps;
  };
  try {
    double best_score = 1e30;
    for (size_t c = 0; c < cand.size(); ++c) {
      const double us = time_us(cand[c], rcap);
      double score = us;
      for (size_t w = 1; w < widths.size(); ++w) score += time_us(cand[c], widths[w]);
      (void)us;
      if (c == 0) res.default_us = score;
      if (score < best_score) {
        best_score = score;
        res.best_us = score;
        res.best = cand[c];
        if (res.best.cpl == 0) res.best.cpl = sizeof(T) == 8 ? 2 : 4;
      }
      ++res.tried;
    }
  } catch (...) {
    profiler().suspended--;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    throw;
  }
  profiler().suspended--;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  cx.spmm_cache[key_of(o, rcap, sizeof(T))] = res.best;
  return res;
}

template <class T>
SpmmCfg spmm_config(const Ops& o, int rcap) {
  const auto k = key_of(o, rcap, sizeof(T));
  auto it = o.ctx->spmm_cache.find(k);
  if (it != o.ctx->spmm_cache.end()) return it->second;
  return tune_spmm<T>(o, rcap).best;
}

template SpmmTuneResult tune_spmm<double>(const Ops&, int);
template SpmmTuneResult tune_spmm<float>(const Ops&, int);
template SpmmCfg spmm_config<double>(const Ops&, int);
template SpmmCfg spmm_config<float>(const Ops&, int);

}  // namespace lrc
