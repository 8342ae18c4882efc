#include "prof.hpp"

namespace lrc {

Profiler& profiler() {
  static Profiler p;
  return p;
}

void Profiler::clear() {
  for (auto& v : ev) {
    for (auto& pr : v) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
    v.clear();
  }
}

void Profiler::read(double* ms, int* count) {
  for (int k = 0; k < K_COUNT; ++k) {
    double t = 0.0;
    for (auto& pr : ev[k]) {
      (void)hipEventSynchronize(pr.second);
      float x = 0.0f;
      if (hipEventElapsedTime(&x, pr.first, pr.second) == hipSuccess) t += x;
    }
    if (ms) ms[k] = t;
    if (count) count[k] = int(ev[k].size());
  }
}

ProfScope::ProfScope(KClass k_, hipStream_t s_) : k(k_), s(s_) {
  Profiler& p = profiler();
  if (!p.on) return;
  hipEvent_t e0;
  if (hipEventCreate(&e0) != hipSuccess) return;
  if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); e1 = nullptr; return; }
  (void)hipEventRecord(e0, s);
  p.ev[k].push_back({e0, e1});
}

ProfScope::~ProfScope() {
  if (e1) (void)hipEventRecord(e1, s);
}

}  // namespace lrc
