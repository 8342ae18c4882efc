#include "prof.hpp"

#include <algorithm>
#include <string>

namespace lrc {

const char* kclass_name(int c) {
  static const char* names[K_NBASE] = {"spmm", "gram", "gram_reduce", "chol", "tsmm", "jacobi",
                                       "jacobi_replay", "small_gemm", "select", "prec_gather",
                                       "prec_product", "residual", "vector", "qrcp", "mlp",
                                       "graph", "gram_bf16"};
  static std::vector<std::string> full;
  if (full.empty())
    for (int k = 0; k < K_COUNT; ++k)
      full.push_back(std::string(names[k / 2]) + ((k & 1) ? ".f32" : ".f64"));
  return (c >= 0 && c < K_COUNT) ? full[c].c_str() : "?";
}

Work combine_work(const std::vector<Work>& items) {
  Work w;
  std::vector<std::pair<size_t, size_t>> span;   // group range of each item
  std::vector<std::function<double(const std::vector<double>&)>> fs;
  for (const auto& it : items) {
    if (!it.valid()) return Work();
    w.bytes = it.bytes;
    span.emplace_back(w.groups.size(), it.groups.size());
    w.groups.insert(w.groups.end(), it.groups.begin(), it.groups.end());
    fs.push_back(it.f);
  }
  if (fs.empty()) return Work();
  w.f = [span, fs](const std::vector<double>& v) {
    double t = 0.0;
    for (size_t i = 0; i < fs.size(); ++i)
      t += fs[i](std::vector<double>(v.begin() + span[i].first,
                                     v.begin() + span[i].first + span[i].second));
    return t;
  };
  return w;
}

Profiler& profiler() {
  static Profiler p;
  return p;
}

void Profiler::clear() {
  for (auto& v : ev) {
    for (auto& l : v) {
      (void)hipEventDestroy(l.e0);
      (void)hipEventDestroy(l.e1);
    }
    v.clear();
  }
  log_used = 0;
}

void Profiler::read(double* ms, int* count, double* work, int* unit) {
  std::vector<int> snap(static_cast<size_t>(log_used));
  if (log_used > 0) {
    (void)hipDeviceSynchronize();
    (void)hipMemcpy(snap.data(), log_dev, sizeof(int) * size_t(log_used), hipMemcpyDeviceToHost);
  }
  for (int k = 0; k < K_COUNT; ++k) {
    double t = 0.0, wsum = 0.0;
    int u = 0;
    for (auto& l : ev[k]) {
      (void)hipEventSynchronize(l.e1);
      float x = 0.0f;
      if (hipEventElapsedTime(&x, l.e0, l.e1) == hipSuccess) t += x;
      if (l.w.valid() && !l.slots.empty()) {
        std::vector<double> wv;
        for (size_t g = 0; g < l.w.groups.size(); ++g) {
          double sum = 0.0;
          for (size_t j = 0; j < l.w.groups[g].size(); ++j) {
            const int sl = l.slots[g][j];
            sum += sl >= 0 ? double(snap[size_t(sl)]) : double(l.w.groups[g][j].c);
          }
          wv.push_back(sum);
        }
        wsum += l.w.f(wv);
        u = l.w.bytes ? 1 : 2;
      }
    }
    if (ms) ms[k] = t;
    if (count) count[k] = int(ev[k].size());
    if (work) work[k] = wsum;
    if (unit) unit[k] = u;
  }
}

ProfScope::ProfScope(int cls, hipStream_t s_, Work w) : s(s_) {
  Profiler& p = profiler();
  if (p.mode == 0 || p.suspended > 0 || cls < 0 || cls >= K_COUNT) return;
  Profiler::Launch l;
  if (p.mode == 2 && w.valid()) {
    for (auto& g : w.groups) {
      std::vector<int> sl;
      for (auto& t : g) {
        if (!t.dev) {
          sl.push_back(-1);
          continue;
        }
        if (p.log_used >= p.log_cap) {
          const int cap = std::max(1 << 16, 2 * p.log_cap);
          int* nd = nullptr;
          if (hipMalloc(&nd, sizeof(int) * size_t(cap)) != hipSuccess) return;
          if (p.log_dev) {
            (void)hipDeviceSynchronize();
            (void)hipMemcpy(nd, p.log_dev, sizeof(int) * size_t(p.log_used),
                            hipMemcpyDeviceToDevice);
            (void)hipFree(p.log_dev);
          }
          p.log_dev = nd;
          p.log_cap = cap;
        }
        (void)hipMemcpyAsync(p.log_dev + p.log_used, t.dev, sizeof(int), hipMemcpyDeviceToDevice,
                             s);
        sl.push_back(p.log_used++);
      }
      l.slots.push_back(sl);
    }
    l.w = std::move(w);
  }
  if (hipEventCreate(&l.e0) != hipSuccess) return;
  if (hipEventCreate(&l.e1) != hipSuccess) {
    (void)hipEventDestroy(l.e0);
    return;
  }
  (void)hipEventRecord(l.e0, s);
  e1 = l.e1;
  p.ev[cls].push_back(std::move(l));
}

ProfScope::~ProfScope() {
  if (e1) (void)hipEventRecord(e1, s);
}

}  // namespace lrc
