// Opt-in timing of kernel classes with HIP events recorded on the stream each
// kernel is launched on.  Off by default.  Mode 1 brackets every launch of a
// class with an event pair; mode 2 additionally snapshots, before the events,
// the device-resident widths the launch reads (one 4-byte device copy each),
// so that the algorithmic work of every launch (bytes or flops, from a model
// written next to the launch) can be totalled afterwards.
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <vector>

namespace lrc {

enum KClass {
  K_SPMM = 0, K_GRAM, K_GRAM_REDUCE, K_CHOL, K_TSMM, K_JACOBI, K_REPLAY, K_SMALL_GEMM,
  K_SELECT, K_PREC_GATHER, K_PREC_PRODUCT, K_RESIDUAL, K_VECTOR, K_QRCP, K_MLP, K_GRAPH,
  K_GRAM_BF16, K_NBASE
};
// class index = base * 2 + (fp32 ? 1 : 0)
constexpr int K_COUNT = 2 * K_NBASE;
inline int kcls(KClass k, bool f32) { return 2 * int(k) + (f32 ? 1 : 0); }
const char* kclass_name(int c);

// One width the launch reads: the device int at `dev` when non-null, else `c`.
struct WTerm {
  const int* dev;
  int c;
};
// Work model of a launch: widths w_g = sum of the terms of group g; the model
// maps them to algorithmic work (unit: bytes if `bytes`, else flops).
struct Work {
  bool bytes = true;
  std::vector<std::vector<WTerm>> groups;
  std::function<double(const std::vector<double>&)> f;
  bool valid() const { return bool(f); }
};

// Work of a batched launch: the sum of its items' models.
Work combine_work(const std::vector<Work>& items);

struct Profiler {
  int mode = 0;   // 0 off, 1 events, 2 events + work
  int suspended = 0;   // > 0 while a stream is being captured into a graph
  struct Launch {
    hipEvent_t e0, e1;
    Work w;
    std::vector<std::vector<int>> slots;   // log slot of each device term (-1 const)
  };
  std::vector<Launch> ev[K_COUNT];
  int* log_dev = nullptr;     // snapshot slots on the device
  int log_cap = 0, log_used = 0;
  void clear();
  // per class: summed ms, launches, summed algorithmic work and its unit
  // (0 none, 1 bytes, 2 flops); synchronises the recorded events
  void read(double* ms, int* count, double* work, int* unit);
};
Profiler& profiler();

struct ProfScope {
  hipEvent_t e1 = nullptr;
  hipStream_t s;
  ProfScope(int cls, hipStream_t s_, Work w = Work());
  ~ProfScope();
};

template <class T> inline bool is_f32() { return sizeof(T) == 4; }

}  // namespace lrc
