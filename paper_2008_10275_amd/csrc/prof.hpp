// Opt-in timing of kernel classes with HIP events (recorded on the stream each
// kernel is launched on).  Off by default; when on, every launch of a class is
// bracketed by an event pair and the durations are summed on request.
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

namespace lrc {

enum KClass {
  K_SPMM = 0, K_GRAM, K_GRAM_REDUCE, K_CHOL, K_TSMM, K_JACOBI, K_REPLAY, K_SMALL_GEMM,
  K_SELECT, K_PREC_GATHER, K_PREC_PRODUCT, K_RESIDUAL, K_VECTOR, K_COUNT
};

inline const char* kclass_name(int k) {
  static const char* names[K_COUNT] = {"spmm", "gram", "gram_reduce", "chol", "tsmm", "jacobi",
                                       "jacobi_replay", "small_gemm", "select", "prec_gather",
                                       "prec_product", "residual_fp64", "vector"};
  return (k >= 0 && k < K_COUNT) ? names[k] : "?";
}

struct Profiler {
  bool on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[K_COUNT];
  void clear();
  // durations in ms and launch counts per class (synchronises the events)
  void read(double* ms, int* count);
};
Profiler& profiler();

struct ProfScope {
  KClass k;
  hipStream_t s;
  hipEvent_t e1 = nullptr;
  ProfScope(KClass k_, hipStream_t s_);
  ~ProfScope();
};

}  // namespace lrc
