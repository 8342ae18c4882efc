// Allocation-free variant of the device truncation (lrc_truncate_noalloc_dev).
//
// The truncation needs device scratch beyond its inputs and outputs: the
// Gram partial sums, the first CholeskyQR pass's factors, the k x k arena of
// the Cholesky / QR / Jacobi stages and the rotation log.  lrc_truncate_dev
// allocates it per call; this entry point carves it from one fixed array in
// the library's code object instead, so that it calls no hipMalloc or hipFree
// and no allocating library routine.  The array lives once per device until
// the process ends; its device address is looked up once per device at
// lrc_create (hipGetSymbolAddress with that device current) and kept in a
// per-device table: host code never passes the array's own name to a kernel.
#include <hip/hip_runtime.h>

#include <cstring>
#include <mutex>

#include "handles.hpp"
#include "prof.hpp"

static constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB per device
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace lrc {
namespace {

constexpr size_t kHeader = 4096;                     // c, s and small outputs
constexpr int kMaxDevices = 64;

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

}  // namespace

void noalloc_init_device(int device) {
  LRC_CHECK(device >= 0 && device < kMaxDevices, ST_EINVAL, "noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (g_scratch[device]) return;
  void* p = nullptr;
  LRC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
  LRC_CHECK(p != nullptr, ST_EDEVICE, "noalloc: scratch symbol has no device address");
  g_scratch[device] = p;
}

static unsigned char* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (device < 0 || device >= kMaxDevices) return nullptr;
  return static_cast<unsigned char*>(g_scratch[device]);
}

}  // namespace lrc

using namespace lrc;

extern "C" lrc_status lrc_truncate_noalloc_dev(lrc_ctx ctx, int dtype, int64_t n, int64_t m,
                                               int k, const void* A, int lda, const double* c,
                                               const void* B, int ldb, int rank_cap, double tol,
                                               void* U, int ldu, double* s, void* V, int ldv,
                                               int* rank) {
  if (!ctx) return LRC_EINVAL;
  return guarded(&ctx->c, [&]() -> lrc_status {
    LRC_CHECK(dtype == 0 || dtype == 1, ST_EINVAL, "truncate_noalloc: dtype must be 0 or 1");
    LRC_CHECK(n >= 1 && m >= 1 && k >= 1 && k <= kTruncCap, ST_EINVAL,
              "truncate_noalloc: need n, m >= 1 and 1 <= k <= 128");
    LRC_CHECK(rank_cap >= 1 && rank_cap <= 64 && rank_cap <= ldu && rank_cap <= ldv, ST_EINVAL,
              "truncate_noalloc: rank_cap in [1, 64] and <= ldu, ldv");
    LRC_CHECK(A && B && c && U && V && s && rank && lda >= k && ldb >= k, ST_EINVAL,
              "truncate_noalloc: bad pointers or leading dimensions");
    LRC_CHECK(profiler().mode == 0, ST_EINVAL,
              "truncate_noalloc: kernel timing (lrc_profile_enable) allocates; switch it off");
    const size_t need = dtype == 0 ? trunc_workspace_bytes<double>(n, m)
                                   : trunc_workspace_bytes<float>(n, m);
    LRC_CHECK(need <= kScratchBytes - kHeader, ST_EINVAL,
              "truncate_noalloc: n + m rows need " + std::to_string(need) +
                  " bytes of scratch, more than the fixed " +
                  std::to_string(kScratchBytes - kHeader) +
                  " (n + m <= 32768 always fits)");
    unsigned char* base = scratch_of(ctx->c.device);
    LRC_CHECK(base != nullptr, ST_EINVAL, "truncate_noalloc: scratch not set up for this device");
    hipStream_t st = ctx->c.stream;
    double* cd = reinterpret_cast<double*>(base);          // k <= 128 core weights
    double* sd = cd + kTruncCap;                           // 64 singular values
    double* outs = sd + 64;                                // norm and rank
    int* rk = reinterpret_cast<int*>(outs + 2);
    LRC_HIP(hipMemcpyAsync(cd, c, size_t(k) * sizeof(double), hipMemcpyHostToDevice, st));
    CoreView cv{};
    cv.nb = 1;
    cv.s[0] = cd;
    cv.coef[0] = 1.0;
    cv.wdev[0] = nullptr;
    cv.wconst[0] = k;
    auto run = [&](auto* tag) {
      using T = std::remove_pointer_t<decltype(tag)>;
      Truncator<T> tr;
      tr.bind(base + kHeader, kScratchBytes - kHeader, n, m, st);
      BlockView<T> av = view1<T>(static_cast<const T*>(A), lda, nullptr, k);
      BlockView<T> bv = view1<T>(static_cast<const T*>(B), ldb, nullptr, k);
      tr.run(av, n, bv, m, cv, rank_cap, tol, static_cast<T*>(U), ldu, static_cast<T*>(V), ldv,
             sd, rk, outs, st);
      LRC_HIP(hipMemcpyAsync(rank, rk, sizeof(int), hipMemcpyDeviceToHost, st));
      LRC_HIP(hipStreamSynchronize(st));
      if (*rank > 0)
        LRC_HIP(hipMemcpyAsync(s, sd, size_t(*rank) * sizeof(double), hipMemcpyDeviceToHost, st));
      int flags = 0;
      LRC_HIP(hipMemcpyAsync(&flags, tr.st.info, sizeof(int), hipMemcpyDeviceToHost, st));
      LRC_HIP(hipStreamSynchronize(st));
      if (flags & 2) throw Error(ST_EBREAKDOWN, "truncate_noalloc: Cholesky breakdown");
    };
    if (dtype == 0) run(static_cast<double*>(nullptr));
    else run(static_cast<float*>(nullptr));
    return LRC_OK;
  });
}
