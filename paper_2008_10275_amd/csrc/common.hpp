// Shared host/device definitions of the low-rank ChebyshevT library.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdlib>
#include <stdexcept>
#include <string>
#include <vector>

namespace lrc {

// Error carried from the library internals to the C-ABI boundary.
struct Error : std::runtime_error {
  int code;
  Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

enum : int {
  ST_OK = 0, ST_NOTCONV = 1, ST_EINVAL = -1, ST_ENOMEM = -2, ST_EDEVICE = -3,
  ST_ESINGULAR = -4, ST_EBREAKDOWN = -5, ST_ECALLBACK = -6
};

#define LRC_HIP(call)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (call);                                                             \
    if (e_ != hipSuccess)                                                               \
      throw ::lrc::Error(e_ == hipErrorOutOfMemory ? ::lrc::ST_ENOMEM : ::lrc::ST_EDEVICE, \
                         std::string(#call) + ": " + hipGetErrorString(e_));            \
  } while (0)

#define LRC_CHECK(cond, code, msg)                   \
  do {                                               \
    if (!(cond)) throw ::lrc::Error((code), (msg));  \
  } while (0)

// Owning device buffer (raw bytes).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  explicit DevBuf(size_t b) { alloc(b); }
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) { o.p = nullptr; o.bytes = 0; }
  DevBuf& operator=(DevBuf&& o) noexcept {
    if (this != &o) { release(); p = o.p; bytes = o.bytes; o.p = nullptr; o.bytes = 0; }
    return *this;
  }
  ~DevBuf() { release(); }
  void alloc(size_t b) {
    release();
    if (b == 0) return;
    LRC_HIP(hipMalloc(&p, b));
    bytes = b;
    // debugging aid: LRC_POISON=1 fills fresh buffers with 0xFF bytes (NaN for
    // floating point) so that a read of never-written memory shows up as NaN
    static const bool poison = std::getenv("LRC_POISON") != nullptr;
    if (poison) {
      LRC_HIP(hipMemset(p, 0xFF, b));
      LRC_HIP(hipDeviceSynchronize());
    }
  }
  // grow-only reallocation (contents are not preserved)
  void reserve(size_t b) { if (b > bytes) alloc(b); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
};

template <class T>
inline DevBuf upload(const T* h, size_t count, hipStream_t s) {
  DevBuf b(count * sizeof(T));
  if (count) {
    LRC_HIP(hipMemcpyAsync(b.p, h, count * sizeof(T), hipMemcpyHostToDevice, s));
  }
  return b;
}

template <class T>
inline DevBuf upload(const std::vector<T>& v, hipStream_t s) { return upload(v.data(), v.size(), s); }

__host__ __device__ inline int round_up(int x, int m) { return (x + m - 1) / m * m; }
__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Leading dimension of every tall factor: columns padded to a multiple of 8
// (32 B for float, 64 B for double) so that vector loads stay aligned.
inline int ld_for(int cols) { return round_up(cols < 1 ? 1 : cols, 8); }

// ---------------------------------------------------------------------------
// Views of concatenated low-rank factors, passed to kernels by value.
// A tall operand  [X_0 | X_1 | ... ]  (rows x sum(width_b)) is a list of column
// blocks; a block's width is either a constant or read from device memory
// (the rank of a low-rank object that only the device knows).  Optional row
// scaling (diagonal D_i applied to the rows of a right factor).
constexpr int kMaxBlocks = 16;

template <class T>
struct BlockView {
  const T* ptr[kMaxBlocks];
  const double* rowscale[kMaxBlocks];
  const int* wdev[kMaxBlocks];
  int wconst[kMaxBlocks];
  int ld[kMaxBlocks];
  int cap[kMaxBlocks];   // host-known upper bound of each block's width
  int nb;
};

// upper bound of the total width of a view (host side)
template <class T>
inline int view_cap(const BlockView<T>& v) {
  int c = 0;
  for (int b = 0; b < v.nb; ++b) c += v.cap[b];
  return c;
}

// Diagonal core of a concatenation: block b contributes coef_b * s_b[j]
// (s_b == nullptr means all ones) for its width (same widths as the views).
struct CoreView {
  const double* s[kMaxBlocks];
  double coef[kMaxBlocks];
  const int* wdev[kMaxBlocks];
  int wconst[kMaxBlocks];
  int nb;
};

template <class T>
__device__ inline int block_width(const BlockView<T>& v, int b) {
  return v.wdev[b] ? *v.wdev[b] : v.wconst[b];
}
__device__ inline int core_width(const CoreView& c, int b) {
  return c.wdev[b] ? *c.wdev[b] : c.wconst[b];
}

}  // namespace lrc
