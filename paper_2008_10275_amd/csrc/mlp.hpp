// Surrogate network state on the device (see k_mlp.hip).
#pragma once
#include "common.hpp"

namespace lrc {

constexpr int kMlpK0 = 32;   // padded input width (d0 <= 32)
constexpr int kMlpH = 64;    // hidden width capacity (d1, d2 in {32, 64})
constexpr int kMlpN3 = 32;   // padded output width (d3 <= 32)

struct Mlp {
  int d0 = 0, d1 = 0, d2 = 0, d3 = 0, np = 0, t = 0, bcap = 0;
  // fp32 master parameters (packed W1 b1 W2 b2 W3 b3, W out x in), gradients,
  // Adam moments; bf16 padded weight copies and fp32 padded biases
  DevBuf P, Gr, Mo, Vo, W1b, W2b, W3b, bb;
  // input range (lo, hi) and target mean / deviation, fp64
  DevBuf sc;
  // activations of the last batch (Bp rows)
  DevBuf Xb, H1, G1, H2, G2, Y, Ts, dYf, dYb, dZ2, dZ1, lossd;
  void init(const int* sizes, const float* params, hipStream_t s);
  void sync(hipStream_t s);
  void reserve(int B);
  void fit(int B, const double* X, const double* T, hipStream_t s);
  void targets(int B, const double* T, hipStream_t s);
  void forward(int B, const double* X, hipStream_t s);
  void backward(int B, hipStream_t s);
  void adam(float lr, float beta1, float beta2, float eps, hipStream_t s);
  void outputs(int B, double* out, hipStream_t s);
  const double* lo() const;
  const double* hi() const;
  const double* mean() const;
  const double* sd() const;
};

}  // namespace lrc
