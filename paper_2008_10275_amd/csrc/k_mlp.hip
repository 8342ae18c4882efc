// Surrogate network for a learned initial guess: a 3-layer perceptron
// d0 -> d1 -> d2 -> d3 (GELU, GELU, linear) mapping normalised parameters to
// standardised coefficients on a snapshot basis.  Weights and activations are
// bf16, products accumulate in fp32 on MFMA (v_mfma_f32_16x16x32_bf16), the
// optimiser (Adam) keeps fp32 master weights.  Every training step is a fixed
// sequence of launches on the context stream; nothing synchronises the host.
#include <cmath>

#include "mlp.hpp"
#include "prof.hpp"

namespace lrc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ----------------------------------------------------------------- GELU
// Exact form z Phi(z) with the erf-based normal CDF, and its derivative.
__device__ inline float gelu_f(float z) { return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f)); }
__device__ inline float gelu_d(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// ----------------------------------------------------------------- GEMM
// C (M x N) = A (M x K) * B (K x N), bf16 operands read through strides
// (A(m, k) = A[m * sam + k * sak], B(k, n) = B[k * sbk + n * sbn]), fp32
// accumulation.  M, N multiples of 16 and K of 32 (operands zero-padded in
// memory).  One wave per 16 x 16 output tile; MFMA lane layout (gfx950,
// 16x16x32 bf16): A lane l -> A[l % 16][8 (l / 16) + e], B lane l ->
// B[8 (l / 16) + e][l % 16], D lane l, value i -> D[4 (l / 16) + i][l % 16].
enum { EP_GELU = 0, EP_LINEAR = 1, EP_DZ = 2, EP_GRAD = 3 };

struct GemmArgs {
  const __bf16* A;
  const __bf16* B;
  int M, N, K;
  int sam, sak, sbk, sbn;
  int mvalid, nvalid;        // rows / columns that are real (the rest are written as 0)
  const float* bias;         // EP_GELU, EP_LINEAR: per column
  const __bf16* G;           // EP_DZ: gelu'(Z) of the same shape as C (ld ldc)
  __bf16* Cb;                // EP_GELU: H, EP_DZ: dZ (bf16, ld ldc)
  __bf16* Gout;              // EP_GELU: gelu'(Z) (bf16, ld ldc)
  float* Cf;                 // EP_LINEAR, EP_GRAD: fp32 output (ld ldcf)
  int ldc, ldcf;
};

template <int EP>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(GemmArgs a) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tiles_n = a.N / 16;
  const int tile = blockIdx.x * 4 + wave;
  if (tile >= (a.M / 16) * tiles_n) return;
  const int m0 = (tile / tiles_n) * 16, n0 = (tile % tiles_n) * 16;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  const int r = lane & 15, g = lane >> 4;
  for (int k0 = 0; k0 < a.K; k0 += 32) {
    bf16x8 av, bv;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int kk = k0 + 8 * g + e;
      av[e] = a.A[size_t(m0 + r) * a.sam + size_t(kk) * a.sak];
      bv[e] = a.B[size_t(kk) * a.sbk + size_t(n0 + r) * a.sbn];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc, 0, 0, 0);
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + 4 * g + i, n = n0 + r;
    const bool ok = m < a.mvalid && n < a.nvalid;
    const float v = acc[i];
    if constexpr (EP == EP_GELU) {
      const float z = v + a.bias[n];
      a.Cb[size_t(m) * a.ldc + n] = __bf16(ok ? gelu_f(z) : 0.0f);
      a.Gout[size_t(m) * a.ldc + n] = __bf16(ok ? gelu_d(z) : 0.0f);
    } else if constexpr (EP == EP_LINEAR) {
      a.Cf[size_t(m) * a.ldcf + n] = ok ? v + a.bias[n] : 0.0f;
    } else if constexpr (EP == EP_DZ) {
      a.Cb[size_t(m) * a.ldc + n] = __bf16(ok ? v * float(a.G[size_t(m) * a.ldc + n]) : 0.0f);
    } else {
      if (ok) a.Cf[size_t(m) * a.ldcf + n] = v;
    }
  }
}

template <int EP>
static void gemm(const GemmArgs& a, hipStream_t s) {
  LRC_CHECK(a.M % 16 == 0 && a.N % 16 == 0 && a.K % 32 == 0, ST_EINVAL, "mlp: bad GEMM shape");
  const int tiles = (a.M / 16) * (a.N / 16);
  hipLaunchKernelGGL((mlp_gemm_kernel<EP>), dim3((tiles + 3) / 4), dim3(256), 0, s, a);
  LRC_HIP(hipGetLastError());
}

// ----------------------------------------------------------------- scaling
// Inputs: fp64 (B x d0, row-major raw parameters) -> bf16 (Bp x 32) mapped by
// x -> 2 (x - lo) / (hi - lo) - 1; padding rows and columns are zero.
__global__ void mlp_inputs_kernel(const double* __restrict__ X, int B, int Bp, int d0,
                                  const double* __restrict__ lo, const double* __restrict__ hi,
                                  __bf16* __restrict__ Xb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Bp * kMlpK0) return;
  const int m = e / kMlpK0, c = e % kMlpK0;
  float v = 0.0f;
  if (m < B && c < d0) v = float(2.0 * (X[size_t(m) * d0 + c] - lo[c]) / (hi[c] - lo[c]) - 1.0);
  Xb[e] = __bf16(v);
}

// Per-column range of the inputs and mean / standard deviation of the
// targets (population form; a zero deviation becomes 1).  One workgroup.
__global__ __launch_bounds__(256) void mlp_fit_kernel(const double* __restrict__ X, int B, int d0,
                                                      const double* __restrict__ T, int d3,
                                                      double* lo, double* hi, double* mean,
                                                      double* sd) {
  for (int c = threadIdx.x; c < d0 + d3; c += blockDim.x) {
    if (c < d0) {
      double a = X[c], b = X[c];
      for (int m = 1; m < B; ++m) {
        const double x = X[size_t(m) * d0 + c];
        a = fmin(a, x);
        b = fmax(b, x);
      }
      if (!(b > a)) { a -= 1.0; b += 1.0; }
      lo[c] = a;
      hi[c] = b;
    } else {
      const int j = c - d0;
      double s1 = 0.0;
      for (int m = 0; m < B; ++m) s1 += T[size_t(m) * d3 + j];
      const double mu = s1 / B;
      double s2 = 0.0;
      for (int m = 0; m < B; ++m) {
        const double d = T[size_t(m) * d3 + j] - mu;
        s2 += d * d;
      }
      const double v = sqrt(s2 / B);
      mean[j] = mu;
      sd[j] = v > 0.0 ? v : 1.0;
    }
  }
}

// Standardised targets (fp32, Bp x kMlpN3, zero padding).
__global__ void mlp_targets_kernel(const double* __restrict__ T, int B, int Bp, int d3,
                                   const double* __restrict__ mean, const double* __restrict__ sd,
                                   float* __restrict__ Ts) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= Bp * kMlpN3) return;
  const int m = e / kMlpN3, c = e % kMlpN3;
  Ts[e] = (m < B && c < d3) ? float((T[size_t(m) * d3 + c] - mean[c]) / sd[c]) : 0.0f;
}

// Network outputs back to coefficient units (fp64, B x d3).
__global__ void mlp_outputs_kernel(const float* __restrict__ Y, int B, int d3,
                                   const double* __restrict__ mean, const double* __restrict__ sd,
                                   double* __restrict__ out) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= B * d3) return;
  const int m = e / d3, c = e % d3;
  out[e] = double(Y[size_t(m) * kMlpN3 + c]) * sd[c] + mean[c];
}

// ----------------------------------------------------------------- loss
// loss = mean (Y - T)^2 over the B x d3 real entries; dY = 2 (Y - T) / (B d3)
// in fp32 and bf16.  One workgroup (fixed reduction order).
__global__ __launch_bounds__(1024) void mlp_loss_kernel(const float* __restrict__ Y,
                                                        const float* __restrict__ T, int B, int Bp,
                                                        int d3, float* dYf, __bf16* dYb,
                                                        float* loss_out) {
  __shared__ float red[1024];
  float acc = 0.0f;
  const float sc = 2.0f / float(B * d3);
  for (int e = threadIdx.x; e < Bp * kMlpN3; e += blockDim.x) {
    const int m = e / kMlpN3, c = e % kMlpN3;
    float d = 0.0f;
    if (m < B && c < d3) {
      d = Y[e] - T[e];
      acc += d * d;
    }
    dYf[e] = sc * d;
    dYb[e] = __bf16(sc * d);
  }
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if (int(threadIdx.x) < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0 && loss_out) *loss_out = red[0] / float(B * d3);
}

// Bias gradients db_l[n] = sum over the batch of dZ_l[:, n] (fixed order).
__global__ void mlp_bias_grad_kernel(const float* __restrict__ dYf, const __bf16* __restrict__ dZ2,
                                     const __bf16* __restrict__ dZ1, int Bp, int d1, int d2, int d3,
                                     float* db1, float* db2, float* db3) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < d3) {
    float s = 0.0f;
    for (int m = 0; m < Bp; ++m) s += dYf[size_t(m) * kMlpN3 + c];
    db3[c] = s;
  } else if (c < d3 + d2) {
    const int j = c - d3;
    float s = 0.0f;
    for (int m = 0; m < Bp; ++m) s += float(dZ2[size_t(m) * kMlpH + j]);
    db2[j] = s;
  } else if (c < d3 + d2 + d1) {
    const int j = c - d3 - d2;
    float s = 0.0f;
    for (int m = 0; m < Bp; ++m) s += float(dZ1[size_t(m) * kMlpH + j]);
    db1[j] = s;
  }
}

// ----------------------------------------------------------------- Adam
// Bias-corrected Adam on the fp32 master parameters (packed W1 b1 W2 b2 W3 b3,
// W stored out x in); b1t = beta1^t, b2t = beta2^t.
__global__ void mlp_adam_kernel(float* p, const float* g, float* m, float* v, int n, float lr,
                                float beta1, float beta2, float eps, float b1t, float b2t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float mh = mi / (1.0f - b1t), vh = vi / (1.0f - b2t);
  p[i] -= lr * mh / (sqrtf(vh) + eps);
}

// bf16 copies of the weights, padded for the MFMA shapes: W1b (d1 x 32),
// W2b (d2 x d1), W3b (kMlpN3 x d2), all out x in row-major; fp32 biases with
// zero padding.
__global__ void mlp_sync_kernel(const float* __restrict__ p, int d0, int d1, int d2, int d3,
                                __bf16* W1b, __bf16* W2b, __bf16* W3b, float* b1, float* b2,
                                float* b3) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int o1 = 0, ob1 = o1 + d1 * d0, o2 = ob1 + d1, ob2 = o2 + d2 * d1, o3 = ob2 + d2,
            ob3 = o3 + d3 * d2;
  if (e < d1 * kMlpK0) {
    const int n = e / kMlpK0, k = e % kMlpK0;
    W1b[e] = __bf16(k < d0 ? p[o1 + n * d0 + k] : 0.0f);
  }
  if (e < d2 * d1) W2b[e] = __bf16(p[o2 + e]);
  if (e < kMlpN3 * d2) {
    const int n = e / d2, k = e % d2;
    W3b[e] = __bf16(n < d3 ? p[o3 + n * d2 + k] : 0.0f);
  }
  if (e < d1) b1[e] = p[ob1 + e];
  if (e < d2) b2[e] = p[ob2 + e];
  if (e < kMlpN3) b3[e] = e < d3 ? p[ob3 + e] : 0.0f;
}

// ----------------------------------------------------------------- host side
static int blocks(int64_t n, int t = 256) { return int((n + t - 1) / t); }

void Mlp::init(const int* sizes, const float* params, hipStream_t s) {
  d0 = sizes[0];
  d1 = sizes[1];
  d2 = sizes[2];
  d3 = sizes[3];
  LRC_CHECK(d0 >= 1 && d0 <= kMlpK0 && d1 >= 32 && d1 <= kMlpH && d1 % 32 == 0 && d2 >= 32 &&
                d2 <= kMlpH && d2 % 32 == 0 && d3 >= 1 && d3 <= kMlpN3,
            ST_EINVAL, "mlp: sizes must satisfy d0 <= 32, d1, d2 in {32, 64}, d3 <= 32");
  np = d1 * d0 + d1 + d2 * d1 + d2 + d3 * d2 + d3;
  std::vector<float> h(params, params + np);
  P = upload(h, s);
  Gr.alloc(size_t(np) * 4);
  Mo.alloc(size_t(np) * 4);
  Vo.alloc(size_t(np) * 4);
  LRC_HIP(hipMemsetAsync(Mo.p, 0, Mo.bytes, s));
  LRC_HIP(hipMemsetAsync(Vo.p, 0, Vo.bytes, s));
  W1b.alloc(size_t(kMlpH) * kMlpK0 * 2);
  W2b.alloc(size_t(kMlpH) * kMlpH * 2);
  W3b.alloc(size_t(kMlpN3) * kMlpH * 2);
  bb.alloc(size_t(3) * kMlpH * 4);
  sc.alloc(size_t(2 * kMlpK0 + 2 * kMlpN3) * 8);
  // identity scaling until fitted: inputs already in [-1, 1], targets standardised
  std::vector<double> id(2 * kMlpK0 + 2 * kMlpN3);
  for (int c = 0; c < kMlpK0; ++c) { id[c] = -1.0; id[kMlpK0 + c] = 1.0; }
  for (int c = 0; c < kMlpN3; ++c) { id[2 * kMlpK0 + c] = 0.0; id[2 * kMlpK0 + kMlpN3 + c] = 1.0; }
  LRC_HIP(hipMemcpyAsync(sc.p, id.data(), id.size() * 8, hipMemcpyHostToDevice, s));
  t = 0;
  sync(s);
  LRC_HIP(hipStreamSynchronize(s));
}

void Mlp::sync(hipStream_t s) {
  float* b = bb.as<float>();
  hipLaunchKernelGGL(mlp_sync_kernel, dim3(blocks(kMlpH * kMlpH)), dim3(256), 0, s,
                     P.as<float>(), d0, d1, d2, d3, W1b.as<__bf16>(), W2b.as<__bf16>(),
                     W3b.as<__bf16>(), b, b + kMlpH, b + 2 * kMlpH);
  LRC_HIP(hipGetLastError());
}

void Mlp::reserve(int B) {
  const int Bp = (B + 31) / 32 * 32;
  if (Bp <= bcap) return;
  bcap = Bp;
  Xb.alloc(size_t(Bp) * kMlpK0 * 2);
  H1.alloc(size_t(Bp) * kMlpH * 2);
  G1.alloc(size_t(Bp) * kMlpH * 2);
  H2.alloc(size_t(Bp) * kMlpH * 2);
  G2.alloc(size_t(Bp) * kMlpH * 2);
  Y.alloc(size_t(Bp) * kMlpN3 * 4);
  Ts.alloc(size_t(Bp) * kMlpN3 * 4);
  dYf.alloc(size_t(Bp) * kMlpN3 * 4);
  dYb.alloc(size_t(Bp) * kMlpN3 * 2);
  dZ2.alloc(size_t(Bp) * kMlpH * 2);
  dZ1.alloc(size_t(Bp) * kMlpH * 2);
  lossd.alloc(4 * 4);
}

const double* Mlp::lo() const { return sc.as<double>(); }
const double* Mlp::hi() const { return sc.as<double>() + kMlpK0; }
const double* Mlp::mean() const { return sc.as<double>() + 2 * kMlpK0; }
const double* Mlp::sd() const { return sc.as<double>() + 2 * kMlpK0 + kMlpN3; }

void Mlp::fit(int B, const double* X, const double* T, hipStream_t s) {
  double* base = sc.as<double>();
  hipLaunchKernelGGL(mlp_fit_kernel, dim3(1), dim3(256), 0, s, X, B, d0, T, d3, base,
                     base + kMlpK0, base + 2 * kMlpK0, base + 2 * kMlpK0 + kMlpN3);
  LRC_HIP(hipGetLastError());
}

void Mlp::forward(int B, const double* X, hipStream_t s) {
  reserve(B);
  const int Bp = (B + 31) / 32 * 32;
  ProfScope ps(kcls(K_MLP, true), s);
  hipLaunchKernelGGL(mlp_inputs_kernel, dim3(blocks(Bp * kMlpK0)), dim3(256), 0, s, X, B, Bp,
                     d0, lo(), hi(), Xb.as<__bf16>());
  const float* b = bb.as<float>();
  GemmArgs g{};
  // layer 1: Z1 = X W1^T + b1, H1 = gelu(Z1)
  g = GemmArgs{Xb.as<__bf16>(), W1b.as<__bf16>(), Bp, d1, kMlpK0, kMlpK0, 1, 1, kMlpK0,
               B, d1, b, nullptr, H1.as<__bf16>(), G1.as<__bf16>(), nullptr, kMlpH, 0};
  gemm<EP_GELU>(g, s);
  // layer 2
  g = GemmArgs{H1.as<__bf16>(), W2b.as<__bf16>(), Bp, d2, d1, kMlpH, 1, 1, d1,
               B, d2, b + kMlpH, nullptr, H2.as<__bf16>(), G2.as<__bf16>(), nullptr, kMlpH, 0};
  gemm<EP_GELU>(g, s);
  // layer 3 (linear)
  g = GemmArgs{H2.as<__bf16>(), W3b.as<__bf16>(), Bp, kMlpN3, d2, kMlpH, 1, 1, d2,
               B, d3, b + 2 * kMlpH, nullptr, nullptr, nullptr, Y.as<float>(), 0, kMlpN3};
  gemm<EP_LINEAR>(g, s);
}

void Mlp::backward(int B, hipStream_t s) {
  const int Bp = (B + 31) / 32 * 32;
  ProfScope ps(kcls(K_MLP, true), s);
  float* gr = Gr.as<float>();
  const int o1 = 0, ob1 = o1 + d1 * d0, o2 = ob1 + d1, ob2 = o2 + d2 * d1, o3 = ob2 + d2,
            ob3 = o3 + d3 * d2;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(1024), 0, s, Y.as<float>(), Ts.as<float>(),
                     B, Bp, d3, dYf.as<float>(), dYb.as<__bf16>(), lossd.as<float>());
  GemmArgs g{};
  // dW3 = dY^T H2   (d3 x d2), A(m, k) = dY[k][m]
  g = GemmArgs{dYb.as<__bf16>(), H2.as<__bf16>(), kMlpN3, d2, Bp, 1, kMlpN3, kMlpH, 1,
               d3, d2, nullptr, nullptr, nullptr, nullptr, gr + o3, 0, d2};
  gemm<EP_GRAD>(g, s);
  // dZ2 = (dY W3) o gelu'(Z2): B(k, n) = W3b[k][n]
  g = GemmArgs{dYb.as<__bf16>(), W3b.as<__bf16>(), Bp, d2, kMlpN3, kMlpN3, 1, d2, 1,
               B, d2, nullptr, G2.as<__bf16>(), dZ2.as<__bf16>(), nullptr, nullptr, kMlpH, 0};
  gemm<EP_DZ>(g, s);
  // dW2 = dZ2^T H1
  g = GemmArgs{dZ2.as<__bf16>(), H1.as<__bf16>(), d2, d1, Bp, 1, kMlpH, kMlpH, 1,
               d2, d1, nullptr, nullptr, nullptr, nullptr, gr + o2, 0, d1};
  gemm<EP_GRAD>(g, s);
  // dZ1 = (dZ2 W2) o gelu'(Z1)
  g = GemmArgs{dZ2.as<__bf16>(), W2b.as<__bf16>(), Bp, d1, d2, kMlpH, 1, d1, 1,
               B, d1, nullptr, G1.as<__bf16>(), dZ1.as<__bf16>(), nullptr, nullptr, kMlpH, 0};
  gemm<EP_DZ>(g, s);
  // dW1 = dZ1^T X   (d1 x d0; columns padded to 16)
  g = GemmArgs{dZ1.as<__bf16>(), Xb.as<__bf16>(), d1, (d0 + 15) / 16 * 16, Bp, 1, kMlpH, kMlpK0, 1,
               d1, d0, nullptr, nullptr, nullptr, nullptr, gr + o1, 0, d0};
  gemm<EP_GRAD>(g, s);
  hipLaunchKernelGGL(mlp_bias_grad_kernel, dim3(blocks(d1 + d2 + d3)), dim3(256), 0, s,
                     dYf.as<float>(), dZ2.as<__bf16>(), dZ1.as<__bf16>(), Bp, d1, d2, d3,
                     gr + ob1, gr + ob2, gr + ob3);
  LRC_HIP(hipGetLastError());
}

void Mlp::targets(int B, const double* T, hipStream_t s) {
  reserve(B);
  const int Bp = (B + 31) / 32 * 32;
  hipLaunchKernelGGL(mlp_targets_kernel, dim3(blocks(Bp * kMlpN3)), dim3(256), 0, s, T, B, Bp,
                     d3, mean(), sd(), Ts.as<float>());
  LRC_HIP(hipGetLastError());
}

void Mlp::adam(float lr, float beta1, float beta2, float eps, hipStream_t s) {
  ++t;
  const float b1t = std::pow(beta1, float(t)), b2t = std::pow(beta2, float(t));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(blocks(np)), dim3(256), 0, s, P.as<float>(),
                     Gr.as<float>(), Mo.as<float>(), Vo.as<float>(), np, lr, beta1, beta2, eps,
                     b1t, b2t);
  LRC_HIP(hipGetLastError());
  sync(s);
}

void Mlp::outputs(int B, double* out, hipStream_t s) {
  hipLaunchKernelGGL(mlp_outputs_kernel, dim3(blocks(B * d3)), dim3(256), 0, s, Y.as<float>(), B,
                     d3, mean(), sd(), out);
  LRC_HIP(hipGetLastError());
}

}  // namespace lrc
