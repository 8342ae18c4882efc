// Dense tall-skinny kernels on MFMA (gfx950): Gram products of concatenated
// factors, tall-skinny times small products, and the fp64 true residual.
// All use the 16x16x4 MFMA shapes (f32 and f64) with the lane layout
//   A operand  lane l -> A[l % 16][l / 16]   (16 x 4)
//   B operand  lane l -> B[l / 16][l % 16]   (4 x 16)
//   D, f32     lane l, value i -> D[4 (l / 16) + i][l % 16]
//   D, f64     lane l, value i -> D[(l / 16) + 4 i][l % 16]   (rows interleaved)
// (both result layouts were checked on gfx950 with a one-wave probe).
#include <algorithm>

#include "kernels.hpp"
#include "prof.hpp"

namespace lrc {

template <class T>
static std::vector<WTerm> view_terms(const BlockView<T>& v) {
  std::vector<WTerm> t;
  for (int b = 0; b < v.nb; ++b) t.push_back({v.wdev[b], v.wconst[b]});
  return t;
}


typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

template <class T> struct Mfma;
template <> struct Mfma<float> {
  typedef floatx4 acc_t;
  static __device__ inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int drow(int lane, int i) { return 4 * (lane >> 4) + i; }
};
template <> struct Mfma<double> {
  typedef doublex4 acc_t;
  static __device__ inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int drow(int lane, int i) { return (lane >> 4) + 4 * i; }
};

constexpr int kKCAP = 192;          // max total columns of a concatenation
constexpr int kKT = kKCAP / 16;     // 12 tiles per dimension
constexpr int kTiles = kKT * (kKT + 1) / 2;   // 78 upper tiles
constexpr int kGramRows = 32;       // rows staged per chunk

// column -> (block, local column) tables of a view, built in LDS
// (columns beyond kKCAP are dropped; the Gram reduction reports the overflow)
template <class T>
__device__ inline int build_coltab(const BlockView<T>& v, unsigned char* blk, short* loc) {
  int k = 0;
  for (int b = 0; b < v.nb; ++b) {
    const int w = block_width(v, b);
    for (int c = threadIdx.x; c < w && k + c < kKCAP; c += blockDim.x) {
      blk[k + c] = (unsigned char)b;
      loc[k + c] = (short)c;
    }
    k += w;
  }
  return k < kKCAP ? k : kKCAP;
}

template <class T>
__device__ inline T view_at(const BlockView<T>& v, int b, int lc, int64_t row) {
  T x = v.ptr[b][row * v.ld[b] + lc];
  if (v.rowscale[b]) x *= T(v.rowscale[b][row]);
  return x;
}

// ============================================================== Gram
template <class T>
struct GramArgs {
  BlockView<T> X[2];
  int64_t rows[2];
  int nwg0;          // workgroups of job 0; the rest belong to job 1
  int nwg1;
};

__device__ inline void tile_of(int t, int KT, int& bi, int& bj) {
  // enumerate (bi <= bj) row by row
  bi = 0;
  int rem = t;
  while (rem >= KT - bi) { rem -= KT - bi; ++bi; }
  bj = bi + rem;
}

template <class T, class Tacc>
__global__ __launch_bounds__(256) void gram_kernel(GramArgs<T> a, Tacc* __restrict__ partial) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T stage[kGramRows][kKCAP + 4];
  __shared__ unsigned char blk[kKCAP];
  __shared__ short loc[kKCAP];
  const int job = blockIdx.x < a.nwg0 ? 0 : 1;
  const int wg = job == 0 ? blockIdx.x : blockIdx.x - a.nwg0;
  const int nwg = job == 0 ? a.nwg0 : a.nwg1;
  const BlockView<T>& X = a.X[job];
  const int64_t rows = a.rows[job];
  const int k = build_coltab(X, blk, loc);
  const int KT = (k + 15) / 16;
  const int T_ = KT * (KT + 1) / 2;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  constexpr int MAXT = (kTiles + 3) / 4;
  acc_t acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = acc_t{};
  int tbi[MAXT], tbj[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int tt = wave + 4 * t;
    if (tt < T_) tile_of(tt, KT, tbi[t], tbj[t]);
    else { tbi[t] = -1; tbj[t] = -1; }
  }
  __syncthreads();
  // contiguous row range of this workgroup, in chunks
  const int64_t per = ceil_div(ceil_div(rows, kGramRows), nwg) * kGramRows;
  const int64_t r0 = int64_t(wg) * per, r1 = std::min<int64_t>(rows, r0 + per);
  const int kp = KT * 16;
  for (int64_t c0 = r0; c0 < r1; c0 += kGramRows) {
    const int nr = int(std::min<int64_t>(kGramRows, r1 - c0));
    for (int e = threadIdx.x; e < kGramRows * kp; e += blockDim.x) {
      const int rr = e / kp, c = e - rr * kp;
      T v = T(0);
      if (rr < nr && c < k) v = view_at(X, blk[c], loc[c], c0 + rr);
      stage[rr][c] = v;
    }
    __syncthreads();
    for (int kk = 0; kk < kGramRows; kk += 4) {
      const int rr = kk + (lane >> 4), cc = lane & 15;
#pragma unroll
      for (int t = 0; t < MAXT; ++t) {
        if (tbi[t] < 0) continue;
        acc[t] = Mfma<T>::op(stage[rr][tbi[t] * 16 + cc], stage[rr][tbj[t] * 16 + cc], acc[t]);
      }
    }
    __syncthreads();
  }
  // write the compact upper tiles of this workgroup
  Tacc* out = partial + (size_t(blockIdx.x) * kTiles) * 256;
#pragma unroll
  for (int t = 0; t < MAXT; ++t) {
    const int tt = wave + 4 * t;
    if (tt >= T_) continue;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      out[size_t(tt) * 256 + Mfma<T>::drow(lane, i) * 16 + (lane & 15)] = Tacc(acc[t][i]);
  }
}

template <class T, class Tacc>
__global__ void gram_reduce_kernel(GramArgs<T> a, const Tacc* __restrict__ partial, double* G0,
                                   double* G1, int kcap, int* k0, int* k1, int* info) {
  const int job = blockIdx.y;
  const BlockView<T>& X = a.X[job];
  int ktot = 0;
  for (int b = 0; b < X.nb; ++b) ktot += block_width(X, b);
  const int kg = ktot < kKCAP ? ktot : kKCAP;     // columns the Gram kernel saw
  const int k = kg < kcap ? kg : kcap;
  const int KT = (kg + 15) / 16;
  const int T_ = KT * (KT + 1) / 2;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int t = e / 256, w = e & 255;
  if (e == 0 && ktot > kcap && info) atomicOr(info, 8);
  if (job == 0 && e == 0 && k0) *k0 = k;
  if (job == 1 && e == 0 && k1) *k1 = k;
  if (t >= T_) return;
  int bi, bj;
  tile_of(t, KT, bi, bj);
  const int r = bi * 16 + w / 16, c = bj * 16 + (w & 15);
  if (r >= k || c >= k || r > c) return;
  const int w0 = job == 0 ? 0 : a.nwg0;
  const int nw = job == 0 ? a.nwg0 : a.nwg1;
  double s = 0.0;
  for (int i = 0; i < nw; ++i) s += double(partial[(size_t(w0 + i) * kTiles + t) * 256 + w]);
  double* G = job == 0 ? G0 : G1;
  G[size_t(r) * kcap + c] = s;
  G[size_t(c) * kcap + r] = s;
}

static int gram_wgs(int64_t rows) {
  if (rows <= 0) return 1;
  return int(std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(rows, 256))));
}

size_t gram_workspace_bytes(int64_t rows_a, int64_t rows_b, int kcap, bool fp64) {
  (void)kcap;
  return size_t(gram_wgs(rows_a) + gram_wgs(rows_b)) * kTiles * 256 * (fp64 ? 8 : 4);
}

template <class T>
void launch_gram(const GramJob<T>* jobs, int njobs, int kcap, double* ws_partial, size_t ws_bytes,
                 int* info, hipStream_t s) {
  LRC_CHECK(njobs >= 1 && njobs <= 2, ST_EINVAL, "gram: one or two jobs");
  LRC_CHECK(kcap <= kKCAP, ST_EINVAL, "gram: at most 192 columns");
  GramArgs<T> a;
  a.X[0] = jobs[0].X;
  a.rows[0] = jobs[0].rows;
  a.nwg0 = gram_wgs(jobs[0].rows);
  if (njobs == 2) {
    a.X[1] = jobs[1].X;
    a.rows[1] = jobs[1].rows;
    a.nwg1 = gram_wgs(jobs[1].rows);
  } else {
    a.X[1] = jobs[0].X;
    a.rows[1] = 0;
    a.nwg1 = 0;
  }
  // fp32 products accumulate in fp32 inside a workgroup; fp64 in fp64
  const size_t need = size_t(a.nwg0 + a.nwg1) * kTiles * 256 * sizeof(T);
  LRC_CHECK(need <= ws_bytes, ST_EINVAL, "gram: workspace too small");
  {
    // algorithmic flops: the k(k+1)/2 distinct entries of each Gram matrix,
    // 2 flops per row each
    Work w;
    w.bytes = false;
    const double r0 = double(a.rows[0]), r1 = double(a.rows[1]);
    w.groups = {view_terms(jobs[0].X), view_terms(njobs > 1 ? jobs[1].X : jobs[0].X)};
    w.f = [=](const std::vector<double>& v) {
      return r0 * v[0] * (v[0] + 1.0) + r1 * v[1] * (v[1] + 1.0);
    };
    ProfScope ps(kcls(K_GRAM, is_f32<T>()), s, w);
    hipLaunchKernelGGL((gram_kernel<T, T>), dim3(a.nwg0 + a.nwg1), dim3(256), 0, s, a,
                       reinterpret_cast<T*>(ws_partial));
  }
  ProfScope ps(kcls(K_GRAM_REDUCE, is_f32<T>()), s);
  const int elems = kTiles * 256;
  hipLaunchKernelGGL((gram_reduce_kernel<T, T>), dim3(ceil_div(elems, 256), njobs), dim3(256), 0,
                     s, a, reinterpret_cast<const T*>(ws_partial), jobs[0].G,
                     njobs == 2 ? jobs[1].G : jobs[0].G, kcap, jobs[0].kout,
                     njobs == 2 ? jobs[1].kout : nullptr, info);
  LRC_HIP(hipGetLastError());
}
template void launch_gram<float>(const GramJob<float>*, int, int, double*, size_t, int*,
                                 hipStream_t);
template void launch_gram<double>(const GramJob<double>*, int, int, double*, size_t, int*,
                                  hipStream_t);

// ============================================================== TSMM  Y = X * M
// Output columns are processed in slices of 64 (grid.y); one workgroup stages
// the k x 64 slice of M and 64-row blocks of X (in k-chunks of 32) in LDS.
constexpr int kTsRows = 64;
constexpr int kTsK = 32;
constexpr int kTsSlice = 64;
constexpr int kTsKCAP = 128;

template <class T>
struct TsmmArgs {
  TsmmJob<T> job[2];
  int nwg0, nwg1;
};

template <class T>
__global__ __launch_bounds__(256) void tsmm_kernel(TsmmArgs<T> a) {
  typedef typename Mfma<T>::acc_t acc_t;
  __shared__ T Ms[kTsKCAP][kTsSlice + 4];
  __shared__ T Xs[kTsRows][kTsK + 1];
  __shared__ unsigned char blk[kKCAP];
  __shared__ short loc[kKCAP];
  const int jb = blockIdx.x < a.nwg0 ? 0 : 1;
  const int wg = jb == 0 ? blockIdx.x : blockIdx.x - a.nwg0;
  const int nwg = jb == 0 ? a.nwg0 : a.nwg1;
  const TsmmJob<T>& J = a.job[jb];
  const int k = build_coltab(J.X, blk, loc);
  const int r = *J.r_dev;
  const int cs = blockIdx.y * kTsSlice;          // first output column of the slice
  if (cs >= r || k > kTsKCAP) return;
  const int rs = min(kTsSlice, r - cs);
  const int kp = (k + 3) / 4 * 4;
  const int RT = (rs + 15) / 16;
  for (int e = threadIdx.x; e < kp * kTsSlice; e += blockDim.x) {
    const int i = e / kTsSlice, c = e - i * kTsSlice;
    Ms[i][c] = (i < k && c < rs) ? T(J.M[size_t(i) * J.ldm + cs + c]) : T(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t row0 = int64_t(wg) * kTsRows; row0 < J.rows; row0 += int64_t(nwg) * kTsRows) {
    acc_t acc[kTsSlice / 16];
#pragma unroll
    for (int t = 0; t < kTsSlice / 16; ++t) acc[t] = acc_t{};
    const int nr = int(std::min<int64_t>(kTsRows, J.rows - row0));
    for (int k0 = 0; k0 < kp; k0 += kTsK) {
      const int kc = std::min(kTsK, kp - k0);
      for (int e = threadIdx.x; e < kTsRows * kTsK; e += blockDim.x) {
        const int rr = e / kTsK, c = e - rr * kTsK;
        T v = T(0);
        if (rr < nr && c < kc && k0 + c < k) v = view_at(J.X, blk[k0 + c], loc[k0 + c], row0 + rr);
        Xs[rr][c] = v;
      }
      __syncthreads();
      for (int kk = 0; kk < kc; kk += 4) {
        const T xa = Xs[wave * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int t = 0; t < kTsSlice / 16; ++t) {
          if (t < RT) acc[t] = Mfma<T>::op(xa, Ms[k0 + kk + (lane >> 4)][t * 16 + (lane & 15)], acc[t]);
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < kTsSlice / 16; ++t) {
      if (t >= RT) continue;
      const int c = t * 16 + (lane & 15);
      if (c >= rs) continue;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = wave * 16 + Mfma<T>::drow(lane, i);
        if (rr < nr) J.Y[(row0 + rr) * J.ldy + cs + c] = acc[t][i];
      }
    }
  }
}

template <class T>
void launch_tsmm(const TsmmJob<T>* jobs, int njobs, int kcap, int rcap, hipStream_t s) {
  LRC_CHECK(njobs >= 1 && njobs <= 2, ST_EINVAL, "tsmm: one or two jobs");
  LRC_CHECK(kcap <= kTsKCAP && rcap <= kTsKCAP, ST_EINVAL, "tsmm: capacity exceeded");
  TsmmArgs<T> a;
  a.job[0] = jobs[0];
  a.nwg0 = int(std::min<int64_t>(1024, std::max<int64_t>(1, ceil_div(jobs[0].rows, kTsRows))));
  if (njobs == 2) {
    a.job[1] = jobs[1];
    a.nwg1 = int(std::min<int64_t>(256, std::max<int64_t>(1, ceil_div(jobs[1].rows, kTsRows))));
  } else {
    a.job[1] = jobs[0];
    a.nwg1 = 0;
  }
  const int slices = int(ceil_div(rcap, kTsSlice));
  // algorithmic flops: 2 rows k r per job
  Work w;
  w.bytes = false;
  const double r0 = double(a.nwg0 > 0 ? jobs[0].rows : 0), r1 = double(a.nwg1 > 0 ? jobs[1].rows : 0);
  w.groups = {view_terms(jobs[0].X), {{jobs[0].r_dev, 0}},
              view_terms(njobs > 1 ? jobs[1].X : jobs[0].X),
              {{njobs > 1 ? jobs[1].r_dev : jobs[0].r_dev, 0}}};
  w.f = [=](const std::vector<double>& v) { return 2.0 * (r0 * v[0] * v[1] + r1 * v[2] * v[3]); };
  ProfScope ps(kcls(K_TSMM, is_f32<T>()), s, w);
  hipLaunchKernelGGL((tsmm_kernel<T>), dim3(a.nwg0 + a.nwg1, slices), dim3(256), 0, s, a);
  LRC_HIP(hipGetLastError());
}
template void launch_tsmm<float>(const TsmmJob<float>*, int, int, int, hipStream_t);
template void launch_tsmm<double>(const TsmmJob<double>*, int, int, int, hipStream_t);

// ============================================================== fp64 residual
// R = A * (core-scaled B)^T entry by entry on fp64 MFMA; only the per-column
// sums of squares leave the kernel (R itself is never stored).
constexpr int kResCols = 64;
constexpr int kResRows = 64;
constexpr int kResK = 32;
constexpr int kResRowGroups = 64;

__global__ __launch_bounds__(256) void residual_kernel(BlockView<double> A, int64_t n,
                                                       BlockView<double> B, CoreView core,
                                                       int64_t m, double* __restrict__ part) {
  __shared__ double Bs[kResCols][kKCAP + 1];
  __shared__ double As[kResRows][kResK + 1];
  __shared__ unsigned char blk[kKCAP];
  __shared__ short loc[kKCAP];
  __shared__ double coef[kKCAP];
  __shared__ double colacc[4][kResCols];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // core coefficients per concatenated column
  {
    int k = 0;
    for (int b = 0; b < core.nb; ++b) {
      const int w = core_width(core, b);
      for (int c = threadIdx.x; c < w && k + c < kKCAP; c += blockDim.x)
        coef[k + c] = core.coef[b] * (core.s[b] ? core.s[b][c] : 1.0);
      k += w;
    }
  }
  const int kB = build_coltab(B, blk, loc);
  const int64_t j0 = int64_t(blockIdx.x) * kResCols;
  const int kp = (kB + 3) / 4 * 4;
  __syncthreads();
  for (int e = threadIdx.x; e < kResCols * kp; e += blockDim.x) {
    const int jj = e / kp, c = e - jj * kp;
    double v = 0.0;
    if (j0 + jj < m && c < kB) v = view_at(B, blk[c], loc[c], j0 + jj) * coef[c];
    Bs[jj][c] = v;
  }
  __syncthreads();
  const int kA = build_coltab(A, blk, loc);   // same total width as B
  (void)kA;
  __syncthreads();
  double csum[4] = {0.0, 0.0, 0.0, 0.0};
  const int64_t per = ceil_div(ceil_div(n, kResRows), gridDim.y) * kResRows;
  const int64_t r0 = int64_t(blockIdx.y) * per, r1 = std::min<int64_t>(n, r0 + per);
  for (int64_t row0 = r0; row0 < r1; row0 += kResRows) {
    const int nr = int(std::min<int64_t>(kResRows, r1 - row0));
    doublex4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = doublex4{};
    for (int k0 = 0; k0 < kp; k0 += kResK) {
      const int kc = std::min(kResK, kp - k0);
      for (int e = threadIdx.x; e < kResRows * kResK; e += blockDim.x) {
        const int rr = e / kResK, c = e - rr * kResK;
        double v = 0.0;
        if (rr < nr && c < kc && k0 + c < kB) v = view_at(A, blk[k0 + c], loc[k0 + c], row0 + rr);
        As[rr][c] = v;
      }
      __syncthreads();
      for (int kk = 0; kk < kc; kk += 4) {
        const double xa = As[wave * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int t = 0; t < 4; ++t)
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(
              xa, Bs[t * 16 + (lane & 15)][k0 + kk + (lane >> 4)], acc[t], 0, 0, 0);
      }
      __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) csum[t] += acc[t][i] * acc[t][i];
  }
  // reduce lanes with the same column (l, l+16, l+32, l+48), then waves
#pragma unroll
  for (int t = 0; t < 4; ++t) {
    double v = csum[t];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < 16) colacc[wave][t * 16 + lane] = v;
  }
  __syncthreads();
  if (threadIdx.x < kResCols) {
    const double v = colacc[0][threadIdx.x] + colacc[1][threadIdx.x] + colacc[2][threadIdx.x] +
                     colacc[3][threadIdx.x];
    const int64_t j = j0 + threadIdx.x;
    if (j < m) part[size_t(blockIdx.y) * m + j] = v;
  }
}

__global__ void residual_reduce_kernel(const double* __restrict__ part, int groups, int64_t m,
                                       double* __restrict__ colsq) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int g = 0; g < groups; ++g) s += part[size_t(g) * m + j];
  colsq[j] = s;
}

size_t residual_workspace_bytes(int64_t n, int64_t m) {
  (void)n;
  return size_t(kResRowGroups) * size_t(m) * sizeof(double);
}

void launch_residual_fp64(const BlockView<double>& A, int64_t n, const BlockView<double>& B,
                          CoreView core, int64_t m, int kcap, double* colsq, double* ws,
                          size_t ws_bytes, hipStream_t s) {
  LRC_CHECK(kcap <= kKCAP, ST_EINVAL, "residual: at most 192 columns");
  LRC_CHECK(ws_bytes >= residual_workspace_bytes(n, m), ST_EINVAL, "residual: workspace too small");
  const int groups = int(std::min<int64_t>(kResRowGroups, std::max<int64_t>(1, ceil_div(n, kResRows))));
  dim3 grid(unsigned(ceil_div(m, kResCols)), unsigned(groups));
  // algorithmic flops: every entry of the n x m residual is a k-term dot product
  Work w;
  w.bytes = false;
  const double nm = double(n) * double(m);
  w.groups = {view_terms(A)};
  w.f = [=](const std::vector<double>& v) { return 2.0 * nm * v[0]; };
  ProfScope ps(kcls(K_RESIDUAL, false), s, w);
  hipLaunchKernelGGL(residual_kernel, grid, dim3(256), 0, s, A, n, B, core, m, ws);
  hipLaunchKernelGGL(residual_reduce_kernel, dim3(unsigned(ceil_div(m, 256))), dim3(256), 0, s, ws,
                     groups, m, colsq);
  LRC_HIP(hipGetLastError());
}

}  // namespace lrc
