// Sparse kernels: fused CSR SpMM of the q operators against a tall factor, the
// level-scheduled supernodal triangular solves of the preconditioner, and the
// small vector kernels of the single-column (median parameter) solve.
#include <algorithm>

#include "kernels.hpp"
#include "prof.hpp"

namespace lrc {

// ============================================================== SpMM
// Every row of K_i is handled by `lpr` consecutive lanes; each lane owns CPL
// consecutive columns of the factor.  Rows of U are contiguous (row-major), so
// each nonzero K_i(row, j) costs one coalesced read of row j of U.  The grid's
// y dimension runs over the q operators that share U.
template <class T, int CPL>
__global__ __launch_bounds__(256) void spmm_kernel(SpmmArgs<T> a0, const SpmmArgs<T>* ab,
                                                   const int* done, int lpr) {
  if (done && done[blockIdx.z]) return;
  const SpmmArgs<T>& args = ab ? ab[blockIdx.z] : a0;
  if (int(blockIdx.y) >= args.q) return;
  const DevCsr<T> K = args.op[blockIdx.y];
  T* __restrict__ W = args.W[blockIdx.y];
  const T* __restrict__ U = args.U;
  const int ldu = args.ldu, ldw = args.ldw;
  const int r = args.r_dev ? *args.r_dev : args.r_const;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rpw = 64 / lpr;                       // rows per wave
  const int sub = lane / lpr;
  const int chunk = lane - sub * lpr;
  const int c0 = chunk * CPL;
  if (sub >= rpw || c0 >= r) return;
  const int64_t rows_per_block = int64_t(rpw) * (blockDim.x >> 6);
  for (int64_t row = int64_t(blockIdx.x) * rows_per_block + int64_t(wave) * rpw + sub; row < K.n;
       row += int64_t(gridDim.x) * rows_per_block) {
    T acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = T(0);
    const int e0 = K.rowptr[row], e1 = K.rowptr[row + 1];
    for (int e = e0; e < e1; ++e) {
      const T v = K.val[e];
      const T* __restrict__ u = U + int64_t(K.col[e]) * ldu + c0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[c] += v * u[c];
    }
    T* w = W + row * ldw + c0;
    if (c0 + CPL <= r) {
#pragma unroll
      for (int c = 0; c < CPL; ++c) w[c] = acc[c];
    } else {
#pragma unroll
      for (int c = 0; c < CPL; ++c)
        if (c0 + c < r) w[c] = acc[c];
    }
  }
}

template <class T>
SpmmLaunch<T> make_spmm(const DevCsr<T>* ops, int q, const T* U, int ldu, const int* r_dev,
                        int r_const, int rcap, T* const* W, int ldw, int cpl) {
  LRC_CHECK(q >= 1 && q <= kMaxOps, ST_EINVAL, "spmm: bad operator count");
  LRC_CHECK(rcap >= 1, ST_EINVAL, "spmm: rank capacity must be positive");
  LRC_CHECK(ldu % 8 == 0 && ldw % 8 == 0 && ldu >= rcap && ldw >= rcap, ST_EINVAL,
            "spmm: leading dimensions must be multiples of 8 and cover the rank capacity");
  LRC_CHECK(cpl == 2 || cpl == 4 || cpl == 8, ST_EINVAL, "spmm: columns per lane must be 2, 4 or 8");
  const int lpr = int(ceil_div(rcap, cpl));
  LRC_CHECK(lpr <= 64, ST_EINVAL, "spmm: rank capacity too large for the lane mapping");
  SpmmLaunch<T> l;
  SpmmArgs<T>& a = l.a;
  int64_t n = 0;
  for (int i = 0; i < q; ++i) {
    a.op[i] = ops[i];
    a.W[i] = W[i];
    n = std::max(n, ops[i].n);
  }
  a.q = q;
  a.U = U;
  a.ldu = ldu;
  a.r_dev = r_dev;
  a.r_const = r_const;
  a.ldw = ldw;
  l.cpl = cpl;
  l.lpr = lpr;
  const int rpw = 64 / lpr;
  const int64_t rows_per_block = int64_t(rpw) * 4;
  l.blocks = int(std::max<int64_t>(std::min<int64_t>(ceil_div(n, rows_per_block), 256 * 32), 1));
  l.q = q;
  // algorithmic bytes: values + int32 columns + row pointers of every operator,
  // U read once, every W_i written (all n rows)
  double fixed = 0.0, wrows = 0.0;
  for (int i = 0; i < q; ++i) {
    fixed += double(ops[i].nnz) * (sizeof(T) + 4) + double(ops[i].n + 1) * 4;
    wrows += double(ops[i].n);
  }
  const double nr = double(n);
  l.work.groups = {{{r_dev, r_const}}};
  l.work.f = [=](const std::vector<double>& v) { return fixed + (nr + wrows) * v[0] * sizeof(T); };
  return l;
}

template <class T>
void enqueue_spmm(const SpmmLaunch<T>& l, Batched<SpmmArgs<T>> b, hipStream_t s) {
  ProfScope ps(kcls(K_SPMM, is_f32<T>()), s, b.dev ? Work() : l.work);
  const dim3 grid(unsigned(l.blocks), unsigned(l.q), unsigned(b.n));
  switch (l.cpl) {
    case 2:
      hipLaunchKernelGGL((spmm_kernel<T, 2>), grid, dim3(256), 0, s, l.a, b.dev, b.done, l.lpr);
      break;
    case 4:
      hipLaunchKernelGGL((spmm_kernel<T, 4>), grid, dim3(256), 0, s, l.a, b.dev, b.done, l.lpr);
      break;
    default:
      hipLaunchKernelGGL((spmm_kernel<T, 8>), grid, dim3(256), 0, s, l.a, b.dev, b.done, l.lpr);
      break;
  }
  LRC_HIP(hipGetLastError());
}

template <class T>
void launch_spmm(const DevCsr<T>* ops, int q, const T* U, int ldu, const int* r_dev, int r_const,
                 int rcap, T* const* W, int ldw, int cpl, hipStream_t s) {
  enqueue_spmm(make_spmm(ops, q, U, ldu, r_dev, r_const, rcap, W, ldw, cpl), Batched<SpmmArgs<T>>(),
               s);
}

template SpmmLaunch<float> make_spmm<float>(const DevCsr<float>*, int, const float*, int,
                                            const int*, int, int, float* const*, int, int);
template SpmmLaunch<double> make_spmm<double>(const DevCsr<double>*, int, const double*, int,
                                              const int*, int, int, double* const*, int, int);
template void enqueue_spmm<float>(const SpmmLaunch<float>&, Batched<SpmmArgs<float>>, hipStream_t);
template void enqueue_spmm<double>(const SpmmLaunch<double>&, Batched<SpmmArgs<double>>,
                                   hipStream_t);
template void launch_spmm<float>(const DevCsr<float>*, int, const float*, int, const int*, int,
                                 int, float* const*, int, int, hipStream_t);
template void launch_spmm<double>(const DevCsr<double>*, int, const double*, int, const int*,
                                  int, int, double* const*, int, int, hipStream_t);

// ============================================================== preconditioner
// Each level of the supernode tree is processed in two launches:
//  1. gather: every front row of the level's supernodes is assembled into a
//     dense staging block (forward: b(perm) + children's contribution rows;
//     backward: [y_own ; x(boundary)]), one thread per entry;
//  2. product: one workgroup per (supernode, 16 output rows); the 4 waves
//     split the input dimension, each accumulates a 16 x 64 tile on MFMA
//     (16x16x4), and the partial tiles are summed through LDS.
typedef float floatx4_s __attribute__((ext_vector_type(4)));
typedef double doublex4_s __attribute__((ext_vector_type(4)));
template <class T> struct PMfma;
template <> struct PMfma<float> {
  typedef floatx4_s acc_t;
  static __device__ inline acc_t op(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ inline int drow(int lane, int i) { return 4 * (lane >> 4) + i; }
};
template <> struct PMfma<double> {
  typedef doublex4_s acc_t;
  static __device__ inline acc_t op(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ inline int drow(int lane, int i) { return (lane >> 4) + 4 * i; }
};

constexpr int kKMAX = 64;      // max columns per apply
constexpr int kPT = 16;        // output rows per product workgroup

template <class T, bool FWD>
__global__ __launch_bounds__(256) void prec_gather_kernel(PrecDev<T> P, const int2* __restrict__ rows,
                                                          int nrows, const int64_t* __restrict__ soff,
                                                          PrecItem<T> a0, const PrecItem<T>* ab,
                                                          const int* done, int ldw, int kcap) {
  if (done && done[blockIdx.z]) return;
  const PrecItem<T>& it = ab ? ab[blockIdx.z] : a0;
  const T* __restrict__ R = it.R;
  const int ldr = it.ldr;
  const T* __restrict__ y = it.y;
  const T* __restrict__ x = it.x;
  const T* __restrict__ cb = it.cb;
  T* __restrict__ stage = it.stage;
  const int k = it.k_dev ? *it.k_dev : it.k_const;
  const int64_t total = int64_t(nrows) * kcap;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int item = int(e / kcap);
    const int c = int(e - int64_t(item) * kcap);
    if (c >= k) continue;
    const int2 sp = rows[item];
    const int sn = sp.x, p = sp.y;
    const int ns = P.ns[sn], j0 = P.j0[sn];
    T v;
    if (FWD) {
      v = (p < ns) ? R[int64_t(P.perm[j0 + p]) * ldr + c] : T(0);
      const int64_t fr = P.front_off[sn] + p;
      for (int64_t q = P.asm_ptr[fr]; q < P.asm_ptr[fr + 1]; ++q) v += cb[P.asm_src[q] * ldw + c];
    } else {
      v = (p < ns) ? y[int64_t(j0 + p) * ldw + c]
                   : x[int64_t(P.bnd[P.bnd_off[sn] + p - ns]) * ldw + c];
    }
    stage[(soff[sn] + p) * ldw + c] = v;
  }
}

template <class T, bool FWD>
__global__ __launch_bounds__(256) void prec_product_kernel(PrecDev<T> P, const int2* __restrict__ tasks,
                                                           const int64_t* __restrict__ soff,
                                                           PrecItem<T> a0, const PrecItem<T>* ab,
                                                           const int* done, int ldw) {
  typedef typename PMfma<T>::acc_t acc_t;
  __shared__ T red[4][kPT][kKMAX + 1];
  if (done && done[blockIdx.z]) return;
  const PrecItem<T>& it = ab ? ab[blockIdx.z] : a0;
  const T* __restrict__ stage = it.stage;
  T* __restrict__ y = it.y;
  T* __restrict__ x = it.x;
  T* __restrict__ cb = it.cb;
  T* __restrict__ Z = it.Z;
  const int ldz = it.ldz;
  const int2 task = tasks[blockIdx.x];
  const int sn = task.x, row0 = task.y;
  const int k = it.k_dev ? *it.k_dev : it.k_const;
  const int KT = (k + 15) / 16;
  const int ns = P.ns[sn], f = ns + P.nb[sn], j0 = P.j0[sn];
  const int nin = FWD ? ns : f;
  const int nout = FWD ? f : ns;
  const T* __restrict__ M = FWD ? it.fw + P.fw_off[sn] : it.bw + P.bw_off[sn];
  const int ldM = FWD ? f : ns;                  // column-major: element (row, i) at i * ldM + row
  const T* __restrict__ In = stage + soff[sn] * ldw;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int chunk = ((nin + 3) / 4 + 3) / 4 * 4;
  const int i0 = wave * chunk, i1 = min(nin, i0 + chunk);
  const int orow = row0 + (lane & 15);
  const bool rowok = orow < nout;
  acc_t acc[kKMAX / 16];
#pragma unroll
  for (int t = 0; t < kKMAX / 16; ++t) acc[t] = acc_t{};
  for (int kk = i0; kk < i1; kk += 4) {
    const int i = kk + (lane >> 4);
    const bool iok = i < i1;
    const T a = (iok && rowok) ? M[int64_t(i) * ldM + orow] : T(0);
#pragma unroll
    for (int t = 0; t < kKMAX / 16; ++t) {
      if (t < KT) {
        const int c = t * 16 + (lane & 15);
        const T b = (iok && c < k) ? In[int64_t(i) * ldw + c] : T(0);
        acc[t] = PMfma<T>::op(a, b, acc[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < kKMAX / 16; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wave][PMfma<T>::drow(lane, v)][t * 16 + (lane & 15)] = acc[t][v];
  __syncthreads();
  for (int e = threadIdx.x; e < kPT * kKMAX; e += blockDim.x) {
    const int r = e / kKMAX, c = e - r * kKMAX;
    const int row = row0 + r;
    if (c >= k || row >= nout) continue;
    const T v = red[0][r][c] + red[1][r][c] + red[2][r][c] + red[3][r][c];
    if (FWD) {
      if (row < ns) y[int64_t(j0 + row) * ldw + c] = v;
      else cb[(P.cb_off[sn] + row - ns) * ldw + c] = v + In[int64_t(row) * ldw + c];
    } else {
      x[int64_t(j0 + row) * ldw + c] = v;
      Z[int64_t(P.perm[j0 + row]) * ldz + c] = v;
    }
  }
}

// algorithmic bytes of one level: a staged row is read from its source and
// written once; a product reads the level's dense blocks once plus the staged
// input rows, and writes its output rows (k columns each)
template <class T>
static Work gather_work(const LevelTasks& L, const int* k_dev, int k_const) {
  Work w;
  const double rows = double(L.nrows);
  w.groups = {{{k_dev, k_const}}};
  w.f = [=](const std::vector<double>& v) { return 2.0 * rows * v[0] * sizeof(T); };
  return w;
}
template <class T>
static Work product_work(const LevelTasks& L, const int* k_dev, int k_const) {
  Work w;
  const double blk = L.blk, io = double(L.in_rows + L.out_rows);
  w.groups = {{{k_dev, k_const}}};
  w.f = [=](const std::vector<double>& v) { return (blk + io * v[0]) * sizeof(T); };
  return w;
}

template <class T>
void enqueue_prec_apply(const PrecDev<T>& P, const std::vector<LevelTasks>& fwd,
                        const std::vector<LevelTasks>& bwd, const PrecItem<T>& it,
                        Batched<PrecItem<T>> b, int kcap, int ldw, hipStream_t s) {
  LRC_CHECK(kcap >= 1 && kcap <= kKMAX, ST_EINVAL,
            "preconditioner apply: at most 64 right-hand sides per call");
  LRC_CHECK(ldw >= kcap && it.ldr >= kcap && it.ldz >= kcap, ST_EINVAL,
            "preconditioner apply: leading dimension smaller than the column capacity");
  auto gblocks = [&](int nrows) {
    return unsigned(std::min<int64_t>(std::max<int64_t>(ceil_div(int64_t(nrows) * kcap, 256), 1), 65535));
  };
  const bool batched = b.dev != nullptr;
  for (int pass = 0; pass < 2; ++pass) {
    const bool fw = pass == 0;
    for (const auto& L : fw ? fwd : bwd) {
      if (L.count == 0) continue;
      {
        ProfScope ps(kcls(K_PREC_GATHER, is_f32<T>()), s,
                     batched ? Work() : gather_work<T>(L, it.k_dev, it.k_const));
        const dim3 grid(gblocks(L.nrows), 1, b.n);
        if (fw)
          hipLaunchKernelGGL((prec_gather_kernel<T, true>), grid, dim3(256), 0, s, P, L.rows,
                             L.nrows, P.soff_fwd, it, b.dev, b.done, ldw, kcap);
        else
          hipLaunchKernelGGL((prec_gather_kernel<T, false>), grid, dim3(256), 0, s, P, L.rows,
                             L.nrows, P.soff_bwd, it, b.dev, b.done, ldw, kcap);
      }
      {
        ProfScope ps(kcls(K_PREC_PRODUCT, is_f32<T>()), s,
                     batched ? Work() : product_work<T>(L, it.k_dev, it.k_const));
        const dim3 grid(L.count, 1, b.n);
        if (fw)
          hipLaunchKernelGGL((prec_product_kernel<T, true>), grid, dim3(256), 0, s, P, L.tasks,
                             P.soff_fwd, it, b.dev, b.done, ldw);
        else
          hipLaunchKernelGGL((prec_product_kernel<T, false>), grid, dim3(256), 0, s, P, L.tasks,
                             P.soff_bwd, it, b.dev, b.done, ldw);
      }
    }
  }
  LRC_HIP(hipGetLastError());
}

template <class T>
void launch_prec_apply(const PrecDev<T>& P, const std::vector<LevelTasks>& fwd,
                       const std::vector<LevelTasks>& bwd, const T* R, int ldr, T* Z, int ldz,
                       const int* k_dev, int k_const, int kcap, T* ws_y, T* ws_x, T* ws_cb,
                       T* ws_stage, int ldw, hipStream_t s) {
  const PrecItem<T> it{P.fw, P.bw, R, ldr, Z, ldz, k_dev, k_const, ws_y, ws_x, ws_cb, ws_stage};
  enqueue_prec_apply(P, fwd, bwd, it, Batched<PrecItem<T>>(), kcap, ldw, s);
}

template void enqueue_prec_apply<float>(const PrecDev<float>&, const std::vector<LevelTasks>&,
                                        const std::vector<LevelTasks>&, const PrecItem<float>&,
                                        Batched<PrecItem<float>>, int, int, hipStream_t);
template void enqueue_prec_apply<double>(const PrecDev<double>&, const std::vector<LevelTasks>&,
                                         const std::vector<LevelTasks>&, const PrecItem<double>&,
                                         Batched<PrecItem<double>>, int, int, hipStream_t);
template void launch_prec_apply<float>(const PrecDev<float>&, const std::vector<LevelTasks>&,
                                       const std::vector<LevelTasks>&, const float*, int, float*,
                                       int, const int*, int, int, float*, float*, float*, float*,
                                       int, hipStream_t);
template void launch_prec_apply<double>(const PrecDev<double>&, const std::vector<LevelTasks>&,
                                        const std::vector<LevelTasks>&, const double*, int,
                                        double*, int, const int*, int, int, double*, double*,
                                        double*, double*, int, hipStream_t);

// ============================================================== vectors
template <class Tin, class Tout>
__global__ void cast_kernel(const Tin* __restrict__ x, int ldx, Tout* __restrict__ y, int ldy,
                            int64_t rows, const int* cols_dev, int cols_const, int colcap) {
  const int cols = cols_dev ? *cols_dev : cols_const;
  const int64_t total = rows * colcap;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e / colcap;
    const int c = int(e - r * colcap);
    if (c < cols) y[r * ldy + c] = Tout(x[r * ldx + c]);
  }
}

template <class Tin, class Tout>
void launch_cast(const Tin* x, int ldx, Tout* y, int ldy, int64_t rows, const int* cols_dev,
                 int cols_const, int colcap, hipStream_t s) {
  const int64_t total = rows * colcap;
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>(ceil_div(total, 256), 1), 8192);
  hipLaunchKernelGGL((cast_kernel<Tin, Tout>), dim3(unsigned(blocks)), dim3(256), 0, s, x, ldx, y,
                     ldy, rows, cols_dev, cols_const, colcap);
  LRC_HIP(hipGetLastError());
}
template void launch_cast<double, float>(const double*, int, float*, int, int64_t, const int*, int,
                                         int, hipStream_t);
template void launch_cast<float, double>(const float*, int, double*, int, int64_t, const int*, int,
                                         int, hipStream_t);
template void launch_cast<double, double>(const double*, int, double*, int, int64_t, const int*,
                                          int, int, hipStream_t);
template void launch_cast<float, float>(const float*, int, float*, int, int64_t, const int*, int,
                                        int, hipStream_t);

// ============================================================== median-parameter solve
// Lockstep preconditioned Chebyshev iteration on one column per item (the
// upper-median parameter's system): every kernel's grid z runs over the items.
constexpr int kMedBlocks = 256;   // residual partial sums per item (fixed: deterministic sums)

// dl = alpha dl + beta z ; x += dl   (alpha, beta from the item's control state)
__global__ __launch_bounds__(256) void med_update_kernel(const MedItem* __restrict__ items,
                                                         const MedCtl* __restrict__ ctl,
                                                         const int* __restrict__ done) {
  const int j = blockIdx.z;
  if (done[j]) return;
  const MedItem& a = items[j];
  const double al = ctl[j].alpha, be = ctl[j].beta;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n;
       i += int64_t(gridDim.x) * blockDim.x) {
    const double d = al * a.dl[i * 8] + be * a.z[i * 8];
    a.dl[i * 8] = d;
    a.x[i * 8] += d;
  }
}

// r = f - sum_t coef_t W_t, and per-block partial sums of r^2
__global__ __launch_bounds__(256) void med_resid_kernel(const MedItem* __restrict__ items,
                                                        const int* __restrict__ done) {
  __shared__ double sh[256];
  const int j = blockIdx.z;
  if (done[j]) return;
  const MedItem& a = items[j];
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < a.n;
       i += int64_t(gridDim.x) * blockDim.x) {
    double v = a.f[i];
    for (int t = 0; t < a.q; ++t) v -= a.coef[t] * a.W[(int64_t(t) * a.n + i) * 8];
    a.r[i * 8] = v;
    acc += v * v;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) a.part[blockIdx.x] = sh[0];
}

// One workgroup per item: the residual norm, the stopping test, and the next
// step's coefficients (rho_0 = c/dc with (alpha, beta) = (0, 1/dc); then
// rho' = 1 / (2 dc/c - rho), alpha = rho' rho, beta = 2 rho' / c).
__global__ __launch_bounds__(256) void med_check_kernel(const MedItem* __restrict__ items,
                                                        MedCtl* __restrict__ ctl,
                                                        int* __restrict__ done, int after_update) {
  __shared__ double sh[256];
  const int j = blockIdx.x;
  if (done[j]) return;
  const MedItem& a = items[j];
  sh[threadIdx.x] = threadIdx.x < kMedBlocks ? a.part[threadIdx.x] : 0.0;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  MedCtl c = ctl[j];
  c.norm = sqrt(sh[0]);
  if (after_update) ++c.iters;
  if (!isfinite(c.norm)) c.state = 2;
  else if (c.norm <= c.target) c.state = 1;
  else if (c.iters >= c.max_iter) c.state = 2;
  if (c.state == 0) {
    if (!after_update) {
      c.rho = c.c / c.dc;
      c.alpha = 0.0;
      c.beta = 1.0 / c.dc;
    } else {
      const double rn = 1.0 / (2.0 * c.dc / c.c - c.rho);
      c.alpha = rn * c.rho;
      c.beta = 2.0 * rn / c.c;
      c.rho = rn;
    }
  }
  ctl[j] = c;
  if (c.state) done[j] = 1;
}

void launch_med_update(const MedItem* items, const MedCtl* ctl, const int* done, int nb,
                       int64_t nmax, hipStream_t s) {
  const int64_t blocks = std::min<int64_t>(std::max<int64_t>(ceil_div(nmax, 256), 1), 2048);
  ProfScope ps(kcls(K_VECTOR, false), s);
  hipLaunchKernelGGL(med_update_kernel, dim3(unsigned(blocks), 1, unsigned(nb)), dim3(256), 0, s,
                     items, ctl, done);
  LRC_HIP(hipGetLastError());
}
void launch_med_resid(const MedItem* items, const int* done, int nb, hipStream_t s) {
  ProfScope ps(kcls(K_VECTOR, false), s);
  hipLaunchKernelGGL(med_resid_kernel, dim3(kMedBlocks, 1, unsigned(nb)), dim3(256), 0, s, items,
                     done);
  LRC_HIP(hipGetLastError());
}
void launch_med_check(const MedItem* items, MedCtl* ctl, int* done, int nb, int after_update,
                      hipStream_t s) {
  ProfScope ps(kcls(K_VECTOR, false), s);
  hipLaunchKernelGGL(med_check_kernel, dim3(unsigned(nb)), dim3(256), 0, s, items, ctl, done,
                     after_update);
  LRC_HIP(hipGetLastError());
}
int med_partials() { return kMedBlocks; }

__global__ void fill_kernel(double* p, int64_t count, double v) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += int64_t(gridDim.x) * blockDim.x)
    p[i] = v;
}
void launch_fill(double* p, int64_t count, double v, hipStream_t s) {
  if (count <= 0) return;
  const int64_t blocks = std::min<int64_t>(ceil_div(count, 256), 4096);
  hipLaunchKernelGGL(fill_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, p, count, v);
  LRC_HIP(hipGetLastError());
}

__global__ void copy_cols_kernel(const double* __restrict__ src, int lds, double* __restrict__ dst,
                                 int ldd, int64_t rows, int cols) {
  const int64_t total = rows * cols;
  for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
       e += int64_t(gridDim.x) * blockDim.x) {
    const int64_t r = e / cols;
    const int c = int(e - r * cols);
    dst[r * ldd + c] = src[r * lds + c];
  }
}
void launch_copy_cols(const double* src, int lds, double* dst, int ldd, int64_t rows, int cols,
                      hipStream_t s) {
  if (rows * cols == 0) return;
  const int64_t blocks = std::min<int64_t>(ceil_div(rows * cols, 256), 8192);
  hipLaunchKernelGGL(copy_cols_kernel, dim3(unsigned(blocks)), dim3(256), 0, s, src, lds, dst, ldd,
                     rows, cols);
  LRC_HIP(hipGetLastError());
}

}  // namespace lrc
