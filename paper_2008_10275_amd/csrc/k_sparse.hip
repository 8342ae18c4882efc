// Sparse kernels: fused CSR SpMM of the q operators against a tall factor, the
// level-scheduled supernodal triangular solves of the preconditioner, and the
// small vector kernels of the single-column (median parameter) solve.
#include <algorithm>

#include "kernels.hpp"
#include "gmem.hpp"
#include "prof.hpp"

namespace lrc {

// 16-byte vector of T
template <class T> struct V16;
template <> struct V16<float> {
  typedef float4 t;
  static constexpr int n = 4;
  static __device__ inline t zero() { return make_float4(0.f, 0.f, 0.f, 0.f); }
  static __device__ inline void add(t& a, const t& b) { a.x += b.x; a.y += b.y; a.z += b.z; a.w += b.w; }
  static __device__ inline void fma(t& a, float s, const t& b) {
    a.x += s * b.x; a.y += s * b.y; a.z += s * b.z; a.w += s * b.w;
  }
};
template <> struct V16<double> {
  typedef double2 t;
  static constexpr int n = 2;
  static __device__ inline t zero() { return make_double2(0.0, 0.0); }
  static __device__ inline void add(t& a, const t& b) { a.x += b.x; a.y += b.y; }
  static __device__ inline void fma(t& a, double s, const t& b) { a.x += s * b.x; a.y += s * b.y; }
};

// ============================================================== SpMM
// Every row of K_i is handled by `lpr` consecutive lanes; a lane owns NV
// 16-byte vectors of the factor's columns, interleaved with stride lpr, so
// that every load of a row of U and every store of a row of W_i is one
// contiguous span per instruction (whole cache lines, not 8-byte pieces).
// lpr follows the device rank (lanes past it would idle).  The nonzeros of a
// row are taken in batches, their column indices loaded before the U rows
// they select (padding slots reuse the row's first column with a zero value),
// so that a row costs two dependent load rounds per batch after the row
// pointers.  Operators whose rows are about equally long (stencils, up to 27
// entries) also carry a padded column-major copy: a row then needs no row
// pointers, and a wave's index loads for consecutive rows are contiguous.
// The row of W: a lane's NV vectors of the accumulated row.
template <class T, int NV>
__device__ __forceinline__ void spmm_store(const typename V16<T>::t* acc, int64_t row,
                                           T* __restrict__ W, int ldw, int r, int nvec, int lpr,
                                           int chunk, bool wpad) {
  typedef typename V16<T>::t V;
  constexpr int VW = V16<T>::n;
  T* __restrict__ wr = W + row * ldw;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int j = chunk + v * lpr;
    if (j >= nvec) break;
    if ((j + 1) * VW <= r) {
      gstore(reinterpret_cast<V*>(wr + j * VW), acc[v]);
    } else {
      // the row's last, partial vector (static element indices: the
      // accumulator stays in registers).  With wpad the columns past the rank
      // (inside the row's padding: ldw >= the rank rounded up to 8) are written
      // as zeros, so that the store is one whole vector.
      T ap[VW];
      *reinterpret_cast<V*>(ap) = acc[v];
      if (wpad) {
#pragma unroll
        for (int x = 0; x < VW; ++x)
          if (j * VW + x >= r) ap[x] = T(0);
        gstore(reinterpret_cast<V*>(wr + j * VW), *reinterpret_cast<const V*>(ap));
      } else {
#pragma unroll
        for (int x = 0; x < VW; ++x)
          if (j * VW + x < r) gmem(wr)[j * VW + x] = ap[x];
      }
    }
  }
}

// One row of one operator: acc = K(row, :) U, stored to W.
template <class T, int NV, int NZB>
__device__ __forceinline__ void spmm_row(const DevCsr<T>& K, int64_t row,
                                         const T* __restrict__ U, int ldu, T* __restrict__ W,
                                         int ldw, int r, int nvec, int lpr, int chunk, bool wpad) {
  typedef typename V16<T>::t V;
  V acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = V16<T>::zero();
  const int e0 = gmem(K.rowptr)[row], e1 = gmem(K.rowptr)[row + 1];
  for (int e = e0; e < e1; e += NZB) {
    int cj[NZB];
    T vj[NZB];
#pragma unroll
    for (int u = 0; u < NZB; ++u) {
      const bool ok = e + u < e1;
      const int x = ok ? e + u : e0;
      cj[u] = gmem(K.col)[x];
      const T val = gmem(K.val)[x];
      vj[u] = ok ? val : T(0);
    }
#pragma unroll
    for (int u = 0; u < NZB; ++u) {
      const V* ur = reinterpret_cast<const V*>(U + int64_t(cj[u]) * ldu);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int j = chunk + v * lpr;
        if (NV == 1 || j < nvec) V16<T>::fma(acc[v], vj[u], gload(ur + j));
      }
    }
  }
  spmm_store<T, NV>(acc, row, W, ldw, r, nvec, lpr, chunk, wpad);
}

// The same product from the padded copy: visited row x's EW entries are one
// round of coalesced index and value loads (consecutive rows adjacent), then
// the factor rows they select; padding slots add 0 times a valid row, so the
// sum (taken in the row's entry order) has the CSR path's bits.
template <class T, int NV, int EW>
__device__ __forceinline__ void spmm_row_ell(const DevCsr<T>& K, int64_t x, int64_t row,
                                             const T* __restrict__ U, int ldu, T* __restrict__ W,
                                             int ldw, int r, int nvec, int lpr, int chunk,
                                             bool wpad) {
  typedef typename V16<T>::t V;
  V acc[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) acc[v] = V16<T>::zero();
  int cj[EW];
  T vj[EW];
#pragma unroll
  for (int u = 0; u < EW; ++u) {
    cj[u] = gmem(K.ecol)[int64_t(u) * K.nrows + x];
    vj[u] = gmem(K.eval)[int64_t(u) * K.nrows + x];
  }
#pragma unroll
  for (int u = 0; u < EW; ++u) {
    const V* ur = reinterpret_cast<const V*>(U + int64_t(cj[u]) * ldu);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int j = chunk + v * lpr;
      if (NV == 1 || j < nvec) V16<T>::fma(acc[v], vj[u], gload(ur + j));
    }
  }
  spmm_store<T, NV>(acc, row, W, ldw, r, nvec, lpr, chunk, wpad);
}

// Workgroups per operator and row block: consecutive workgroups of one XCD
// (hardware workgroup w runs on XCD w mod 8) take the q operators of one row
// block, so that the rows of U one operator loads serve the others from that
// XCD's L2 while every row keeps a single dependent chain.  The grid is a
// multiple of 8 q.  The nonzeros of a row are taken NZB at a time: the
// operator's longest row when it is 5 or 9 (the stencils' own widths: no
// padded slot on interior rows), else 4.
// WIDE: the launch holds an operator whose padded copy is 27 entries wide;
// the narrower instantiation leaves that path out, whose 27 index and value
// registers per lane would otherwise set the register count (and so the
// occupancy) of every launch.
template <class T, int NV, bool WIDE>
__global__ __launch_bounds__(512) void spmm_kernel(SpmmArgs<T> a0, const SpmmArgs<T>* ab,
                                                   const int* done, int lpr_cap) {
  constexpr int VW = V16<T>::n;
  if (done && done[blockIdx.z]) return;
  // the item's fields are copied through a pointer of one address space
  // (device array or kernel argument), so that they arrive in scalar
  // registers instead of through generic per-lane loads
  const SpmmArgs<T>* ap = ab ? ab + blockIdx.z : nullptr;
  const int q = ap ? ap->q : a0.q;
  const int L = blockIdx.x, xcd = L & 7, kx = L >> 3;
  const int op = kx % q, rb = (kx / q) * 8 + xcd;   // row block of this workgroup's sweep
  const int nrb = int(gridDim.x) / q;                // row blocks per sweep
  if (rb >= nrb) return;
  DevCsr<T> K;
  T* W;
  const T* U;
  const int* r_dev;
  int r_const, ldu, ldw, wpad_i, skip;
  if (ap) {
    K = ap->op[op];
    W = ap->W[op];
    U = ap->U;
    r_dev = ap->r_dev;
    r_const = ap->r_const;
    ldu = ap->ldu;
    ldw = ap->ldw;
    wpad_i = ap->wpad;
    skip = ap->skip_empty;
  } else {
    K = a0.op[op];
    W = a0.W[op];
    U = a0.U;
    r_dev = a0.r_dev;
    r_const = a0.r_const;
    ldu = a0.ldu;
    ldw = a0.ldw;
    wpad_i = a0.wpad;
    skip = a0.skip_empty;
  }
  const int r = __builtin_amdgcn_readfirstlane(r_dev ? *r_dev : r_const);
  if (r <= 0) return;
  const int nvec = (r + VW - 1) / VW;            // vectors per row
  const int lpr = min(lpr_cap, (nvec + NV - 1) / NV);
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int rpw = 64 / lpr;                       // rows per wave
  const int sub = lane / lpr;
  const int chunk = lane - sub * lpr;
  if (sub >= rpw || chunk >= nvec) return;
  const int64_t rows_per_block = int64_t(rpw) * (blockDim.x >> 6);
  const int64_t stride = int64_t(nrb) * rows_per_block;
  const int64_t first = int64_t(rb) * rows_per_block + int64_t(wave) * rpw + sub;
  const int maxrow = __builtin_amdgcn_readfirstlane(K.maxrow);
  const bool wpad = wpad_i != 0;
  // with a row list only the non-empty rows are visited (the solid box of
  // K_1, K_2: a sixth of the rows); the list is read in order, so a wave's
  // lookups are one contiguous span
  const int* __restrict__ rl = skip ? K.rows : nullptr;
  const int64_t nvis = rl ? K.nrows : K.n;
  // the padded copy covers exactly the visited rows (all rows, or the list)
  const int ew = __builtin_amdgcn_readfirstlane((rl || !K.rows) ? K.ew : 0);
#define LRC_ELL(EW)                                                                               \
  for (int64_t x = first; x < nvis; x += stride)                                                  \
    spmm_row_ell<T, NV, EW>(K, x, rl ? int64_t(gmem(rl)[x]) : x, U, ldu, W, ldw, r, nvec, lpr,    \
                            chunk, wpad)
  if (ew == 5) {
    LRC_ELL(5);
  } else if (ew == 7) {
    LRC_ELL(7);
  } else if (ew == 9) {
    LRC_ELL(9);
  } else if (WIDE && ew == 27) {
    LRC_ELL(27);
  } else if (maxrow <= 5) {
    for (int64_t x = first; x < nvis; x += stride)
      spmm_row<T, NV, 5>(K, rl ? int64_t(gmem(rl)[x]) : x, U, ldu, W, ldw, r, nvec, lpr, chunk, wpad);
  } else if (maxrow <= 9) {
    for (int64_t x = first; x < nvis; x += stride)
      spmm_row<T, NV, 9>(K, rl ? int64_t(gmem(rl)[x]) : x, U, ldu, W, ldw, r, nvec, lpr, chunk, wpad);
  } else {
    for (int64_t x = first; x < nvis; x += stride)
      spmm_row<T, NV, 4>(K, rl ? int64_t(gmem(rl)[x]) : x, U, ldu, W, ldw, r, nvec, lpr, chunk, wpad);
  }
#undef LRC_ELL
}

template <class T>
SpmmLaunch<T> make_spmm(const DevCsr<T>* ops, int q, const T* U, int ldu, const int* r_dev,
                        int r_const, int rcap, T* const* W, int ldw, SpmmCfg cfg,
                        bool skip_empty) {
  const int cpl = cfg.cpl > 0 ? cfg.cpl : (sizeof(T) == 8 ? 2 : 4);
  LRC_CHECK(q >= 1 && q <= kMaxOps, ST_EINVAL, "spmm: bad operator count");
  LRC_CHECK(rcap >= 1, ST_EINVAL, "spmm: rank capacity must be positive");
  LRC_CHECK(ldu % 8 == 0 && ldw % 8 == 0 && ldu >= rcap && ldw >= rcap, ST_EINVAL,
            "spmm: leading dimensions must be multiples of 8 and cover the rank capacity");
  LRC_CHECK(cpl == 1 || cpl == 2 || cpl == 4 || cpl == 8, ST_EINVAL,
            "spmm: columns per lane must be 1, 2, 4 or 8");
  LRC_CHECK(cfg.waves >= 1 && cfg.waves <= 8 && cfg.max_blocks >= 1, ST_EINVAL,
            "spmm: 1..8 waves per workgroup");
  // a lane owns nv 16-byte vectors (cpl columns, at least one vector)
  constexpr int VW = 16 / int(sizeof(T));
  const int nv = std::max(1, cpl / VW);
  const int lpr = int(ceil_div(ceil_div(rcap, VW), nv));
  LRC_CHECK(lpr <= 64, ST_EINVAL, "spmm: rank capacity too large for the lane mapping");
  auto al16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  LRC_CHECK(al16(U), ST_EINVAL, "spmm: the factor must be 16-byte aligned");
  for (int i = 0; i < q; ++i)
    LRC_CHECK(al16(W[i]), ST_EINVAL, "spmm: the products must be 16-byte aligned");
  SpmmLaunch<T> l;
  SpmmArgs<T>& a = l.a;
  int64_t n = 0;
  for (int i = 0; i < q; ++i) {
    a.op[i] = ops[i];
    a.W[i] = W[i];
    n = std::max(n, ops[i].n);
  }
  a.q = q;
  l.wide = false;
  for (int i = 0; i < q; ++i) l.wide = l.wide || ops[i].ew > 9;
  a.U = U;
  a.ldu = ldu;
  a.r_dev = r_dev;
  a.r_const = r_const;
  a.ldw = ldw;
  a.wpad = 1;   // the solver's own product buffers; callers' buffers clear it
  a.skip_empty = skip_empty ? 1 : 0;
  l.cpl = cpl;
  l.nv = nv;
  l.lpr = lpr;
  l.waves = cfg.waves;
  const int rpw = 64 / lpr;
  const int64_t rows_per_block = int64_t(rpw) * cfg.waves;
  // row blocks per sweep, a multiple of 8; q workgroups each
  int64_t rbs = std::max<int64_t>(std::min<int64_t>(ceil_div(n, rows_per_block), cfg.max_blocks), 1);
  rbs = (rbs + 7) / 8 * 8;
  LRC_CHECK(rbs * q < (int64_t(1) << 31), ST_EINVAL, "spmm: grid too large");
  l.blocks = int(rbs * q);
  l.q = q;
  // algorithmic bytes: values + int32 columns of every operator, U read once,
  // and per visited row its row pointers and its row of W_i (all n rows, or
  // the non-empty rows with their list entries)
  double fixed = 0.0, wrows = 0.0;
  for (int i = 0; i < q; ++i) {
    const bool list = skip_empty && ops[i].rows;
    fixed += double(ops[i].nnz) * (sizeof(T) + 4) +
             (list ? double(ops[i].nrows) * 12 : double(ops[i].n + 1) * 4);
    wrows += list ? double(ops[i].nrows) : double(ops[i].n);
  }
  const double nr = double(n);
  l.work.groups = {{{r_dev, r_const}}};
  l.work.f = [=](const std::vector<double>& v) { return fixed + (nr + wrows) * v[0] * sizeof(T); };
  return l;
}

template <class T>
void enqueue_spmm(const SpmmLaunch<T>& l, Batched<SpmmArgs<T>> b, hipStream_t s) {
  ProfScope ps(kcls(K_SPMM, is_f32<T>()), s, l.work);
  const dim3 grid(unsigned(l.blocks), 1, unsigned(b.n)), blk(64 * l.waves);
#define LRC_SPMM(NV)                                                                              \
  do {                                                                                            \
    if (l.wide)                                                                                   \
      hipLaunchKernelGGL((spmm_kernel<T, NV, true>), grid, blk, 0, s, l.a, b.dev, b.done, l.lpr);  \
    else                                                                                          \
      hipLaunchKernelGGL((spmm_kernel<T, NV, false>), grid, blk, 0, s, l.a, b.dev, b.done, l.lpr); \
  } while (0)
  switch (l.nv) {
    case 1: LRC_SPMM(1); break;
    case 2: LRC_SPMM(2); break;
    default: LRC_SPMM(4); break;
  }
#undef LRC_SPMM
  LRC_HIP(hipGetLastError());
}

template <class T>
void launch_spmm(const DevCsr<T>* ops, int q, const T* U, int ldu, const int* r_dev, int r_const,
                 int rcap, T* const* W, int ldw, int cpl, hipStream_t s) {
  SpmmCfg cfg;
  cfg.cpl = cpl;
  enqueue_spmm(make_spmm(ops, q, U, ldu, r_dev, r_const, rcap, W, ldw, cfg), Batched<SpmmArgs<T>>(),
               s);
}

template SpmmLaunch<float> make_spmm<float>(const DevCsr<float>*, int, const float*, int,
                                            const int*, int, int, float* const*, int, SpmmCfg,
                                            bool);
template SpmmLaunch<double> make_spmm<double>(const DevCsr<double>*, int, const double*, int,
                                              const int*, int, int, double* const*, int, SpmmCfg,
                                              bool);
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
//     backward: [y_own ; x(boundary)]), from a precomputed source descriptor
//     per row, 16 bytes per thread;
//  2. product: one task per (supernode, 16 output rows), a 16 x 16k tile
//     accumulated on MFMA (16x16x4).  Levels whose inputs are short give every
//     wave its own task; long inputs are split over NW waves of one workgroup
//     whose partial tiles are summed through LDS (levels with more tasks than
//     resident waves keep one wave per task up to 256 inputs).  The input
//     loop issues the loads of eight MFMA steps (four in single-wave forward
//     tasks) before their products.
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
constexpr int kPT = 16;        // output rows per product task

template <class T, bool FWD>
__global__ __launch_bounds__(256) void prec_gather_kernel(const GatherRow* __restrict__ rows,
                                                          int nrows, int vpr,
                                                          const int64_t* __restrict__ asm_src,
                                                          PrecItem<T> a0, const PrecItem<T>* ab,
                                                          const int* done, int ldw) {
  typedef typename V16<T>::t vec;
  constexpr int VN = V16<T>::n;
  // the done flag, the item and the thread's first row descriptor are read in
  // one round (all are valid memory whatever the flag says); the empty asm
  // statement keeps them ahead of the exit, so that a launch does not wait
  // on one round per pointer
  const int64_t total = int64_t(nrows) * vpr;
  const int64_t e0 = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  const int dn = done ? done[blockIdx.z] : 0;
  PrecItem<T> it;
  if (ab)
    it = ab[blockIdx.z];
  else
    it = a0;
  const GatherRow g0 = e0 < total ? rows[int(e0 / vpr)] : GatherRow{};
  asm volatile("" ::"v"(dn), "v"(g0.src), "v"(g0.na));
  if (dn) return;
  for (int64_t e = e0; e < total; e += int64_t(gridDim.x) * blockDim.x) {
    const int row = int(e / vpr);
    const int c = int(e - int64_t(row) * vpr) * VN;
    const GatherRow g = e == e0 ? g0 : rows[row];
    vec v;
    if (FWD) {
      v = V16<T>::zero();
      if (g.src >= 0) v = gload(reinterpret_cast<const vec*>(it.R + int64_t(g.src) * it.ldr + c));
      for (int q = 0; q < g.na; ++q)
        V16<T>::add(v, gload(reinterpret_cast<const vec*>(it.cb + gmem(asm_src)[g.a0 + q] * ldw +
                                                          c)));
    } else {
      const T* src = g.src >= 0 ? it.y + int64_t(g.src) * ldw : it.x + int64_t(-g.src - 1) * ldw;
      v = gload(reinterpret_cast<const vec*>(src + c));
    }
    gstore(reinterpret_cast<vec*>(it.stage + int64_t(row) * ldw + c), v);
  }
}

// DIRECT: the inputs are read where they live instead of from the staged
// front (backward: y rows and x boundary rows; forward levels without
// contributions: R rows by the permutation), so the level needs no gather.
template <class T, bool FWD, int NW, int KTM, bool DIRECT, int U>
__global__ __launch_bounds__(NW > 4 ? 64 * NW : 256) void prec_product_kernel(
    PrecDev<T> P, const int2* __restrict__ tasks, int ntasks, const int64_t* __restrict__ soff,
    PrecItem<T> a0, const PrecItem<T>* ab, const int* done, int ldw) {
  typedef typename PMfma<T>::acc_t acc_t;
  constexpr int WPB = NW > 4 ? NW : 4;    // waves per workgroup
  constexpr int TPB = WPB / NW;           // tasks per workgroup
  __shared__ T red[NW > 1 ? NW : 1][KTM * 4][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  // workgroups are dealt to the 8 XCDs in turn (w -> XCD w % 8): the grid (a
  // multiple of 8) gives XCD x the contiguous eighth x of the task range, so
  // that the tasks of one supernode, which all read its input rows, share an L2
  const int bx = int(blockIdx.x & 7) * int(gridDim.x >> 3) + int(blockIdx.x >> 3);
  const int tk = bx * TPB + wave / NW;   // uniform per workgroup when NW > 1
  const bool live = tk < ntasks;
  const int wv = wave % NW;
  // Launches of the upper levels are short, so their cost is the chain of
  // dependent loads before the first product: the done flag, the item and the
  // task are read in one round, the supernode's fields and the width in the
  // next (all valid memory whatever the flag says; a wave past the last task
  // reads task 0); the empty asm statement keeps these loads ahead of the
  // exit (uniform per workgroup when NW > 1).
  const int dn = done ? done[blockIdx.z] : 0;
  PrecItem<T> it;
  if (ab)
    it = ab[blockIdx.z];
  else
    it = a0;
  const int2 task = tasks[live ? tk : 0];
  const int sn = task.x, row0 = task.y;
  const int k = it.k_dev ? *it.k_dev : it.k_const;
  const int ns = P.ns[sn], f = ns + P.nb[sn], j0 = P.j0[sn];
  const int leaf = FWD ? 0 : P.leaf[sn];
  asm volatile("" ::"v"(dn), "v"(k), "v"(f), "v"(j0), "v"(leaf));
  if (!live || dn) return;
  const int nin = FWD ? ns : f;
  const int nout = FWD ? f : ns;
  const T* __restrict__ M = FWD ? it.fw + P.fw_off[sn] : it.bw + P.bw_off[sn];
  const int ldM = FWD ? f : ns;                  // column-major: element (row, i) at i * ldM + row
  const T* __restrict__ In = DIRECT ? nullptr : it.stage + soff[sn] * ldw;
  const int* __restrict__ bnd = DIRECT && !FWD ? P.bnd + P.bnd_off[sn] : nullptr;
  // source row number of input i: direct inputs look it up (forward: the
  // permutation; backward: the boundary list past ns), which the loop fetches
  // one iteration ahead so that an iteration waits on one round of loads
  auto in_idx = [&](int i) -> int {
    if (!DIRECT) return i;
    if (FWD) return gmem(P.perm)[j0 + i];
    return i < ns ? j0 + i : gmem(bnd)[i - ns];
  };
  auto in_row = [&](int i, int idx) -> const T* {
    if (!DIRECT) return In + int64_t(idx) * ldw;
    if (FWD) return it.R + int64_t(idx) * it.ldr;
    return (i < ns ? it.y : it.x) + int64_t(idx) * ldw;
  };
  // The diagonal parts of the blocks are triangular (forward: L^-1 on the
  // first ns rows, backward: U^-1 on the first ns columns), so a task whose
  // 16 output rows lie in the diagonal part reads only the inputs that meet
  // the triangle: forward i < row0 + 16, backward i >= row0.
  const int lo = FWD ? 0 : row0;
  const int hi = (FWD && row0 + kPT <= ns) ? row0 + kPT : nin;
  const int chunk = NW == 1 ? hi - lo : (hi - lo + 4 * NW - 1) / (4 * NW) * 4;
  const int i0 = lo + wv * chunk, i1 = min(hi, i0 + chunk);
  const int orow = row0 + (lane & 15);
  const bool rowok = orow < nout;
  acc_t acc[KTM];
#pragma unroll
  for (int t = 0; t < KTM; ++t) acc[t] = acc_t{};
  int nidx[DIRECT ? U : 1];
  if constexpr (DIRECT) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 4 * u + (lane >> 4);
      nidx[u] = i < i1 ? in_idx(i) : 0;
    }
  }
  for (int kk = i0; kk < i1; kk += 4 * U) {
    T a[U], b[U][KTM];
    const T* rp[U];
    if constexpr (DIRECT) {
      int cidx[U];
#pragma unroll
      for (int u = 0; u < U; ++u) cidx[u] = nidx[u];
      if (kk + 4 * U < i1) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int i = kk + 4 * U + 4 * u + (lane >> 4);
          nidx[u] = i < i1 ? in_idx(i) : 0;
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = kk + 4 * u + (lane >> 4);
        rp[u] = i < i1 ? in_row(i, cidx[u]) : nullptr;
      }
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int i = kk + 4 * u + (lane >> 4);
        rp[u] = i < i1 ? in_row(i, i) : nullptr;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = kk + 4 * u + (lane >> 4);
      const bool iok = i < i1;
      a[u] = (iok && rowok) ? gmem(M)[int64_t(i) * ldM + orow] : T(0);
#pragma unroll
      for (int t = 0; t < KTM; ++t) {
        const int c = t * 16 + (lane & 15);
        b[u][t] = (iok && c < k) ? gmem(rp[u])[c] : T(0);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int t = 0; t < KTM; ++t) acc[t] = PMfma<T>::op(a[u], b[u][t], acc[t]);
  }
  auto store = [&](int r, int c, T v) {
    const int row = row0 + r;
    if (c >= k || row >= nout) return;
    if (FWD) {
      if (row < ns) gmem(it.y)[int64_t(j0 + row) * ldw + c] = v;
      else
        gmem(it.cb)[(P.cb_off[sn] + row - ns) * ldw + c] =
            DIRECT ? v : v + gmem(In)[int64_t(row) * ldw + c];
    } else {
      if (!leaf) gmem(it.x)[int64_t(j0 + row) * ldw + c] = v;
      const int64_t zo = int64_t(gmem(P.perm)[j0 + row]) * it.ldz + c;
      if (it.Z64)
        gmem(it.Z64)[zo] = double(v);
      else
        gmem(it.Z)[zo] = v;
    }
  };
  if (NW == 1) {
#pragma unroll
    for (int t = 0; t < KTM; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) store(PMfma<T>::drow(lane, v), t * 16 + (lane & 15), acc[t][v]);
    return;
  }
  // partial tiles in lane order; the workgroup sums them in a fixed order
#pragma unroll
  for (int t = 0; t < KTM; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) red[wv][t * 4 + v][lane] = acc[t][v];
  __syncthreads();
  for (int e = threadIdx.x; e < KTM * 4 * 64; e += blockDim.x) {
    const int tv = e >> 6, l = e & 63;
    T sum = red[0][tv][l];
#pragma unroll
    for (int w = 1; w < NW; ++w) sum += red[w][tv][l];
    store(PMfma<T>::drow(l, tv & 3), (tv >> 2) * 16 + (l & 15), sum);
  }
}

// algorithmic bytes of one level: a staged row is read from its source and
// written once; a product reads the level's dense blocks once plus the staged
// input rows, and writes its output rows (k columns each)
// (kterms: the widths of all items of the launch; their sum is v[0])
template <class T>
static Work gather_work(const LevelTasks& L, const std::vector<WTerm>& kterms) {
  Work w;
  const double rows = double(L.nrows);
  w.groups = {kterms};
  w.f = [=](const std::vector<double>& v) { return 2.0 * rows * v[0] * sizeof(T); };
  return w;
}
// (z64: the backward output rows of the solution go out in fp64, z_rows of
// them per level, each k columns wider by 8 - sizeof(T) bytes)
template <class T>
static Work product_work(const LevelTasks& L, const std::vector<WTerm>& kterms,
                         double z_rows = 0.0) {
  Work w;
  const double blk = L.blk * double(kterms.size()), io = double(L.in_rows + L.out_rows);
  const double zx = z_rows * (8.0 - sizeof(T));
  w.groups = {kterms};
  w.f = [=](const std::vector<double>& v) { return (blk + io * v[0]) * sizeof(T) + zx * v[0]; };
  return w;
}

template <class T>
void check_prec_item(const PrecItem<T>& it, int kcap, int ldw) {
  constexpr int VN = V16<T>::n;
  auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  LRC_CHECK(kcap >= 1 && kcap <= kKMAX, ST_EINVAL,
            "preconditioner apply: at most 64 right-hand sides per call");
  LRC_CHECK(ldw >= kcap && it.ldr >= kcap && it.ldz >= kcap, ST_EINVAL,
            "preconditioner apply: leading dimension smaller than the column capacity");
  LRC_CHECK(it.ldr % VN == 0 && ldw % VN == 0 && ldw >= (kcap + VN - 1) / VN * VN &&
                it.ldr >= (kcap + VN - 1) / VN * VN,
            ST_EINVAL, "preconditioner apply: leading dimensions must be multiples of 16 bytes");
  LRC_CHECK(al(it.R) && al(it.y) && al(it.x) && al(it.cb) && al(it.stage), ST_EINVAL,
            "preconditioner apply: operands must be 16-byte aligned");
}

template <class T, bool FWD, int NW>
static void launch_product_nw(int KTM, dim3 grid, dim3 blk, hipStream_t s, const PrecDev<T>& P,
                              const LevelTasks& L, const int64_t* soff, const PrecItem<T>& it,
                              const Batched<PrecItem<T>>& b, int ldw) {
  // eight MFMA steps of loads in flight per wave (four for single-wave forward
  // tasks, whose inputs are at most 64 long: more only costs occupancy there)
  constexpr int U = (NW == 1 && FWD) ? 4 : 8;
#define LRC_PP(KT)                                                                                \
  do {                                                                                            \
    if (L.direct)                                                                                 \
      hipLaunchKernelGGL((prec_product_kernel<T, FWD, NW, KT, true, U>), grid, blk, 0, s, P,       \
                         L.tasks, L.count, soff, it, b.dev, b.done, ldw);                         \
    else                                                                                          \
      hipLaunchKernelGGL((prec_product_kernel<T, FWD, NW, KT, false, U>), grid, blk, 0, s, P,      \
                         L.tasks, L.count, soff, it, b.dev, b.done, ldw);                         \
  } while (0)
  switch (KTM) {
    case 1: LRC_PP(1); break;
    case 2: LRC_PP(2); break;
    case 3: LRC_PP(3); break;
    default: LRC_PP(4); break;
  }
#undef LRC_PP
}

// ILU(0) triangular solves, one launch per level: a thread takes one (row,
// column) of the level, y_i = r_i - sum_{j < i} L_ij y_j forward and
// z_i = (y_i - sum_{j > i} U_ij z_j) / U_ii backward; the rows a level reads
// belong to earlier launches.  Threads of one row are consecutive, so the
// reads of a neighbour's row are contiguous.
template <class T, bool FWD>
__global__ __launch_bounds__(256) void ilu_level_kernel(PrecDev<T> P, int off, int count,
                                                        PrecItem<T> it0, const PrecItem<T>* ab,
                                                        const int* done, int ldw) {
  if (done && done[blockIdx.z]) return;
  const PrecItem<T>& it = ab ? ab[blockIdx.z] : it0;
  const int k = it.k_dev ? *it.k_dev : it.k_const;
  if (k <= 0) return;
  const int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= int64_t(count) * k) return;
  const int c = int(t % k);
  const int row = (FWD ? P.irows_f : P.irows_b)[off + int(t / k)];
  const T* __restrict__ lu = it.fw;
  const int d = P.idiag[row];
  if (FWD) {
    T acc = it.R[int64_t(row) * it.ldr + c];
    for (int e = P.irp[row]; e < d; ++e) acc -= lu[e] * it.y[int64_t(P.icol[e]) * ldw + c];
    it.y[int64_t(row) * ldw + c] = acc;
  } else {
    T acc = it.y[int64_t(row) * ldw + c];
    for (int e = d + 1; e < P.irp[row + 1]; ++e) acc -= lu[e] * it.Z[int64_t(P.icol[e]) * it.ldz + c];
    it.Z[int64_t(row) * it.ldz + c] = acc / lu[d];
  }
}

template <class T>
static void enqueue_ilu_apply(const PrecDev<T>& P, const std::vector<LevelTasks>& fwd,
                              const std::vector<LevelTasks>& bwd, const PrecItem<T>& it,
                              Batched<PrecItem<T>> b, int kcap, int ldw, hipStream_t s,
                              const std::vector<WTerm>& kt) {
  for (int pass = 0; pass < 2; ++pass) {
    const bool fw = pass == 0;
    for (const auto& L : fw ? fwd : bwd) {
      if (L.count == 0) continue;
      Work w;
      w.groups = {kt};
      const double nnz = double(L.ilu_nnz), rows = double(L.count);
      w.f = [=](const std::vector<double>& v) {
        return nnz * (sizeof(T) + 4) + (nnz + 2.0 * rows) * v[0] * sizeof(T);
      };
      ProfScope ps(kcls(K_PREC_PRODUCT, is_f32<T>()), s, w);
      const dim3 grid(unsigned(ceil_div(int64_t(L.count) * kcap, 256)), 1, b.n);
      if (fw)
        hipLaunchKernelGGL((ilu_level_kernel<T, true>), grid, dim3(256), 0, s, P, L.ilu_off,
                           L.count, it, b.dev, b.done, ldw);
      else
        hipLaunchKernelGGL((ilu_level_kernel<T, false>), grid, dim3(256), 0, s, P, L.ilu_off,
                           L.count, it, b.dev, b.done, ldw);
    }
  }
  LRC_HIP(hipGetLastError());
}

template <class T>
void enqueue_prec_apply(const PrecDev<T>& P, const std::vector<LevelTasks>& fwd,
                        const std::vector<LevelTasks>& bwd, const PrecItem<T>& it,
                        Batched<PrecItem<T>> b, int kcap, int ldw, hipStream_t s,
                        const std::vector<WTerm>* kterms) {
  check_prec_item(it, kcap, ldw);
  const std::vector<WTerm> kt = kterms ? *kterms : std::vector<WTerm>{{it.k_dev, it.k_const}};
  if (P.kind == 1) {
    enqueue_ilu_apply(P, fwd, bwd, it, b, kcap, ldw, s, kt);
    return;
  }
  constexpr int VN = V16<T>::n;
  const int vpr = (kcap + VN - 1) / VN;
  const int KTM = (kcap + 15) / 16;
  auto gblocks = [&](int nrows) {
    return unsigned(std::min<int64_t>(std::max<int64_t>(ceil_div(int64_t(nrows) * vpr, 256), 1), 65535));
  };
  for (int pass = 0; pass < 2; ++pass) {
    const bool fw = pass == 0;
    for (const auto& L : fw ? fwd : bwd) {
      if (L.count == 0) continue;
      if (!L.direct) {
        ProfScope ps(kcls(K_PREC_GATHER, is_f32<T>()), s, gather_work<T>(L, kt));
        const dim3 grid(gblocks(L.nrows), 1, b.n);
        if (fw)
          hipLaunchKernelGGL((prec_gather_kernel<T, true>), grid, dim3(256), 0, s, L.grows,
                             L.nrows, vpr, P.asm_src, it, b.dev, b.done, ldw);
        else
          hipLaunchKernelGGL((prec_gather_kernel<T, false>), grid, dim3(256), 0, s, L.grows,
                             L.nrows, vpr, P.asm_src, it, b.dev, b.done, ldw);
      }
      {
        ProfScope ps(kcls(K_PREC_PRODUCT, is_f32<T>()), s,
                     product_work<T>(L, kt, (!fw && it.Z64) ? double(L.z_rows) : 0.0));
        // waves per task by the level's longest input; a level with more tasks
        // than the GPU holds waves is throughput-bound: one wave per task there
        // (no partial tiles to sum) unless the inputs are long
        const bool wide = L.count >= 8192;
        const int NW = (L.nin_max <= 64 || (wide && L.nin_max <= 256)) ? 1
                       : L.nin_max <= 256 ? 4 : L.nin_max <= 512 ? 8 : 16;
        const int tpb = NW == 1 ? 4 : 1;
        const dim3 grid(unsigned(round_up(ceil_div(L.count, tpb), 8)), 1, b.n),
            blk(NW > 4 ? 64 * NW : 256);
        const int64_t* so = fw ? P.soff_fwd : P.soff_bwd;
        if (fw) {
          if (NW == 1) launch_product_nw<T, true, 1>(KTM, grid, blk, s, P, L, so, it, b, ldw);
          else if (NW == 4) launch_product_nw<T, true, 4>(KTM, grid, blk, s, P, L, so, it, b, ldw);
          else if (NW == 8) launch_product_nw<T, true, 8>(KTM, grid, blk, s, P, L, so, it, b, ldw);
          else launch_product_nw<T, true, 16>(KTM, grid, blk, s, P, L, so, it, b, ldw);
        } else {
          if (NW == 1) launch_product_nw<T, false, 1>(KTM, grid, blk, s, P, L, so, it, b, ldw);
          else if (NW == 4) launch_product_nw<T, false, 4>(KTM, grid, blk, s, P, L, so, it, b, ldw);
          else if (NW == 8) launch_product_nw<T, false, 8>(KTM, grid, blk, s, P, L, so, it, b, ldw);
          else launch_product_nw<T, false, 16>(KTM, grid, blk, s, P, L, so, it, b, ldw);
        }
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
  enqueue_prec_apply(P, fwd, bwd, it, Batched<PrecItem<T>>(), kcap, ldw, s, nullptr);
}

template void check_prec_item<float>(const PrecItem<float>&, int, int);
template void check_prec_item<double>(const PrecItem<double>&, int, int);
template void enqueue_prec_apply<float>(const PrecDev<float>&, const std::vector<LevelTasks>&,
                                        const std::vector<LevelTasks>&, const PrecItem<float>&,
                                        Batched<PrecItem<float>>, int, int, hipStream_t,
                                        const std::vector<WTerm>*);
template void enqueue_prec_apply<double>(const PrecDev<double>&, const std::vector<LevelTasks>&,
                                         const std::vector<LevelTasks>&, const PrecItem<double>&,
                                         Batched<PrecItem<double>>, int, int, hipStream_t,
                                         const std::vector<WTerm>*);
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
    const double zi = a.z32 ? double(a.z32[i * 8]) : a.z[i * 8];
    const double d = al * a.dl[i * 8] + be * zi;
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
    if (a.r32) a.r32[i * 8] = float(v);
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

// Batched copy of low-rank factors with a precision change: U (n rows), V (m
// rows), the core s and the rank, the first min(rank, colcap) columns.
template <class Tin, class Tout>
__global__ __launch_bounds__(256) void cast_lr_kernel(const CastItem<Tin, Tout>* __restrict__ items,
                                                      const int* __restrict__ done) {
  if (done && done[blockIdx.z]) return;
  const CastItem<Tin, Tout>& c = items[blockIdx.z];
  const int cols = __builtin_amdgcn_readfirstlane(min(*c.r, c.colcap));
  if (cols > 0) {
    // lpr = the power of two >= cols lanes per row (cols <= 64 <= blockDim)
    int lg = 0;
    while ((1 << lg) < cols) ++lg;
    const int rpb = int(blockDim.x) >> lg, col = int(threadIdx.x) & ((1 << lg) - 1);
    const int64_t rows = c.n + c.m;
    if (col < cols)
      for (int64_t row = int64_t(blockIdx.x) * rpb + (threadIdx.x >> lg); row < rows;
           row += int64_t(gridDim.x) * rpb) {
        if (row < c.n) c.U2[row * c.ldu2 + col] = Tout(c.U[row * c.ldu + col]);
        else c.V2[(row - c.n) * c.ldv2 + col] = Tout(c.V[(row - c.n) * c.ldv + col]);
      }
  }
  if (blockIdx.x == 0) {
    for (int t = threadIdx.x; t < cols; t += blockDim.x) c.s2[t] = c.s[t];
    if (threadIdx.x == 0) *c.r2 = cols;
  }
}

template <class Tin, class Tout>
void launch_cast_lr(const CastItem<Tin, Tout>* items, const int* done, int nb, int64_t rows_max,
                    int colcap, hipStream_t s) {
  LRC_CHECK(colcap >= 0 && colcap <= 64, ST_EINVAL, "cast: at most 64 columns");
  const int64_t blocks =
      std::min<int64_t>(std::max<int64_t>(ceil_div(rows_max * colcap, 256), 1), 4096);
  ProfScope ps(kcls(K_VECTOR, false), s);
  hipLaunchKernelGGL((cast_lr_kernel<Tin, Tout>), dim3(unsigned(blocks), 1, unsigned(nb)),
                     dim3(256), 0, s, items, done);
  LRC_HIP(hipGetLastError());
}
template void launch_cast_lr<double, float>(const CastItem<double, float>*, const int*, int,
                                            int64_t, int, hipStream_t);
template void launch_cast_lr<float, double>(const CastItem<float, double>*, const int*, int,
                                            int64_t, int, hipStream_t);
template void launch_cast_lr<double, double>(const CastItem<double, double>*, const int*, int,
                                             int64_t, int, hipStream_t);
template void launch_cast_lr<float, float>(const CastItem<float, float>*, const int*, int,
                                           int64_t, int, hipStream_t);

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
