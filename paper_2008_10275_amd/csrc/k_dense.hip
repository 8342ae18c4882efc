// Dense tall-skinny kernels on MFMA (gfx950): Gram products of concatenated
// factors, tall-skinny times small products, and the fp64 true residual.
// All use the 16x16x4 MFMA shapes (f32 and f64) with the lane layout
//   A operand  lane l -> A[l % 16][l / 16]   (16 x 4)
//   B operand  lane l -> B[l / 16][l % 16]   (4 x 16)
//   D, f32     lane l, value i -> D[4 (l / 16) + i][l % 16]
//   D, f64     lane l, value i -> D[(l / 16) + 4 i][l % 16]   (rows interleaved)
// (both result layouts were checked on gfx950 with a one-wave probe).
#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>

#include "gmem.hpp"
#include "kernels.hpp"
#include "prof.hpp"

namespace lrc {

template <class T>
static std::vector<WTerm> view_terms(const BlockView<T>& v) {
  std::vector<WTerm> t;
  for (int b = 0; b < v.nb; ++b) t.push_back({v.wdev[b], v.wconst[b]});
  return t;
}


// Workgroups of kernel `fn` (block of `threads`) resident on the whole current
// device at once, cached per kernel and device: grids sized to this run in a
// single round.
static int resident_wgs(const void* fn, int threads) {
  static std::mutex mu;
  static std::map<std::pair<const void*, int>, int> cache;
  int dev = 0;
  LRC_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(mu);
  const auto key = std::make_pair(fn, dev);
  const auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  int per_cu = 0, cus = 0;
  LRC_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, threads, 0));
  LRC_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int v = std::max(1, per_cu) * std::max(1, cus);
  cache[key] = v;
  return v;
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
  T x = gmem(v.ptr[b])[row * v.ld[b] + lc];
  if (v.rowscale[b]) x *= T(gmem(v.rowscale[b])[row]);
  return x;
}

// ============================================================== Gram
// G = X^T X for up to two operands (the A and B sides of a truncation) in one
// launch, k <= 128 columns.  Each wave streams rows straight from HBM in the
// MFMA operand layout: for a 4-row slab, lane l holds row (l / 16) at columns
// 16 t + (l % 16), so the A operand of tile (bi, bj) is the lane's value for
// t = bi and the B operand its value for t = bj; all 36 upper tiles of the
// 8 x 8 tile grid accumulate in registers (tiles beyond the device width are
// skipped).  fp64 splits the tiles over two wave groups to halve the
// accumulator registers.  The waves of a workgroup are summed through LDS in a
// fixed order, one partial per workgroup is written, and a second kernel sums
// the partials in a fixed order (results are bitwise reproducible).
constexpr int kGK = 128;                       // columns of the Gram / TSMM kernels
constexpr int kGT = kGK / 16;                  // 8 tiles per dimension
constexpr int kGN = kGT * (kGT + 1) / 2;       // 36 upper tiles
constexpr int kGramWgMax = 512;


template <class T>
__device__ inline int view_width(const BlockView<T>& v) {
  int k = 0;
  for (int b = 0; b < v.nb; ++b) k += block_width(v, b);
  return k;
}

// A concatenated column c of a view, ready for branch-free loads: columns
// past the width point at a valid address (their values are never used);
// for row-scaled views `sc` is a valid row-scale array of the view and `ss`
// is 1 when the column's own block is scaled by it, 0 otherwise.
template <class T>
struct ColRef {
  const T* p;
  const double* sc;
  int ld;
  int ss;
};

template <class T>
__device__ inline ColRef<T> resolve_col(const BlockView<T>& v, int c) {
  ColRef<T> r{v.ptr[0], nullptr, 0, 0};
  for (int b = 0; b < v.nb; ++b)
    if (!r.sc && v.rowscale[b]) r.sc = v.rowscale[b];
  int off = 0;
  for (int b = 0; b < v.nb; ++b) {
    const int w = block_width(v, b);
    if (c >= off && c < off + w) {
      r.p = v.ptr[b] + (c - off);
      r.ld = v.ld[b];
      if (v.rowscale[b]) { r.sc = v.rowscale[b]; r.ss = 1; }
    }
    off += w;
  }
  return r;
}

// Load row min(row, rmax) of a column (always a valid address; rows are
// below 2^31 / ld, so offsets are 32-bit).  Callers mask rows they must not
// count at the point of use, so that loads stay in flight.  SCALED requires a
// row-scaled view (so that c.sc is a valid array).
template <class T, bool SCALED>
__device__ inline T col_load(const ColRef<T>& c, int64_t row, int64_t rmax) {
  const int r = int(row < rmax ? row : rmax);
  T x = gmem(c.p)[r * c.ld];
  if constexpr (SCALED) {
    const double f = gmem(c.sc)[r];
    x *= c.ss ? T(f) : T(1);
  }
  return x;
}

template <class T>
__host__ inline bool view_scaled(const BlockView<T>& v) {
  for (int b = 0; b < v.nb; ++b)
    if (v.rowscale[b]) return true;
  return false;
}

// upper-tile enumeration of a KTM x KTM tile grid, row by row
template <int KTM>
struct TileTab {
  static constexpr int N = KTM * (KTM + 1) / 2;
  int bi[N], bj[N];
  constexpr TileTab() : bi(), bj() {
    int u = 0;
    for (int i = 0; i < KTM; ++i)
      for (int j = i; j < KTM; ++j) { bi[u] = i; bj[u] = j; ++u; }
  }
};
__host__ __device__ constexpr int gtile_id(int bi, int bj) {
  return bi * kGT - bi * (bi - 1) / 2 + (bj - bi);
}
__device__ inline void gtile_of(int id, int& bi, int& bj) {
  bi = 0;
  int rem = id;
  while (rem >= kGT - bi) { rem -= kGT - bi; ++bi; }
  bj = bi + rem;
}

// Gram accumulation over the rows [r0, r1) of one operand for one wave of
// tile group G: rows r0 + 8 (stream + NS i) + {0..7} per step, PD steps in
// flight.  The loop is branch-free: all KTM column loads and all tiles of the
// group are issued whatever the device width (tiles past it are computed on
// valid data and never written), so that the scheduler keeps every load PD
// steps ahead of its MFMAs.
template <class T, int KTM, int NG, int G, int PD, bool SCALED>
__device__ inline void gram_rows(const ColRef<T>* cr, int KT, int64_t r0, int64_t r1, int stream,
                                 int sub, typename Mfma<T>::acc_t* acc) {
  constexpr TileTab<KTM> tt{};
  constexpr int NS = 4 / NG;
  const int64_t step = 8 * NS;
  // Columns past the width (inside the last 16-column tile) read valid but
  // unrelated data: they only reach Gram entries of columns >= k, which are
  // never used.  Rows past r1 belong to the next workgroup and are zeroed
  // when consumed (masking at the load would make every load wait at once).
  T xa[PD][KTM] = {}, xb[PD][KTM] = {};
  const int64_t rl = r1 - 1;
  int64_t q = r0 + 8 * stream;
#pragma unroll
  for (int d = 0; d < PD; ++d) {
    const int64_t ra = q + d * step + sub, rb = ra + 4;
#pragma unroll
    for (int t = 0; t < KTM; ++t) {
      if (t < KT) {
        xa[d][t] = col_load<T, SCALED>(cr[t], ra, rl);
        xb[d][t] = col_load<T, SCALED>(cr[t], rb, rl);
      }
    }
  }
  for (; q < r1; q += PD * step) {
#pragma unroll
    for (int d = 0; d < PD; ++d) {
      const int64_t ra = q + d * step + sub, rb = ra + 4;
      const bool oa = ra < r1, ob = rb < r1;
      T ya[KTM], yb[KTM];
#pragma unroll
      for (int t = 0; t < KTM; ++t) {
        ya[t] = oa ? xa[d][t] : T(0);
        yb[t] = ob ? xb[d][t] : T(0);
      }
#pragma unroll
      for (int u = G; u < tt.N; u += NG) {
        if (tt.bj[u] < KT) {
          acc[u / NG] = Mfma<T>::op(ya[tt.bi[u]], ya[tt.bj[u]], acc[u / NG]);
          acc[u / NG] = Mfma<T>::op(yb[tt.bi[u]], yb[tt.bj[u]], acc[u / NG]);
        }
      }
      const int64_t na = ra + PD * step, nb = na + 4;
#pragma unroll
      for (int t = 0; t < KTM; ++t) {
        if (t < KT) {
          xa[d][t] = col_load<T, SCALED>(cr[t], na, rl);
          xb[d][t] = col_load<T, SCALED>(cr[t], nb, rl);
        }
      }
    }
  }
}

template <class T, int KTM, int NG, int PD, bool SCALED>
__device__ inline void gram_rows_g(int g, const ColRef<T>* cr, int KT, int64_t r0, int64_t r1,
                                   int stream, int sub, typename Mfma<T>::acc_t* acc) {
  if (g == 0) gram_rows<T, KTM, NG, 0, PD, SCALED>(cr, KT, r0, r1, stream, sub, acc);
  if constexpr (NG > 1)
    if (g == 1) gram_rows<T, KTM, NG, 1, PD, SCALED>(cr, KT, r0, r1, stream, sub, acc);
  if constexpr (NG > 2) {
    if (g == 2) gram_rows<T, KTM, NG, 2, PD, SCALED>(cr, KT, r0, r1, stream, sub, acc);
    if (g == 3) gram_rows<T, KTM, NG, 3, PD, SCALED>(cr, KT, r0, r1, stream, sub, acc);
  }
}

// (wave groups sharing the tiles, prefetch depth) of a tile grid, chosen so
// that accumulators + operand ring fit the registers
// (KTK: the kernel's own grid bound; a narrow grid inside a wide kernel keeps
// the wide kernel's register budget, so only narrow kernels go deeper)
template <class T, int KTM, int KTK>
struct GramCfg {
  static constexpr bool F64 = sizeof(T) == 8;
  static constexpr int NG = KTM <= 4 ? 1 : KTM <= 6 ? 2 : (F64 ? 4 : 2);
  static constexpr int PD = KTM <= 2 ? (KTK <= 4 ? 8 : 4)
                          : KTM <= 4 ? (KTK <= 4 || !F64 ? 4 : 2)
                          : KTM <= 6 ? (F64 ? 2 : 4) : 2;
};

// One workgroup's share of one operand for a KTM x KTM tile grid: stream
// the rows, sum the waves' tiles in LDS (fixed order), write the partial.
template <class T, int KTM, int KTK, bool SCALED1>
__device__ __forceinline__ void gram_body(const GramArgs<T>& a, int job, int wg, int nwg, int KT,
                                          T* red) {
  typedef typename Mfma<T>::acc_t acc_t;
  constexpr int NG = GramCfg<T, KTM, KTK>::NG, PD = GramCfg<T, KTM, KTK>::PD;
  constexpr TileTab<KTM> tt{};
  constexpr int NTM = TileTab<KTM>::N;
  constexpr int MAXT = (NTM + NG - 1) / NG;
  constexpr int NS = 4 / NG;                 // row streams per workgroup
  const BlockView<T>& X = a.X[job];
  const int64_t rows = a.rows[job];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = wave % NG, stream = wave / NG;
  ColRef<T> cr[KTM];
#pragma unroll
  for (int t = 0; t < KTM; ++t) cr[t] = resolve_col(X, 16 * t + (lane & 15));
  acc_t acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = acc_t{};
  const int64_t per = ceil_div(ceil_div(rows, int64_t(8)), int64_t(nwg)) * 8;
  const int64_t r0 = int64_t(wg) * per, r1 = std::min<int64_t>(rows, r0 + per);
  if (r0 < r1) {
    // the row-scaled operand is the short V side: no deep prefetch there, so
    // that it does not raise the register budget of the long side
    if (SCALED1 && job == 1)
      gram_rows_g<T, KTM, NG, 1, true>(g, cr, KT, r0, r1, stream, lane >> 4, acc);
    else
      gram_rows_g<T, KTM, NG, PD, false>(g, cr, KT, r0, r1, stream, lane >> 4, acc);
  }
  // sum the row streams in LDS (fixed order)
  for (int s = 0; s < NS; ++s) {
    if (stream == s) {
#pragma unroll
      for (int u = 0; u < NTM; ++u) {
        if (u % NG == g && tt.bj[u] < KT) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            T* d = &red[u * 256 + Mfma<T>::drow(lane, i) * 16 + (lane & 15)];
            *d = s == 0 ? acc[u / NG][i] : *d + acc[u / NG][i];
          }
        }
      }
    }
    __syncthreads();
  }
  // partial layout: tiles of the full 8 x 8 grid (ids of gtile_id)
  T* out = a.partial + size_t(blockIdx.x) * kGN * 256;
  for (int e = threadIdx.x; e < NTM * 256; e += blockDim.x) {
    const int u = e >> 8;
    if (tt.bj[u] < KT) gmem(out)[gtile_id(tt.bi[u], tt.bj[u]) * 256 + (e & 255)] = red[e];
  }
}

// The host bound KTM of the width sizes LDS; the tile grid actually used
// follows the device width (a wave-uniform branch), so that a wide capacity
// with a narrow operand runs the narrow grid's schedule.
template <class T, int KTM, bool SCALED1>
__global__ __launch_bounds__(256, 2) void gram_kernel(GramArgs<T> a0, const GramArgs<T>* ab,
                                                   const int* done) {
  if (done && done[blockIdx.z]) return;
  const GramArgs<T>& a = ab ? ab[blockIdx.z] : a0;
  if (int(blockIdx.x) >= a.nwg0 + a.nwg1) return;   // batched grids take the largest item
  __shared__ T red[TileTab<KTM>::N * 256];
  const int job = int(blockIdx.x) < a.nwg0 ? 0 : 1;
  const int wg = job == 0 ? blockIdx.x : blockIdx.x - a.nwg0;
  const int nwg = job == 0 ? a.nwg0 : a.nwg1;
  const int k = min(view_width(a.X[job]), 16 * KTM);
  const int KT = __builtin_amdgcn_readfirstlane((k + 15) / 16);
  if constexpr (KTM >= 8)
    if (KT > 6) return gram_body<T, 8, KTM, SCALED1>(a, job, wg, nwg, KT, red);
  if constexpr (KTM >= 6)
    if (KT > 4) return gram_body<T, 6, KTM, SCALED1>(a, job, wg, nwg, KT, red);
  if constexpr (KTM >= 4)
    if (KT > 2) return gram_body<T, 4, KTM, SCALED1>(a, job, wg, nwg, KT, red);
  gram_body<T, 2, KTM, SCALED1>(a, job, wg, nwg, KT, red);
}

// ---------------------------------------------------------- BF16 first pass
// The same Gram products with the fp32 operands rounded to bf16 as they are
// loaded and multiplied on v_mfma_f32_16x16x32_bf16 (fp32 accumulation): a
// lane holds 8 consecutive rows of one column of a 16-column tile (rows 8 s
// + e of a 32-row step, s = lane / 16, column lane % 16), which is the A
// operand of X^T and the B operand of X alike, so the fragments of every
// column tile serve all tiles of the upper triangle.  A step covers 32 rows
// with one MFMA per tile (8 with the fp32 16x16x4 form); the partials have
// the fp32 kernel's layout and are summed by its reduction.
typedef __bf16 bf16x8_g __attribute__((ext_vector_type(8)));

template <int KTM, int NG, int G, bool SCALED>
__device__ inline void gram_rows_bf16(const ColRef<float>* cr, int KT, int64_t r0, int64_t r1,
                                      int stream, int nstream, int sub, floatx4* acc) {
  constexpr TileTab<KTM> tt{};
  const int64_t rl = r1 - 1;
  const int64_t step = 32 * int64_t(nstream);
  float cur[KTM][8];
  int64_t q = r0 + 32 * stream;
#pragma unroll
  for (int t = 0; t < KTM; ++t)
#pragma unroll
    for (int e = 0; e < 8; ++e) cur[t][e] = t < KT ? col_load<float, SCALED>(cr[t], q + 8 * sub + e, rl) : 0.0f;
  for (; q < r1; q += step) {
    bf16x8_g fr[KTM];
#pragma unroll
    for (int t = 0; t < KTM; ++t)
#pragma unroll
      for (int e = 0; e < 8; ++e) fr[t][e] = __bf16(q + 8 * sub + e < r1 ? cur[t][e] : 0.0f);
    const int64_t qn = q + step;
#pragma unroll
    for (int t = 0; t < KTM; ++t)
      if (t < KT)
#pragma unroll
        for (int e = 0; e < 8; ++e) cur[t][e] = col_load<float, SCALED>(cr[t], qn + 8 * sub + e, rl);
#pragma unroll
    for (int u = G; u < tt.N; u += NG)
      if (tt.bj[u] < KT)
        acc[u / NG] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fr[tt.bi[u]], fr[tt.bj[u]],
                                                              acc[u / NG], 0, 0, 0);
  }
}

template <int KTM, bool SCALED1>
__device__ __forceinline__ void gram_body_bf16(const GramArgs<float>& a, int job, int wg, int nwg,
                                               int KT, float* red) {
  constexpr int NG = KTM <= 4 ? 1 : 2;
  constexpr TileTab<KTM> tt{};
  constexpr int NTM = TileTab<KTM>::N;
  constexpr int MAXT = (NTM + NG - 1) / NG;
  constexpr int NS = 4 / NG;
  const BlockView<float>& X = a.X[job];
  const int64_t rows = a.rows[job];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = wave % NG, stream = wave / NG;
  ColRef<float> cr[KTM];
#pragma unroll
  for (int t = 0; t < KTM; ++t) cr[t] = resolve_col(X, 16 * t + (lane & 15));
  floatx4 acc[MAXT];
#pragma unroll
  for (int t = 0; t < MAXT; ++t) acc[t] = floatx4{};
  const int64_t per = ceil_div(ceil_div(rows, int64_t(32)), int64_t(nwg)) * 32;
  const int64_t r0 = int64_t(wg) * per, r1 = std::min<int64_t>(rows, r0 + per);
  if (r0 < r1) {
    const bool sc = SCALED1 && job == 1;
    if (g == 0) {
      if (sc) gram_rows_bf16<KTM, NG, 0, true>(cr, KT, r0, r1, stream, NS, lane >> 4, acc);
      else gram_rows_bf16<KTM, NG, 0, false>(cr, KT, r0, r1, stream, NS, lane >> 4, acc);
    }
    if constexpr (NG > 1)
      if (g == 1) {
        if (sc) gram_rows_bf16<KTM, NG, 1, true>(cr, KT, r0, r1, stream, NS, lane >> 4, acc);
        else gram_rows_bf16<KTM, NG, 1, false>(cr, KT, r0, r1, stream, NS, lane >> 4, acc);
      }
  }
  for (int s = 0; s < NS; ++s) {
    if (stream == s) {
#pragma unroll
      for (int u = 0; u < NTM; ++u) {
        if (u % NG == g && tt.bj[u] < KT) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float* d = &red[u * 256 + Mfma<float>::drow(lane, i) * 16 + (lane & 15)];
            *d = s == 0 ? acc[u / NG][i] : *d + acc[u / NG][i];
          }
        }
      }
    }
    __syncthreads();
  }
  float* out = a.partial + size_t(blockIdx.x) * kGN * 256;
  for (int e = threadIdx.x; e < NTM * 256; e += blockDim.x) {
    const int u = e >> 8;
    if (tt.bj[u] < KT) gmem(out)[gtile_id(tt.bi[u], tt.bj[u]) * 256 + (e & 255)] = red[e];
  }
}

template <int KTM, bool SCALED1>
__global__ __launch_bounds__(256, 2) void gram_bf16_kernel(GramArgs<float> a0,
                                                         const GramArgs<float>* ab,
                                                         const int* done) {
  if (done && done[blockIdx.z]) return;
  const GramArgs<float>& a = ab ? ab[blockIdx.z] : a0;
  if (int(blockIdx.x) >= a.nwg0 + a.nwg1) return;
  __shared__ float red[TileTab<KTM>::N * 256];
  const int job = int(blockIdx.x) < a.nwg0 ? 0 : 1;
  const int wg = job == 0 ? blockIdx.x : blockIdx.x - a.nwg0;
  const int nwg = job == 0 ? a.nwg0 : a.nwg1;
  const int k = min(view_width(a.X[job]), 16 * KTM);
  const int KT = __builtin_amdgcn_readfirstlane((k + 15) / 16);
  if constexpr (KTM >= 8)
    if (KT > 6) return gram_body_bf16<8, SCALED1>(a, job, wg, nwg, KT, red);
  if constexpr (KTM >= 6)
    if (KT > 4) return gram_body_bf16<6, SCALED1>(a, job, wg, nwg, KT, red);
  if constexpr (KTM >= 4)
    if (KT > 2) return gram_body_bf16<4, SCALED1>(a, job, wg, nwg, KT, red);
  gram_body_bf16<2, SCALED1>(a, job, wg, nwg, KT, red);
}

// G[r][c] = sum over the job's workgroup partials (fixed order), both triangles
// written; also publishes the width k = min(width, kcap) and flags widths
// beyond the capacity (info bit 8).
template <class T>
__global__ __launch_bounds__(1024) void gram_reduce_kernel(GramRedArgs<T> r0, const GramRedArgs<T>* rb,
                                                           const int* done) {
  __shared__ double sh[16][64];
  if (done && done[blockIdx.z]) return;
  const GramRedArgs<T>& ra = rb ? rb[blockIdx.z] : r0;
  const GramArgs<T>& a = ra.g;
  const T* __restrict__ partial = a.partial;
  double* G0 = ra.G0;
  double* G1 = ra.G1;
  const int kcap = ra.kcap;
  int* k0 = ra.k0;
  int* k1 = ra.k1;
  int* info = ra.info;
  const int job = blockIdx.y;
  const int ktot = view_width(a.X[job]);
  const int kg = min(ktot, kGK);
  const int k = min(kg, kcap);
  const int KT = (kg + 15) / 16;
  const int tid = threadIdx.x, grp = tid >> 6, l = tid & 63;
  const int e = blockIdx.x * 64 + l;
  const int id = e >> 8, w = e & 255;
  if (blockIdx.x == 0 && tid == 0) {
    if (ktot > min(kcap, kGK) && info) atomicOr(info, 8);
    if (job == 0 && k0) *k0 = k;
    if (job == 1 && k1) *k1 = k;
  }
  int tbi = 0, tbj = 0;
  if (id < kGN) gtile_of(id, tbi, tbj);
  const bool valid = id < kGN && tbj < KT;
  const int w0 = job == 0 ? 0 : a.nwg0;
  const int nw = job == 0 ? a.nwg0 : a.nwg1;
  // partials p = grp, grp + 16, ... summed in that order; eight loads are
  // issued before their additions
  double s = 0.0;
  if (valid) {
    const T* __restrict__ pp = partial + (size_t(w0) * kGN + id) * 256 + w;
    constexpr size_t st = size_t(kGN) * 256;
    int p = grp;
    for (; p + 16 * 7 < nw; p += 16 * 8) {
      T v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = gmem(pp)[size_t(p + 16 * u) * st];
#pragma unroll
      for (int u = 0; u < 8; ++u) s += double(v[u]);
    }
    for (; p < nw; p += 16) s += double(gmem(pp)[size_t(p) * st]);
  }
  sh[grp][l] = s;
  __syncthreads();
  if (grp != 0 || !valid) return;
  double t = 0.0;
#pragma unroll
  for (int x = 0; x < 16; ++x) t += sh[x][l];
  const int r = tbi * 16 + (w >> 4), c = tbj * 16 + (w & 15);
  if (r >= k || c >= k || r > c) return;
  double* G = job == 0 ? G0 : G1;
  gmem(G)[size_t(r) * kcap + c] = t;
  gmem(G)[size_t(c) * kcap + r] = t;
}

template <class T>
using GramFn = void (*)(GramArgs<T>, const GramArgs<T>*, const int*);

// the width bound picks the LDS class; the kernel follows the device width
template <class T>
static GramFn<T> gram_fn(int kb, bool sc1) {
  if (kb <= 32) return sc1 ? gram_kernel<T, 2, true> : gram_kernel<T, 2, false>;
  if (kb <= 64) return sc1 ? gram_kernel<T, 4, true> : gram_kernel<T, 4, false>;
  if (kb <= 96) return sc1 ? gram_kernel<T, 6, true> : gram_kernel<T, 6, false>;
  return sc1 ? gram_kernel<T, 8, true> : gram_kernel<T, 8, false>;
}

static GramFn<float> gram_bf16_fn(int kb, bool sc1) {
  if (kb <= 32) return sc1 ? gram_bf16_kernel<2, true> : gram_bf16_kernel<2, false>;
  if (kb <= 64) return sc1 ? gram_bf16_kernel<4, true> : gram_bf16_kernel<4, false>;
  if (kb <= 96) return sc1 ? gram_bf16_kernel<6, true> : gram_bf16_kernel<6, false>;
  return sc1 ? gram_bf16_kernel<8, true> : gram_bf16_kernel<8, false>;
}

static int gram_wgs(int64_t rows) {
  // about 128 rows per workgroup for short operands (so that their serial
  // load chains stay short), at most kGramWgMax workgroups for long ones
  if (rows <= 0) return 1;
  return int(std::min<int64_t>(kGramWgMax, std::max<int64_t>(1, ceil_div(rows, int64_t(128)))));
}

size_t gram_workspace_bytes(int64_t rows_a, int64_t rows_b, int kcap, bool fp64) {
  (void)kcap;
  return size_t(gram_wgs(rows_a) + gram_wgs(rows_b)) * kGN * 256 * (fp64 ? 8 : 4);
}

template <class T>
GramLaunch<T> make_gram(const GramJob<T>* jobs, int njobs, int kcap, double* ws_partial,
                        size_t ws_bytes, int* info) {
  LRC_CHECK(njobs >= 1 && njobs <= 2, ST_EINVAL, "gram: one or two jobs");
  LRC_CHECK(kcap <= kGK, ST_EINVAL, "gram: at most 128 columns");
  GramLaunch<T> l;
  GramArgs<T>& a = l.g;
  l.kb = std::min(kGK, std::max(view_cap(jobs[0].X), njobs > 1 ? view_cap(jobs[1].X) : 0));
  l.sc1 = njobs > 1 && view_scaled(jobs[1].X);
  a.X[0] = jobs[0].X;
  a.rows[0] = jobs[0].rows;
  if (njobs == 2) {
    a.X[1] = jobs[1].X;
    a.rows[1] = jobs[1].rows;
    a.nwg1 = gram_wgs(jobs[1].rows);
  } else {
    a.X[1] = jobs[0].X;
    a.rows[1] = 0;
    a.nwg1 = 0;
  }
  // the long operand takes the resident slots the short one leaves
  const int slots = resident_wgs(reinterpret_cast<const void*>(gram_fn<T>(l.kb, l.sc1)), 256);
  a.nwg0 = std::min(gram_wgs(jobs[0].rows), std::max(1, slots - a.nwg1));
  a.partial = reinterpret_cast<T*>(ws_partial);
  const size_t need = size_t(a.nwg0 + a.nwg1) * kGN * 256 * sizeof(T);
  LRC_CHECK(need <= ws_bytes, ST_EINVAL, "gram: workspace too small");
  LRC_CHECK(!view_scaled(jobs[0].X), ST_EINVAL, "gram: the first operand cannot be row-scaled");
  l.r = GramRedArgs<T>{a, jobs[0].G, njobs == 2 ? jobs[1].G : jobs[0].G, kcap, jobs[0].kout,
                       njobs == 2 ? jobs[1].kout : nullptr, info};
  l.njobs = njobs;
  l.grid = a.nwg0 + a.nwg1;
  // algorithmic flops: the k(k+1)/2 distinct entries of each Gram matrix, 2 flops per row each
  l.work.bytes = false;
  const double r0 = double(a.rows[0]), r1 = double(a.rows[1]);
  l.work.groups = {view_terms(jobs[0].X), view_terms(njobs > 1 ? jobs[1].X : jobs[0].X)};
  l.work.f = [=](const std::vector<double>& v) {
    return r0 * v[0] * (v[0] + 1.0) + r1 * v[1] * (v[1] + 1.0);
  };
  return l;
}

template <class T>
void enqueue_gram(const GramLaunch<T>& l, Batched<GramArgs<T>> bg, Batched<GramRedArgs<T>> br,
                  hipStream_t s) {
  if constexpr (sizeof(T) == 4) {
    if (l.bf16) {
      ProfScope ps(kcls(K_GRAM_BF16, true), s, l.work);
      const dim3 grid(l.grid, 1, bg.n), blk(256);
      gram_bf16_fn(l.kb, l.sc1)<<<grid, blk, 0, s>>>(l.g, bg.dev, bg.done);
    }
  }
  if (!l.bf16) {
    ProfScope ps(kcls(K_GRAM, is_f32<T>()), s, l.work);
    const GramArgs<T>& a = l.g;
    const dim3 grid(l.grid, 1, bg.n), blk(256);
    gram_fn<T>(l.kb, l.sc1)<<<grid, blk, 0, s>>>(a, bg.dev, bg.done);
  }
  ProfScope ps(kcls(K_GRAM_REDUCE, is_f32<T>()), s);
  hipLaunchKernelGGL((gram_reduce_kernel<T>), dim3(kGN * 256 / 64, l.njobs, br.n), dim3(1024), 0,
                     s, l.r, br.dev, br.done);
  LRC_HIP(hipGetLastError());
}

template <class T>
void launch_gram(const GramJob<T>* jobs, int njobs, int kcap, double* ws_partial, size_t ws_bytes,
                 int* info, hipStream_t s) {
  enqueue_gram(make_gram(jobs, njobs, kcap, ws_partial, ws_bytes, info), Batched<GramArgs<T>>(),
               Batched<GramRedArgs<T>>(), s);
}
template GramLaunch<float> make_gram<float>(const GramJob<float>*, int, int, double*, size_t, int*);
template GramLaunch<double> make_gram<double>(const GramJob<double>*, int, int, double*, size_t,
                                              int*);
template void enqueue_gram<float>(const GramLaunch<float>&, Batched<GramArgs<float>>,
                                  Batched<GramRedArgs<float>>, hipStream_t);
template void enqueue_gram<double>(const GramLaunch<double>&, Batched<GramArgs<double>>,
                                   Batched<GramRedArgs<double>>, hipStream_t);
template void launch_gram<float>(const GramJob<float>*, int, int, double*, size_t, int*,
                                 hipStream_t);
template void launch_gram<double>(const GramJob<double>*, int, int, double*, size_t, int*,
                                  hipStream_t);

// ============================================================== TSMM  Y = X * M
// Each wave streams 16-row tiles of X straight from HBM into the MFMA
// A-operand layout (lane l: row l % 16, column 4 q + l / 16 at step q),
// loading the next tile while the current one multiplies; M (k x r, at most
// 16 NT columns) sits in LDS for the whole launch, and the accumulators are
// stored to Y directly, so the row loop has no barrier.  The device widths
// (k of the view, r of *r_dev) bound the steps and tiles at run time; the
// template bounds (KQ, NT) only size registers and LDS.
constexpr int kTsThreads = 512;
constexpr int kTsPad = 16;
constexpr int kTsKCAP = kGK;

template <class T, int KQ, bool SCALED>
__device__ __forceinline__ void ts_load(T (&a)[KQ], const ColRef<T>* cols, int kq, int k, int g,
                                        int64_t row, int64_t rows) {
  // addresses are always valid (rows clamped, absent columns alias a real
  // one); entries outside the operand are zeroed at the select, so that all
  // loads stay in flight together
#pragma unroll
  for (int q = 0; q < KQ; ++q)
    if (q < kq) {
      const int c = 4 * q + g;
      const T x = col_load<T, SCALED>(cols[c], row, rows - 1);
      a[q] = (c < k && row < rows) ? x : T(0);
    }
}

// NTU (<= NT) output tiles are multiplied; the caller picks NTU from the
// uniform tile count so that no accumulator update is guarded.  TRI: M is
// upper triangular (the inverse factor of the first pass), so output tile t
// takes only the input steps q < 4 (t + 1).
template <class T, int KQ, int NT, int NTU, bool TRI>
__device__ __forceinline__ void ts_tile(const T (&a)[KQ], const T* Ms, int kq, int g, int rl,
                                        int lane, int64_t row0, int64_t rows, int r,
                                        T* __restrict__ Y, int64_t ldy) {
  constexpr int S = 16 * NT + kTsPad;
  typedef typename Mfma<T>::acc_t acc_t;
  acc_t acc[NTU];
#pragma unroll
  for (int t = 0; t < NTU; ++t) acc[t] = acc_t{};
#pragma unroll
  for (int q = 0; q < KQ; ++q)
    if (q < kq) {
      const T* br = Ms + (4 * q + g) * S + rl;
#pragma unroll
      for (int t = 0; t < NTU; ++t)
        if (!TRI || q < 4 * (t + 1)) acc[t] = Mfma<T>::op(a[q], br[16 * t], acc[t]);
    }
#pragma unroll
  for (int t = 0; t < NTU; ++t) {
    const int c = 16 * t + rl;
    if (c < r) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int64_t row = row0 + Mfma<T>::drow(lane, i);
        if (row < rows) gmem(Y)[row * ldy + c] = acc[t][i];
      }
    }
  }
}

// A wave keeps D row tiles in flight in a register ring of D x KQU operands.
template <class T, int KQU, int NT, int NTU, int D, bool SCALED, bool TRI>
__device__ __forceinline__ void ts_rows(const ColRef<T>* cols, const T* Ms, int k, int r,
                                        int64_t t0, int64_t t1, int64_t rows, T* Y, int64_t ldy) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 6);
  const int g = lane >> 4, rl = lane & 15;
  const int kq = (k + 3) >> 2;
  constexpr int nw = kTsThreads / 64;
  T buf[D][KQU];
  const int64_t q0 = t0 + wave;
  if (q0 >= t1) return;   // also covers an empty operand (no row to clamp to)
#pragma unroll
  for (int d = 0; d < D; ++d) {
    const int64_t tt = q0 + int64_t(d) * nw;
    if (tt < t1) ts_load<T, KQU, SCALED>(buf[d], cols, kq, k, g, tt * 16 + rl, rows);
  }
  for (int64_t q = q0; q < t1; q += int64_t(D) * nw) {
#pragma unroll
    for (int d = 0; d < D; ++d) {
      const int64_t tt = q + int64_t(d) * nw;
      if (tt < t1) {
        ts_tile<T, KQU, NT, NTU, TRI>(buf[d], Ms, kq, g, rl, lane, tt * 16, rows, r, Y, ldy);
        // re-read the column table from LDS rather than keeping it live
        __asm__ volatile("" ::: "memory");
        const int64_t tn = tt + int64_t(D) * nw;
        if (tn < t1) ts_load<T, KQU, SCALED>(buf[d], cols, kq, k, g, tn * 16 + rl, rows);
      }
    }
  }
}

template <class T, int KQU, int NT, int D, bool SCALED, bool TRI>
__device__ __forceinline__ void ts_rows_nt(const ColRef<T>* cols, const T* Ms, int k, int r,
                                           int64_t t0, int64_t t1, int64_t rows, T* Y,
                                           int64_t ldy) {
  const int rt = (r + 15) >> 4;
  // eight output tiles hold 32 accumulators per lane: half the ring depth
  constexpr int D8 = D >= 4 ? D / 2 : D;
  if constexpr (NT >= 8)
    if (rt > 4) return ts_rows<T, KQU, NT, 8, D8, SCALED, TRI>(cols, Ms, k, r, t0, t1, rows, Y, ldy);
  if constexpr (NT >= 4)
    if (rt > 2) return ts_rows<T, KQU, NT, 4, D, SCALED, TRI>(cols, Ms, k, r, t0, t1, rows, Y, ldy);
  ts_rows<T, KQU, NT, 2, D, SCALED, TRI>(cols, Ms, k, r, t0, t1, rows, Y, ldy);
}

// The ring holds 2 KQ operands whatever the width: narrow inputs keep more
// tiles in flight.  (The row-scaled operand is the short V side: one class.)
template <class T, int KQ, int NT, bool SCALED, bool TRI>
__device__ __forceinline__ void ts_rows_by_width(const ColRef<T>* cols, const T* Ms, int k, int r,
                                                 int64_t t0, int64_t t1, int64_t rows, T* Y,
                                                 int64_t ldy) {
  const int kq = (k + 3) >> 2;
  if constexpr (!SCALED) {
    if constexpr (KQ >= 32) {
      if (kq <= 8) return ts_rows_nt<T, 8, NT, 8, false, TRI>(cols, Ms, k, r, t0, t1, rows, Y, ldy);
      if (kq <= 16) return ts_rows_nt<T, 16, NT, 4, false, TRI>(cols, Ms, k, r, t0, t1, rows, Y, ldy);
    } else {
      if (kq <= 8) return ts_rows_nt<T, 8, NT, 4, false, TRI>(cols, Ms, k, r, t0, t1, rows, Y, ldy);
    }
  }
  ts_rows_nt<T, KQ, NT, 2, SCALED, TRI>(cols, Ms, k, r, t0, t1, rows, Y, ldy);
}

template <class T, int KQ, int NT, bool SCALED1, bool TRI>
__global__ __launch_bounds__(kTsThreads) void tsmm_kernel(TsmmArgs<T> a0, const TsmmArgs<T>* ab,
                                                          const int* done) {
  if (done && done[blockIdx.z]) return;
  const TsmmArgs<T>& a = ab ? ab[blockIdx.z] : a0;
  if (int(blockIdx.x) >= a.nwg0 + a.nwg1) return;   // batched grids take the largest item
  constexpr int KP = 4 * KQ, NC = 16 * NT, S = NC + kTsPad;
  __shared__ T Ms[KP * S];
  __shared__ ColRef<T> cols[KP];
  const int jb = int(blockIdx.x) < a.nwg0 ? 0 : 1;
  const int wg = jb == 0 ? blockIdx.x : blockIdx.x - a.nwg0;
  const int nwg = jb == 0 ? a.nwg0 : a.nwg1;
  const TsmmJob<T>& J = a.job[jb];
  // wave-uniform widths (scalar branches on the steps and tile classes)
  const int k = __builtin_amdgcn_readfirstlane(min(view_width(J.X), KP));
  const int r = __builtin_amdgcn_readfirstlane(min(*J.r_dev, NC));
  if (r <= 0) return;
  const int kp = (k + 3) & ~3;
  for (int e = threadIdx.x; e < kp * NC; e += blockDim.x) {
    const int i = e / NC, c = e - i * NC;
    Ms[i * S + c] = (i < k && c < r) ? T(J.M[size_t(i) * J.ldm + c]) : T(0);
  }
  for (int c = threadIdx.x; c < KP; c += blockDim.x) cols[c] = resolve_col(J.X, c);
  __syncthreads();
  const int64_t nrt = (J.rows + 15) / 16;
  const int64_t per = (nrt + nwg - 1) / nwg;
  const int64_t t0 = int64_t(wg) * per, t1 = min(nrt, t0 + per);
  if (SCALED1 && jb == 1)
    ts_rows_by_width<T, KQ, NT, true, TRI>(cols, Ms, k, r, t0, t1, J.rows, J.Y, J.ldy);
  else
    ts_rows_by_width<T, KQ, NT, false, TRI>(cols, Ms, k, r, t0, t1, J.rows, J.Y, J.ldy);
}

template <class T>
using TsmmFn = void (*)(TsmmArgs<T>, const TsmmArgs<T>*, const int*);

template <class T, bool TRI>
static TsmmFn<T> tsmm_fn_t(int kb, int rb, bool sc1) {
  if (kb <= 64) {
    if (rb <= 64) return sc1 ? tsmm_kernel<T, 16, 4, true, TRI> : tsmm_kernel<T, 16, 4, false, TRI>;
    return sc1 ? tsmm_kernel<T, 16, 8, true, TRI> : tsmm_kernel<T, 16, 8, false, TRI>;
  }
  if (rb <= 64) return sc1 ? tsmm_kernel<T, 32, 4, true, TRI> : tsmm_kernel<T, 32, 4, false, TRI>;
  return sc1 ? tsmm_kernel<T, 32, 8, true, TRI> : tsmm_kernel<T, 32, 8, false, TRI>;
}
template <class T>
static TsmmFn<T> tsmm_fn(int kb, int rb, bool sc1, bool tri) {
  return tri ? tsmm_fn_t<T, true>(kb, rb, sc1) : tsmm_fn_t<T, false>(kb, rb, sc1);
}

static int64_t tsmm_tiles(int64_t rows) { return (std::max<int64_t>(rows, 1) + 15) / 16; }
// at least one row tile per wave
static int tsmm_wgs_max(int64_t rows) {
  return int(std::min<int64_t>(1 << 20, ceil_div(tsmm_tiles(rows), kTsThreads / 64)));
}

template <class T>
TsmmLaunch<T> make_tsmm(const TsmmJob<T>* jobs, int njobs, int kcap, int rcap, bool tri) {
  LRC_CHECK(njobs >= 1 && njobs <= 2, ST_EINVAL, "tsmm: one or two jobs");
  LRC_CHECK(kcap <= kTsKCAP && rcap <= kTsKCAP, ST_EINVAL, "tsmm: capacity exceeded");
  LRC_CHECK(!view_scaled(jobs[0].X), ST_EINVAL, "tsmm: the first operand cannot be row-scaled");
  TsmmLaunch<T> l;
  TsmmArgs<T>& a = l.a;
  // host bounds of the device widths select the register / LDS class
  l.kb = std::min(kcap, std::max(view_cap(jobs[0].X), njobs > 1 ? view_cap(jobs[1].X) : 0));
  l.rb = rcap;
  l.sc1 = njobs > 1 && view_scaled(jobs[1].X);
  l.tri = tri;
  // one round of resident workgroups, shared by the jobs in proportion to
  // their row tiles
  const int slots =
      resident_wgs(reinterpret_cast<const void*>(tsmm_fn<T>(l.kb, l.rb, l.sc1, l.tri)), kTsThreads);
  a.job[0] = jobs[0];
  if (njobs == 2) {
    a.job[1] = jobs[1];
    const double t0 = double(tsmm_tiles(jobs[0].rows)), t1 = double(tsmm_tiles(jobs[1].rows));
    const int share = int(std::ceil(double(slots) * t1 / (t0 + t1)));
    a.nwg1 = std::min(tsmm_wgs_max(jobs[1].rows), std::max(1, share));
  } else {
    a.job[1] = jobs[0];
    a.nwg1 = 0;
  }
  a.nwg0 = std::min(tsmm_wgs_max(jobs[0].rows), std::max(1, slots - a.nwg1));
  l.grid = a.nwg0 + a.nwg1;
  // algorithmic bytes: X read once plus Y written once per job
  const double r0 = double(jobs[0].rows), r1 = double(njobs > 1 ? jobs[1].rows : 0);
  l.work.groups = {view_terms(jobs[0].X), {{jobs[0].r_dev, 0}},
                   view_terms(njobs > 1 ? jobs[1].X : jobs[0].X),
                   {{njobs > 1 ? jobs[1].r_dev : jobs[0].r_dev, 0}}};
  l.work.f = [=](const std::vector<double>& v) {
    return double(sizeof(T)) * (r0 * (v[0] + v[1]) + r1 * (v[2] + v[3]));
  };
  return l;
}

template <class T>
void enqueue_tsmm(const TsmmLaunch<T>& l, Batched<TsmmArgs<T>> b, hipStream_t s) {
  LRC_CHECK(l.kb <= kTsKCAP && l.rb <= kTsKCAP, ST_EINVAL, "tsmm: capacity exceeded");
  ProfScope ps(kcls(K_TSMM, is_f32<T>()), s, l.work);
  const dim3 grid(l.grid, 1, b.n), blk(kTsThreads);
  tsmm_fn<T>(l.kb, l.rb, l.sc1, l.tri)<<<grid, blk, 0, s>>>(l.a, b.dev, b.done);
  LRC_HIP(hipGetLastError());
}

template <class T>
void launch_tsmm(const TsmmJob<T>* jobs, int njobs, int kcap, int rcap, hipStream_t s) {
  enqueue_tsmm(make_tsmm(jobs, njobs, kcap, rcap), Batched<TsmmArgs<T>>(), s);
}
template TsmmLaunch<float> make_tsmm<float>(const TsmmJob<float>*, int, int, int, bool);
template TsmmLaunch<double> make_tsmm<double>(const TsmmJob<double>*, int, int, int, bool);
template void enqueue_tsmm<float>(const TsmmLaunch<float>&, Batched<TsmmArgs<float>>, hipStream_t);
template void enqueue_tsmm<double>(const TsmmLaunch<double>&, Batched<TsmmArgs<double>>,
                                   hipStream_t);
template void launch_tsmm<float>(const TsmmJob<float>*, int, int, int, hipStream_t);
template void launch_tsmm<double>(const TsmmJob<double>*, int, int, int, hipStream_t);

// ============================================================== fp64 residual
// R = A * (core-scaled B)^T entry by entry on fp64 MFMA; only the per-column
// sums of squares leave the kernel (R itself is never stored).
//
// A workgroup owns NC = 16 NT columns of R and a contiguous range of 16-row
// tiles.  The scaled B block (K x NC) sits in LDS for the whole launch; each
// wave streams its row tiles straight from HBM into the MFMA A-operand layout
// (lane l: row l % 16, column 4 q + l / 16 at step q), loading the next tile
// while the current one multiplies, so the row loop has no barrier.  Workgroups
// of one row range but different column blocks are placed on the same XCD so
// that they share its L2 copy of those rows.
constexpr int kResThreads = 256;
constexpr int kResRowGroups = 128;   // most partial rows per column
constexpr int kResBPad = 16;          // LDS row padding of B (doubles)

struct ResCol {
  const double* p;   // first element of the column
  int64_t ld;        // row stride
};

template <int KQ>
__device__ __forceinline__ void res_load(double (&a)[KQ], const ResCol* acol, int kq, int g,
                                         int64_t row, bool ok) {
#pragma unroll
  for (int q = 0; q < KQ; ++q)
    if (q < kq) {
      const ResCol e = acol[4 * q + g];
      a[q] = (ok && e.p) ? gmem(e.p)[row * e.ld] : 0.0;
    }
}

template <int NT, int KQ>
__device__ __forceinline__ void res_tile(const double (&a)[KQ], const double* Bs, int kq, int g,
                                         int rl, double (&csum)[NT]) {
  constexpr int S = 16 * NT + kResBPad;
  doublex4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = doublex4{};
#pragma unroll
  for (int q = 0; q < KQ; ++q)
    if (q < kq) {
      const double* br = Bs + (4 * q + g) * S + rl;
#pragma unroll
      for (int t = 0; t < NT; ++t)
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[q], br[16 * t], acc[t], 0, 0, 0);
    }
  // every lane holds four rows of column 16 t + (lane % 16)
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int i = 0; i < 4; ++i) csum[t] += acc[t][i] * acc[t][i];
}

template <int NT, int KQ>
__global__ __launch_bounds__(kResThreads) void residual_kernel(BlockView<double> A, int64_t n,
                                                               BlockView<double> B, CoreView core,
                                                               int64_t m, int gx, int gy,
                                                               double* __restrict__ part) {
  constexpr int NC = 16 * NT, KP = 4 * KQ, S = NC + kResBPad;
  static_assert(KP <= kKCAP, "residual: width beyond the column tables");
  __shared__ double Bs[KP * S];
  __shared__ ResCol acol[KP];
  __shared__ double coef[KP];
  __shared__ unsigned char blk[kKCAP];
  __shared__ short loc[kKCAP];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int g = lane >> 4, rl = lane & 15;
  // XCD-aware placement: consecutive workgroups of one XCD take the column
  // blocks of one row range (gx * gy is a multiple of 8)
  const int tot = gx * gy, L = blockIdx.x;
  const int id = (L & 7) * (tot >> 3) + (L >> 3);
  const int cb = id % gx, rg = id / gx;
  const int64_t j0 = int64_t(cb) * NC;
  {
    int k = 0;
    for (int b = 0; b < core.nb; ++b) {
      const int w = core_width(core, b);
      for (int c = threadIdx.x; c < w && k + c < KP; c += blockDim.x)
        coef[k + c] = core.coef[b] * (core.s[b] ? core.s[b][c] : 1.0);
      k += w;
    }
  }
  const int kb = min(build_coltab(B, blk, loc), KP);
  const int kp = (kb + 3) & ~3, kq = kp >> 2;
  __syncthreads();
  for (int e = threadIdx.x; e < NC * kp; e += blockDim.x) {
    const int jj = e / kp, c = e - jj * kp;
    double v = 0.0;
    if (j0 + jj < m && c < kb) v = view_at(B, blk[c], loc[c], j0 + jj) * coef[c];
    Bs[c * S + jj] = v;
  }
  __syncthreads();
  build_coltab(A, blk, loc);   // same total width as B; A carries no row scaling
  __syncthreads();
  for (int c = threadIdx.x; c < KP; c += blockDim.x) {
    ResCol e{nullptr, 0};
    if (c < kb) e = ResCol{A.ptr[blk[c]] + loc[c], int64_t(A.ld[blk[c]])};
    acol[c] = e;
  }
  __syncthreads();

  const int64_t nrt = (n + 15) / 16;
  const int64_t per = (nrt + gy - 1) / gy;
  const int64_t t0 = int64_t(rg) * per, t1 = min(nrt, t0 + per);
  double csum[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) csum[t] = 0.0;
  double a0[KQ], a1[KQ];
  const int nw = kResThreads / 64;
  int64_t tile = t0 + wave;
  res_load<KQ>(a0, acol, kq, g, tile * 16 + rl, tile < t1 && tile * 16 + rl < n);
  for (; tile < t1; tile += 2 * nw) {
    const int64_t tb = tile + nw, tc = tile + 2 * nw;
    res_load<KQ>(a1, acol, kq, g, tb * 16 + rl, tb < t1 && tb * 16 + rl < n);
    res_tile<NT, KQ>(a0, Bs, kq, g, rl, csum);
    if (tb >= t1) break;
    res_load<KQ>(a0, acol, kq, g, tc * 16 + rl, tc < t1 && tc * 16 + rl < n);
    res_tile<NT, KQ>(a1, Bs, kq, g, rl, csum);
  }
  // lanes l, l+16, l+32, l+48 share a column; then the waves
  __syncthreads();   // Bs is reused for the wave partials
  double* colacc = Bs;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    double v = csum[t];
    v += __shfl_xor(v, 16);
    v += __shfl_xor(v, 32);
    if (lane < 16) colacc[wave * NC + t * 16 + lane] = v;
  }
  __syncthreads();
  for (int jj = threadIdx.x; jj < NC; jj += blockDim.x) {
    double v = 0.0;
    for (int w = 0; w < nw; ++w) v += colacc[w * NC + jj];
    if (j0 + jj < m) gmem(part)[size_t(rg) * m + j0 + jj] = v;
  }
}

__global__ void residual_reduce_kernel(const double* __restrict__ part, int groups, int64_t m,
                                       double* __restrict__ colsq) {
  const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double s = 0.0;
  for (int g = 0; g < groups; ++g) s += gmem(part)[size_t(g) * m + j];
  colsq[j] = s;
}

size_t residual_workspace_bytes(int64_t n, int64_t m) {
  (void)n;
  return size_t(kResRowGroups) * size_t(m) * sizeof(double);
}

template <int NT, int KQ>
static void launch_res(const BlockView<double>& A, int64_t n, const BlockView<double>& B,
                       const CoreView& core, int64_t m, double* ws, hipStream_t s, int* gy_out) {
  constexpr int NC = 16 * NT;
  const int gx = int(ceil_div(m, NC));
  // about 1024 workgroups, a multiple of 8 row groups
  int gy = int(ceil_div(int64_t(1024), int64_t(gx)));
  gy = std::min(kResRowGroups, std::max(8, (gy + 7) / 8 * 8));
  *gy_out = gy;
  hipLaunchKernelGGL((residual_kernel<NT, KQ>), dim3(unsigned(gx * gy)), dim3(kResThreads), 0, s,
                     A, n, B, core, m, gx, gy, ws);
}

void launch_residual_fp64(const BlockView<double>& A, int64_t n, const BlockView<double>& B,
                          CoreView core, int64_t m, int kcap, double* colsq, double* ws,
                          size_t ws_bytes, hipStream_t s) {
  LRC_CHECK(kcap >= 0 && kcap <= kKCAP, ST_EINVAL, "residual: at most 192 columns");
  LRC_CHECK(view_cap(A) <= kKCAP && A.nb == B.nb && B.nb == core.nb, ST_EINVAL,
            "residual: inconsistent views");
  for (int b = 0; b < A.nb; ++b)
    LRC_CHECK(!A.rowscale[b], ST_EINVAL, "residual: row scaling of the left factor");
  LRC_CHECK(ws_bytes >= residual_workspace_bytes(n, m), ST_EINVAL, "residual: workspace too small");
  if (m <= 0) return;
  // algorithmic flops: every entry of the n x m residual is a k-term dot product
  Work w;
  w.bytes = false;
  const double nm = double(n) * double(m);
  w.groups = {view_terms(A)};
  w.f = [=](const std::vector<double>& v) { return 2.0 * nm * v[0]; };
  ProfScope ps(kcls(K_RESIDUAL, false), s, w);
  // kcap bounds the device widths; the tile shape follows it and m
  const int need = int(std::min<int64_t>(8, ceil_div(m, 16)));
  int gy = 8;
  if (kcap <= 64) {
    if (need > 4) launch_res<8, 16>(A, n, B, core, m, ws, s, &gy);
    else if (need > 2) launch_res<4, 16>(A, n, B, core, m, ws, s, &gy);
    else launch_res<2, 16>(A, n, B, core, m, ws, s, &gy);
  } else if (kcap <= 128) {
    if (need > 2) launch_res<4, 32>(A, n, B, core, m, ws, s, &gy);
    else launch_res<2, 32>(A, n, B, core, m, ws, s, &gy);
  } else {
    if (need > 2) launch_res<4, 48>(A, n, B, core, m, ws, s, &gy);
    else launch_res<2, 48>(A, n, B, core, m, ws, s, &gy);
  }
  hipLaunchKernelGGL(residual_reduce_kernel, dim3(unsigned(ceil_div(m, 256))), dim3(256), 0, s, ws,
                     gy, m, colsq);
  LRC_HIP(hipGetLastError());
}

}  // namespace lrc
