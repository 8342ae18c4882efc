// Small fp64 kernels of the truncation (k x k with k <= 128): equilibrated,
// shift-guarded Cholesky of a Gram matrix with the inverse of its factor,
// small matrix products, the SVD of the core (pivoted Householder QR, then
// one-sided Jacobi on R^T, with the rotations logged and replayed per row when
// they do not fit in LDS), and the rank selection.
#include <algorithm>

#include "kernels.hpp"
#include "prof.hpp"

namespace lrc {

// Batched launches: item = blockIdx.z; a done item does nothing.
#define LRC_ITEM(Type, name, a0, ab, done)        \
  if ((done) && (done)[blockIdx.z]) return;        \
  const Type& name = (ab) ? (ab)[blockIdx.z] : (a0);

constexpr int SK = 128;                         // capacity of the small kernels


// ============================================================== Cholesky + inverse
// One workgroup per side (A, B).  G is equilibrated (unit diagonal) and
// factorised G_s = R^T R right-looking; the rows are scaled only at the end
// (the trailing update divides by the pivot instead), so that each step needs
// a single barrier: step j reads row j and writes rows > j.  A pivot at or
// below tau = eps k restarts the factorisation of G_s + shift I (shift 10 tau,
// then 100 times larger): the shift bounds ||R^-1|| by shift^-1/2, which keeps
// X R^-1 well conditioned for the second pass.  Columns whose Gram diagonal
// vanishes are treated as absent.  R^-1 by 16 x 16 blocks.  Outputs (ld = kcap):
//   Rout = R D^{-1}   (so that X = Q Rout),  Tout = D R^{-1}  (so that Q = X Tout).

constexpr int kCholThreads = 512;
constexpr int kCL = SK + 1;   // row stride of the k x k matrix in LDS
typedef double doublex4_c __attribute__((ext_vector_type(4)));
__device__ inline doublex4_c mfma64(double a, double b, doublex4_c c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// value of v in lane `src` (uniform), through scalar registers
__device__ inline double lane_bcast(double v, int src) {
  const long long b = __double_as_longlong(v);
  const unsigned lo = unsigned(__builtin_amdgcn_readlane(int(b & 0xffffffffll), src));
  const unsigned hi = unsigned(__builtin_amdgcn_readlane(int(b >> 32), src));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
// Blocked right-looking Cholesky in 16-column panels: the diagonal block is
// factorised (and inverted) by one wave in registers with lane shuffles, the
// panel row R_IJ = R_II^-T A_IJ and the trailing update A_JL -= R_IJ^T R_IL
// run as 16 x 16 x 16 fp64 MFMA tile products; three barriers per panel.  The
// matrix is padded to whole tiles with identity rows.  R^-1 follows by block
// diagonals: W_IJ = sum_{I<L<=J} R_IL X_LJ, X_IJ = -X_II W_IJ, with the
// off-diagonal blocks of X kept in the (otherwise unused) lower triangle.
__global__ __launch_bounds__(kCholThreads) void chol_kernel(CholArgs a0, const CholArgs* ab,
                                                            const int* done) {
  LRC_ITEM(CholArgs, ca, a0, ab, done)
  const TruncState& st = ca.st;
  const int pass = ca.pass, kcap = ca.kcap;
  const double eps = ca.eps;
  __shared__ double A[SK * kCL];
  __shared__ double Tb[SK / 16][16][17];    // inverses of the diagonal blocks
  __shared__ double dsc[SK];
  __shared__ double s_gm;
  __shared__ int s_fail;
  const int side = blockIdx.x;
  const int k = *st.k;
  const double* G = st.G[side];
  double* Rout = pass == 1 ? st.R1[side] : st.R2[side];
  double* Tout = pass == 1 ? st.T1[side] : st.R2i[side];
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  const int nwv = nt >> 6;
  if (k == 0) return;
  const int nbk = (k + 15) / 16, kp = nbk * 16;
  // G is read from global memory once: the scale and the first attempt take it from LDS
  for (int i = wave; i < k; i += nwv)
    for (int j = lane; j < k; j += 64) A[i * kCL + j] = G[size_t(i) * kcap + j];
  __syncthreads();
  if (tid < 64) {
    double gm = 0.0;
    for (int j = tid; j < k; j += 64) gm = fmax(gm, A[j * kCL + j]);
    for (int o = 32; o > 0; o >>= 1) gm = fmax(gm, __shfl_xor(gm, o));
    if (tid == 0) s_gm = gm;
  }
  __syncthreads();
  for (int j = tid; j < k; j += nt) {
    const double g = A[j * kCL + j];
    dsc[j] = (g > 1e-300 && g > 1e-28 * s_gm) ? 1.0 / sqrt(g) : 0.0;
    // a non-finite diagonal means non-finite operand data: a breakdown, not
    // a vanishing column to be dropped
    if (!isfinite(g)) atomicOr(st.info, 2);
  }
  __syncthreads();
  const double tau = eps * k;
  double shift = ca.shift0;
  bool fail = true;
  const int lr = lane >> 4, lc = lane & 15;   // MFMA slice row group, column
  for (int attempt = 0; attempt < 6 && fail; ++attempt) {
    // equilibrated (and shifted) Gram, identity on dead columns and padding
    for (int e = tid; e < kp * kp; e += nt) {
      const int i = e / kp, j = e - i * kp;
      double v;
      if (i < k && j < k) {
        const double di = dsc[i], dj = dsc[j];
        const double g = attempt == 0 ? A[i * kCL + j] : G[size_t(i) * kcap + j];
        v = (di == 0.0 || dj == 0.0) ? (i == j ? 1.0 : 0.0) : di * g * dj + (i == j ? shift : 0.0);
      } else {
        v = i == j ? 1.0 : 0.0;
      }
      A[i * kCL + j] = v;
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();
    for (int I = 0; I < nbk; ++I) {
      const int o = 16 * I;
      if (wave == 0) {
        // lane c < 16 holds column c of the diagonal block (rows 0..15)
        // (the reciprocal square root of each pivot scales its row and is the
        // inverse's diagonal: no division on the dependent chain)
        double a[16], x[16], rinv[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) a[r] = lc < 16 ? A[(o + r) * kCL + o + lc] : 0.0;
        bool bad = false;
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) {
          const double piv = lane_bcast(a[jj], jj);
          if (!(piv > tau) && o + jj < k) bad = true;
          const double pv = fmax(piv, 1e-300);
          const double ri = rsqrt(pv);
          rinv[jj] = ri;
          a[jj] = lane == jj ? pv * ri : (lane > jj ? a[jj] * ri : a[jj]);
#pragma unroll
          for (int ii = jj + 1; ii < 16; ++ii) {
            const double t = lane_bcast(a[jj], ii);     // r_{jj, ii}
            if (lane >= ii) a[ii] -= t * a[jj];
          }
        }
        // R_II back to LDS first: the inverse reads its rows there (one
        // broadcast load per entry, in the wave's own LDS order)
        if (lane < 16) {
#pragma unroll
          for (int r = 0; r < 16; ++r) A[(o + r) * kCL + o + lane] = r <= lane ? a[r] : 0.0;
        }
        // x = column lc of the inverse of the upper-triangular block (x[t] = 0
        // for t > lc; the newest x[t] enters the sum last, which keeps the
        // dependent chain at one product per row)
#pragma unroll
        for (int ii = 15; ii >= 0; --ii) {
          double acc = 0.0;
#pragma unroll
          for (int tt = 15; tt > ii; --tt) acc = fma(A[(o + ii) * kCL + o + tt], x[tt], acc);
          x[ii] = ii == lane ? rinv[ii] : (ii < lane ? -acc * rinv[ii] : 0.0);
        }
        if (lane < 16) {
#pragma unroll
          for (int r = 0; r < 16; ++r) Tb[I][r][lane] = x[r];
        }
        if (bad && lane == 0) s_fail = 1;
      }
      __syncthreads();
      if (s_fail) break;                       // same value in every thread
      // panel row: R_IJ = X_II^T A_IJ, one wave per tile
      for (int J = I + 1 + wave; J < nbk; J += nwv) {
        doublex4_c acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4)
          acc = mfma64(Tb[I][kk + lr][lc], A[(o + kk + lr) * kCL + 16 * J + lc], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) A[(o + lr + 4 * v) * kCL + 16 * J + lc] = acc[v];
      }
      __syncthreads();
      // trailing update of the upper tiles: A_JL -= R_IJ^T R_IL, I < J <= L
      const int nr = nbk - I - 1;
      for (int tt = wave; tt < nr * (nr + 1) / 2; tt += nwv) {
        int J = 0, rem = tt;
        while (rem >= nr - J) { rem -= nr - J; ++J; }
        const int L = I + 1 + J + rem;
        J += I + 1;
        doublex4_c acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4)
          acc = mfma64(A[(o + kk + lr) * kCL + 16 * J + lc], A[(o + kk + lr) * kCL + 16 * L + lc], acc);
#pragma unroll
        for (int v = 0; v < 4; ++v) A[(16 * J + lr + 4 * v) * kCL + 16 * L + lc] -= acc[v];
      }
      __syncthreads();
    }
    fail = s_fail != 0;
    if (fail) {
      shift = shift == 0.0 ? 10.0 * tau : 100.0 * shift;
      if (tid == 0) atomicOr(st.info, 1);
      __syncthreads();
    }
  }
  if (fail) {
    // give up on factorising: identity factor (the truncation then works on the
    // equilibrated columns as they are) and report the breakdown
    for (int e = tid; e < kp * kp; e += nt) {
      const int i = e / kp, j = e - i * kp;
      if (j >= i) A[i * kCL + j] = (i == j) ? 1.0 : 0.0;
    }
    for (int e = tid; e < nbk * 256; e += nt) {
      const int I = e >> 8, r = (e >> 4) & 15, c = e & 15;
      Tb[I][r][c] = r == c ? 1.0 : 0.0;
    }
    if (tid == 0) atomicOr(st.info, 2);
  }
  __syncthreads();
  // Rout = R D^{-1} (only the leading k x k block: every consumer reads
  // within the device width)
  for (int e = tid; e < k * k; e += nt) {
    const int i = e / k, j = e - i * k;
    double v = 0.0;
    if (j >= i && dsc[j] != 0.0) v = A[i * kCL + j] / dsc[j];
    Rout[size_t(i) * kcap + j] = v;
  }
  // X = R^{-1} by block diagonals; X_IJ (I < J) lives in the lower tile (J, I)
  for (int d = 1; d < nbk; ++d) {
    // W_IJ = sum_{L = I+1..J} R_IL X_LJ into the tile of X_IJ
    for (int I = wave; I + d < nbk; I += nwv) {
      const int J = I + d;
      doublex4_c acc = {0.0, 0.0, 0.0, 0.0};
      for (int L = I + 1; L <= J; ++L) {
#pragma unroll
        for (int kk = 0; kk < 16; kk += 4) {
          const double xv = L == J ? Tb[J][kk + lr][lc]
                                   : A[(16 * J + kk + lr) * kCL + 16 * L + lc];
          acc = mfma64(A[(16 * I + lc) * kCL + 16 * L + kk + lr], xv, acc);
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(16 * J + lr + 4 * v) * kCL + 16 * I + lc] = acc[v];
    }
    __syncthreads();
    // X_IJ = -X_II W_IJ, in place
    for (int I = wave; I + d < nbk; I += nwv) {
      const int J = I + d;
      doublex4_c acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4)
        acc = mfma64(Tb[I][lc][kk + lr], A[(16 * J + kk + lr) * kCL + 16 * I + lc], acc);
#pragma unroll
      for (int v = 0; v < 4; ++v) A[(16 * J + lr + 4 * v) * kCL + 16 * I + lc] = -acc[v];
    }
    __syncthreads();
  }
  // Tout = D R^{-1} (leading k x k block)
  for (int e = tid; e < k * k; e += nt) {
    const int i = e / k, j = e - i * k;
    double v = 0.0;
    if (j >= i) {
      const int I = i >> 4, J = j >> 4;
      const double xv = I == J ? Tb[I][i & 15][j & 15] : A[(16 * J + (i & 15)) * kCL + 16 * I + (j & 15)];
      v = dsc[i] * xv;
    }
    Tout[size_t(i) * kcap + j] = v;
  }
}

void enqueue_chol(const CholArgs& a, Batched<CholArgs> b, hipStream_t s) {
  LRC_CHECK(a.kcap <= SK, ST_EINVAL, "truncation: at most 128 concatenated columns");
  ProfScope ps(kcls(K_CHOL, false), s);
  hipLaunchKernelGGL(chol_kernel, dim3(2, 1, b.n), dim3(kCholThreads), 0, s, a, b.dev, b.done);
  LRC_HIP(hipGetLastError());
}

// ============================================================== small products
// C = op(A) diag(mid) op(B)[:, colperm] diag(colscale), all k x k (or k x r
// output columns), fp64, ld kcap.  One 16 x 16 output tile per workgroup: the
// tile's 16-row panel of op(A) and 16-column panel of op(B) (inner length at
// most 128) are staged in LDS with one round of loads, each coalesced along
// the index that is contiguous in memory, and every thread then sums its
// entry over the whole inner length.
__global__ __launch_bounds__(256) void small_gemm_kernel(SmallGemmArgs a0, const SmallGemmArgs* ab,
                                                         const int* done) {
  __shared__ double As[16][SK + 1];
  __shared__ double Bs[SK][17];
  __shared__ double mid[SK];
  // blockIdx.z = item * 2 + job
  const int item = blockIdx.z >> 1;
  if (done && done[item]) return;
  const SmallGemmArgs& a = ab ? ab[item] : a0;
  if (int(blockIdx.z & 1) >= a.njobs) return;
  const SmallGemm g = a.g[blockIdx.z & 1];   // by value: fields read once
  const int k = *a.k;
  const int ncols = g.ncols_dev ? *g.ncols_dev : k;
  const int kin = g.inner_dev ? *g.inner_dev : k;
  const int ti = blockIdx.y * 16, tj = blockIdx.x * 16;
  if (ti >= k || tj >= ncols) return;
  const int tid = threadIdx.x;
  if (g.use_core) {
    int off = 0;
    for (int b = 0; b < a.core.nb; ++b) {
      const int w = core_width(a.core, b);
      for (int c = tid; c < w && off + c < SK; c += blockDim.x)
        mid[off + c] = a.core.coef[b] * (a.core.s[b] ? a.core.s[b][c] : 1.0);
      off += w;
    }
  }
  const int kc = a.kcap;
  const double* __restrict__ Ap = g.A;
  const double* __restrict__ Bp = g.B;
  const int* __restrict__ cp = g.colperm;
  const bool ta = g.transA != 0, tb = g.transB != 0;
  // eight entries of each panel per thread; indices are clamped inside the
  // leading blocks the producers wrote (finite values), so that every load is
  // issued at once, and entries outside the operands are zeroed by a product
  // with a 0/1 mask (a select would let the compiler move each load into a
  // branch of its own and wait for it there)
  constexpr int PE = 16 * SK / 256;
  double va[PE], vb[PE];
  if (kin > 0) {
    // the column permutation first (its loads together, outside the panel loop)
    int jcs[PE];
#pragma unroll
    for (int u = 0; u < PE; ++u) {
      const int e = tid + 256 * u;
      jcs[u] = min(tj + (tb ? e / SK : (e & 15)), ncols - 1);
    }
    if (cp) {
#pragma unroll
      for (int u = 0; u < PE; ++u) jcs[u] = cp[jcs[u]];
    }
#pragma unroll
    for (int u = 0; u < PE; ++u) {
      const int e = tid + 256 * u;
      const int li = ta ? (e & 15) : e / SK, pa = ta ? (e >> 4) : e % SK;
      const int i = ti + li;
      const int ic = min(i, k - 1), pc = min(pa, kin - 1);
      const double x = ta ? Ap[size_t(pc) * kc + ic] : Ap[size_t(ic) * kc + pc];
      va[u] = x * ((i < k && pa < kin) ? 1.0 : 0.0);
      const int lj = tb ? e / SK : (e & 15), pb = tb ? e % SK : (e >> 4);
      const int j = tj + lj;
      const int qc = min(pb, kin - 1), jc = jcs[u];
      const double y = tb ? Bp[size_t(jc) * kc + qc] : Bp[size_t(qc) * kc + jc];
      vb[u] = y * ((pb < kin && j < ncols) ? 1.0 : 0.0);
    }
  } else {
#pragma unroll
    for (int u = 0; u < PE; ++u) va[u] = vb[u] = 0.0;
  }
#pragma unroll
  for (int u = 0; u < PE; ++u) {
    const int e = tid + 256 * u;
    As[ta ? (e & 15) : e / SK][ta ? (e >> 4) : e % SK] = va[u];
    Bs[tb ? e % SK : (e >> 4)][tb ? e / SK : (e & 15)] = vb[u];
  }
  __syncthreads();
  if (g.use_core) {
    for (int e = tid; e < 16 * SK; e += 256) {
      const int lj = e & 15, p = e >> 4;
      if (p < kin) Bs[p][lj] *= mid[p];
    }
    __syncthreads();
  }
  const int li = tid >> 4, lj = tid & 15;
  const int i = ti + li, j = tj + lj;
  double acc = 0.0;
  // (entries past the inner length were staged as zeros)
  for (int p0 = 0; p0 < kin; p0 += 16) {
#pragma unroll
    for (int q = 0; q < 16; ++q) acc += As[li][p0 + q] * Bs[p0 + q][lj];
  }
  if (i < k && j < ncols) {
    if (g.colscale) acc *= g.colscale[j];
    const int io = g.rowperm ? g.rowperm[i] : i;
    g.C[size_t(io) * kc + j] = acc;
  }
}

SmallGemmArgs make_small_gemm(const SmallGemm* jobs, int njobs, CoreView core, const int* k,
                              int kcap) {
  SmallGemmArgs a;
  a.g[0] = jobs[0];
  a.g[1] = njobs > 1 ? jobs[1] : jobs[0];
  a.core = core;
  a.k = k;
  a.kcap = kcap;
  a.njobs = njobs;
  return a;
}

void enqueue_small_gemm(const SmallGemmArgs& a, Batched<SmallGemmArgs> b, hipStream_t s) {
  const int t = (a.kcap + 15) / 16;
  ProfScope ps(kcls(K_SMALL_GEMM, false), s);
  hipLaunchKernelGGL(small_gemm_kernel, dim3(t, t, 2 * b.n), dim3(256), 0, s, a, b.dev, b.done);
  LRC_HIP(hipGetLastError());
}

// ============================================================== one-sided Jacobi
// Round-robin ("tournament") pairing of kp (even) indices: in round t, slot a
// pairs positions a and kp-1-a of the rotated list [0, 1 + (t + i) mod (kp-1)].
__device__ inline int rr_player(int pos, int t, int kp) {
  if (pos == 0) return 0;
  // pos - 1 and t are both below kp - 1: one conditional subtraction
  // replaces the integer modulo
  const int x = pos - 1 + t;
  return 1 + (x >= kp - 1 ? x - (kp - 1) : x);
}

// One-sided (Hestenes) Jacobi SVD of X = R^T (k x kj), R from the pivoted QR
// of the core: X Y = Z with orthogonal columns, sigma_a = ||z_a||, so that
// R = Y diag(sigma) (Z diag(1/sigma))^T.  The QR's column pivoting makes the
// columns of X graded and nearly orthogonal, so few sweeps are needed.  X is
// kept in LDS by columns; a round rotates kp/2 disjoint pairs (p, q), one
// team of 16, 32 or 64 lanes per pair (the three dot products reduced with
// lane shuffles), chosen so that x_p^T x_q = 0 afterwards:
//   zeta = (b - a) / (2 g),  t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
//   c = 1 / sqrt(1 + t^2),  s = c t,  [x_p, x_q] <- [c x_p - s x_q, s x_p + c x_q]
// with a = ||x_p||^2, b = ||x_q||^2, g = x_p^T x_q; a pair is rotated when
// |g| > 1e-14 sqrt(a b) (rounding level of the products), so every singular
// value comes out with an absolute error of a few ulps of ||M|| and the
// columns of Z are orthogonal to working accuracy whatever their norms.
// Y accumulates in LDS next to X when both fit; otherwise the (c, s) of every
// round are logged and the replay kernel rebuilds Y.  Outputs: sigma (st.lam,
// Jacobi order), V_M = Z diag(1/sigma) (st.VP, k x kj), Y (st.VM) or the log.
constexpr int kJacThreads = 512;
constexpr int kJacLds = 18432;              // doubles (144 KiB)
constexpr int kJacE = 16;                   // column entries per lane (k <= 16 * 8)
static_assert(SK * SK <= kJacLds, "X must fit in LDS at the largest width");
static_assert(kJacE * 8 >= SK, "a team of 8 lanes must hold a column");
// One round for the pairs of one team size TL (16 lanes per pair while at
// most 32 pairs fit the 8 waves, else 8): a lane keeps its E >= k / TL entries
// of both columns in registers between the dot products and the rotation, so
// that a round reads each column from LDS once and writes it once.
// Sum of a double over the 16 lanes of a DPP row, in every lane: four
// rotate-and-add steps (row_ror 8, 4, 2, 1) on the two 32-bit halves, which
// stay inside the row (no LDS permute).
template <int ROT>
__device__ __forceinline__ double row_ror(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b & 0xffffffffll), 0x120 + ROT, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0x120 + ROT, 0xf, 0xf, false);
  return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double row_sum16(double x) {
  x += row_ror<8>(x);
  x += row_ror<4>(x);
  x += row_ror<2>(x);
  x += row_ror<1>(x);
  return x;
}

// 1/x and 1/sqrt(x) from the hardware estimates refined by two Newton steps
// each (quadratic convergence from the estimate's ~2^-23 to the last bits);
// x finite and normal.  The fp64 divide and square root expand to long
// dependent sequences that set the length of a Jacobi round.
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  r = fma(r, fma(-x, r, 1.0), r);
  return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  y = fma(0.5 * y, fma(-x * y, y, 1.0), y);
  return y;
}

// E: column entries per lane actually live (k <= TL E), so that a narrow core
// issues no work for the empty slots
template <int TL, int E>
__device__ __forceinline__ int jacobi_pair(double* X, double* Y, bool fuse, int k, int kj, int p,
                                           int q, int tl, double* cs, double& dmax) {
  double* xp = X + p * k;
  double* xq = X + q * k;
  double u[E], v[E];
  double al = 0.0, be = 0.0, ga = 0.0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = tl + e * TL;
    u[e] = i < k ? xp[i] : 0.0;
    v[e] = i < k ? xq[i] : 0.0;
  }
#pragma unroll
  for (int e = 0; e < E; ++e) {
    al = fma(u[e], u[e], al);
    be = fma(v[e], v[e], be);
    ga = fma(u[e], v[e], ga);
  }
  if constexpr (TL == 16) {
    // a team is one DPP row
    al = row_sum16(al);
    be = row_sum16(be);
    ga = row_sum16(ga);
  } else {
#pragma unroll
    for (int o = TL >> 1; o > 0; o >>= 1) {
      al += __shfl_xor(al, o);
      be += __shfl_xor(be, o);
      ga += __shfl_xor(ga, o);
    }
  }
  double c = 1.0, s = 0.0;
  // squared relative coupling g^2 / (a b) (the exit test needs no accuracy)
  const double ab = al * be, g2 = ga * ga;
  if (ab > 1e-300) dmax = fmax(dmax, g2 * __builtin_amdgcn_rcp(ab));
  // rotate when |g| > 1e-14 sqrt(a b); where a b underflows only the guard
  // |g| > 1e-300 applies: pairs of tiny columns are still rotated, so that
  // the singular vectors of small singular values stay orthogonal
  if (fabs(ga) > 1e-300 && (g2 > 1e-28 * ab || !(ab > 0.0))) {
    const double zeta = (be - al) * (0.5 * rcp_nr(ga));
    const double az = fabs(zeta);
    // sqrt(1 + zeta^2) without overflow for huge |zeta|
    const double w = fma(az, az, 1.0);
    const double hyp = az > 1e150 ? az : w * rsq_nr(w);
    const double tt = zeta >= 0.0 ? rcp_nr(az + hyp) : -rcp_nr(az + hyp);
    c = rsq_nr(fma(tt, tt, 1.0));
    s = c * tt;
  }
  cs[0] = c;
  cs[1] = s;
  if (s == 0.0) return 0;
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int i = tl + e * TL;
    if (i < k) {
      xp[i] = c * u[e] - s * v[e];
      xq[i] = s * u[e] + c * v[e];
    }
  }
  if (fuse) {
    double* yp = Y + p * kj;
    double* yq = Y + q * kj;
    for (int b = tl; b < kj; b += TL) {
      const double a1 = yp[b], a2 = yq[b];
      yp[b] = c * a1 - s * a2;
      yq[b] = s * a1 + c * a2;
    }
  }
  return 1;
}

__global__ __launch_bounds__(kJacThreads) void jacobi_kernel(JacArgs a0, const JacArgs* ab,
                                                            const int* done) {
  LRC_ITEM(JacArgs, ja_, a0, ab, done)
  const TruncState& st = ja_.st;
  const int kcap = ja_.kcap, max_rounds = ja_.max_rounds;
  __shared__ double lds[kJacLds];
  __shared__ double s_sig[SK];
  const int k = *st.k, kj = *st.kj;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  if (kj <= 0 || k <= 0) {
    if (tid == 0) *st.rounds = -1;
    return;
  }
  const int kp = kj + (kj & 1);
  const int npair = kp / 2;
  const bool fuse = kj * k + kj * kj <= kJacLds;
  double* X = lds;                 // column a at X + a * k
  double* Y = lds + kj * k;        // column a at Y + a * kj (when fused)
  for (int e = tid; e < kj * k; e += nt) {
    const int a = e / k, i = e - a * k;
    X[e] = st.W[size_t(a) * kcap + i];
  }
  if (fuse)
    for (int e = tid; e < kj * kj; e += nt) Y[e] = (e / kj == e % kj) ? 1.0 : 0.0;
  __syncthreads();
  const bool wide = npair > (kJacThreads / 16);   // more pairs than 16-lane teams
  const int TL = wide ? 8 : 16;
  const int slot = wave * (64 / TL) + lane / TL;
  const int tl = lane % TL;
  // Sweeps end when none rotates, or once the largest relative coupling
  // |x_p^T x_q| / (||x_p|| ||x_q||) met in a sweep is below 1e-7 (its square
  // below 1e-14): convergence
  // is quadratic, so the next sweep would only meet couplings near 1e-14,
  // the rounding level of the dot products themselves (a sweep spent on
  // rounding noise is saved).
  __shared__ double s_dmax[kJacThreads / 64];
  int round = 0;
  bool converged = false;
  for (int sweep = 0; sweep < 30 && round < max_rounds; ++sweep) {
    int any = 0;
    double dmax = 0.0;
    for (int t = 0; t < kp - 1 && round < max_rounds; ++t, ++round) {
      if (slot < npair) {
        int p = rr_player(slot, t, kp), q = rr_player(kp - 1 - slot, t, kp);
        if (p > q) { const int x = p; p = q; q = x; }
        double cs[2] = {1.0, 0.0};
        if (q < kj) {
          if (wide)
            any |= jacobi_pair<8, SK / 8>(X, Y, fuse, k, kj, p, q, tl, cs, dmax);
          else if (k <= 16)
            any |= jacobi_pair<16, 1>(X, Y, fuse, k, kj, p, q, tl, cs, dmax);
          else if (k <= 32)
            any |= jacobi_pair<16, 2>(X, Y, fuse, k, kj, p, q, tl, cs, dmax);
          else if (k <= 64)
            any |= jacobi_pair<16, 4>(X, Y, fuse, k, kj, p, q, tl, cs, dmax);
          else
            any |= jacobi_pair<16, SK / 16>(X, Y, fuse, k, kj, p, q, tl, cs, dmax);
        }
        if (!fuse && tl == 0) {
          st.rot[(size_t(round) * (SK / 2) + slot) * 2 + 0] = cs[0];
          st.rot[(size_t(round) * (SK / 2) + slot) * 2 + 1] = cs[1];
        }
      }
      __syncthreads();
    }
    for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o));
    if (lane == 0) s_dmax[wave] = dmax;
    if (!__syncthreads_or(any)) { converged = true; break; }
    double dm = 0.0;
    for (int w = 0; w < kJacThreads / 64; ++w) dm = fmax(dm, s_dmax[w]);
    if (dm < 1e-14) { converged = true; break; }
  }
  for (int a = tid; a < kj; a += nt) {
    double sq = 0.0;
    for (int i = 0; i < k; ++i) sq = fma(X[a * k + i], X[a * k + i], sq);
    s_sig[a] = sqrt(sq);
  }
  __syncthreads();
  for (int e = tid; e < kj * k; e += nt) {
    const int c = e / kj, a = e - c * kj;
    const double sg = s_sig[a];
    st.VP[size_t(c) * kcap + a] = sg > 0.0 ? X[a * k + c] * (1.0 / sg) : 0.0;
  }
  for (int a = tid; a < kj; a += nt) st.lam[a] = s_sig[a];
  if (fuse)
    for (int e = tid; e < kj * kj; e += nt) {
      const int b = e / kj, a = e - b * kj;
      st.VM[size_t(b) * kcap + a] = Y[a * kj + b];
    }
  if (tid == 0) {
    *st.rounds = fuse ? -1 : round;
    st.kj[1] = round;   // diagnostic: rounds taken
    if (!converged) atomicOr(st.info, 4);
  }
}

// V = J_0 J_1 ... J_{T-1}: every row of V evolves independently.  A workgroup
// (one wave) owns kRepRows rows; lane a applies pair a's rotation to them.  The
// rotation log is staged through LDS in batches of kRepBatch rounds.
constexpr int kRepRows = 4;
constexpr int kRepBatch = 16;
__global__ __launch_bounds__(64) void jacobi_replay_kernel(RepArgs a0, const RepArgs* ab,
                                                           const int* done) {
  LRC_ITEM(RepArgs, ra_, a0, ab, done)
  const TruncState& st = ra_.st;
  const int kcap = ra_.kcap;
  __shared__ double row[kRepRows][SK];
  __shared__ double2 rb[kRepBatch][SK / 2];
  const int k = *st.kj;
  const int kp = k + (k & 1);
  const int i0 = blockIdx.x * kRepRows;
  if (i0 >= k) return;
  const int T = *st.rounds;
  if (T < 0) return;                  // the Jacobi kernel already wrote V
  const int lane = threadIdx.x;
  for (int r = 0; r < kRepRows; ++r)
    for (int j = lane; j < kp; j += 64) row[r][j] = (j == i0 + r) ? 1.0 : 0.0;
  const int npair = kp / 2;
  const double2* rot = reinterpret_cast<const double2*>(st.rot);
  for (int t0 = 0; t0 < T; t0 += kRepBatch) {
    const int nb = min(kRepBatch, T - t0);
    __syncthreads();
    for (int e = lane; e < nb * (SK / 2); e += 64) rb[e / (SK / 2)][e % (SK / 2)] = rot[size_t(t0) * (SK / 2) + e];
    __syncthreads();
    for (int tb = 0; tb < nb; ++tb) {
      if (lane < npair) {
        const int tr = (t0 + tb) % (kp - 1);
        int p = rr_player(lane, tr, kp), q = rr_player(kp - 1 - lane, tr, kp);
        if (p > q) { int x = p; p = q; q = x; }
        const double2 cs = rb[tb][lane];
        if (cs.y != 0.0) {
#pragma unroll
          for (int r = 0; r < kRepRows; ++r) {
            const double vp = row[r][p], vq = row[r][q];
            row[r][p] = cs.x * vp - cs.y * vq;
            row[r][q] = cs.y * vp + cs.x * vq;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int r = 0; r < kRepRows; ++r) {
    const int i = i0 + r;
    if (i >= k) break;
    for (int j = lane; j < k; j += 64) st.VM[size_t(i) * kcap + j] = row[r][j];
  }
}

void enqueue_replay(const RepArgs& a, Batched<RepArgs> b, hipStream_t s) {
  ProfScope ps(kcls(K_REPLAY, false), s);
  hipLaunchKernelGGL(jacobi_replay_kernel, dim3((a.kcap + kRepRows - 1) / kRepRows, 1, b.n),
                     dim3(64), 0, s, a, b.dev, b.done);
  LRC_HIP(hipGetLastError());
}

// ============================================================== pivoted QR of the core
// Householder QR with column pivoting of the core M (k x k), M P = Q R, in
// fp64 and without forming M^T M: 8-lane teams hold one column of M each
// (rows tl + 8 t), the same threads hold one row of Q each (Q <- Q H_j after
// every step, so Q's first kj columns are ready at the end).  Step j takes the
// column with the largest trailing norm (recomputed exactly each step: no
// downdating), builds the reflector from its rows >= j (beta = -sign(x_j)
// ||x||, v_j = 1, v_i = x_i / (x_j - beta), tau = (beta - x_j) / beta), and
// applies it to the other columns and to Q.  It stops once the trailing block's
// Frobenius norm is at most 1e-3 of the truncation's tail budget
// max(tol ||M||_F, abs_tol): what is left cannot move the rank decision or any
// kept singular value by more than (1e-3 budget)^2 / sigma.  For factors held
// in fp32 it also stops at 1e-7 ||M||_F, their rounding level.  Outputs: R (kj x
// k, by original column, so that M = Q R) in st.W, Q (k x kj) in st.H, the
// pivot order in st.piv and kj in st.kj.  Two barriers per step; every wave
// takes the pivot decision itself from the same LDS data (same order of
// operations, so the same result in every wave).
constexpr int kQrThreads = 1024;
constexpr int kQrTeam = 8;
constexpr int kQrSlots = SK / kQrTeam;
static_assert(kQrThreads / kQrTeam == SK, "one team per column");
__device__ inline double team8_sum(double v) {
  v += __shfl_xor(v, 4);
  v += __shfl_xor(v, 2);
  v += __shfl_xor(v, 1);
  return v;
}
// NS: slots per lane actually live (k <= 8 NS), so that a narrow core issues
// no work for the empty slots.  Waves whose teams all lie beyond k only keep
// the barriers: the pivot search runs in the waves that hold columns, and
// wave 0 publishes the stop decision for the others.
template <int NS>
__device__ __forceinline__ void qrcp_body(const QrArgs& qa_, int k, double* nrm, double* vb,
                                          double* s_tau, int* s_stop) {
  const TruncState& st = qa_.st;
  const int kcap = qa_.kcap;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int team = tid >> 3, tl = tid & 7;
  const bool inside = team < k;
  const bool wave_live = wave * (64 / kQrTeam) < k;
  double mc[NS], qr[NS];
  double ss = 0.0;
#pragma unroll
  for (int t = 0; t < NS; ++t) {
    const int i = tl + kQrTeam * t;
    mc[t] = (inside && i < k) ? st.M[size_t(i) * kcap + team] : 0.0;   // M[i][team]
    qr[t] = (inside && i == team) ? 1.0 : 0.0;                          // Q[team][i]
    ss = fma(mc[t], mc[t], ss);
  }
  ss = team8_sum(ss);
  if (tl == 0) nrm[team] = inside ? ss : -1.0;
  __syncthreads();
  bool active = inside;
  double thr2 = 0.0;
  int kj = 0;
  for (int j = 0; j < k; ++j) {
    int p = -1;
    if (wave_live) {
      double best = -1.0, tot = 0.0;
      int bi = SK;
      for (int c = lane; c < k; c += 64) {
        const double v = nrm[c];
        if (v >= 0.0) {
          tot += v;
          if (v > best) { best = v; bi = c; }
        }
      }
      for (int o = 32; o > 0; o >>= 1) {
        tot += __shfl_xor(tot, o);
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (j == 0) {
        const double b1 = qa_.tol > 0.0 ? 1e-3 * qa_.tol : 0.0;
        const double b2 = 1e-3 * qa_.abs_tol;
        // factors held in fp32 resolve nothing below their rounding level: the
        // directions there are noise of the data, not of the method
        const double b3 = qa_.data_eps;
        thr2 = fmax(fmax(b1 * b1, b3 * b3) * tot, b2 * b2);
      }
      const bool stop = !(tot > thr2) || !(best > 0.0) || bi >= k;   // the same in every wave
      if (wave == 0 && lane == 0) *s_stop = stop ? 1 : 0;
      p = stop ? -1 : bi;
      if (!stop && team == p) {
        double s2 = 0.0, x0 = 0.0;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const int i = tl + kQrTeam * t;
          if (i >= j && i < k) s2 = fma(mc[t], mc[t], s2);
          if (i == j) x0 = mc[t];
        }
        s2 = team8_sum(s2);
        x0 = team8_sum(x0);
        const double nx = sqrt(s2);               // s2 >= best > 0
        const double beta = x0 >= 0.0 ? -nx : nx;
        // |x0 - beta| = |x0| + ||x|| >= |beta| > 0; the refined estimate
        // needs a normal operand
        const bool normal = nx > 1e-290;
        const double inv = normal ? rcp_nr(x0 - beta) : 1.0 / (x0 - beta);
        const double rb = normal ? rcp_nr(beta) : 1.0 / beta;
#pragma unroll
        for (int t = 0; t < NS; ++t) {
          const int i = tl + kQrTeam * t;
          if (i < k) vb[i] = i < j ? 0.0 : (i == j ? 1.0 : mc[t] * inv);
        }
        if (tl == 0) {
          *s_tau = (beta - x0) * rb;
          st.W[size_t(j) * kcap + p] = beta;
          st.piv[j] = p;
        }
      }
    }
    __syncthreads();
    if (*s_stop) break;                         // the same in every wave
    const double tau = *s_tau;
    if (active && team != p) {
      double w = 0.0;
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int i = tl + kQrTeam * t;
        if (i < k) w = fma(vb[i], mc[t], w);
      }
      w = team8_sum(w) * tau;
      double s2 = 0.0, rj = 0.0;
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int i = tl + kQrTeam * t;
        if (i < k) {
          mc[t] = fma(-w, vb[i], mc[t]);
          if (i > j) s2 = fma(mc[t], mc[t], s2);
          if (i == j) rj = mc[t];
        }
      }
      s2 = team8_sum(s2);
      rj = team8_sum(rj);
      if (tl == 0) {
        nrm[team] = s2;
        st.W[size_t(j) * kcap + team] = rj;
      }
    } else if (inside && team != p && tl == 0) {
      st.W[size_t(j) * kcap + team] = 0.0;       // chosen at an earlier step
    }
    if (team == p) {
      active = false;
      if (tl == 0) nrm[p] = -1.0;
    }
    // Q <- Q H_j (row `team` of Q)
    if (inside) {
      double w = 0.0;
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int c = tl + kQrTeam * t;
        if (c < k) w = fma(qr[t], vb[c], w);
      }
      w = team8_sum(w) * tau;
#pragma unroll
      for (int t = 0; t < NS; ++t) {
        const int c = tl + kQrTeam * t;
        if (c < k) qr[t] = fma(-w, vb[c], qr[t]);
      }
    }
    kj = j + 1;
    __syncthreads();
  }
  if (inside) {
#pragma unroll
    for (int t = 0; t < NS; ++t) {
      const int c = tl + kQrTeam * t;
      if (c < kj) st.H[size_t(team) * kcap + c] = qr[t];
    }
  }
  if (tid == 0) *st.kj = kj;
}

__global__ __launch_bounds__(kQrThreads) void qrcp_kernel(QrArgs a0, const QrArgs* ab,
                                                          const int* done) {
  LRC_ITEM(QrArgs, qa_, a0, ab, done)
  __shared__ double nrm[SK];     // trailing squared norm of each column (-1: chosen or absent)
  __shared__ double vb[SK];      // reflector of the current step
  __shared__ double s_tau;
  __shared__ int s_stop;
  const int k = *qa_.st.k;
  if (k <= 8) qrcp_body<1>(qa_, k, nrm, vb, &s_tau, &s_stop);
  else if (k <= 16) qrcp_body<2>(qa_, k, nrm, vb, &s_tau, &s_stop);
  else if (k <= 32) qrcp_body<4>(qa_, k, nrm, vb, &s_tau, &s_stop);
  else if (k <= 64) qrcp_body<8>(qa_, k, nrm, vb, &s_tau, &s_stop);
  else qrcp_body<kQrSlots>(qa_, k, nrm, vb, &s_tau, &s_stop);
}

void enqueue_qrcp(const QrArgs& a, Batched<QrArgs> b, hipStream_t s) {
  LRC_CHECK(a.kcap <= SK, ST_EINVAL, "truncation: at most 128 concatenated columns");
  ProfScope ps(kcls(K_QRCP, false), s);
  hipLaunchKernelGGL(qrcp_kernel, dim3(1, 1, b.n), dim3(kQrThreads), 0, s, a, b.dev, b.done);
  LRC_HIP(hipGetLastError());
}

void enqueue_jacobi(const JacArgs& a, Batched<JacArgs> b, hipStream_t s) {
  ProfScope ps(kcls(K_JACOBI, false), s);
  hipLaunchKernelGGL(jacobi_kernel, dim3(1, 1, b.n), dim3(kJacThreads), 0, s, a, b.dev, b.done);
  LRC_HIP(hipGetLastError());
}

// R_A = R2_A R1_A, R_B = R2_B R1_B (into the G buffers); M = R_A diag(core) R_B^T
void make_core_gemms(const TruncState& st, const CoreView& core, int kcap, SmallGemmArgs* out) {
  SmallGemm j2[2];
  for (int x = 0; x < 2; ++x) j2[x] = SmallGemm{st.R2[x], st.R1[x], st.G[x], nullptr, nullptr, nullptr, 0, 0, 0};
  out[0] = make_small_gemm(j2, 2, core, st.k, kcap);
  SmallGemm jm{st.G[0], st.G[1], st.M, nullptr, nullptr, nullptr, 0, 1, 1};
  out[1] = make_small_gemm(&jm, 1, core, st.k, kcap);
}

// U_M = Q Y (into st.W); after the selection XA = R2i_A U_M[:, order],
// XB = R2i_B V_M[:, order] (unit columns: no scaling)
void make_finish_gemms(const TruncState& st, int kcap, const int* rank_out, SmallGemmArgs* out) {
  CoreView none{};
  none.nb = 0;
  SmallGemm ju{st.H, st.VM, st.W, nullptr, nullptr, st.kj, 0, 0, 0, nullptr, st.kj};
  out[0] = make_small_gemm(&ju, 1, none, st.k, kcap);
  SmallGemm jx[2];
  jx[0] = SmallGemm{st.R2i[0], st.W, st.XA, st.order, nullptr, rank_out, 0, 0, 0};
  jx[1] = SmallGemm{st.R2i[1], st.VP, st.XB, st.order, nullptr, rank_out, 0, 0, 0};
  out[1] = make_small_gemm(jx, 2, none, st.k, kcap);
}

// ============================================================== rank selection
// sigma from the Jacobi kernel; order by decreasing sigma;
// r' = min(cap, smallest r with tail <= max(tol * ||sigma||, abs_tol)).
constexpr int kSelThreads = 256;
__global__ __launch_bounds__(kSelThreads) void select_kernel(SelArgs a0, const SelArgs* ab,
                                                             const int* done) {
  LRC_ITEM(SelArgs, sa_, a0, ab, done)
  const TruncState& st = sa_.st;
  const int rank_cap = sa_.rank_cap;
  const double tol = sa_.tol;
  double* s_out = sa_.s_out;
  int* rank_out = sa_.rank_out;
  double* norm_out = sa_.norm_out;
  __shared__ double sig[SK];
  __shared__ double srt[SK];
  __shared__ int ord[SK];
  __shared__ int rsel;
  const int k = *st.kj;          // candidate singular directions
  const int tid = threadIdx.x;
  for (int j = tid; j < k; j += blockDim.x) sig[j] = st.lam[j];
  __syncthreads();
  for (int j = tid; j < k; j += blockDim.x) {
    int pos = 0;
    const double sj = sig[j];
    for (int i = 0; i < k; ++i) {
      const double si = sig[i];
      if (si > sj || (si == sj && i < j)) ++pos;
    }
    ord[pos] = j;
    srt[pos] = sj;
  }
  __syncthreads();
  if (tid == 0) {
    double tot = 0.0;
    for (int j = k - 1; j >= 0; --j) tot += srt[j] * srt[j];
    const double total = sqrt(tot);
    int r = 0;
    if (total > 0.0) {
      // smallest r with sqrt(sum_{j >= r} s_j^2) <= max(tol * total, abs_tol)
      r = k;
      double tail = 0.0;
      const double lim = fmax(tol * total, sa_.abs_tol);
      for (int j = k - 1; j >= 0; --j) {
        const double t2 = tail + srt[j] * srt[j];
        if (sqrt(t2) <= lim) { tail = t2; r = j; }
        else break;
      }
    }
    r = min(r, rank_cap);
    rsel = r;
    *rank_out = r;
    *norm_out = total;
  }
  __syncthreads();
  const int r = rsel;
  for (int j = tid; j < k; j += blockDim.x) {
    st.order[j] = ord[j];
    if (j < r) s_out[j] = srt[j];
  }
}

void enqueue_select(const SelArgs& a, Batched<SelArgs> b, hipStream_t s) {
  ProfScope ps(kcls(K_SELECT, false), s);
  hipLaunchKernelGGL(select_kernel, dim3(1, 1, b.n), dim3(kSelThreads), 0, s, a, b.dev, b.done);
  LRC_HIP(hipGetLastError());
}

// ============================================================== batch control
__global__ __launch_bounds__(64) void batch_check_kernel(BCtl* __restrict__ ctl,
                                                        int* __restrict__ done, int nb,
                                                        int after_update) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nb || done[j]) return;
  BCtl c = ctl[j];
  const double nr = *c.norm;
  c.last = nr;
  if (after_update) {
    ++c.iters;
    if (nr < 0.7 * c.best) {
      c.best = nr;
      c.stall = 0;
    } else {
      c.best = fmin(c.best, nr);
      ++c.stall;
    }
  } else {
    c.best = nr;
    c.stall = 0;
  }
  if (!isfinite(nr)) c.state = 2;
  else if (nr <= c.target) c.state = 1;
  else if (c.iters >= c.max_iter || c.stall >= c.stall_limit) c.state = 2;
  ctl[j] = c;
  if (c.state) done[j] = 1;
}

void launch_batch_check(BCtl* ctl, int* done, int nb, int after_update, hipStream_t s) {
  ProfScope ps(K_VECTOR * 2, s);
  hipLaunchKernelGGL(batch_check_kernel, dim3(unsigned(ceil_div(nb, 64))), dim3(64), 0, s, ctl,
                     done, nb, after_update);
  LRC_HIP(hipGetLastError());
}

}  // namespace lrc
