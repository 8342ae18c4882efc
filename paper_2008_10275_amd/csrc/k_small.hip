// Small fp64 kernels of the truncation (k x k with k <= 128): equilibrated,
// shift-guarded Cholesky of a Gram matrix with the inverse of its factor,
// small matrix products, the symmetric eigen-decomposition of the core's Gram
// by parallel two-sided Jacobi (rotations logged, then replayed per row), and
// the rank selection.
#include <algorithm>

#include "kernels.hpp"
#include "prof.hpp"

namespace lrc {

// Batched launches: item = blockIdx.z; a done item does nothing.
#define LRC_ITEM(Type, name, a0, ab, done)        \
  if ((done) && (done)[blockIdx.z]) return;        \
  const Type& name = (ab) ? (ab)[blockIdx.z] : (a0);

constexpr int SK = 128;                         // capacity of the small kernels
constexpr int SKP = SK * (SK + 1) / 2;          // packed upper triangle


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
__device__ inline int pu(int i, int j, int k) {   // packed upper by rows, i <= j
  return i * k - (i * (i - 1)) / 2 + (j - i);
}

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
  }
  __syncthreads();
  const double tau = eps * k;
  double shift = 0.0;
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

// ============================================================== Jacobi
// Round-robin ("tournament") pairing of kp (even) indices: in round t, slot a
// pairs positions a and kp-1-a of the rotated list [0, 1 + (t + i) mod (kp-1)].
__device__ inline int rr_player(int pos, int t, int kp) {
  if (pos == 0) return 0;
  return 1 + (pos - 1 + t) % (kp - 1);
}

// Two-sided Jacobi on the symmetric H (k x k, padded to even kp with a zero
// row/column).  H is kept as its packed upper triangle, twice: every round
// reads one copy and writes the rotated matrix H <- J^T H J into the other,
// so a single barrier per round separates the rounds.  A round applies kp/2
// disjoint rotations; each wave computes all of them itself from the copy it
// reads (no broadcast), and the 2 x 2 blocks (pair a, pair b), a <= b, are
// rotated once each (the lower triangle is the same storage).  Rounds without
// a rotation (the same decision in every wave) are skipped.  Up to kJFuse
// the eigenvectors V = prod J accumulate in LDS next to H and are written to
// st.VM (st.rounds = -1 marks this); beyond, the (c, s) of every round are
// logged and V is rebuilt per row by the replay kernel.
constexpr int kJFuse = 88;
constexpr int kJacThreads = 1024;
constexpr int kJacLds = 2 * SKP;            // doubles: two packed copies of H at kp <= 128
static_assert(2 * (kJFuse * (kJFuse + 1) / 2) + kJFuse * (kJFuse + 1) <= kJacLds,
              "fused eigenvectors must fit next to the two packed copies");
__global__ __launch_bounds__(kJacThreads) void jacobi_kernel(JacArgs a0, const JacArgs* ab,
                                                            const int* done) {
  LRC_ITEM(JacArgs, ja_, a0, ab, done)
  const TruncState& st = ja_.st;
  const int kcap = ja_.kcap, max_rounds = ja_.max_rounds;
  __shared__ double lds[kJacLds];
  __shared__ double2 csw[kJacThreads / 64][SK / 2];
  __shared__ short2 pqw[kJacThreads / 64][SK / 2];
  __shared__ double s_floor;
  const int k = *st.kj;
  const int kp = k + (k & 1);
  const bool fuse = k <= kJFuse;
  const int tid = threadIdx.x, nt = blockDim.x, lane = tid & 63, wave = tid >> 6;
  if (k <= 1) {
    if (tid == 0) {
      if (k == 1) {
        st.VM[0] = 1.0;
        st.lam[0] = st.H[0];
      }
      *st.rounds = -1;
    }
    return;
  }
  const int np = kp * (kp + 1) / 2;
  double* Hs[2] = {lds, lds + np};
  double* V = lds + 2 * np;                 // kp x (kp + 1) when fused
  const int P = kp + 1;
  for (int e = tid; e < kp * kp; e += nt) {
    const int i = e / kp, j = e - i * kp;
    if (j >= i) Hs[0][pu(i, j, kp)] = (j < k) ? st.H[size_t(i) * kcap + j] : 0.0;
    if (fuse) V[i * P + j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  // Off-diagonal entries below max(1e-16, 0.01 tol^2) * trace(H) are not
  // rotated: 1e-16 is the rounding noise of the squared core, and a truncation
  // at relative tolerance tol needs the eigenvalues of H = M^T M (squared
  // singular values) to no better than a small fraction of tol^2 * ||M||_F^2.
  if (tid < 64) {
    double tr = 0.0;
    for (int i = tid; i < k; i += 64) tr += fabs(Hs[0][pu(i, i, kp)]);
    for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o);
    if (tid == 0)
      s_floor = fmax(fmax(1e-16, 0.01 * ja_.tol * ja_.tol) * tr, 0.01 * ja_.abs_tol * ja_.abs_tol);
  }
  __syncthreads();
  const double floor_abs = s_floor;
  const int npair = kp / 2;
  const int nblk = npair * (npair + 1) / 2;     // <= 2080: at most 3 blocks per thread
  // this thread's blocks (pair a, pair b), a <= b, in row-major order of the
  // upper triangle of the pair grid
  int ba[3], bb[3], nmy = 0;
  for (int e = tid; e < nblk; e += nt) {
    int a = 0, rem = e;
    while (rem >= npair - a) { rem -= npair - a; ++a; }
    ba[nmy] = a;
    bb[nmy] = a + rem;
    ++nmy;
  }
  int round = 0, cur = 0;
  bool converged = false;
  for (int sweep = 0; sweep < 30 && round < max_rounds; ++sweep) {
    int nrot = 0;
    // pair slot `lane` of round t: positions lane and kp-1-lane of the rotated
    // list [0, 1 + (t + i) mod (kp - 1)]; the residues advance by one a round
    int c0 = lane == 0 ? 0 : lane - 1, c1 = kp - 2 - lane;
    for (int t = 0; t < kp - 1 && round < max_rounds; ++t, ++round) {
      const double* H = Hs[cur];
      double* Hn = Hs[cur ^ 1];
      bool rot = false;
      const int x0 = lane == 0 ? 0 : 1 + c0, x1 = 1 + c1;
      c0 = c0 + 1 == kp - 1 ? 0 : c0 + 1;
      c1 = c1 + 1 == kp - 1 ? 0 : c1 + 1;
      if (lane < npair) {
        const int p = min(x0, x1), q = max(x0, x1);
        const double hpp = H[pu(p, p, kp)], hqq = H[pu(q, q, kp)], hpq = H[pu(p, q, kp)];
        double c = 1.0, sn = 0.0;
        if (fabs(hpq) > floor_abs) {
          // the rotation of angle |theta| <= pi/4 with tan 2 theta = 2 h_pq / (h_qq - h_pp),
          // from the half-angle formulas: cos 2 theta = |d| / rho >= 0,
          // sin 2 theta = sign(d) e / rho, c = sqrt((1 + cos 2 theta) / 2),
          // s = sin 2 theta / (2 c)  (two reciprocal square roots, no division)
          const double d = hqq - hpp, e = 2.0 * hpq;
          const double ri = rsqrt(fma(d, d, e * e));
          const double c2 = fabs(d) * ri, s2 = (d >= 0.0 ? e : -e) * ri;
          const double h = 0.5 + 0.5 * c2;
          const double hi = rsqrt(h);
          c = h * hi;
          sn = 0.5 * s2 * hi;
          rot = true;
        }
        csw[wave][lane] = make_double2(c, sn);
        pqw[wave][lane] = make_short2(short(p), short(q));
        if (!fuse && wave == 0) {
          st.rot[(size_t(round) * (SK / 2) + lane) * 2 + 0] = c;
          st.rot[(size_t(round) * (SK / 2) + lane) * 2 + 1] = sn;
        }
      }
      const int rr = __popcll(__ballot(rot));
      if (rr == 0) continue;          // H unchanged: no update, no barrier
      nrot += rr;
      // Hn <- J^T H J over the blocks (pair a, pair b), a <= b
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        if (u >= nmy) break;
        const int a = ba[u], b = bb[u];
        const double2 ja = csw[wave][a], jb = csw[wave][b];
        const short2 qa2 = pqw[wave][a], qb2 = pqw[wave][b];
        const int pa = qa2.x, qa = qa2.y, pb = qb2.x, qb = qb2.y;
        auto at = [&](int x, int y) { return x <= y ? pu(x, y, kp) : pu(y, x, kp); };
        const int i00 = at(pa, pb), i01 = at(pa, qb), i10 = at(qa, pb), i11 = at(qa, qb);
        const double h00 = H[i00], h01 = H[i01], h10 = H[i10], h11 = H[i11];
        const double l00 = ja.x * h00 - ja.y * h10, l01 = ja.x * h01 - ja.y * h11;
        const double l10 = ja.y * h00 + ja.x * h10, l11 = ja.y * h01 + ja.x * h11;
        double r00 = jb.x * l00 - jb.y * l01, r01 = jb.y * l00 + jb.x * l01;
        double r10 = jb.x * l10 - jb.y * l11, r11 = jb.y * l10 + jb.x * l11;
        if (a == b && ja.y != 0.0) r01 = r10 = 0.0;   // the rotated pair is diagonalised
        Hn[i00] = r00;
        Hn[i01] = r01;
        Hn[i11] = r11;
        if (a != b) Hn[i10] = r10;        // a == b: (qa, pa) is (pa, qa)'s storage
      }
      if (fuse) {
        // V <- V J: columns (p_a, q_a) of every row
        for (int e = tid; e < kp * npair; e += nt) {
          const int i = e / npair, a = e - i * npair;
          const double2 ja = csw[wave][a];
          if (ja.y == 0.0) continue;
          const short2 q2 = pqw[wave][a];
          const double vp = V[i * P + q2.x], vq = V[i * P + q2.y];
          V[i * P + q2.x] = ja.x * vp - ja.y * vq;
          V[i * P + q2.y] = ja.y * vp + ja.x * vq;
        }
      }
      cur ^= 1;
      __syncthreads();
    }
    if (nrot == 0) { converged = true; break; }
  }
  const double* H = Hs[cur];
  if (fuse) {
    for (int e = tid; e < k * k; e += nt) {
      const int i = e / k, j = e - i * k;
      st.VM[size_t(i) * kcap + j] = V[i * P + j];
    }
  }
  for (int j = tid; j < k; j += nt) st.lam[j] = H[pu(j, j, kp)];
  if (tid == 0) {
    *st.rounds = fuse ? -1 : round;
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

constexpr int kJL = SK + 1;   // row stride of full k x k matrices in LDS

// ============================================================== pivoted Cholesky
// Diagonally pivoted Cholesky of H = M^T M:  Pi^T H Pi = R^T R, stopped once
// the trace of the remaining Schur complement (the energy of the directions
// left out) is below max(1e-16, (tol / 10)^2) trace(H): the rounding level of
// H, or 1% of the truncation's tail budget if that is larger.  With tol = 0
// every positive pivot is kept.  The rank kj it reveals is the dimension of
// the eigenproblem solved next, on R R^T, whose eigenvectors Y give H's as
// Pi R^T Y.  R R^T is close to diagonal after pivoting, so far fewer Jacobi
// sweeps are needed than on H itself.
// Pivoting is logical: the trailing matrix stays indexed by the original
// columns (a step updates the entries of the columns not yet chosen), rows of
// R are first written by original column to st.VP, and R R^T (which does not
// depend on the column order) is formed from those rows.  Two barriers per
// step.  Outputs: R (kj x k, upper trapezoidal in pivot order, zero rows below
// kj) in st.W, R R^T (kj x kj) in st.H, the pivot order in st.piv, kj in st.kj.
constexpr int kPivThreads = 1024;
__global__ __launch_bounds__(kPivThreads) void pivchol_kernel(PivArgs a0, const PivArgs* ab,
                                                              const int* done) {
  LRC_ITEM(PivArgs, pa_, a0, ab, done)
  const TruncState& st = pa_.st;
  const int kcap = pa_.kcap;
  const double tol = pa_.tol;
  __shared__ double A[SK * kJL];
  __shared__ double dg[SK];
  __shared__ int pos[SK];
  __shared__ unsigned char rem[SK];
  __shared__ int s_p, s_stop;
  __shared__ double s_thr;
  const int k = *st.k;
  const int tid = threadIdx.x, nt = blockDim.x;
  double* Ro = st.VP;   // rows of R by original column (scratch)
  for (int e = tid; e < k * k; e += nt) {
    const int i = e / k, j = e - i * k;
    A[i * kJL + j] = st.H[size_t(i) * kcap + j];
  }
  for (int i = tid; i < k; i += nt) {
    dg[i] = st.H[size_t(i) * kcap + i];
    rem[i] = 1;
  }
  __syncthreads();
  if (tid < 64) {
    double tr = 0.0;
    for (int i = tid; i < k; i += 64) tr += fabs(dg[i]);
    for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o);
    // 1% of the tail budget (relative, or absolute when that is larger)
    if (tid == 0)
      s_thr = fmax(tol > 0.0 ? fmax(1e-16, 0.01 * tol * tol) * tr : 0.0,
                   0.01 * pa_.abs_tol * pa_.abs_tol);
  }
  int r = k;
  for (int j = 0; j < k; ++j) {
    if (tid < 64) {
      double best = -1.0, sum = 0.0;
      int bi = k;
      for (int i = tid; i < k; i += 64) {
        if (!rem[i]) continue;
        const double v = dg[i];
        sum += v;
        if (v > best || (v == best && i < bi)) { best = v; bi = i; }
      }
      for (int o = 32; o > 0; o >>= 1) {
        sum += __shfl_xor(sum, o);
        const double ob = __shfl_xor(best, o);
        const int oi = __shfl_xor(bi, o);
        if (ob > best || (ob == best && oi < bi)) { best = ob; bi = oi; }
      }
      if (tid == 0) {
        const bool stop = !(sum > s_thr) || !(best > 0.0) || bi >= k;
        s_stop = stop ? 1 : 0;
        s_p = bi;
        if (!stop) {
          pos[j] = bi;
          rem[bi] = 0;
        }
      }
    }
    __syncthreads();
    if (s_stop) { r = j; break; }
    const int p = s_p;
    const double d = dg[p];
    const double inv = 1.0 / sqrt(d);
    // row j of R by original column: R[j][p] = sqrt(d), R[j][x] = A[p][x] / sqrt(d)
    // for columns not chosen yet, 0 for those chosen before
    for (int x = tid; x < k; x += nt)
      Ro[size_t(j) * kcap + x] = x == p ? d * inv : (rem[x] ? A[p * kJL + x] * inv : 0.0);
    // trailing update of the remaining columns (row p is only read)
    const double id = 1.0 / d;
    for (int e = tid; e < k * k; e += nt) {
      const int x = e / k, y = e - x * k;
      if (!rem[x] || !rem[y]) continue;
      const double v = A[x * kJL + y] - A[p * kJL + x] * A[p * kJL + y] * id;
      A[x * kJL + y] = v;
      if (x == y) dg[x] = v;
    }
    __syncthreads();
  }
  // the columns never chosen follow in original order
  if (tid == 0) {
    int q = r;
    for (int x = 0; x < k; ++x)
      if (rem[x]) pos[q++] = x;
  }
  __syncthreads();
  // R in pivot order, and R R^T from the rows by original column (staged in LDS)
  for (int e = tid; e < k * k; e += nt) {
    const int a = e / k, c = e - a * k;
    const double v = (a < r && c >= a) ? Ro[size_t(a) * kcap + pos[c]] : 0.0;
    st.W[size_t(a) * kcap + c] = v;
    A[a * kJL + c] = a < r ? Ro[size_t(a) * kcap + c] : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < r * r; e += nt) {
    const int a = e / r, b = e - a * r;
    if (b < a) continue;
    double acc = 0.0;
    for (int x = 0; x < k; ++x) acc += A[a * kJL + x] * A[b * kJL + x];
    st.H[size_t(a) * kcap + b] = acc;
    st.H[size_t(b) * kcap + a] = acc;
  }
  for (int i = tid; i < k; i += nt) st.piv[i] = pos[i];
  if (tid == 0) *st.kj = r;
}

// ============================================================== core + Jacobi
// R_A = R2_A R1_A, R_B = R2_B R1_B;  M = R_A diag(core) R_B^T;  H = M^T M;
// pivoted Cholesky of H, then the Jacobi rounds on R R^T.  Scratch: R1
// buffers are overwritten by R_A, R_B; H by R R^T.
void enqueue_pivchol(const PivArgs& a, Batched<PivArgs> b, hipStream_t s) {
  LRC_CHECK(a.kcap <= SK, ST_EINVAL, "truncation: at most 128 concatenated columns");
  ProfScope ps(kcls(K_PIVCHOL, false), s);
  hipLaunchKernelGGL(pivchol_kernel, dim3(1, 1, b.n), dim3(kPivThreads), 0, s, a, b.dev, b.done);
  LRC_HIP(hipGetLastError());
}

void enqueue_jacobi(const JacArgs& a, Batched<JacArgs> b, hipStream_t s) {
  ProfScope ps(kcls(K_JACOBI, false), s);
  hipLaunchKernelGGL(jacobi_kernel, dim3(1, 1, b.n), dim3(kJacThreads), 0, s, a, b.dev, b.done);
  LRC_HIP(hipGetLastError());
}

// R_A = R2_A R1_A, R_B = R2_B R1_B (into the G buffers); M = R_A diag(core) R_B^T; H = M^T M
void make_core_gemms(const TruncState& st, const CoreView& core, int kcap, SmallGemmArgs* out) {
  SmallGemm j2[2];
  for (int x = 0; x < 2; ++x) j2[x] = SmallGemm{st.R2[x], st.R1[x], st.G[x], nullptr, nullptr, nullptr, 0, 0, 0};
  out[0] = make_small_gemm(j2, 2, core, st.k, kcap);
  SmallGemm jm{st.G[0], st.G[1], st.M, nullptr, nullptr, nullptr, 0, 1, 1};
  out[1] = make_small_gemm(&jm, 1, core, st.k, kcap);
  SmallGemm jh{st.M, st.M, st.H, nullptr, nullptr, nullptr, 1, 0, 0};
  out[2] = make_small_gemm(&jh, 1, core, st.k, kcap);
}

// VP = Pi R^T Y, W = M VP; after the selection XA = R2i_A W[:, order] diag(1 / ||W_j||),
// XB = R2i_B VP[:, order] diag(1 / ||VP_j||)
void make_finish_gemms(const TruncState& st, int kcap, const int* rank_out, SmallGemmArgs* out) {
  CoreView none{};
  none.nb = 0;
  SmallGemm jv{st.W, st.VM, st.VP, nullptr, nullptr, st.kj, 1, 0, 0, st.piv, st.kj};
  out[0] = make_small_gemm(&jv, 1, none, st.k, kcap);
  SmallGemm jw{st.M, st.VP, st.W, nullptr, nullptr, st.kj, 0, 0, 0};
  out[1] = make_small_gemm(&jw, 1, none, st.k, kcap);
  SmallGemm jx[2];
  jx[0] = SmallGemm{st.R2i[0], st.W, st.XA, st.order, st.invsig, rank_out, 0, 0, 0};
  jx[1] = SmallGemm{st.R2i[1], st.VP, st.XB, st.order, st.invnu, rank_out, 0, 0, 0};
  out[2] = make_small_gemm(jx, 2, none, st.k, kcap);
}

// ============================================================== rank selection
// W = M V (columns: M v_j = sigma_j u_j); sigma_j = ||W[:, j]||; order by
// decreasing sigma; r' = min(cap, smallest r with tail <= tol * ||sigma||).
// Then XA = R2i_A * W[:, order] diag(1/sigma), XB = R2i_B * V[:, order].
constexpr int kSelThreads = 1024;
constexpr int kSelRG = kSelThreads / SK;   // row groups of the column norms
__global__ __launch_bounds__(kSelThreads) void select_kernel(SelArgs a0, const SelArgs* ab,
                                                             const int* done) {
  LRC_ITEM(SelArgs, sa_, a0, ab, done)
  const TruncState& st = sa_.st;
  const int kcap = sa_.kcap, rank_cap = sa_.rank_cap;
  const double tol = sa_.tol;
  double* s_out = sa_.s_out;
  int* rank_out = sa_.rank_out;
  double* norm_out = sa_.norm_out;
  __shared__ double sig[SK];
  __shared__ double srt[SK];
  __shared__ int ord[SK];
  __shared__ int rsel;
  __shared__ double om[SK], nu[SK];
  __shared__ double pw[kSelRG][SK], pv[kSelRG][SK];
  __shared__ double s_lfloor;
  const int kr = *st.k;          // rows of W and VP
  const int k = *st.kj;          // candidate singular directions
  const int tid = threadIdx.x;
  if (tid < 64) {
    double tr = 0.0;
    for (int j = tid; j < k; j += 64) tr += fabs(st.lam[j]);
    for (int o = 32; o > 0; o >>= 1) tr += __shfl_xor(tr, o);
    if (tid == 0) s_lfloor = 64.0 * 1e-16 * tr;
  }
  __syncthreads();
  // sigma_j = ||M VP_j|| / ||VP_j|| (= lambda_j / sqrt(lambda_j)) is the more
  // accurate value where lambda_j is well above the Jacobi floor; at the
  // rounding level both norms are noise, and sqrt(lambda_j) is used instead.
  // column norms of W and VP: row group g sums rows g, g + kSelRG, ...; the
  // groups are added in a fixed order
  {
    const int j = tid % SK, grp = tid / SK;
    double a = 0.0, b = 0.0;
    if (j < k)
      for (int i = grp; i < kr; i += kSelRG) {
        const double w = st.W[size_t(i) * kcap + j];
        const double v = st.VP[size_t(i) * kcap + j];
        a += w * w;
        b += v * v;
      }
    pw[grp][j] = a;
    pv[grp][j] = b;
  }
  __syncthreads();
  for (int j = tid; j < k; j += blockDim.x) {
    double a = 0.0, b = 0.0;
#pragma unroll
    for (int g = 0; g < kSelRG; ++g) {
      a += pw[g][j];
      b += pv[g][j];
    }
    om[j] = sqrt(a);
    nu[j] = sqrt(b);
    const double lj = st.lam[j];
    sig[j] = (lj > s_lfloor && nu[j] > 0.0) ? om[j] / nu[j] : sqrt(fmax(lj, 0.0));
  }
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
    const int o = ord[j];
    st.order[j] = o;
    st.invsig[j] = om[o] > 0.0 ? 1.0 / om[o] : 0.0;
    st.invnu[j] = nu[o] > 0.0 ? 1.0 / nu[o] : 0.0;
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
