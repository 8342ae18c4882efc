// Small fp64 kernels of the truncation (k x k with k <= 128): equilibrated,
// shift-guarded Cholesky of a Gram matrix with the inverse of its factor,
// small matrix products, the symmetric eigen-decomposition of the core's Gram
// by parallel two-sided Jacobi (rotations logged, then replayed per row), and
// the rank selection.
#include <algorithm>

#include "kernels.hpp"
#include "prof.hpp"

namespace lrc {

constexpr int SK = 128;                         // capacity of the small kernels
constexpr int SKP = SK * (SK + 1) / 2;          // packed upper triangle

__device__ inline int pk(int i, int j, int k) {  // packed upper by rows, i <= j
  return i * k - (i * (i - 1)) / 2 + (j - i);
}

// ============================================================== Cholesky + inverse
// One workgroup per side (A, B).  G is equilibrated (unit diagonal), factorised
// G_s = R^T R; a failed pivot restarts with a diagonal shift; columns whose
// Gram diagonal vanishes are treated as absent.  Outputs (ld = kcap):
//   Rout = R D^{-1}   (so that X = Q Rout),  Tout = D R^{-1}  (so that Q = X Tout).
__global__ __launch_bounds__(256) void chol_kernel(TruncState st, int pass, int kcap,
                                                   double eps) {
  __shared__ double Rp[SKP];
  __shared__ double Xp[SKP];
  __shared__ double Wt[(SK / 16) * 256];
  __shared__ double dsc[SK];
  __shared__ int fail;
  const int side = blockIdx.x;
  const int k = *st.k;
  const double* G = st.G[side];
  double* Rout = pass == 1 ? st.R1[side] : st.R2[side];
  double* Tout = pass == 1 ? st.T1[side] : st.R2i[side];
  const int tid = threadIdx.x, nt = blockDim.x;
  if (k == 0) return;
  // equilibration
  __shared__ double gmax;
  if (tid == 0) {
    double m = 0.0;
    for (int j = 0; j < k; ++j) m = fmax(m, G[size_t(j) * kcap + j]);
    gmax = m;
  }
  __syncthreads();
  for (int j = tid; j < k; j += nt) {
    const double g = G[size_t(j) * kcap + j];
    dsc[j] = (g > 1e-300 && g > 1e-28 * gmax) ? 1.0 / sqrt(g) : 0.0;
  }
  __syncthreads();
  double shift = 0.0;
  const double tau = eps * k;
  for (int attempt = 0; attempt < 6; ++attempt) {
    for (int e = tid; e < k * k; e += nt) {
      const int i = e / k, j = e - i * k;
      if (j < i) continue;
      double v;
      if (dsc[i] == 0.0 || dsc[j] == 0.0) v = (i == j) ? 1.0 : 0.0;
      else v = dsc[i] * G[size_t(i) * kcap + j] * dsc[j] + (i == j ? shift : 0.0);
      Rp[pk(i, j, k)] = v;
    }
    if (tid == 0) fail = 0;
    __syncthreads();
    for (int j = 0; j < k; ++j) {
      if (tid == 0) {
        const double p = Rp[pk(j, j, k)];
        if (!(p > tau)) fail = 1;
        else Rp[pk(j, j, k)] = sqrt(p);
      }
      __syncthreads();
      if (fail) break;
      const double rjj = Rp[pk(j, j, k)];
      for (int c = j + 1 + tid; c < k; c += nt) Rp[pk(j, c, k)] /= rjj;
      __syncthreads();
      // trailing update, 16 x 16 thread grid over (row a, column b >= a)
      {
        const int ty = tid >> 4, tx = tid & 15;
        for (int a = j + 1 + ty; a < k; a += 16) {
          const double rja = Rp[pk(j, a, k)];
          const int base = pk(a, 0, k);            // row a starts at base + a
          for (int b = a + tx; b < k; b += 16) Rp[base + b] -= rja * Rp[pk(j, b, k)];
        }
      }
      __syncthreads();
    }
    if (!fail) break;
    shift = (shift == 0.0) ? 10.0 * tau : shift * 100.0;
    if (tid == 0) atomicOr(st.info, 1);
    __syncthreads();
  }
  if (fail) {
    // give up on factorising: identity factor (the truncation then works on the
    // equilibrated columns as they are) and report the breakdown
    for (int e = tid; e < k * k; e += nt) {
      const int i = e / k, j = e - i * k;
      if (j >= i) Rp[pk(i, j, k)] = (i == j) ? 1.0 : 0.0;
    }
    if (tid == 0) atomicOr(st.info, 2);
    __syncthreads();
  }
  // Rout = R D^{-1}
  for (int e = tid; e < kcap * kcap; e += nt) {
    const int i = e / kcap, j = e - i * kcap;
    double v = 0.0;
    if (i < k && j < k && j >= i && dsc[j] != 0.0) v = Rp[pk(i, j, k)] / dsc[j];
    Rout[e] = v;
  }
  // blocked inverse of the upper-triangular R (16 x 16 blocks)
  const int nbk = (k + 15) / 16;
  for (int t = tid; t < nbk * 16; t += nt) {
    const int I = t / 16, J = t;                 // column J inside diagonal block I
    if (J >= k) continue;
    const int lo = I * 16;
    for (int i = J; i >= lo; --i) {
      double s = (i == J) ? 1.0 : 0.0;
      for (int p = i + 1; p <= J; ++p) s -= Rp[pk(i, p, k)] * Xp[pk(p, J, k)];
      Xp[pk(i, J, k)] = s / Rp[pk(i, i, k)];
    }
  }
  __syncthreads();
  for (int d = 1; d < nbk; ++d) {
    const int npairs = nbk - d;
    // W_IJ = sum_{r in blocks I+1..J} R[I][r] X[r][J]
    for (int e = tid; e < npairs * 256; e += nt) {
      const int I = e / 256, w = e & 255, J = I + d;
      const int i = I * 16 + w / 16, j = J * 16 + (w & 15);
      double s = 0.0;
      if (i < k && j < k)
        for (int r = (I + 1) * 16; r <= j; ++r) s += Rp[pk(i, r, k)] * Xp[pk(r, j, k)];
      Wt[e] = s;
    }
    __syncthreads();
    // X_IJ = -X_II W_IJ
    for (int e = tid; e < npairs * 256; e += nt) {
      const int I = e / 256, w = e & 255, J = I + d;
      const int ii = w / 16, jj = w & 15;
      const int i = I * 16 + ii, j = J * 16 + jj;
      if (i >= k || j >= k) continue;
      double s = 0.0;
      for (int q = ii; q < 16 && I * 16 + q < k; ++q)
        s -= Xp[pk(i, I * 16 + q, k)] * Wt[I * 256 + q * 16 + jj];
      Xp[pk(i, j, k)] = s;
    }
    __syncthreads();
  }
  // Tout = D R^{-1}
  for (int e = tid; e < kcap * kcap; e += nt) {
    const int i = e / kcap, j = e - i * kcap;
    double v = 0.0;
    if (i < k && j < k && j >= i) v = dsc[i] * Xp[pk(i, j, k)];
    Tout[e] = v;
  }
}

void launch_chol(TruncState st, int pass, int kcap, double eps_gram, hipStream_t s) {
  LRC_CHECK(kcap <= SK, ST_EINVAL, "truncation: at most 128 concatenated columns");
  ProfScope ps(kcls(K_CHOL, false), s);
  hipLaunchKernelGGL(chol_kernel, dim3(2), dim3(256), 0, s, st, pass, kcap, eps_gram);
  LRC_HIP(hipGetLastError());
}

// ============================================================== small products
// C = op(A) diag(mid) op(B)[:, colperm] diag(colscale), all k x k (or k x r
// output columns), fp64, ld kcap.  One 16 x 16 output tile per workgroup.
struct SmallGemm {
  const double* A;
  const double* B;
  double* C;
  const int* colperm;        // optional
  const double* colscale;    // optional (per output column)
  const int* ncols_dev;      // optional: output columns (default k)
  int transA, transB;
  int use_core;              // mid = core coefficients
};

struct SmallGemmArgs {
  SmallGemm g[2];
  CoreView core;
  const int* k;
  int kcap;
};

__global__ __launch_bounds__(256) void small_gemm_kernel(SmallGemmArgs a) {
  __shared__ double As[16][17];
  __shared__ double Bs[16][17];
  __shared__ double mid[SK];
  const SmallGemm& g = a.g[blockIdx.z];
  const int k = *a.k;
  const int ncols = g.ncols_dev ? *g.ncols_dev : k;
  const int ti = blockIdx.y * 16, tj = blockIdx.x * 16;
  if (ti >= k || tj >= ncols) return;
  if (g.use_core) {
    int off = 0;
    for (int b = 0; b < a.core.nb; ++b) {
      const int w = core_width(a.core, b);
      for (int c = threadIdx.x; c < w && off + c < SK; c += blockDim.x)
        mid[off + c] = a.core.coef[b] * (a.core.s[b] ? a.core.s[b][c] : 1.0);
      off += w;
    }
  }
  const int li = threadIdx.x / 16, lj = threadIdx.x & 15;
  const int i = ti + li, j = tj + lj;
  const int jc = (j < ncols) ? (g.colperm ? g.colperm[j] : j) : 0;
  double acc = 0.0;
  for (int p0 = 0; p0 < k; p0 += 16) {
    __syncthreads();
    {
      const int p = p0 + lj;
      double v = 0.0;
      if (i < k && p < k) v = g.transA ? g.A[size_t(p) * a.kcap + i] : g.A[size_t(i) * a.kcap + p];
      As[li][lj] = v;
      const int pb = p0 + li;
      double w = 0.0;
      if (pb < k && j < ncols) w = g.transB ? g.B[size_t(jc) * a.kcap + pb] : g.B[size_t(pb) * a.kcap + jc];
      if (g.use_core && pb < k) w *= mid[pb];
      Bs[li][lj] = w;
    }
    __syncthreads();
#pragma unroll
    for (int p = 0; p < 16; ++p) acc += As[li][p] * Bs[p][lj];
  }
  if (i < k && j < ncols) {
    if (g.colscale) acc *= g.colscale[j];
    g.C[size_t(i) * a.kcap + j] = acc;
  }
}

static void small_gemm(const SmallGemm* jobs, int njobs, CoreView core, const int* k, int kcap,
                       hipStream_t s) {
  SmallGemmArgs a;
  a.g[0] = jobs[0];
  a.g[1] = njobs > 1 ? jobs[1] : jobs[0];
  a.core = core;
  a.k = k;
  a.kcap = kcap;
  const int t = (kcap + 15) / 16;
  ProfScope ps(kcls(K_SMALL_GEMM, false), s);
  hipLaunchKernelGGL(small_gemm_kernel, dim3(t, t, njobs), dim3(256), 0, s, a);
}

// ============================================================== Jacobi
// Round-robin ("tournament") pairing of kp (even) indices: in round t, slot a
// pairs positions a and kp-1-a of the rotated list [0, 1 + (t + i) mod (kp-1)].
__device__ inline int rr_player(int pos, int t, int kp) {
  if (pos == 0) return 0;
  return 1 + (pos - 1 + t) % (kp - 1);
}

// Two-sided Jacobi on the symmetric H (k x k, padded to even kp with a zero
// row/column), stored in full in LDS (both triangles kept equal).  Every round
// applies kp/2 disjoint rotations H <- J^T H J; the (c, s) of each round are
// logged so that V = prod J can be rebuilt per row.
constexpr int kJL = SK + 1;   // LDS row pitch of H (odd: fewer bank conflicts)
__global__ __launch_bounds__(1024) void jacobi_kernel(TruncState st, int kcap, int max_rounds) {
  __shared__ double Hs[SK * kJL];
  __shared__ double cs_c[SK / 2], cs_s[SK / 2];
  __shared__ unsigned char pp[SK / 2], qq[SK / 2];                 // pair a = (pp[a], qq[a])
  __shared__ int nrot, rrot;
  const int k = *st.k;
  const int kp = k + (k & 1);
  const int tid = threadIdx.x, nt = blockDim.x;
  if (k <= 1) {
    if (tid == 0) *st.rounds = 0;
    return;
  }
  for (int e = tid; e < kp * kp; e += nt) {
    const int i = e / kp, j = e - i * kp;
    Hs[i * kJL + j] = (i < k && j < k) ? st.H[size_t(i) * kcap + j] : 0.0;
  }
  const int npair = kp / 2;
  __syncthreads();
  // Off-diagonal entries below 1e-16 * trace(H) are rounding noise of the
  // squared core and are not rotated; the eigenvalues are then accurate to
  // that absolute level (singular values to ~1e-8 of the largest).
  __shared__ double hscale;
  if (tid == 0) {
    double tr = 0.0;
    for (int i = 0; i < k; ++i) tr += fabs(Hs[i * kJL + i]);
    hscale = 1e-16 * tr;
  }
  __syncthreads();
  const double floor_abs = hscale;
  // thread layout of the update phase: 16 threads per pair a (one per column
  // group), each sweeping the columns j of rows pp[a], qq[a]
  int round = 0;
  for (int sweep = 0; sweep < 30 && round < max_rounds; ++sweep) {
    if (tid == 0) nrot = 0;
    __syncthreads();
    for (int t = 0; t < kp - 1 && round < max_rounds; ++t, ++round) {
      if (tid == 0) rrot = 0;
      __syncthreads();
      if (tid < npair) {
        // pair slot tid of round t: positions tid and kp-1-tid of the rotated list
        const int x0 = tid == 0 ? 0 : 1 + (tid - 1 + t) % (kp - 1);
        const int x1 = 1 + (kp - 2 - tid + t) % (kp - 1);
        const int p = min(x0, x1), q = max(x0, x1);
        pp[tid] = (unsigned char)p;
        qq[tid] = (unsigned char)q;
        const double hpp = Hs[p * kJL + p], hqq = Hs[q * kJL + q], hpq = Hs[p * kJL + q];
        double c = 1.0, s = 0.0;
        if (fabs(hpq) > floor_abs) {
          const double zeta = (hqq - hpp) / (2.0 * hpq);
          const double tt = (zeta >= 0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          c = 1.0 / sqrt(1.0 + tt * tt);
          s = c * tt;
          atomicAdd(&rrot, 1);
        }
        cs_c[tid] = c;
        cs_s[tid] = s;
        st.rot[(size_t(round) * (SK / 2) + tid) * 2 + 0] = c;
        st.rot[(size_t(round) * (SK / 2) + tid) * 2 + 1] = s;
      }
      __syncthreads();
      if (rrot == 0) continue;          // nothing rotated in this round
      if (tid == 0) nrot += rrot;
      // H <- J^T H (rows), then H <- H J (columns), done as one pass over the
      // 2 x 2 blocks (pair a, pair b): each block is owned by one thread.
      for (int e = tid; e < npair * npair; e += nt) {
        const int a = e / npair, b = e - a * npair;
        const double ca = cs_c[a], sa = cs_s[a], cb = cs_c[b], sb = cs_s[b];
        if (sa == 0.0 && sb == 0.0) continue;
        const int pa = pp[a], qa = qq[a], pb = pp[b], qb = qq[b];
        const double h00 = Hs[pa * kJL + pb], h01 = Hs[pa * kJL + qb];
        const double h10 = Hs[qa * kJL + pb], h11 = Hs[qa * kJL + qb];
        const double l00 = ca * h00 - sa * h10, l01 = ca * h01 - sa * h11;
        const double l10 = sa * h00 + ca * h10, l11 = sa * h01 + ca * h11;
        double r00 = cb * l00 - sb * l01, r01 = sb * l00 + cb * l01;
        double r10 = cb * l10 - sb * l11, r11 = sb * l10 + cb * l11;
        if (a == b) r01 = r10 = 0.0;      // the rotated pair is diagonalised
        Hs[pa * kJL + pb] = r00;
        Hs[pa * kJL + qb] = r01;
        Hs[qa * kJL + pb] = r10;
        Hs[qa * kJL + qb] = r11;
      }
      __syncthreads();
    }
    __syncthreads();
    if (nrot == 0) break;
    __syncthreads();
  }
  if (tid == 0) {
    *st.rounds = round;
    if (nrot != 0) atomicOr(st.info, 4);
  }
}

// V = J_0 J_1 ... J_{T-1}: every row of V evolves independently.  A workgroup
// (one wave) owns kRepRows rows; lane a applies pair a's rotation to them.  The
// rotation log is staged through LDS in batches of kRepBatch rounds.
constexpr int kRepRows = 4;
constexpr int kRepBatch = 16;
__global__ __launch_bounds__(64) void jacobi_replay_kernel(TruncState st, int kcap) {
  __shared__ double row[kRepRows][SK];
  __shared__ double2 rb[kRepBatch][SK / 2];
  const int k = *st.k;
  const int kp = k + (k & 1);
  const int i0 = blockIdx.x * kRepRows;
  if (i0 >= k) return;
  const int T = *st.rounds;
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

void launch_jacobi_replay(TruncState st, int kcap, hipStream_t s) {
  ProfScope ps(kcls(K_REPLAY, false), s);
  hipLaunchKernelGGL(jacobi_replay_kernel, dim3((kcap + kRepRows - 1) / kRepRows), dim3(64), 0, s,
                     st, kcap);
  LRC_HIP(hipGetLastError());
}

// ============================================================== core + Jacobi
// R_A = R2_A R1_A, R_B = R2_B R1_B;  M = R_A diag(core) R_B^T;  H = M^T M;
// then the Jacobi rounds.  Scratch: R1 buffers are overwritten by R_A, R_B.
void launch_core_jacobi(TruncState st, CoreView core, int kcap, int max_rounds, hipStream_t s) {
  LRC_CHECK(kcap <= SK, ST_EINVAL, "truncation: at most 128 concatenated columns");
  // R_A, R_B into the G buffers (the Grams are no longer needed)
  SmallGemm j2[2];
  for (int x = 0; x < 2; ++x) {
    j2[x] = SmallGemm{st.R2[x], st.R1[x], st.G[x], nullptr, nullptr, nullptr, 0, 0, 0};
  }
  small_gemm(j2, 2, core, st.k, kcap, s);
  // M = R_A diag(core) R_B^T
  SmallGemm jm{st.G[0], st.G[1], st.M, nullptr, nullptr, nullptr, 0, 1, 1};
  small_gemm(&jm, 1, core, st.k, kcap, s);
  // H = M^T M
  SmallGemm jh{st.M, st.M, st.H, nullptr, nullptr, nullptr, 1, 0, 0};
  small_gemm(&jh, 1, core, st.k, kcap, s);
  ProfScope ps(kcls(K_JACOBI, false), s);
  hipLaunchKernelGGL(jacobi_kernel, dim3(1), dim3(1024), 0, s, st, kcap, max_rounds);
  LRC_HIP(hipGetLastError());
}

// ============================================================== rank selection
// W = M V (columns: M v_j = sigma_j u_j); sigma_j = ||W[:, j]||; order by
// decreasing sigma; r' = min(cap, smallest r with tail <= tol * ||sigma||).
// Then XA = R2i_A * W[:, order] diag(1/sigma), XB = R2i_B * V[:, order].
__global__ __launch_bounds__(256) void select_kernel(TruncState st, int kcap, int rank_cap,
                                                     double tol, double* s_out, int* rank_out,
                                                     double* norm_out) {
  __shared__ double sig[SK];
  __shared__ double srt[SK];
  __shared__ int ord[SK];
  __shared__ int rsel;
  const int k = *st.k;
  const int tid = threadIdx.x;
  for (int j = tid; j < k; j += blockDim.x) {
    double a = 0.0;
    for (int i = 0; i < k; ++i) {
      const double w = st.W[size_t(i) * kcap + j];
      a += w * w;
    }
    sig[j] = sqrt(a);
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
      // smallest r with sqrt(sum_{j >= r} s_j^2) <= tol * total
      r = k;
      double tail = 0.0;
      for (int j = k - 1; j >= 0; --j) {
        const double t2 = tail + srt[j] * srt[j];
        if (sqrt(t2) <= tol * total) { tail = t2; r = j; }
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
    st.invsig[j] = srt[j] > 0.0 ? 1.0 / srt[j] : 0.0;
    if (j < r) s_out[j] = srt[j];
  }
}

void launch_trunc_finish(TruncState st, int kcap, int rank_cap, double tol, double* s_out,
                         int* rank_out, double* norm_out, hipStream_t s) {
  CoreView none{};
  none.nb = 0;
  SmallGemm jw{st.M, st.VM, st.W, nullptr, nullptr, nullptr, 0, 0, 0};
  small_gemm(&jw, 1, none, st.k, kcap, s);
  {
    ProfScope ps(kcls(K_SELECT, false), s);
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(256), 0, s, st, kcap, rank_cap, tol, s_out,
                       rank_out, norm_out);
  }
  // XA = R2i_A W[:, order] diag(1 / sigma),  XB = R2i_B V[:, order]
  SmallGemm jx[2];
  jx[0] = SmallGemm{st.R2i[0], st.W, st.XA, st.order, st.invsig, rank_out, 0, 0, 0};
  jx[1] = SmallGemm{st.R2i[1], st.VM, st.XB, st.order, nullptr, rank_out, 0, 0, 0};
  small_gemm(jx, 2, none, st.k, kcap, s);
  LRC_HIP(hipGetLastError());
}

}  // namespace lrc
